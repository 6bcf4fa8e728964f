// Batched FP32 Krylov solves of the request server (library-internal).
//
// The request server attaches one KBatcher to the mixed-precision solvers it
// creates.  Their FP32 BiCGSTAB solves (the bulk of a crack-length increment)
// then run in an engine thread that groups the solves in flight by grid
// (one size class per grid) and advances each group by a fixed chunk of
// iterations with batched kernels, replayed from a captured HIP graph; a
// solve joins or leaves its group at chunk boundaries.
#pragma once

#include <cstddef>

struct pff_solver;

namespace pff {

struct KBatcher;

struct KBatcherStats {
  long long chunks;        // chunks launched
  long long rve_chunks;    // sum over chunks of the solves in them
  long long solves;        // solves finished
  long long iterations;    // BiCGSTAB iterations of the finished solves
  long long graphs;        // graphs captured (one per size class and batch size)
  int max_batch;           // largest batch of one chunk
};

// Starts the engine thread on `device`.  bmax: solves per chunk (larger groups
// wait), chunk: iterations per chunk, graph: replay chunks from captured graphs.
KBatcher* kbatcher_create(int device, int bmax, int chunk, int graph);
void kbatcher_destroy(KBatcher* kb);
void kbatcher_stats(KBatcher* kb, KBatcherStats* out);
// Route the FP32 inner solves of s through kb (null: solve on the solver's stream).
void kbatcher_attach(pff_solver* s, KBatcher* kb);
// A solver of the request server keeps the fixed launch shapes: with many
// RVEs on the device at once, the grid-sized shapes of a lone solver (more,
// smaller blocks) measured slower (p50 latency 22.2 against 25.1 s on a
// 64-request stream at 32 slots).
void serving_shapes(pff_solver* s);

}  // namespace pff
