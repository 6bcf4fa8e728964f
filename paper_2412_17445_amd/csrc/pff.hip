// Host driver and C ABI of the crack-length-controlled phase-field FFT solver.
//
// Paper: Aranda & Segurado, Sec. 3.2 and Algorithm 2.  One increment:
//   a <- a + delta_a; Newton from the committed fields; per iteration the
//   FP64 residual pass (constitutive update fused into its first FFT pass),
//   BiCGSTAB on the matrix-free tangent (FFT passes with fused prologue and
//   epilogue), the relaxed update; history committed after convergence.
#include "pff.h"

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <map>
#include <memory>
#include <thread>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <stdexcept>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

#include "batch.hpp"
#include "krylov.hpp"
#include "pipes.hpp"

using namespace pff;

namespace {

struct Fail : std::runtime_error {
  int code;
  Fail(const std::string& m, int c) : std::runtime_error(m), code(c) {}
};

#define HC(expr)                                                                          \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      throw Fail(std::string(#expr) + ": " + hipGetErrorString(e_),                       \
                 e_ == hipErrorOutOfMemory ? PFF_ERR_OOM : PFF_ERR_DEVICE);               \
  } while (0)

#define LAUNCH_CHECK() HC(hipGetLastError())

constexpr size_t kLdsBudget = 64 * 1024;
constexpr uint64_t kShadowSeed = 0x5EED;
constexpr double kDiverged = 1e8;
constexpr int kBisection = 100;
constexpr int kMaxCycles = 8;
constexpr int kNumVec = 13;          // Krylov work vectors
constexpr int kTimSlots = 60;        // pass timing: 6 kernels x 5 apply variants x 2 precisions
constexpr double kInner32 = 5e-2;        // relative residual of each FP32 inner solve (mixed)
constexpr int kMixedMaxit32 = 3000;      // FP32 BiCGSTAB iteration cap per inner solve
constexpr int kMaxRefine = 8;            // FP64 refinement steps per Newton iteration
constexpr double kRefineContract = 0.5;  // a refinement step must at least halve the defect

// device scalar slots
enum {
  SC_SIG = 0,      // 6 sums of sigma
  SC_GAMMA = 6, SC_F1 = 7, SC_F2 = 8,
  SC_NW = 9, SC_NEPS = 10, SC_NDPHI = 11, SC_NPHI = 12,
  SC_ETA = 13,     // 2 slots: ||b - J x||^2, ||b||^2 of the FP64 check
  SC_DISS = 15,    // dissipation: sum of Gc gamma_f
  SC_F3 = 24,      // constraint residual F3 = w_a Gamma + w_E E - tau
  SC_NSIG = 25,    // ||sigma||^2 (Mandel components of the strain unknowns)
  SC_NH2 = 26,     // ||2H||^2
  SC_CG = 16,      // CG scratch (16..23); staggered scheme: [17] max |d eps~|, [18..21] stagger norms
  SC_KS = 32,      // Krylov scalars
  SC_COUNT = 64
};

// Stage plan of one axis: radix 8 stages, then one 4 or 2, then 3s (all with
// unrolled butterflies), then every other prime factor in ascending order
// (generic radix stage).
bool make_plan(int n, AxisPlan& pl) {
  if (n < 1 || n > 512) return false;
  pl.n = n;
  pl.nstage = 0;
  int a = 0, b = 0, m = n;
  while (m % 2 == 0) { m /= 2; ++a; }
  while (m % 3 == 0) { m /= 3; ++b; }
  while (a >= 3) { pl.radix[pl.nstage++] = 8; a -= 3; }
  if (a == 2) pl.radix[pl.nstage++] = 4;
  else if (a == 1) pl.radix[pl.nstage++] = 2;
  for (int i = 0; i < b; ++i) pl.radix[pl.nstage++] = 3;
  for (int p = 5; m > 1; p += 2) {
    while (m % p == 0) {
      if (pl.nstage >= kMaxStages) return false;
      pl.radix[pl.nstage++] = p;
      m /= p;
    }
  }
  if (pl.nstage > kMaxStages) return false;
  pl.dn = make_fastdiv((uint32_t)n);
  int Ns = 1;
  for (int st = 0; st < pl.nstage; ++st) {
    pl.dnb[st] = make_fastdiv((uint32_t)(n / pl.radix[st]));
    pl.dns[st] = make_fastdiv((uint32_t)Ns);
    Ns *= pl.radix[st];
  }
  return true;
}

// A graph under construction: kernel nodes appended in launch order (see launch_k).
struct GraphRec {
  hipGraph_t g = nullptr;
  hipGraphNode_t last = nullptr;
};

template <typename T> struct DevTables {
  cpx<T>* tw[3] = {nullptr, nullptr, nullptr};
  T* hs[3] = {nullptr, nullptr, nullptr};
  T* hc[3] = {nullptr, nullptr, nullptr};
  T* q2[3] = {nullptr, nullptr, nullptr};
  T* fh = nullptr;   // f / |f| in Mandel components under mixed macroscopic conditions
};

}  // namespace

struct pff_solver {
  // problem
  int nx = 0, ny = 0, nz = 0, nxh = 0, dim = 0, C = 0;
  long long N = 0, Nh = 0, M = 0;
  Material mat{};
  pff_params prm{};
  double fm[6] = {0, 0, 0, 0, 0, 0};   // f in Mandel form
  double fh[6] = {0, 0, 0, 0, 0, 0};   // f / |f| (mixed macroscopic conditions)
  int mixed_bc = 0;                     // 1: PFF_BC_MIXED
  std::vector<uint8_t> h_pid, h_mask;
  bool has_mask = false;
  std::vector<pff_phase> phases;
  hipStream_t stream = nullptr;
  GridDesc g{};
  AxisPlan plan[3]{};
  bool plan_any = false;    // some axis has a prime factor above 3 (generic FFT stages)
  DevTables<double> td;
  DevTables<float> tf;
  // device memory: every buffer comes from the caller's allocator (or hipMalloc)
  pff_allocator allocator{nullptr, nullptr, nullptr};
  std::vector<std::pair<void*, size_t>> allocs;
  uint8_t *pid = nullptr, *mask = nullptr;
  double *eps_t = nullptr, *phi = nullptr, *Hn = nullptr, *Hcur = nullptr;
  double* lap64 = nullptr;   // 2D: Laplacian of phi for the residual (N)
  double *eps_c = nullptr, *phi_c = nullptr, *phi_guess = nullptr, *dmask = nullptr;
  double* Edev = nullptr;   // [0] current E, [1] committed E
  // tangent state (TsLayout fields x N), Krylov vectors (M each) and the
  // apply's auxiliary field (N): FP64 always, FP32 copies in mixed mode
  double* ts64 = nullptr;
  float* ts32 = nullptr;
  double* kv64[kNumVec] = {};
  float* kv32[kNumVec] = {};
  double* aux64 = nullptr;
  float* aux32 = nullptr;
  long long applies64 = 0;  // FP64 applies (all applies in FP64 mode)
  int fallbacks = 0;        // mixed mode: Newton iterations finished by an FP64 BiCGSTAB
  int refinements = 0;      // mixed mode: FP32 correction solves
  cpx<double>* spec_d = nullptr;
  cpx<float>* spec_f = nullptr;
  double *part0 = nullptr, *part1 = nullptr;
  size_t part_len = 0;
  double* scal = nullptr;
  double* hscal = nullptr;  // pinned mirror
  double* hstage = nullptr; // pinned staging for small uploads
  double* cgv[4] = {};      // CG vectors (N doubles)
  // host state
  bool bootstrapped = false;
  bool ts_valid = false;
  bool trace = false;       // PFF_TRACE=1: per-Newton-iteration log on stderr
  bool ktrace = false;      // PFF_TRACE=2: the first BiCGSTAB scalars of every solve
  int tim_every = 0;        // sampled kernel timing of the tangent apply
  bool tim_whole = false;   // sampled applies carry the whole-apply events only
  // launch tuning (env PFF_AXIS_THREADS, PFF_SPEC_THREADS, PFF_AXIS_TX, PFF_SPEC_TX, PFF_X_ROWS)
  int axis_threads = 0, spec_threads = 0, axis_tx = 64, spec_tx = 64, x_rows = 64;
  double inner32 = 0.0;     // mixed: FP32 inner-solve tolerance (env PFF_INNER32)
  int xcd_remap = 1;        // z pass: consecutive tiles on one XCD (env PFF_XCD_REMAP)
  int zspec = 1;            // z pass with register-resident end stages for nz = 32, 64, 128 (env PFF_ZSPEC)
  int fit_shapes = 1;       // launch shapes sized to the grid's block count (env PFF_FIT_SHAPES)
  int max_substep_depth = 3;  // sub-increments of a failing increment, down to delta_a / 2^depth (env PFF_SUBSTEPS)
  int yreg = 1;             // FP32 y passes with register-resident end stages (env PFF_YREG: 0 off,
                            // 1 / 2 / 3 tiles of 16 / 32 / 64 columns)
  int fused = 1;            // BiCGSTAB steps fused into the applies (env PFF_FUSED): 0 none,
                            // 1 inner products in the epilogues, 2 also the p / s updates in the prologues
  hipEvent_t ev_scal = nullptr;   // marks the scalar copy of a BiCGSTAB iteration
  pff::KBatcher* kb = nullptr;    // request server: FP32 inner solves batched across solvers
  GraphRec* rec = nullptr;        // always null: a solver's passes are launched directly
  hipEvent_t kb_ready = nullptr, kb_done = nullptr;   // hand-over events of a batched solve
  // sampled pass timing per slot 6 * (5 * fp32 + variant) + kernel, variant = mode + 2 * pro
  std::vector<std::array<hipEvent_t, 6>> tim_pending, tim_free;
  std::vector<int> tim_group;
  double tim_ms[kTimSlots] = {};
  long long tim_n[kTimSlots] = {};
  int n = 0;
  double a = 0.0, E = 0.0, E_s = 0.0;   // a: control value tau
  double wa = 1.0, wE = 0.0;              // control weights (tau = wa Q + wE E)
  bool dctl = false;                      // Q = D (dissipation) instead of Gamma
  bool var = false;                       // variational toughness term (finite differences)
  bool var_het = false;                   // ... with more than one toughness (stencil kernel needed)
  double* lgc64 = nullptr;                // l div(Gc grad .) of the last input (N)
  float* lgc32 = nullptr;
  long long applies = 0, kiters = 0;
  std::string err;

  bool mixed() const { return prm.precision == PFF_PREC_MIXED; }

  size_t bytes_alloc = 0;    // device bytes held by this solver
  template <typename T> T* alloc(size_t count) {
    void* p = nullptr;
    const size_t b = std::max<size_t>(count, 1) * sizeof(T);
    if (allocator.alloc) {
      p = allocator.alloc(b, allocator.ctx);
      if (!p) throw Fail("device allocation of " + std::to_string(b) + " bytes failed (caller's allocator)",
                         PFF_ERR_OOM);
      if (reinterpret_cast<uintptr_t>(p) % 256 != 0) {
        allocator.free(p, b, allocator.ctx);
        throw Fail("the caller's allocator returned memory not aligned to 256 bytes", PFF_ERR_ARG);
      }
    } else {
      HC(hipMalloc(&p, b));
    }
    allocs.emplace_back(p, b);
    bytes_alloc += b;
    return static_cast<T*>(p);
  }
  template <typename T> const DevTables<T>& tables() const;
  template <typename T> cpx<T>* spec() const;
};

template <typename T> T* vecs(pff_solver* s, int k);
template <> double* vecs<double>(pff_solver* s, int k) { return s->kv64[k]; }
template <> float* vecs<float>(pff_solver* s, int k) { return s->kv32[k]; }
template <typename T> T* tstate(pff_solver* s);
template <> double* tstate<double>(pff_solver* s) { return s->ts64; }
template <> float* tstate<float>(pff_solver* s) { return s->ts32; }
template <typename T> T* auxf(pff_solver* s);
template <> double* auxf<double>(pff_solver* s) { return s->aux64; }
template <> float* auxf<float>(pff_solver* s) { return s->aux32; }
template <typename T> T* lgcf(pff_solver* s);
template <> double* lgcf<double>(pff_solver* s) { return s->lgc64; }
template <> float* lgcf<float>(pff_solver* s) { return s->lgc32; }

template <> const DevTables<double>& pff_solver::tables<double>() const { return td; }
template <> const DevTables<float>& pff_solver::tables<float>() const { return tf; }
template <> cpx<double>* pff_solver::spec<double>() const { return spec_d; }
template <> cpx<float>* pff_solver::spec<float>() const { return spec_f ? spec_f : (cpx<float>*)spec_d; }

namespace {

template <typename T> SpecTables<T> spec_tables(const pff_solver* s) {
  const DevTables<T>& t = s->tables<T>();
  SpecTables<T> st;
  for (int a = 0; a < 3; ++a) {
    st.hs[a] = t.hs[a];
    st.hc[a] = t.hc[a];
    st.q2[a] = t.q2[a];
  }
  st.invN = T(1.0 / double(s->N));
  st.fh = t.fh;
  return st;
}

int grid1(long long M) {
  long long b = (M + kBlock - 1) / kBlock;
  if (b > 4096) b = 4096;
  return (int)std::max<long long>(b, 1);
}

// Per-pass tiling.  The in-place FFT needs (elements per block) <=
// MAXE * kBlock and the LDS holds the elements plus one twiddle table.
size_t g_lds_budget = kLdsBudget;

int maxe_of(size_t) { return 8; }
int fft_threads(size_t) { return 512; }

int choose_rb(int nx, int np, size_t csz, int rows_max) {
  const size_t cap = size_t(maxe_of(csz)) * fft_threads(csz);
  int rb = 1;
  while (true) {
    const int nr = rb * 2;
    const size_t elems = size_t(nr) * np * nx;
    if (nr > rows_max || elems > cap || (size_t(lds_padded(elems)) + nx) * csz > g_lds_budget || nr * nx > 4096)
      break;
    rb = nr;
  }
  return rb;
}

size_t lds_x(int rb, int np, int nx, size_t csz, int nred) {
  size_t b = (size_t(lds_padded((long long)rb * np * nx)) + nx) * csz;
  return std::max(b, size_t(nred) * fft_threads(csz) * sizeof(double));
}

// columns per tile (a power of two) for a strided-axis pass over nfb fields
// of length n with `threads` threads per block
int choose_tx(int n, int nfb, size_t csz, int nxh, int threads, int tx_max) {
  const size_t cap = size_t(maxe_of(csz)) * threads;
  int tx = 64;
  while (tx > 1 && (tx > tx_max || size_t(nfb) * n * tx > cap ||
                    (size_t(nfb) * n * tx + n) * csz > kLdsBudget))
    tx /= 2;
  while (tx > 1 && tx / 2 >= nxh) tx /= 2;
  return tx;
}

int log2i(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

size_t lds_axis(int n, int nfb, int tx, size_t csz) { return (size_t(nfb) * n * tx + n) * csz; }

// Runs the FFT round trip of pipe P: forward passes with its prologue, the
// spectral stage, inverse passes with its epilogue.
// Kernel launches of the pass runner: queued on the context's stream, or,
// when the context records a graph (the request server's batched chunks),
// appended to that graph as kernel nodes in launch order.  The graph is
// built node by node rather than by stream capture, so that other threads
// issuing HIP calls meanwhile (the server's slots) cannot invalidate it.
template <typename... KArgs, typename... Args>
void launch_k(GraphRec* rec, void (*kern)(KArgs...), dim3 grid, dim3 block, size_t shmem, hipStream_t st,
              Args&&... args) {
  if (!rec) {
    hipLaunchKernelGGL(kern, grid, block, shmem, st, std::forward<Args>(args)...);
    LAUNCH_CHECK();
    return;
  }
  std::tuple<std::decay_t<KArgs>...> vals(std::forward<Args>(args)...);
  void* params[sizeof...(KArgs) > 0 ? sizeof...(KArgs) : 1];
  std::apply([&](auto&... v) {
    int k = 0;
    ((params[k++] = static_cast<void*>(&v)), ...);
  }, vals);
  hipKernelNodeParams kp{};
  kp.func = reinterpret_cast<void*>(kern);
  kp.gridDim = grid;
  kp.blockDim = block;
  kp.sharedMemBytes = (unsigned int)shmem;
  kp.kernelParams = params;
  kp.extra = nullptr;
  hipGraphNode_t node = nullptr;
  HC(hipGraphAddKernelNode(&node, rec->g, rec->last ? &rec->last : nullptr, rec->last ? 1 : 0, &kp));
  rec->last = node;
}

// The batched strided-axis kernel of pipe P, or null where P takes no
// batched launches (it is then never instantiated).
template <class P, int S, bool SPECTRAL, bool ANY>
auto k_axis_b_of() {
  using Fn = void (*)(const BatchEntry<P>*, AxisPlan, const cpx<typename P::real>*, int, int, int, int);
  if constexpr (Batchable<P>::value) return static_cast<Fn>(k_axis_b<P, S, SPECTRAL, ANY>);
  else return static_cast<Fn>(nullptr);
}

// Pipes of plane-strain problems never take the 3D z pass.
template <class P> struct Only2D : std::false_type {};
template <typename T> struct Only2D<TangentPipe<T, 2>> : std::true_type {};
template <> struct Only2D<ResidualPipe<2>> : std::true_type {};
template <> struct Only2D<CompatPipe<2>> : std::true_type {};
template <typename T> struct Only2D<ProjectPipe<T, 2>> : std::true_type {};

// The z pass with register-resident first and last radix stages (k_zspec),
// for z lengths 32, 64 and 128; returns false where it does not apply.
// FP32 tiles run 256 threads, FP64 tiles 128 (the same LDS bytes).
// LDS bytes one workgroup may allocate on the current device (queried once).
size_t lds_per_block_limit() {
  static const size_t lim = [] {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
      return size_t(64) << 10;
    return size_t(v);
  }();
  return lim;
}

template <class P, int N, int TX, class S>
bool launch_zspec_tx(S* s, const typename P::Args& A, const cpx<typename P::real>* tw, cpx<typename P::real>* spec,
                     const BatchEntry<P>* batch, int B) {
  using T = typename P::real;
  const size_t lds = (size_t(ZspecLds<P, N, TX>::ELEMS) + N) * sizeof(cpx<T>);
  if (lds > lds_per_block_limit()) return false;
  const int nkt = (s->g.nxm + TX - 1) / TX;
  const dim3 gs(nkt + s->g.nyq, s->ny, B);
  if constexpr (Batchable<P>::value) {
    if (batch) {
      launch_k(s->rec, k_zspec_b<P, N, TX>, gs, dim3(N / 4 * TX), lds, s->stream, batch, tw, s->xcd_remap);
      return true;
    }
  }
  launch_k(s->rec, k_zspec<P, N, TX>, gs, dim3(N / 4 * TX), lds, s->stream, A, tw, spec, s->xcd_remap);
  return true;
}

// Tile width: TX columns of N / 4 threads each, 256 threads per FP32 tile and
// 128 per FP64 tile.  (At 128^3 FP32, half-width tiles gave the same apply
// time, 177.8 against 178.0 us, and double-width tiles 182.0 us.  The 16
// Nyquist tiles of that grid make the 1025th..1040th tile, a tail after two
// full rounds of two blocks per CU worth about 8 us of the apply; folding the
// Nyquist pencils into the main tiles as a ninth column cost more, +3.5 us,
// and as an extra half-wavefront +13 us, its two code paths taking 249 VGPRs.)
template <class P, int N, class S>
bool launch_zspec_n(S* s, const typename P::Args& A, const cpx<typename P::real>* tw, cpx<typename P::real>* spec,
                    const BatchEntry<P>* batch, int B) {
  using T = typename P::real;
  constexpr int TX = (sizeof(T) == 4 ? 256 : 128) / (N / 4);
  return launch_zspec_tx<P, N, TX>(s, A, tw, spec, batch, B);
}

template <class P, class S>
bool launch_zspec(S* s, const typename P::Args& A, const cpx<typename P::real>* tw, cpx<typename P::real>* spec,
                  const BatchEntry<P>* batch, int B) {
  if constexpr (Only2D<P>::value) {
    return false;
  } else {
    if (!s->zspec) return false;
    switch (s->nz) {
      case 32: return launch_zspec_n<P, 32>(s, A, tw, spec, batch, B);
      case 64: return launch_zspec_n<P, 64>(s, A, tw, spec, batch, B);
      case 128: return launch_zspec_n<P, 128>(s, A, tw, spec, batch, B);
      default: return false;
    }
  }
}

// The y passes of a 3D FP32 tangent apply with register-resident end stages
// (k_yreg) for y lengths 32, 64, 128: tile width 16, 32 or 64 columns
// (context member yreg = 1, 2, 3; 0 keeps k_axis).  Returns false where it
// does not apply.  At 128^3 the FP32 apply takes 171.6 us with 16-column
// tiles, 174.8 with 32, 187.4 with 64, and 177.2 with k_axis.
template <class P, int N, int TX, int SG, class C>
bool launch_yreg_tx(C* s, const typename P::Args& A, const cpx<typename P::real>* tw, cpx<typename P::real>* spec,
                    const BatchEntry<P>* batch, int B) {
  using T = typename P::real;
  const size_t lds = (size_t(YregLds<T, N, TX>::ELEMS) + N) * sizeof(cpx<T>);
  if (lds > lds_per_block_limit()) return false;
  const int nkt = (s->g.nxm + TX - 1) / TX;
  const dim3 gy(nkt + s->g.nyq, s->nz, P::NF * B);
  if (batch) launch_k(s->rec, k_yreg_b<P, N, TX, SG>, gy, dim3(4 * TX), lds, s->stream, batch, tw);
  else launch_k(s->rec, k_yreg<P, N, TX, SG>, gy, dim3(4 * TX), lds, s->stream, A, tw, spec);
  return true;
}

template <class P, int N, int SG, class C>
bool launch_yreg_n(C* s, const typename P::Args& A, const cpx<typename P::real>* tw, cpx<typename P::real>* spec,
                   const BatchEntry<P>* batch, int B) {
  switch (s->yreg) {
    case 1: return launch_yreg_tx<P, N, 16, SG>(s, A, tw, spec, batch, B);
    case 2: return launch_yreg_tx<P, N, 32, SG>(s, A, tw, spec, batch, B);
    case 3: return launch_yreg_tx<P, N, 64, SG>(s, A, tw, spec, batch, B);
    default: return false;
  }
}

template <class P, int SG, class C>
bool launch_yreg(C* s, const typename P::Args& A, const cpx<typename P::real>* tw, cpx<typename P::real>* spec,
                 const BatchEntry<P>* batch, int B) {
  if constexpr (!Batchable<P>::value || P::NF != 7) {
    return false;
  } else {
    if (s->dim != 3 || !s->yreg) return false;
    switch (s->ny) {
      case 32: return launch_yreg_n<P, 32, SG>(s, A, tw, spec, batch, B);
      case 64: return launch_yreg_n<P, 64, SG>(s, A, tw, spec, batch, B);
      case 128: return launch_yreg_n<P, 128, SG>(s, A, tw, spec, batch, B);
      default: return false;
    }
  }
}

// S: a solver, or any context with the same members (tables, spectra,
// plans, launch knobs, stream).  batch: B entries of a batched launch (one
// RVE each, their own arguments, spectra and partials), or null.
template <class P, bool ANY, class S>
void run_passes(S* s, const typename P::Args& A, int& nblk_x, hipEvent_t* ev, const BatchEntry<P>* batch,
                int B) {
  using T = typename P::real;
  constexpr int NF = P::NF;
  constexpr int NP = (NF + 1) / 2;
  const DevTables<T>& tb = s->template tables<T>();
  cpx<T>* spec = s->template spec<T>();
  const size_t csz = sizeof(cpx<T>);
  const int nthr = fft_threads(csz);
  const int nred = std::max(P::NRED_PRO, P::NRED_EPI);
  // rows per x-pass block: at most x_rows, and few enough that the pass has
  // 512 blocks where the grid has the rows (small grids are latency-bound:
  // 256^2 FP64 apply 35.8 -> 31.1 us, 64^2 28.2 -> 23.2 us with one row per block)
  const int rb = choose_rb(s->nx, NP, csz,
                           s->fit_shapes ? std::min(s->x_rows, std::max(1, (int)(((long long)s->ny * s->nz) / 512)))
                                         : s->x_rows);
  const size_t ldsx = lds_x(rb, NP, s->nx, csz, nred);
  if (ldsx > kLdsBudget || size_t(rb) * NP * s->nx > size_t(maxe_of(csz)) * fft_threads(csz))
    throw Fail("grid too large for the LDS budget of the x pass", PFF_ERR_ARG);
  const long long nrows = (long long)s->ny * s->nz;
  nblk_x = (int)((nrows + rb - 1) / rb);
  if ((size_t)nblk_x > s->part_len) throw Fail("partial buffer too small", PFF_ERR_STATE);
  if (ev && ev[0]) HC(hipEventRecord(ev[0], s->stream));
  // batched launches (the request server's FP32 tangent) take the *_b kernels
  constexpr bool BAT = Batchable<P>::value;
  auto axis_launch = [&](auto kern_u, auto kern_b, dim3 grid, int thr, size_t lds, int axis, int ltx, int nfb,
                         int remap) {
    if constexpr (BAT) {
      if (batch) {
        launch_k(s->rec, kern_b, grid, dim3(thr), lds, s->stream, batch, s->plan[axis], tb.tw[axis], axis, ltx,
                 nfb, remap);
        return;
      }
    }
    launch_k(s->rec, kern_u, grid, dim3(thr), lds, s->stream, A, s->plan[axis], tb.tw[axis], spec, axis, ltx, nfb,
             remap);
  };
  if constexpr (BAT) {
    if (batch)
      launch_k(s->rec, k_xfwd<P, ANY, true>, dim3(nblk_x, B), dim3(nthr), ldsx, s->stream, A, s->plan[0], tb.tw[0],
               spec, rb, s->part0, batch);
  }
  if (!BAT || !batch)
    launch_k(s->rec, k_xfwd<P, ANY, false>, dim3(nblk_x), dim3(nthr), ldsx, s->stream, A, s->plan[0], tb.tw[0], spec,
             rb, s->part0, static_cast<const BatchEntry<P>*>(nullptr));
  if (ev && ev[1]) HC(hipEventRecord(ev[1], s->stream));
  // the spectral pass holds all NF fields of a tile
  const int last = s->dim == 2 ? 1 : 2;
  const int nl = s->dim == 2 ? s->ny : s->nz;
  const int sthr = s->spec_threads > 0 ? std::min(s->spec_threads, nthr) : nthr;
  // 2D: one column per spectral tile where fewer than 256 tiles would remain
  // (the whole pass is a few dozen blocks otherwise)
  const int txs = choose_tx(nl, NF, csz, s->g.nxm, sthr,
                            s->dim == 2 && s->fit_shapes ? std::min(s->spec_tx, std::max(1, s->g.nxm / 256))
                                                         : s->spec_tx);
  const size_t ldss = lds_axis(nl, NF, txs, csz);
  if (ldss > kLdsBudget || size_t(NF) * nl * txs > size_t(maxe_of(csz)) * sthr)
    throw Fail("axis too long for the LDS budget", PFF_ERR_ARG);
  const dim3 gs((s->g.nxm + txs - 1) / txs + s->g.nyq, last == 1 ? s->nz : s->ny, B);
  if (s->dim == 2) {
    axis_launch(k_axis<P, -1, true, ANY>, k_axis_b_of<P, -1, true, ANY>(), gs, sthr, ldss, 1, log2i(txs), NF, 0);
    if (ev) {
      for (int k = 2; k <= 4; ++k)
        if (ev[k]) HC(hipEventRecord(ev[k], s->stream));
    }
  } else {
    // forward / inverse y passes: one field per block, wide tiles
    // measured: 256 threads for FP32 tiles, 512 for FP64 (unless set by env)
    const int athr = s->axis_threads > 0 ? std::min(s->axis_threads, nthr) : (csz == 8 ? 256 : 512);
    const int txy = choose_tx(s->ny, 1, csz, s->g.nxm, athr, s->axis_tx);
    const size_t ldsy = lds_axis(s->ny, 1, txy, csz);
    const dim3 gy((s->g.nxm + txy - 1) / txy + s->g.nyq, s->nz, NF * B);
    if (!launch_yreg<P, -1>(s, A, tb.tw[1], spec, batch, B))
      axis_launch(k_axis<P, -1, false, ANY>, k_axis_b_of<P, -1, false, ANY>(), gy, athr, ldsy, 1, log2i(txy), 1, 0);
    if (ev && ev[2]) HC(hipEventRecord(ev[2], s->stream));
    if (!launch_zspec<P>(s, A, tb.tw[2], spec, batch, B)) {
      axis_launch(k_axis<P, -1, true, ANY>, k_axis_b_of<P, -1, true, ANY>(), gs, sthr, ldss, 2, log2i(txs), NF,
                  s->xcd_remap);
    }
    if (ev && ev[3]) HC(hipEventRecord(ev[3], s->stream));
    if (!launch_yreg<P, 1>(s, A, tb.tw[1], spec, batch, B))
      axis_launch(k_axis<P, 1, false, ANY>, k_axis_b_of<P, 1, false, ANY>(), gy, athr, ldsy, 1, log2i(txy), 1, 0);
    if (ev && ev[4]) HC(hipEventRecord(ev[4], s->stream));
  }
  if constexpr (BAT) {
    if (batch)
      launch_k(s->rec, k_xinv<P, ANY, true>, dim3(nblk_x, B), dim3(nthr), ldsx, s->stream, A, s->plan[0], tb.tw[0],
               spec, rb, s->part1, batch);
  }
  if (!BAT || !batch)
    launch_k(s->rec, k_xinv<P, ANY, false>, dim3(nblk_x), dim3(nthr), ldsx, s->stream, A, s->plan[0], tb.tw[0], spec,
             rb, s->part1, static_cast<const BatchEntry<P>*>(nullptr));
  if (ev && ev[5]) HC(hipEventRecord(ev[5], s->stream));
}

// The kernels with the generic-radix FFT stage run only where a grid length
// has a prime factor above 3.
template <class P, class S>
void run_pipeline(S* s, const typename P::Args& A, int& nblk_x, hipEvent_t* ev = nullptr,
                  const BatchEntry<P>* batch = nullptr, int B = 1) {
  if (s->plan_any) run_passes<P, true>(s, A, nblk_x, ev, batch, B);
  else run_passes<P, false>(s, A, nblk_x, ev, batch, B);
}

// ---- live kernel timing (sampled event pairs on the solver stream) -------------

hipEvent_t* timing_acquire(pff_solver* s, int group);
void timing_harvest(pff_solver* s);

void sync_scal(pff_solver* s) {
  HC(hipMemcpyAsync(s->hscal, s->scal, SC_COUNT * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  HC(hipStreamSynchronize(s->stream));
}

// ---- small kernels ------------------------------------------------------------

__global__ void k_lincomb(double* __restrict__ out, double a, const double* __restrict__ x, double b,
                          const double* __restrict__ y, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = a * x[i] + (y ? b * y[i] : 0.0);
}

__global__ void k_axpy(double* x, double a, const double* __restrict__ y, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    x[i] += a * y[i];
}

__global__ void k_mask_to_double(double* __restrict__ out, const uint8_t* __restrict__ m, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = m[i] ? 1.0 : 0.0;
}

// phi0 = m + (1 - m) u
__global__ void k_phi0(double* __restrict__ phi, const double* __restrict__ u,
                       const uint8_t* __restrict__ m, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    phi[i] = m[i] ? 1.0 : u[i];
}

// right-hand side of the Helmholtz solve: b = (1-m) (2|H|/Gc - B m), where b
// holds (1-m) B m on entry
__global__ void k_helm_rhs(double* __restrict__ b, const double* __restrict__ H,
                           const uint8_t* __restrict__ m, const uint8_t* __restrict__ pid, Material mat,
                           long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    b[i] = m[i] ? 0.0 : (H ? 2.0 * fabs(H[i]) / mat.Gc[pid[i]] : 0.0) - b[i];
}

// Finite-difference l div(Gc grad u) of the variational toughness term:
// forward differences of u (masked: u = 0 on the crack mask when mask_in),
// Gc on the faces as the mean of the two voxels, backward differences of
// the fluxes; periodic.  The input u is `in` at stride 1.
template <typename T>
__global__ void k_div_gc_grad(T* __restrict__ out, const T* __restrict__ in, const uint8_t* __restrict__ pid,
                              const uint8_t* __restrict__ mask, int mask_in, Material mat, double l, int nx,
                              int ny, int nz, long long N) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(i % nx);
    const long long yz = i / nx;
    const int y = (int)(yz % ny), z = (int)(yz / ny);
    auto val = [&](long long j) -> double { return (mask_in && mask[j]) ? 0.0 : double(in[j]); };
    const double ui = val(i), gi = mat.Gc[pid[i]];
    double acc = 0.0;
    const long long nb[3][2] = {
        {i - x + (x + 1 == nx ? 0 : x + 1), i - x + (x == 0 ? nx - 1 : x - 1)},
        {i + (long long)((y + 1 == ny ? 0 : y + 1) - y) * nx, i + (long long)((y == 0 ? ny - 1 : y - 1) - y) * nx},
        {i + (long long)((z + 1 == nz ? 0 : z + 1) - z) * nx * ny,
         i + (long long)((z == 0 ? nz - 1 : z - 1) - z) * nx * ny}};
    for (int a = 0; a < 3; ++a) {
      if ((a == 0 && nx == 1) || (a == 1 && ny == 1) || (a == 2 && nz == 1)) continue;
      const long long up = nb[a][0], dn = nb[a][1];
      acc += 0.5 * (gi + mat.Gc[pid[up]]) * (val(up) - ui) - 0.5 * (gi + mat.Gc[pid[dn]]) * (ui - val(dn));
    }
    out[i] = T(l * acc);
  }
}

// per-block partials: max |x_i| over the first n entries
__global__ void __launch_bounds__(kBlock) k_absmax(const double* __restrict__ x, long long n,
                                                   double* __restrict__ partials) {
  __shared__ double lds[kBlock];
  double mx = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    mx = fmax(mx, fabs(x[i]));
  lds[threadIdx.x] = mx;
  __syncthreads();
  for (int h = kBlock / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) lds[threadIdx.x] = fmax(lds[threadIdx.x], lds[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = lds[0];
}

__global__ void __launch_bounds__(kBlock) k_max_final(const double* __restrict__ partials, int nb,
                                                      double* __restrict__ out) {
  __shared__ double lds[kBlock];
  double mx = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) mx = fmax(mx, partials[b]);
  lds[threadIdx.x] = mx;
  __syncthreads();
  for (int h = kBlock / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) lds[threadIdx.x] = fmax(lds[threadIdx.x], lds[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = lds[0];
}

// stagger error partials: ||eps~ - eps~prev||^2, ||f E + eps~||^2,
// ||phi - phi_prev||^2, ||phi||^2
template <int C>
__global__ void __launch_bounds__(kBlock) k_stagger_norms(const double* __restrict__ eps, const double* __restrict__ eps_prev,
                                                          const double* __restrict__ phi,
                                                          const double* __restrict__ phi_prev, Vec16 fm,
                                                          const double* __restrict__ Edev, long long N,
                                                          double* __restrict__ partials) {
  const double E = Edev[0];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
#pragma unroll
    for (int k = 0; k < C; ++k) {
      const double e = eps[k * N + i];
      const double d = e - eps_prev[k * N + i];
      const double t = e + fm.v[k] * E;
      acc[0] += d * d;
      acc[1] += t * t;
    }
    const double p = phi[i], dp = p - phi_prev[i];
    acc[2] += dp * dp;
    acc[3] += p * p;
  }
  write_partials<4>(acc, partials);
}

// predictor guess: phi = max(phi0, (1-m) phi_loc(phase))
__global__ void k_guess(double* __restrict__ phi, const double* __restrict__ phi0,
                        const uint8_t* __restrict__ pid, const uint8_t* __restrict__ m, Vec16 loc,
                        long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double pl = m[i] ? 0.0 : loc.v[pid[i]];
    phi[i] = phi0[i] > pl ? phi0[i] : pl;
  }
}

// Newton update (Algorithm 2): eps_t += alpha d eps, phi += alpha (1-m) d phi,
// partials of ||d eps + f dE||^2, ||eps||^2, ||d phi||^2, ||phi||^2 at the new state.
template <typename TW, int C>
__global__ void __launch_bounds__(kBlock) k_newton_update(double* __restrict__ eps_t, double* __restrict__ phi,
                                                          const TW* __restrict__ x,
                                                          const uint8_t* __restrict__ mask, Vec16 fm,
                                                          const double* __restrict__ Edev, double alpha,
                                                          long long N, double* __restrict__ partials) {
  const double dE = double(x[(long long)(C + 1) * N]);
  const double En = Edev[0] + alpha * dE;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
#pragma unroll
    for (int k = 0; k < C; ++k) {
      const double d = double(x[k * N + i]);
      const double w = d + fm.v[k] * dE;
      const double e = eps_t[k * N + i] + alpha * d;
      eps_t[k * N + i] = e;
      const double et = e + fm.v[k] * En;
      acc[0] += w * w;
      acc[1] += et * et;
    }
    const double dp = mask[i] ? 0.0 : double(x[(long long)C * N + i]);
    const double p = phi[i] + alpha * dp;
    phi[i] = p;
    acc[2] += dp * dp;
    acc[3] += p * p;
  }
  write_partials<4>(acc, partials);
}

__global__ void __launch_bounds__(kBlock) k_widen(double* __restrict__ dst, const float* __restrict__ src,
                                                  long long M) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < M;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = double(src[i]);
}

// out = b - t, partials of (out, out) and (b, b)
__global__ void __launch_bounds__(kBlock) k_resid_pair(double* __restrict__ out, const double* __restrict__ b,
                                                       const double* __restrict__ t, long long M,
                                                       double* __restrict__ partials) {
  double acc[2] = {0.0, 0.0};
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < M;
       i += (long long)gridDim.x * blockDim.x) {
    const double r = b[i] - t[i];
    out[i] = r;
    acc[0] += r * r;
    acc[1] += b[i] * b[i];
  }
  write_partials<2>(acc, partials);
}

__global__ void __launch_bounds__(kBlock) k_narrow_scaled(float* __restrict__ dst, const double* __restrict__ src,
                                                          double scale, long long M) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < M;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = float(scale * src[i]);
}

__global__ void __launch_bounds__(kBlock) k_axpy_widen(double* __restrict__ y, const float* __restrict__ x,
                                                       double a, long long M) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < M;
       i += (long long)gridDim.x * blockDim.x)
    y[i] += a * double(x[i]);
}

__global__ void __launch_bounds__(kBlock) k_add(double* __restrict__ y, const double* __restrict__ x, long long M) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < M;
       i += (long long)gridDim.x * blockDim.x)
    y[i] += x[i];
}

__global__ void k_commit_history(double* __restrict__ Hn, const double* __restrict__ Hcur, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    Hn[i] = fabs(Hcur[i]);
}

struct FinNewton {
  struct Args { double* scal; double* Edev; const void* x; int last_is_float; long long idx; double alpha; };
  __device__ static void run(const Args& F, const double* tot) {
    F.scal[SC_NW] = tot[0];
    F.scal[SC_NEPS] = tot[1];
    F.scal[SC_NDPHI] = tot[2];
    F.scal[SC_NPHI] = tot[3];
    const double dE = F.last_is_float ? double(((const float*)F.x)[F.idx]) : ((const double*)F.x)[F.idx];
    F.Edev[0] = F.Edev[0] + F.alpha * dE;
  }
};

// sums of the residual pass's prologue: sigma (6), ||sigma||^2, ||2H||^2
struct FinSig {
  struct Args { double* scal; };
  __device__ static void run(const Args& F, const double* tot) {
    for (int q = 0; q < 6; ++q) F.scal[SC_SIG + q] = tot[q];
    F.scal[SC_NSIG] = tot[6];
    F.scal[SC_NH2] = tot[7];
  }
};

struct FinResid {
  struct Args {
    double* scal;
    double a;              // control value tau
    double wa, wE;         // F3 = w_a Q + w_E E - tau, Q = Gamma or D
    int dctl;              // 1: Q = D (dissipation control)
    const double* E;
    double* rhs_last;
    float* rhs32_last;
    double* F_last;
  };
  __device__ static void run(const Args& F, const double* tot) {
    const double f3 = F.wa * (F.dctl ? tot[3] : tot[0]) + F.wE * F.E[0] - F.a;
    F.scal[SC_GAMMA] = tot[0];
    F.scal[SC_F1] = tot[1];
    F.scal[SC_F2] = tot[2];
    F.scal[SC_DISS] = tot[3];
    F.scal[SC_F3] = f3;
    F.rhs_last[0] = -f3;
    if (F.rhs32_last) F.rhs32_last[0] = float(-f3);
    if (F.F_last) F.F_last[0] = f3;
  }
};

// ---- templated solver steps -------------------------------------------------------

template <int DIM, typename TW>
struct Impl {
  static constexpr int C = DIM == 2 ? 3 : 6;

  static TW* vec(pff_solver* s, int k) { return vecs<TW>(s, k); }
  enum { X0 = 0, X1, X2, R, RHAT, P, V, S, T, RHS, SOL, VB, VD };

  // variational toughness term of the damage block of the input (d phi' =
  // (1-m) d phi), before the pipeline that consumes it
  static const TW* var_term(pff_solver* s, const TW* v) {
    if (!s->var_het) return nullptr;
    TW* out = lgcf<TW>(s);
    k_div_gc_grad<TW><<<grid1(s->N), kBlock, 0, s->stream>>>(out, v + (long long)C * s->N, s->pid, s->mask, 1,
                                                             s->mat, s->prm.l, s->nx, s->ny, s->nz, s->N);
    LAUNCH_CHECK();
    return out;
  }

  static void fill_tangent_args(pff_solver* s, typename TangentPipe<TW, DIM>::Args& A) {
    A.g = s->g;
    A.mat = s->mat;
    A.l = TW(s->prm.l);
    A.k = TW(s->prm.k_resid);
    for (int k = 0; k < 6; ++k) A.f[k] = TW(s->fm[k]);
    A.ts = tstate<TW>(s);
    A.pid = s->pid;
    A.mask = s->mask;
    A.aux = auxf<TW>(s);
    A.tab = spec_tables<TW>(s);
  }

  // Fused BiCGSTAB apply (mode 1: u = r + beta (v - omega w) -> v, J u -> Jv,
  // alpha = rho / (dv, J u); mode 2: u = r - alpha w -> vout, J u -> Jv,
  // omega = (J u, dv) / (J u, J u)); see TangentPipe.
  static void apply_fused(pff_solver* s, int mode, int pro, const TW* v, const TW* r, const TW* w,
                          TW* vout, TW* Jv, const TW* dv) {
    typename TangentPipe<TW, DIM>::Args A;
    fill_tangent_args(s, A);
    A.v = v;
    A.Jv = Jv;
    A.mode = mode;
    A.pro = pro;
    A.mech = 0;
    A.lgc = pro ? nullptr : var_term(s, v);   // pro modes are off with the variational term
    A.r = r;
    A.w = w;
    A.vout = vout;
    A.dv = dv;
    A.ks = s->scal + SC_KS;
    int nblk = 0;
    const int grp = 5 * (std::is_same<TW, float>::value ? 1 : 0) + mode + 2 * pro;
    hipEvent_t* ev = (s->tim_every > 0 && s->applies % s->tim_every == 0) ? timing_acquire(s, grp) : nullptr;
    run_pipeline<TangentPipe<TW, DIM>>(s, A, nblk, ev);
    const long long last = (long long)(C + 1) * s->N;
    k_fin_fused<TW><<<1, kBlock, 0, s->stream>>>(s->part0, s->part1, nblk, mode, pro, Jv + last,
                                                 pro ? vout + last : nullptr, dv + last, v + last, s->wa,
                                                 s->wE, s->scal + SC_KS);
    LAUNCH_CHECK();
    s->applies++;
    if (std::is_same<TW, double>::value) s->applies64++;
  }

  static void apply(pff_solver* s, const TW* v, TW* Jv, int mech = 0) {
    typename TangentPipe<TW, DIM>::Args A;
    fill_tangent_args(s, A);
    A.v = v;
    A.Jv = Jv;
    A.mode = 0;
    A.pro = 0;
    A.mech = mech;
    A.lgc = var_term(s, v);
    A.r = A.w = A.dv = nullptr;
    A.vout = nullptr;
    A.ks = nullptr;
    int nblk = 0;
    const int grp = 5 * (std::is_same<TW, float>::value ? 1 : 0);
    hipEvent_t* ev = (s->tim_every > 0 && s->applies % s->tim_every == 0) ? timing_acquire(s, grp) : nullptr;
    run_pipeline<TangentPipe<TW, DIM>>(s, A, nblk, ev);
    const long long last = (long long)(C + 1) * s->N;
    typename FinLast<TW>::Args F{Jv + last, s->wa, s->wE, v + last};
    k_reduce<FinLast<TW>><<<1, kBlock, 0, s->stream>>>(s->part0, nblk, 1, F);
    LAUNCH_CHECK();
    s->applies++;
    if (std::is_same<TW, double>::value) s->applies64++;
  }

  // residual at the current state for target a; rhs = -F (FP64, plus the
  // FP32 copy in mixed mode); also refreshes the tangent state(s)
  static void residual(pff_solver* s, double a, double* F_dev) {
    typename ResidualPipe<DIM>::Args A;
    A.g = s->g;
    A.mat = s->mat;
    A.l = s->prm.l;
    A.k = s->prm.k_resid;
    for (int k = 0; k < 6; ++k) A.f[k] = s->fm[k];
    A.eps_t = s->eps_t;
    A.phi = s->phi;
    A.Hn = s->Hn;
    A.Hcur = s->Hcur;
    A.E = s->Edev;
    A.ts = s->ts64;
    A.ts32 = s->ts32;
    A.rhs = vecs<double>(s, RHS);
    A.rhs32 = s->kv32[RHS];
    A.F = F_dev;
    A.pid = s->pid;
    A.mask = s->mask;
    A.tab = spec_tables<double>(s);
    A.lap_ext = nullptr;
    A.lapg = nullptr;
    A.lgc = nullptr;
    if (s->var_het) {
      k_div_gc_grad<double><<<grid1(s->N), kBlock, 0, s->stream>>>(s->lgc64, s->phi, s->pid, s->mask, 0,
                                                                   s->mat, s->prm.l, s->nx, s->ny, s->nz, s->N);
      LAUNCH_CHECK();
      A.lgc = s->lgc64;
    }
    if (DIM == 2) {
      LapPipe::Args LA;
      LA.g = s->g;
      LA.u = s->phi;
      LA.out = s->lap64;
      LA.tab = A.tab;
      LA.pid = nullptr;
      LA.mat = s->mat;
      int nb = 0;
      run_pipeline<LapPipe>(s, LA, nb);
      A.lap_ext = s->lap64;
    }
    if (s->dctl) {
      // Lap(Gc phi) into a CG work vector (free outside the CG solves of the
      // bootstrap and of the staggered Helmholtz problem)
      LapPipe::Args LA;
      LA.g = s->g;
      LA.u = s->phi;
      LA.out = s->cgv[3];
      LA.tab = A.tab;
      LA.pid = s->pid;
      LA.mat = s->mat;
      int nb = 0;
      run_pipeline<LapPipe>(s, LA, nb);
      A.lapg = s->cgv[3];
    }
    int nblk = 0;
    run_pipeline<ResidualPipe<DIM>>(s, A, nblk);
    k_reduce<FinSig><<<1, kBlock, 0, s->stream>>>(s->part0, nblk, 8, FinSig::Args{s->scal});
    LAUNCH_CHECK();
    const long long last = (long long)(C + 1) * s->N;
    FinResid::Args fr{s->scal, a, s->wa, s->wE, s->dctl ? 1 : 0, s->Edev, vecs<double>(s, RHS) + last,
                      s->kv32[RHS] ? s->kv32[RHS] + last : nullptr, F_dev ? F_dev + last : nullptr};
    k_reduce<FinResid><<<1, kBlock, 0, s->stream>>>(s->part1, nblk, 4, fr);
    LAUNCH_CHECK();
    s->ts_valid = true;
  }

  // FP64 solves: the BiCGSTAB direction p is projected onto compatible
  // strains after each update.  At the warm start of an increment many voxels
  // are history ties, and the bordered Jacobian can have a null direction made
  // mostly of incompatible strain (found on the 24^3 particle composite,
  // spectral split and isotropic model alike).  The update p = r + beta (p -
  // omega v) carries the incompatible round-off of p forward with the factor
  // beta every iteration, and the damage rows see it through b : w, so it can
  // grow into that direction; the step projection after the solve cannot
  // undo it, since the direction's compatible part alone is not null.  Every
  // other vector only picks up round-off additively (the strain rows of J v
  // lie in the range of G), so projecting p suffices.
  static void keep_compatible(pff_solver* s, TW* x) {
    if constexpr (std::is_same<TW, double>::value) project_strain(s, x);
  }

  static void reduce_ks(pff_solver* s, int nslot, int which) {
    const int nb = red_blocks(s->M);
    double* ks = s->scal + SC_KS;
    if (which == 0) k_reduce<FinBnorm><<<1, kBlock, 0, s->stream>>>(s->part0, nb, nslot, FinBnorm::Args{ks});
    else if (which == 1) k_reduce<FinRho0><<<1, kBlock, 0, s->stream>>>(s->part0, nb, nslot, FinRho0::Args{ks});
    else if (which == 2) k_reduce<FinAlpha><<<1, kBlock, 0, s->stream>>>(s->part0, nb, nslot, FinAlpha::Args{ks});
    else if (which == 3) k_reduce<FinOmega><<<1, kBlock, 0, s->stream>>>(s->part0, nb, nslot, FinOmega::Args{ks});
    else k_reduce<FinRR><<<1, kBlock, 0, s->stream>>>(s->part0, nb, nslot, FinRR::Args{ks});
    LAUNCH_CHECK();
  }

  // BiCGSTAB with a true-residual check (x_out = J^{-1} b); returns 1 if
  // ||b - J x_out|| <= rtol ||b||.  A run keeps its iterate of smallest
  // recursive residual (three x buffers rotate, no copies); when the run
  // stops, b - J x of that iterate is formed and, if it misses the
  // tolerance, a new run starts from it (the recursive residual of BiCGSTAB
  // can drift from the true one after large intermediate iterates).
  static int bicgstab(pff_solver* s, const TW* b, TW* x_out, double rtol, int maxit, int* iters,
                      double* relres) {
    const long long M = s->M;
    const int nb = red_blocks(M);
    const int g1 = nb;
    double* ks = s->scal + SC_KS;
    // FP64 solves project the direction p after its update (keep_compatible),
    // so they never form p inside the apply prologue (fused mode 2)
    const int fused = std::is_same<TW, double>::value ? std::min(s->fused, 1) : s->fused;
    TW* xb[3] = {vec(s, X0), vec(s, X1), vec(s, X2)};
    TW *r = vec(s, R), *rhat = vec(s, RHAT), *p = vec(s, P), *v = vec(s, V), *sv = vec(s, S),
       *t = vec(s, T);
    k_bicg_init<TW><<<g1, kBlock, 0, s->stream>>>(b, xb[0], r, p, v, M, s->part0);
    LAUNCH_CHECK();
    reduce_ks(s, 1, 0);
    sync_scal(s);
    const double bnorm = s->hscal[SC_KS + KS_BNORM];
    int total = 0, conv = 0, cur = 0, best = 0;
    double true_res = bnorm;
    if (bnorm == 0.0) conv = 1;
    for (int cycle = 0; cycle < kMaxCycles && !conv; ++cycle) {
      double res_best = true_res;     // the run starts at x[best] with its true residual
      cur = best;
      k_bicg_shadow<TW><<<g1, kBlock, 0, s->stream>>>(r, rhat, ks, kShadowSeed, M, s->part0);
      LAUNCH_CHECK();
      reduce_ks(s, 1, 1);
      bool issued = false;   // this iteration's direction apply is already queued
      while (total < maxit) {
        ++total;
        if (fused == 2) {
          // p = r + beta (p - omega v) formed in the prologue; v = J p; alpha = rho / (r_hat, v)
          if (!issued) apply_fused(s, 1, 1, p, r, v, p, v, rhat);
          issued = false;
          // s = r - alpha v formed in the prologue; t = J s; omega = (t, s) / (t, t)
          apply_fused(s, 2, 1, nullptr, r, v, sv, t, sv);
        } else if (fused == 1) {
          // streaming p / s updates; inner products in the apply epilogues
          if (!issued) {
            k_bicg_p<TW><<<g1, kBlock, 0, s->stream>>>(p, r, v, ks, M);
            LAUNCH_CHECK();
            keep_compatible(s, p);
            apply_fused(s, 1, 0, p, nullptr, nullptr, nullptr, v, rhat);
          }
          issued = false;
          k_bicg_s<TW><<<g1, kBlock, 0, s->stream>>>(sv, r, v, ks, M);
          LAUNCH_CHECK();
          apply_fused(s, 2, 0, sv, nullptr, nullptr, nullptr, t, sv);
        } else {
          k_bicg_p<TW><<<g1, kBlock, 0, s->stream>>>(p, r, v, ks, M);
          LAUNCH_CHECK();
          keep_compatible(s, p);
          apply(s, p, v);
          k_dots<TW, 1><<<g1, kBlock, 0, s->stream>>>(rhat, v, nullptr, nullptr, nullptr, nullptr, M, s->part0);
          LAUNCH_CHECK();
          reduce_ks(s, 1, 2);
          k_bicg_s<TW><<<g1, kBlock, 0, s->stream>>>(sv, r, v, ks, M);
          LAUNCH_CHECK();
          apply(s, sv, t);
          k_dots<TW, 2><<<g1, kBlock, 0, s->stream>>>(t, sv, t, t, nullptr, nullptr, M, s->part0);
          LAUNCH_CHECK();
          reduce_ks(s, 2, 3);
        }
        int nxt = 0;
        while (nxt == cur || nxt == best) ++nxt;
        k_bicg_xr<TW><<<g1, kBlock, 0, s->stream>>>(xb[nxt], xb[cur], p, sv, t, r, rhat, ks, M, s->part0);
        LAUNCH_CHECK();
        reduce_ks(s, 2, 4);
        // Copy the scalars, then queue the next iteration's direction apply
        // before waiting for them, so that the device does not idle during
        // the host's decision.  The apply only needs device scalars; when the
        // run stops here its result is not used (a new run zeroes p and v,
        // and x is untouched).
        HC(hipMemcpyAsync(s->hscal, s->scal, SC_COUNT * sizeof(double), hipMemcpyDeviceToHost, s->stream));
        HC(hipEventRecord(s->ev_scal, s->stream));
        if (fused != 0 && total < maxit) {
          if (fused == 1) {
            k_bicg_p<TW><<<g1, kBlock, 0, s->stream>>>(p, r, v, ks, M);
            LAUNCH_CHECK();
            keep_compatible(s, p);
            apply_fused(s, 1, 0, p, nullptr, nullptr, nullptr, v, rhat);
          } else {
            apply_fused(s, 1, 1, p, r, v, p, v, rhat);
          }
          issued = true;
        }
        HC(hipEventSynchronize(s->ev_scal));
        s->kiters++;
        const double flag = s->hscal[SC_KS + KS_FLAG];
        if (flag == 1.0 || flag == 2.0) {   // breakdown before the update
          --total;
          s->kiters--;
          break;
        }
        cur = nxt;
        const double res = std::sqrt(s->hscal[SC_KS + KS_RR]);
        if (s->ktrace && total <= 6) {
          const double* h = s->hscal + SC_KS;
          std::fprintf(stderr, "[kry %d] it %d alpha %.17g omega %.17g rv %.17g ts %.17g tt %.17g rr %.17g\n",
                       (int)sizeof(TW), total, h[KS_ALPHA], h[KS_OMEGA], h[KS_RV], h[KS_TS], h[KS_TT], h[KS_RR]);
        }
        if (res < res_best) {
          best = cur;
          res_best = res;
        }
        if (res <= rtol * bnorm) break;
        if (flag != 0.0 || !std::isfinite(res) || res > kDiverged * bnorm) break;
      }
      // true residual of the best iterate; also resets the scalars of a new run
      apply(s, xb[best], t);
      k_true_resid<TW><<<g1, kBlock, 0, s->stream>>>(r, b, t, p, v, M, s->part0);
      LAUNCH_CHECK();
      k_reduce<FinRestart><<<1, kBlock, 0, s->stream>>>(s->part0, nb, 1, FinRestart::Args{ks});
      LAUNCH_CHECK();
      sync_scal(s);
      true_res = s->hscal[SC_KS + KS_TRUE];
      if (true_res <= rtol * bnorm) conv = 1;
      if (total >= maxit) break;
    }
    k_copy<TW><<<g1, kBlock, 0, s->stream>>>(x_out, xb[best], M);
    LAUNCH_CHECK();
    if (iters) *iters = total;
    if (relres) *relres = bnorm > 0.0 ? true_res / bnorm : 0.0;
    return conv;
  }

  static void newton_update(pff_solver* s, const TW* x, double alpha) {
    const int nb = red_blocks(s->N);
    Vec16 fm{};
    for (int k = 0; k < 6; ++k) fm.v[k] = s->fm[k];
    k_newton_update<TW, C><<<nb, kBlock, 0, s->stream>>>(s->eps_t, s->phi, x, s->mask, fm, s->Edev,
                                                          alpha, s->N, s->part0);
    LAUNCH_CHECK();
    FinNewton::Args F{s->scal, s->Edev, x, std::is_same<TW, float>::value ? 1 : 0,
                      (long long)(C + 1) * s->N, alpha};
    k_reduce<FinNewton><<<1, kBlock, 0, s->stream>>>(s->part0, nb, 4, F);
    LAUNCH_CHECK();
    s->ts_valid = false;
  }

  // x[0 : C N] <- G[x[0 : C N]]: the strain block of an FP64 Krylov vector is
  // projected onto compatible fields.  Exact Newton steps from a compatible
  // state are compatible (the right-hand side and every tangent output lie in
  // the range of G), but round-off is not, and G[sigma] = 0 does not see an
  // incompatible strain: left alone, it accumulates over Newton iterations
  // and moves the iterate along the set of non-physical roots.
  static void project_strain(pff_solver* s, double* x) {
    typename CompatPipe<DIM>::Args A;
    A.g = s->g;
    A.x = x;
    A.tab = spec_tables<double>(s);
    int nblk = 0;
    run_pipeline<CompatPipe<DIM>>(s, A, nblk);
  }

  static void helm_apply(pff_solver* s, const double* u, double* out, int mask_input,
                         const double* H = nullptr) {
    HelmPipe::Args A;
    A.g = s->g;
    A.l = s->prm.l;
    A.u = u;
    A.out = out;
    A.mask_input = mask_input;
    A.mask = s->mask;
    A.tab = spec_tables<double>(s);
    A.H = H;
    A.pid = s->pid;
    A.mat = s->mat;
    int nblk = 0;
    run_pipeline<HelmPipe>(s, A, nblk);
  }

  static double dot(pff_solver* s, const double* a, const double* b, long long n) {
    const int nb = red_blocks(n);
    k_dots<double, 1><<<nb, kBlock, 0, s->stream>>>(a, b, nullptr, nullptr, nullptr, nullptr, n, s->part0);
    LAUNCH_CHECK();
    FinStore::Args fs{s->scal + SC_CG, 1};
    k_reduce<FinStore><<<1, kBlock, 0, s->stream>>>(s->part0, nb, 1, fs);
    LAUNCH_CHECK();
    sync_scal(s);
    return s->hscal[SC_CG];
  }

  // Conjugate gradients on an SPD operator (FP64): x = op^-1 b, x0 = 0,
  // stop at ||r|| <= rtol ||b||; work vectors w[0..2] (r, p, Ap) of length n.
  template <typename Op>
  static int cg(pff_solver* s, Op&& op, const double* b, double* x, double* const* w, long long n,
                double rtol, int maxit, double* relres) {
    const int g = grid1(n);
    double *r = w[0], *p = w[1], *Ap = w[2];
    k_fill<double><<<g, kBlock, 0, s->stream>>>(x, 0.0, n);
    k_copy<double><<<g, kBlock, 0, s->stream>>>(r, b, n);
    k_copy<double><<<g, kBlock, 0, s->stream>>>(p, b, n);
    LAUNCH_CHECK();
    double rr = dot(s, r, r, n);
    const double bnorm = std::sqrt(rr);
    int it = 0;
    if (relres) *relres = 0.0;
    while (bnorm > 0.0 && it < maxit) {
      ++it;
      op(p, Ap);
      const double pAp = dot(s, p, Ap, n);
      if (!(pAp > 0.0)) break;
      const double al = rr / pAp;
      k_lincomb<<<g, kBlock, 0, s->stream>>>(x, 1.0, x, al, p, n);
      k_lincomb<<<g, kBlock, 0, s->stream>>>(r, 1.0, r, -al, Ap, n);
      LAUNCH_CHECK();
      const double rr_new = dot(s, r, r, n);
      if (relres) *relres = std::sqrt(rr_new) / bnorm;
      if (std::sqrt(rr_new) <= rtol * bnorm) break;
      k_lincomb<<<g, kBlock, 0, s->stream>>>(p, 1.0, r, rr_new / rr, p, n);
      LAUNCH_CHECK();
      rr = rr_new;
    }
    return it;
  }

  // Damage field of the Helmholtz problem with history H (signed, as written
  // by the residual pass): (1/l + 2H/Gc) phi - l Lap phi = 2H/Gc off the crack
  // mask, phi = 1 on it (paper eq. LinearOpe_Helm divided by Gc).  phi =
  // m + (1-m) u, CG on u.
  static int helm_solve(pff_solver* s, const double* H, double* phi, double rtol, int maxit) {
    const long long N = s->N;
    const int g = grid1(N);
    double* b = s->cgv[0];
    double* u = s->cgv[1];
    double* w[3] = {s->cgv[2], s->cgv[3], vec(s, X0)};
    k_mask_to_double<<<g, kBlock, 0, s->stream>>>(s->dmask, s->mask, N);
    LAUNCH_CHECK();
    helm_apply(s, s->dmask, b, 0, H);                    // (1-m) B m = -(1-m) l Lap m
    k_helm_rhs<<<g, kBlock, 0, s->stream>>>(b, H, s->mask, s->pid, s->mat, N);
    LAUNCH_CHECK();
    const int it = cg(s, [&](const double* x, double* y) { helm_apply(s, x, y, 1, H); }, b, u, w, N, rtol,
                      maxit, nullptr);
    k_phi0<<<g, kBlock, 0, s->stream>>>(phi, u, s->mask, N);
    LAUNCH_CHECK();
    return it;
  }

  // max |x_i| over n entries (device slot SC_CG + 1, host copy after sync)
  static double absmax(pff_solver* s, const double* x, long long n) {
    const int nb = red_blocks(n);
    k_absmax<<<nb, kBlock, 0, s->stream>>>(x, n, s->part0);
    k_max_final<<<1, kBlock, 0, s->stream>>>(s->part0, nb, s->scal + SC_CG + 1);
    LAUNCH_CHECK();
    sync_scal(s);
    return s->hscal[SC_CG + 1];
  }

  // Mechanical sub-problem of the staggered scheme at fixed phi and E (device
  // Edev[0]): Newton on G[sigma(f E + eps~, phi)] = 0, each step solving
  // G[C_i : d] = -G[sigma_i] by CG with the FP64 tangent restricted to the
  // strain rows; stops when max|d| / (|E| ||f||) < tol.  Returns the Newton
  // count (0: no convergence); CG iterations are added to *cg_total.
  static int mechanical(pff_solver* s, const pff_stagger_params& sp, double nf, long long* cg_total) {
    const long long N = s->N, M = s->M;
    double* rhs = vec(s, RHS);
    double* d = vec(s, SOL);
    double* w[3] = {vec(s, R), vec(s, P), vec(s, V)};
    for (int it = 1; it <= sp.max_newton; ++it) {
      residual(s, 0.0, nullptr);
      k_fill<double><<<grid1(N + 1), kBlock, 0, s->stream>>>(rhs + (long long)C * N, 0.0, N + 1);
      LAUNCH_CHECK();
      const int k = cg(s, [&](const double* x, double* y) { apply(s, x, y, 1); }, rhs, d, w, M, sp.cg_rtol,
                       sp.cg_maxit, nullptr);
      *cg_total += k;
      s->kiters += k;
      project_strain(s, d);
      k_axpy<<<grid1((long long)C * N), kBlock, 0, s->stream>>>(s->eps_t, 1.0, d, (long long)C * N);
      LAUNCH_CHECK();
      s->ts_valid = false;
      if (nf == 0.0) return it;
      const double dm = absmax(s, d, (long long)C * N);
      if (!std::isfinite(dm)) return 0;
      if (dm / nf < sp.tol_mech) return it;
    }
    return 0;
  }

  // One strain-controlled increment (Algorithm 1) from the committed state at
  // load E (device Edev[0]): stagger iterations of the mechanical and the
  // Helmholtz sub-problem until both fields settle.  Leaves the final state in
  // eps_t / phi and its residual pass (sigma, Gamma, history) in the scalars.
  static int stagger(pff_solver* s, const pff_stagger_params& sp, double E, pff_stagger_result* out) {
    const long long N = s->N;
    double* eps_prev = vec(s, X1);
    double* phi_prev = vec(s, X2);
    double fn = 0.0;
    for (int k = 0; k < C; ++k) fn += s->fm[k] * s->fm[k];
    const double nf = std::sqrt(fn) * std::fabs(E);
    Vec16 fm{};
    for (int k = 0; k < 6; ++k) fm.v[k] = s->fm[k];
    long long cgm = 0, cgh = 0;
    int newton = 0, st = 0, conv = 0;
    double err = 0.0;
    for (st = 1; st <= sp.max_stagger; ++st) {
      HC(hipMemcpyAsync(eps_prev, s->eps_t, C * N * sizeof(double), hipMemcpyDeviceToDevice, s->stream));
      HC(hipMemcpyAsync(phi_prev, s->phi, N * sizeof(double), hipMemcpyDeviceToDevice, s->stream));
      const int it = mechanical(s, sp, nf, &cgm);
      if (it == 0) break;
      newton += it;
      residual(s, 0.0, nullptr);                 // history H = max(psi+(eps), Hn) of the new strain
      cgh += helm_solve(s, s->Hcur, s->phi, sp.cg_rtol, sp.cg_maxit);
      const int nb = red_blocks(N);
      k_stagger_norms<C><<<nb, kBlock, 0, s->stream>>>(s->eps_t, eps_prev, s->phi, phi_prev, fm, s->Edev, N,
                                                      s->part0);
      FinStore::Args fs{s->scal + SC_CG + 2, 4};
      k_reduce<FinStore><<<1, kBlock, 0, s->stream>>>(s->part0, nb, 4, fs);
      LAUNCH_CHECK();
      sync_scal(s);
      const double* h = s->hscal + SC_CG + 2;
      // a relative change of zero is zero, also over a zero norm (E = 0)
      auto rel = [](double num, double den) {
        return num == 0.0 ? 0.0 : (den > 0.0 ? num / den : HUGE_VAL);
      };
      err = std::max(rel(std::sqrt(h[0]), std::sqrt(h[1])), rel(std::sqrt(h[2]), std::sqrt(h[3])));
      if (s->trace)
        std::fprintf(stderr, "[pff] stagger %d newton %d err %.3e\n", st, it, err);
      if (std::isnan(err)) break;
      if (err < sp.tol_sta) {
        conv = 1;
        break;
      }
    }
    if (st > sp.max_stagger) st = sp.max_stagger;
    if (conv) residual(s, 0.0, nullptr);         // sigma and Gamma at the final fields
    if (out) {
      out->stagger_iters = st;
      out->newton_iters = newton;
      out->cg_mech = cgm;
      out->cg_helm = cgh;
      out->err = err;
      out->converged = conv;
    }
    return conv;
  }

  // phi0: masked damage-free Helmholtz problem by CG (rtol 1e-14)
  static void initial_damage(pff_solver* s, double* phi0) {
    const long long N = s->N;
    const int g = grid1(N);
    if (!s->has_mask) {
      k_fill<double><<<g, kBlock, 0, s->stream>>>(phi0, 0.0, N);
      LAUNCH_CHECK();
      return;
    }
    double *x = s->cgv[0], *r = s->cgv[1], *p = s->cgv[2], *Ap = s->cgv[3];
    k_mask_to_double<<<g, kBlock, 0, s->stream>>>(s->dmask, s->mask, N);
    LAUNCH_CHECK();
    helm_apply(s, s->dmask, r, 0);                       // (1-m) B m
    k_lincomb<<<g, kBlock, 0, s->stream>>>(r, -1.0, r, 0.0, nullptr, N);   // r = b = -(1-m) B m
    k_fill<double><<<g, kBlock, 0, s->stream>>>(x, 0.0, N);
    k_copy<double><<<g, kBlock, 0, s->stream>>>(p, r, N);
    LAUNCH_CHECK();
    double rr = dot(s, r, r, N);
    const double bnorm = std::sqrt(rr);
    for (int it = 1; it <= 20000 && bnorm > 0.0; ++it) {
      helm_apply(s, p, Ap, 1);
      const double pAp = dot(s, p, Ap, N);
      const double al = rr / pAp;
      k_lincomb<<<g, kBlock, 0, s->stream>>>(x, 1.0, x, al, p, N);
      k_lincomb<<<g, kBlock, 0, s->stream>>>(r, 1.0, r, -al, Ap, N);
      LAUNCH_CHECK();
      const double rr_new = dot(s, r, r, N);
      if (std::sqrt(rr_new) <= 1e-14 * bnorm) break;
      k_lincomb<<<g, kBlock, 0, s->stream>>>(p, 1.0, r, rr_new / rr, p, N);
      LAUNCH_CHECK();
      rr = rr_new;
    }
    k_phi0<<<g, kBlock, 0, s->stream>>>(phi0, x, s->mask, N);
    LAUNCH_CHECK();
  }
};

// ---- batched FP32 inner solves (request server) --------------------------------

}  // namespace

namespace pff {

// One FP32 BiCGSTAB solve handed to the engine: x = J^{-1} b at the solver's
// tangent state, with the run control of Impl::bicgstab (best iterate,
// true-residual check and restart at the end of every run).
struct KJob {
  pff_solver* s = nullptr;
  const float* b = nullptr;
  float* x = nullptr;
  double rtol = 0.0;
  int maxit = 0;
  hipStream_t slot = nullptr;   // the solver's own stream while the engine holds it
  int cycle = 0, total = 0, best = 0, conv = 0;
  double bnorm = 0.0, true_res = 0.0;
  long long applies = 0;
  bool finished = false;        // set under the batcher's lock
  bool failed = false;          // a device error ended the solve
};

// Solves in flight on one grid (a size class): they share launches.  Acts as
// the pass context of run_pipeline (plans, launch knobs, its own twiddles).
struct KClass {
  int nx = 0, ny = 0, nz = 0, dim = 0;
  GridDesc g{};
  AxisPlan plan[3]{};
  bool plan_any = false;
  hipStream_t stream = nullptr;
  int x_rows = 64, spec_threads = 512, spec_tx = 8, axis_threads = 0, axis_tx = 16, xcd_remap = 1, zspec = 1, yreg = 0, fit_shapes = 1;
  GraphRec* rec = nullptr;     // set while a chunk graph is being built
  size_t part_len = 0;
  double* part0 = nullptr;
  double* part1 = nullptr;
  DevTables<float> tf;
  DevTables<double> td;
  long long N = 0, M = 0;
  int C = 0;
  std::vector<KJob*> pending, active;
  // batch arrays (capacity bmax): entries of the two applies, Krylov entries
  void* d_ent1 = nullptr;
  void* d_ent2 = nullptr;
  KryEntry<float>* d_kry = nullptr;
  double* d_flags = nullptr;
  unsigned char* h_ent1 = nullptr;   // pinned staging
  unsigned char* h_ent2 = nullptr;
  KryEntry<float>* h_kry = nullptr;
  double* h_flags = nullptr;
  std::vector<void*> dev_allocs;
  std::map<int, hipGraphExec_t> graphs;   // per batch size
  std::thread th;                         // this class's engine thread
  std::condition_variable cv;             // new solves for it
  template <typename T> const DevTables<T>& tables() const;
  template <typename T> cpx<T>* spec() const { return nullptr; }
};
template <> const DevTables<float>& KClass::tables<float>() const { return tf; }
template <> const DevTables<double>& KClass::tables<double>() const { return td; }

struct KBatcher {
  int device = 0, bmax = 8, chunk = 4, graph = 1;
  std::mutex m;
  std::condition_variable cv_done;
  std::vector<std::unique_ptr<KClass>> classes;
  bool stop = false;
  KBatcherStats st{};
  std::string err;
};

}  // namespace pff

namespace {

size_t entry_bytes(int dim) {
  return dim == 2 ? sizeof(BatchEntry<TangentPipe<float, 2>>) : sizeof(BatchEntry<TangentPipe<float, 3>>);
}

void* kclass_alloc(KClass& c, size_t bytes) {
  void* p = nullptr;
  HC(hipMalloc(&p, bytes));
  c.dev_allocs.push_back(p);
  return p;
}

void class_engine(KBatcher* kb, KClass* c);

// Size class of solver s (created on first use, with its engine thread,
// under the batcher's lock).
KClass* kclass_of(KBatcher* kb, pff_solver* s) {
  for (auto& c : kb->classes)
    if (c->nx == s->nx && c->ny == s->ny && c->nz == s->nz) return c.get();
  auto c = std::make_unique<KClass>();
  c->nx = s->nx;
  c->ny = s->ny;
  c->nz = s->nz;
  c->dim = s->dim;
  c->g = s->g;
  for (int a = 0; a < 3; ++a) c->plan[a] = s->plan[a];
  c->plan_any = s->plan_any;
  c->x_rows = s->x_rows;
  c->spec_threads = s->spec_threads;
  c->spec_tx = s->spec_tx;
  c->axis_threads = s->axis_threads;
  c->axis_tx = s->axis_tx;
  c->xcd_remap = s->xcd_remap;
  c->zspec = s->zspec;
  c->fit_shapes = s->fit_shapes;
  c->yreg = s->yreg;
  c->part_len = s->part_len;
  c->N = s->N;
  c->M = s->M;
  c->C = s->C;
  HC(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
  const int ns[3] = {s->nx, s->ny, s->nz};
  for (int a = 0; a < 3; ++a) {
    c->tf.tw[a] = static_cast<cpx<float>*>(kclass_alloc(*c, ns[a] * sizeof(cpx<float>)));
    HC(hipMemcpy(c->tf.tw[a], s->tf.tw[a], ns[a] * sizeof(cpx<float>), hipMemcpyDeviceToDevice));
  }
  const size_t eb = entry_bytes(c->dim) * kb->bmax;
  c->d_ent1 = kclass_alloc(*c, eb);
  c->d_ent2 = kclass_alloc(*c, eb);
  c->d_kry = static_cast<KryEntry<float>*>(kclass_alloc(*c, sizeof(KryEntry<float>) * kb->bmax));
  c->d_flags = static_cast<double*>(kclass_alloc(*c, 4 * sizeof(double) * kb->bmax));
  HC(hipHostMalloc((void**)&c->h_ent1, eb, hipHostMallocDefault));
  HC(hipHostMalloc((void**)&c->h_ent2, eb, hipHostMallocDefault));
  HC(hipHostMalloc((void**)&c->h_kry, sizeof(KryEntry<float>) * kb->bmax, hipHostMallocDefault));
  HC(hipHostMalloc((void**)&c->h_flags, 4 * sizeof(double) * kb->bmax, hipHostMallocDefault));
  KClass* cp = c.get();
  kb->classes.push_back(std::move(c));
  cp->th = std::thread(class_engine, kb, cp);
  return cp;
}

void kclass_free(KClass& c) {
  for (auto& ge : c.graphs) (void)hipGraphExecDestroy(ge.second);
  c.graphs.clear();
  if (c.stream) (void)hipStreamSynchronize(c.stream);
  for (void* p : c.dev_allocs) (void)hipFree(p);
  c.dev_allocs.clear();
  if (c.h_ent1) (void)hipHostFree(c.h_ent1);
  if (c.h_ent2) (void)hipHostFree(c.h_ent2);
  if (c.h_kry) (void)hipHostFree(c.h_kry);
  if (c.h_flags) (void)hipHostFree(c.h_flags);
  if (c.stream) (void)hipStreamDestroy(c.stream);
  c.stream = nullptr;
}

// The pipe and Krylov entries of one solve (FP32 vectors of the solver).
template <int DIM>
void fill_entries(KClass& c, int b, KJob* j) {
  using I = Impl<DIM, float>;
  using Pipe = TangentPipe<float, DIM>;
  pff_solver* s = j->s;
  float *r = I::vec(s, I::R), *rhat = I::vec(s, I::RHAT), *p = I::vec(s, I::P), *v = I::vec(s, I::V),
        *sv = I::vec(s, I::S), *t = I::vec(s, I::T);
  double* ks = s->scal + SC_KS;
  BatchEntry<Pipe> e1{};
  I::fill_tangent_args(s, e1.A);
  e1.A.mode = 1;
  e1.A.pro = 0;
  e1.A.mech = 0;
  e1.A.lgc = nullptr;
  e1.A.r = e1.A.w = nullptr;
  e1.A.vout = nullptr;
  e1.A.ks = ks;
  e1.spec = s->spec<float>();
  e1.part0 = s->part0;
  e1.part1 = s->part1;
  e1.stop = ks + KS_STOP;
  BatchEntry<Pipe> e2 = e1;
  e1.A.v = p;
  e1.A.Jv = v;
  e1.A.dv = rhat;
  e2.A.mode = 2;
  e2.A.v = sv;
  e2.A.Jv = t;
  e2.A.dv = sv;
  std::memcpy(c.h_ent1 + b * sizeof(e1), &e1, sizeof(e1));
  std::memcpy(c.h_ent2 + b * sizeof(e2), &e2, sizeof(e2));
  KryEntry<float> k{};
  for (int q = 0; q < 3; ++q) k.x[q] = I::vec(s, I::X0 + q);
  k.r = r;
  k.rhat = rhat;
  k.p = p;
  k.v = v;
  k.s = sv;
  k.t = t;
  k.ks = ks;
  k.part = s->part0;
  k.part0 = s->part0;
  k.part1 = s->part1;
  k.wa = s->wa;
  k.wE = s->wE;
  c.h_kry[b] = k;
}

// One BiCGSTAB iteration of every solve of the batch (the kernel sequence of
// Impl::bicgstab with fused applies, one grid dimension over the solves).
// The vector reduction of k_bicg_xr_b and the apply epilogues share the
// solver's partial buffers in stream order, as in the unbatched solve.
template <int DIM>
void batched_iteration(KClass& c, int B) {
  using Pipe = TangentPipe<float, DIM>;
  const long long M = c.M;
  const int g1 = red_blocks(M);
  const long long last = (long long)(c.C + 1) * c.N;
  const typename Pipe::Args none{};
  auto* e1 = static_cast<const BatchEntry<Pipe>*>(c.d_ent1);
  auto* e2 = static_cast<const BatchEntry<Pipe>*>(c.d_ent2);
  int nblk = 0;
  const KryEntry<float>* kry = c.d_kry;
  launch_k(c.rec, k_bicg_p_b<float>, dim3(g1, B), dim3(kBlock), 0, c.stream, kry, M);
  run_pipeline<Pipe>(&c, none, nblk, nullptr, e1, B);
  launch_k(c.rec, k_fin_fused_b<float>, dim3(B), dim3(kBlock), 0, c.stream, kry, nblk, 1, last);
  launch_k(c.rec, k_bicg_s_b<float>, dim3(g1, B), dim3(kBlock), 0, c.stream, kry, M);
  run_pipeline<Pipe>(&c, none, nblk, nullptr, e2, B);
  launch_k(c.rec, k_fin_fused_b<float>, dim3(B), dim3(kBlock), 0, c.stream, kry, nblk, 2, last);
  launch_k(c.rec, k_bicg_xr_b<float>, dim3(g1, B), dim3(kBlock), 0, c.stream, kry, M);
  launch_k(c.rec, k_fin_rr_b<float>, dim3(B), dim3(kBlock), 0, c.stream, kry, g1, kDiverged);
}

template <int DIM>
void launch_chunk(KBatcher* kb, KClass& c, int B) {
  const size_t eb = entry_bytes(c.dim);
  HC(hipMemcpyAsync(c.d_ent1, c.h_ent1, eb * B, hipMemcpyHostToDevice, c.stream));
  HC(hipMemcpyAsync(c.d_ent2, c.h_ent2, eb * B, hipMemcpyHostToDevice, c.stream));
  HC(hipMemcpyAsync(c.d_kry, c.h_kry, sizeof(KryEntry<float>) * B, hipMemcpyHostToDevice, c.stream));
  if (kb->graph) {
    auto it = c.graphs.find(B);
    if (it == c.graphs.end()) {
      GraphRec rec;
      HC(hipGraphCreate(&rec.g, 0));
      c.rec = &rec;
      try {
        for (int k = 0; k < kb->chunk; ++k) batched_iteration<DIM>(c, B);
      } catch (...) {
        c.rec = nullptr;
        (void)hipGraphDestroy(rec.g);
        throw;
      }
      c.rec = nullptr;
      hipGraphExec_t ex = nullptr;
      const hipError_t e = hipGraphInstantiate(&ex, rec.g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(rec.g);
      HC(e);
      it = c.graphs.emplace(B, ex).first;
      kb->st.graphs++;
    }
    HC(hipGraphLaunch(it->second, c.stream));
  } else {
    for (int k = 0; k < kb->chunk; ++k) batched_iteration<DIM>(c, B);
  }
  k_gather_run<float><<<1, 64, 0, c.stream>>>(c.d_kry, B, c.d_flags);
  LAUNCH_CHECK();
  HC(hipMemcpyAsync(c.h_flags, c.d_flags, 4 * sizeof(double) * B, hipMemcpyDeviceToHost, c.stream));
}

// Start of a run of job j: shadow residual, rho, and the device run control.
template <int DIM>
void job_run_start(KJob* j, int cur, double resbest) {
  using I = Impl<DIM, float>;
  pff_solver* s = j->s;
  const int g1 = red_blocks(s->M);
  double* ks = s->scal + SC_KS;
  k_bicg_shadow<float><<<g1, kBlock, 0, s->stream>>>(I::vec(s, I::R), I::vec(s, I::RHAT), ks, kShadowSeed, s->M,
                                                    s->part0);
  LAUNCH_CHECK();
  I::reduce_ks(s, 1, 1);
  k_ks_run_start<<<1, 64, 0, s->stream>>>(ks, double(j->total), double(cur), resbest, j->rtol, double(j->maxit));
  LAUNCH_CHECK();
}

template <int DIM>
void job_finish(KJob* j) {
  using I = Impl<DIM, float>;
  pff_solver* s = j->s;
  k_copy<float><<<red_blocks(s->M), kBlock, 0, s->stream>>>(j->x, I::vec(s, I::X0 + j->best), s->M);
  LAUNCH_CHECK();
  HC(hipEventRecord(s->kb_done, s->stream));
  s->kiters += j->total;
  s->applies += j->applies;
  s->stream = j->slot;
}

// Admission: x = 0, r = b, ||b||; returns false when the solve is finished.
template <int DIM>
bool job_admit(KClass& c, KJob* j) {
  using I = Impl<DIM, float>;
  pff_solver* s = j->s;
  j->slot = s->stream;
  s->stream = c.stream;
  HC(hipStreamWaitEvent(c.stream, s->kb_ready, 0));
  const int g1 = red_blocks(s->M);
  k_bicg_init<float><<<g1, kBlock, 0, s->stream>>>(j->b, I::vec(s, I::X0), I::vec(s, I::R), I::vec(s, I::P),
                                                  I::vec(s, I::V), s->M, s->part0);
  LAUNCH_CHECK();
  I::reduce_ks(s, 1, 0);
  j->best = 0;
  job_run_start<DIM>(j, 0, -1.0);     // ||b|| stays on the device until the run ends
  return true;
}

// End of a run (the device stopped it): the true residual of the best
// iterate decides between convergence, the end of the solve and a new run.
template <int DIM>
bool job_run_end(KJob* j, int total, int best) {
  using I = Impl<DIM, float>;
  pff_solver* s = j->s;
  const int g1 = red_blocks(s->M);
  j->applies += 2LL * (total - j->total);
  j->total = total;
  j->best = best;
  I::apply(s, I::vec(s, I::X0 + best), I::vec(s, I::T));
  s->applies--;                              // counted in j->applies
  j->applies++;
  k_true_resid<float><<<g1, kBlock, 0, s->stream>>>(I::vec(s, I::R), j->b, I::vec(s, I::T), I::vec(s, I::P),
                                                   I::vec(s, I::V), s->M, s->part0);
  LAUNCH_CHECK();
  k_reduce<FinRestart><<<1, kBlock, 0, s->stream>>>(s->part0, g1, 1, FinRestart::Args{s->scal + SC_KS});
  LAUNCH_CHECK();
  sync_scal(s);
  j->bnorm = s->hscal[SC_KS + KS_BNORM];
  j->true_res = s->hscal[SC_KS + KS_TRUE];
  if (j->true_res <= j->rtol * j->bnorm) j->conv = 1;
  if (j->conv || j->total >= j->maxit || ++j->cycle >= kMaxCycles) {
    job_finish<DIM>(j);
    return false;
  }
  job_run_start<DIM>(j, best, j->true_res);
  return true;
}

template <int DIM>
void class_admit(KClass& c, std::vector<KJob*>& in, std::vector<KJob*>& done) {
  for (KJob* j : in) {
    if (job_admit<DIM>(c, j)) c.active.push_back(j);
    else done.push_back(j);
  }
}

template <int DIM>
void class_collect(KClass& c, int B, std::vector<KJob*>& done) {
  HC(hipStreamSynchronize(c.stream));
  std::vector<KJob*> keep;
  for (int b = 0; b < B; ++b) {
    KJob* j = c.active[b];
    const double* f = c.h_flags + 4 * b;
    if (f[0] == 0.0) {
      keep.push_back(j);
      continue;
    }
    // the device stopped this run: the true residual of its best iterate
    if (job_run_end<DIM>(j, int(f[2]), int(f[3]))) keep.push_back(j);
    else done.push_back(j);
  }
  for (size_t b = B; b < c.active.size(); ++b) keep.push_back(c.active[b]);
  c.active.swap(keep);
}

// Engine thread of one size class: admit the solves handed in, run a chunk
// of batched iterations over (at most bmax of) the solves in flight, collect
// the runs the device stopped, repeat.  Device errors end the solves in
// flight with an error.
void class_engine(KBatcher* kb, KClass* cp) {
  KClass& c = *cp;
  (void)hipSetDevice(kb->device);
  std::unique_lock<std::mutex> lk(kb->m);
  for (;;) {
    c.cv.wait(lk, [&] { return kb->stop || !c.pending.empty() || !c.active.empty(); });
    if (c.pending.empty() && c.active.empty()) break;   // stop with nothing in flight
    std::vector<KJob*> in;
    in.swap(c.pending);
    lk.unlock();
    std::vector<KJob*> done;
    int B = 0;
    try {
      if (c.dim == 2) class_admit<2>(c, in, done);
      else class_admit<3>(c, in, done);
      B = (int)std::min<size_t>(c.active.size(), (size_t)kb->bmax);
      if (B > 0) {
        for (int b = 0; b < B; ++b) {
          if (c.dim == 2) fill_entries<2>(c, b, c.active[b]);
          else fill_entries<3>(c, b, c.active[b]);
        }
        if (c.dim == 2) launch_chunk<2>(kb, c, B);
        else launch_chunk<3>(kb, c, B);
        if (c.dim == 2) class_collect<2>(c, B, done);
        else class_collect<3>(c, B, done);
      }
    } catch (const std::exception& e) {
      lk.lock();
      kb->err = e.what();
      for (KJob* j : in) done.push_back(j);
      for (KJob* j : c.active) done.push_back(j);
      c.active.clear();
      for (KJob* j : done) {
        if (j->slot) j->s->stream = j->slot;
        j->failed = true;
        j->finished = true;
      }
      kb->cv_done.notify_all();
      continue;
    }
    lk.lock();
    if (B > 0) {
      kb->st.chunks++;
      kb->st.rve_chunks += B;
      kb->st.max_batch = std::max(kb->st.max_batch, B);
    }
    for (KJob* j : done) {
      j->finished = true;
      kb->st.solves++;
      kb->st.iterations += j->total;
    }
    if (!done.empty()) kb->cv_done.notify_all();
  }
}

// Slot thread: hand the solve to the engine and wait for it.
int kbatcher_solve(pff_solver* s, const float* b, float* x, double rtol, int maxit, int* iters, double* relres) {
  KBatcher* kb = s->kb;
  KJob j;
  j.s = s;
  j.b = b;
  j.x = x;
  j.rtol = rtol;
  j.maxit = maxit;
  HC(hipEventRecord(s->kb_ready, s->stream));
  {
    std::unique_lock<std::mutex> lk(kb->m);
    if (kb->stop) throw Fail("request server is shutting down", PFF_ERR_STATE);
    KClass* c = kclass_of(kb, s);
    c->pending.push_back(&j);
    c->cv.notify_one();
    kb->cv_done.wait(lk, [&] { return j.finished; });
    if (j.failed) throw Fail("batched Krylov engine: " + kb->err, PFF_ERR_DEVICE);
  }
  HC(hipStreamWaitEvent(s->stream, s->kb_done, 0));
  if (iters) *iters = j.total;
  if (relres) *relres = j.bnorm > 0.0 ? j.true_res / j.bnorm : 0.0;
  return j.conv;
}

}  // namespace

namespace pff {

KBatcher* kbatcher_create(int device, int bmax, int chunk, int graph) {
  auto* kb = new (std::nothrow) KBatcher();
  if (!kb) return nullptr;
  kb->device = device;
  kb->bmax = std::max(1, std::min(bmax, 64));
  kb->chunk = std::max(1, std::min(chunk, 64));
  kb->graph = graph ? 1 : 0;
  return kb;
}

void kbatcher_destroy(KBatcher* kb) {
  if (!kb) return;
  {
    std::lock_guard<std::mutex> lk(kb->m);
    kb->stop = true;
    for (auto& c : kb->classes) c->cv.notify_all();
  }
  for (auto& c : kb->classes)
    if (c->th.joinable()) c->th.join();
  (void)hipSetDevice(kb->device);
  for (auto& c : kb->classes) kclass_free(*c);
  delete kb;
}

void kbatcher_stats(KBatcher* kb, KBatcherStats* out) {
  std::lock_guard<std::mutex> lk(kb->m);
  *out = kb->st;
}

void serving_shapes(pff_solver* s) { s->fit_shapes = 0; }

void kbatcher_attach(pff_solver* s, KBatcher* kb) {
  if (kb && (s->var_het || !s->mixed())) kb = nullptr;   // batched: FP32 inner solves, plain toughness term
  if (kb && !s->kb_ready) {
    HC(hipEventCreateWithFlags(&s->kb_ready, hipEventDisableTiming));
    HC(hipEventCreateWithFlags(&s->kb_done, hipEventDisableTiming));
  }
  s->kb = kb;
}

}  // namespace pff

namespace {

// Newton linear solve J dq = -F into the FP64 vector SOL, to the FP64
// relative residual rtol.  FP64 mode: one FP64 BiCGSTAB.  Mixed mode: FP64
// iterative refinement around FP32 solves: BiCGSTAB on the FP32 tangent
// solves J d = r to kInner32, the step is accumulated in FP64 and the defect
// r = -F - J dq is re-evaluated with the FP64 tangent, until it is below
// rtol.  Refinement that stops contracting (the FP32 tangent cannot resolve
// the soft modes of a nearly broken crack, stiffness k) hands the remaining
// defect to an FP64 BiCGSTAB.
template <int DIM>
void newton_linear_solve(pff_solver* s, int* kit, double* eta_out) {
  using I64 = Impl<DIM, double>;
  using I32 = Impl<DIM, float>;
  const double rtol = s->prm.krylov_rtol;
  const int maxit = s->prm.krylov_maxit;
  if (!s->mixed()) {
    I64::bicgstab(s, I64::vec(s, I64::RHS), I64::vec(s, I64::SOL), rtol, maxit, kit, eta_out);
    I64::project_strain(s, I64::vec(s, I64::SOL));
    return;
  }
  const long long M = s->M;
  const int nb = red_blocks(M);
  const double rtol_in = std::max(rtol, s->inner32);
  const int maxit32 = std::min(maxit, kMixedMaxit32);
  double* sol = I64::vec(s, I64::SOL);
  double* defect = I64::vec(s, I64::VB);
  float* rhs32 = I32::vec(s, I32::RHS);
  float* sol32 = I32::vec(s, I32::SOL);
  int k32 = 0, k64 = 0, kk = 0;
  double rr = 0.0, eta = 0.0, eta_prev = 1.0;
  auto solve32 = [&]() {
    if (s->kb) kbatcher_solve(s, rhs32, sol32, rtol_in, maxit32, &kk, &rr);
    else I32::bicgstab(s, rhs32, sol32, rtol_in, maxit32, &kk, &rr);
  };
  solve32();
  k32 += kk;
  k_widen<<<nb, kBlock, 0, s->stream>>>(sol, sol32, M);
  LAUNCH_CHECK();
  I64::project_strain(s, sol);
  for (int ref = 0;; ++ref) {
    I64::apply(s, sol, I64::vec(s, I64::T));
    k_resid_pair<<<nb, kBlock, 0, s->stream>>>(defect, I64::vec(s, I64::RHS), I64::vec(s, I64::T), M,
                                               s->part0);
    LAUNCH_CHECK();
    k_reduce<FinStore><<<1, kBlock, 0, s->stream>>>(s->part0, nb, 2, FinStore::Args{s->scal + SC_ETA, 2});
    LAUNCH_CHECK();
    sync_scal(s);
    const double rr2 = s->hscal[SC_ETA], bb = s->hscal[SC_ETA + 1];
    eta = bb > 0.0 ? std::sqrt(rr2 / bb) : 0.0;
    if (eta <= rtol) break;
    if (ref >= kMaxRefine || !(eta < kRefineContract * eta_prev)) {
      double rr64 = 0.0;
      const double rt = std::min(0.5, rtol / eta);
      I64::bicgstab(s, defect, I64::vec(s, I64::VD), rt, maxit, &k64, &rr64);
      k_add<<<nb, kBlock, 0, s->stream>>>(sol, I64::vec(s, I64::VD), M);
      LAUNCH_CHECK();
      I64::project_strain(s, sol);
      eta *= rr64;
      s->fallbacks++;
      break;
    }
    eta_prev = eta;
    // FP32 solve for the correction, right-hand side scaled to unit norm
    const double rn = std::sqrt(rr2);
    k_narrow_scaled<<<nb, kBlock, 0, s->stream>>>(rhs32, defect, 1.0 / rn, M);
    LAUNCH_CHECK();
    solve32();
    k32 += kk;
    k_axpy_widen<<<nb, kBlock, 0, s->stream>>>(sol, sol32, rn, M);
    LAUNCH_CHECK();
    I64::project_strain(s, sol);
    s->refinements++;
  }
  *kit = k32 + k64;
  *eta_out = eta;
}

template <typename F> void dispatch_dim(pff_solver* s, F&& fn) {
  if (s->dim == 2) fn(std::integral_constant<int, 2>());
  else fn(std::integral_constant<int, 3>());
}

// ---- host-side predictor --------------------------------------------------------

// psi0(+) of a symmetric tensor (3x3, or its in-plane 2x2 block in 2D)
// history driver of the homogeneous strain f (E = 1): psi0(+) of the split
// model, or the whole psi0 of the isotropic one
double psi_plus_host(const double f[9], double lam, double mu, int dim, int iso) {
  double A[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) A[i][j] = 0.5 * (f[3 * i + j] + f[3 * j + i]);
  const int D = dim == 2 ? 2 : 3;
  if (D == 2) A[2][2] = A[0][2] = A[2][0] = A[1][2] = A[2][1] = 0.0;
  // cyclic Jacobi (eigenvalues only)
  for (int sweep = 0; sweep < 50; ++sweep) {
    double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    if (off < 1e-300) break;
    for (int pq = 0; pq < 3; ++pq) {
      const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2, o = 3 - p - q;
      const double apq = A[p][q];
      if (apq == 0.0) continue;
      const double th = (A[q][q] - A[p][p]) / (2.0 * apq);
      const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
      const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
      A[p][p] -= t * apq;
      A[q][q] += t * apq;
      A[p][q] = A[q][p] = 0.0;
      const double aop = A[o][p], aoq = A[o][q];
      A[o][p] = A[p][o] = c * aop - sn * aoq;
      A[o][q] = A[q][o] = sn * aop + c * aoq;
    }
  }
  double tr = 0.0, sq = 0.0;
  for (int a = 0; a < D; ++a) {
    tr += A[a][a];
    const double zp = (iso || A[a][a] > 0.0) ? A[a][a] : 0.0;
    sq += zp * zp;
  }
  const double trp = (iso || tr > 0.0) ? tr : 0.0;
  return 0.5 * lam * trp * trp + mu * sq;
}

pff_status fail(pff_solver* s, const Fail& e) {
  if (s) s->err = e.what();
  return e.code;
}

template <typename F> pff_status guarded(pff_solver* s, F&& fn) {
  if (!s) return PFF_ERR_ARG;
  try {
    s->err.clear();
    return fn();
  } catch (const Fail& e) {
    return fail(s, e);
  } catch (const std::exception& e) {
    s->err = e.what();
    return PFF_ERR_DEVICE;
  }
}

template <typename F> void dispatch(pff_solver* s, F&& fn) {
  if (s->dim == 2) {
    if (s->mixed()) fn(Impl<2, float>{});
    else fn(Impl<2, double>{});
  } else {
    if (s->mixed()) fn(Impl<3, float>{});
    else fn(Impl<3, double>{});
  }
}

template <typename T>
void upload_tables(pff_solver* s, DevTables<T>& t) {
  const int ns[3] = {s->nx, s->ny, s->nz};
  for (int a = 0; a < 3; ++a) {
    const int n = ns[a];
    std::vector<cpx<T>> tw(n);
    std::vector<T> hs(n), hc(n), q2(n);
    for (int j = 0; j < n; ++j) {
      const long double ang = -2.0L * 3.14159265358979323846264338327950288L * (long double)j / n;
      tw[j] = cpx<T>{T(cosl(ang)), T(sinl(ang))};
      const int m = (2 * j < n) ? j : j - n;      // signed frequency, Nyquist reads -n/2
      const long double half = 3.14159265358979323846264338327950288L * (long double)m / n;
      const long double q = 2.0L * half;
      const bool nyq = n % 2 == 0 && 2 * j == n;
      if (s->prm.projection == PFF_PROJ_STANDARD) {
        // r_j = xi_j: the plain frequency, 0 at the Nyquist index (no sign)
        hs[j] = nyq ? T(0) : T(q);
        hc[j] = T(1);
      } else {
        // rotated scheme: r_j = sin(q_j/2) prod_{m != j} cos(q_m/2)
        hs[j] = T(sinl(half));
        hc[j] = nyq ? T(0) : T(cosl(half));
      }
      // Laplacian symbol: spectral (Nyquist kept), or the finite-difference
      // one of the variational toughness term, 4 sin^2(q/2)
      q2[j] = s->prm.gc_form == PFF_GC_VARIATIONAL ? T(4.0L * sinl(half) * sinl(half)) : T(q * q);
    }
    t.tw[a] = s->alloc<cpx<T>>(n);
    t.hs[a] = s->alloc<T>(n);
    t.hc[a] = s->alloc<T>(n);
    t.q2[a] = s->alloc<T>(n);
    HC(hipMemcpy(t.tw[a], tw.data(), n * sizeof(cpx<T>), hipMemcpyHostToDevice));
    HC(hipMemcpy(t.hs[a], hs.data(), n * sizeof(T), hipMemcpyHostToDevice));
    HC(hipMemcpy(t.hc[a], hc.data(), n * sizeof(T), hipMemcpyHostToDevice));
    HC(hipMemcpy(t.q2[a], q2.data(), n * sizeof(T), hipMemcpyHostToDevice));
  }
  if (s->mixed_bc) {
    T fh[6];
    for (int k = 0; k < 6; ++k) fh[k] = T(s->fh[k]);
    t.fh = s->alloc<T>(6);
    HC(hipMemcpy(t.fh, fh, sizeof(fh), hipMemcpyHostToDevice));
  }
}

hipEvent_t* timing_acquire(pff_solver* s, int group) {
  if (s->tim_pending.size() >= 512) timing_harvest(s);
  std::array<hipEvent_t, 6> ev{};
  if (!s->tim_free.empty()) {
    ev = s->tim_free.back();
    s->tim_free.pop_back();
  }
  // whole-apply sampling: only the events before the first and after the
  // last pass (slots 0 and 5); per-pass sampling: all six
  for (int k = 0; k < 6; ++k) {
    const bool want = !s->tim_whole || k == 0 || k == 5;
    if (want && !ev[k]) HC(hipEventCreate(&ev[k]));
    if (!want && ev[k]) {
      (void)hipEventDestroy(ev[k]);
      ev[k] = nullptr;
    }
  }
  s->tim_group.push_back(group);
  s->tim_pending.push_back(ev);
  return s->tim_pending.back().data();
}

void timing_harvest(pff_solver* s) {
  if (s->tim_pending.empty()) return;
  HC(hipEventSynchronize(s->tim_pending.back()[5]));
  for (size_t e = 0; e < s->tim_pending.size(); ++e) {
    auto& ev = s->tim_pending[e];
    const int base = 6 * s->tim_group[e];
    if (ev[1]) {
      float ms[5];
      for (int k = 0; k < 5; ++k) HC(hipEventElapsedTime(&ms[k], ev[k], ev[k + 1]));
      for (int k = 0; k < 5; ++k) {
        s->tim_ms[base + k] += ms[k];
        s->tim_n[base + k] += 1;
      }
    }
    float all = 0.f;
    HC(hipEventElapsedTime(&all, ev[0], ev[5]));
    s->tim_ms[base + 5] += all;
    s->tim_n[base + 5] += 1;
    s->tim_free.push_back(ev);
  }
  s->tim_pending.clear();
  s->tim_group.clear();
}

void destroy_buffers(pff_solver* s) {
  for (auto& ev : s->tim_pending)
    for (auto e : ev)
      if (e) (void)hipEventDestroy(e);
  for (auto& ev : s->tim_free)
    for (auto e : ev)
      if (e) (void)hipEventDestroy(e);
  s->tim_pending.clear();
  s->tim_free.clear();
  s->tim_group.clear();
  if (s->ev_scal) (void)hipEventDestroy(s->ev_scal);
  s->ev_scal = nullptr;
  if (s->kb_ready) (void)hipEventDestroy(s->kb_ready);
  if (s->kb_done) (void)hipEventDestroy(s->kb_done);
  s->kb_ready = s->kb_done = nullptr;
  for (auto& pb : s->allocs) {
    if (s->allocator.alloc) s->allocator.free(pb.first, pb.second, s->allocator.ctx);
    else (void)hipFree(pb.first);
  }
  s->allocs.clear();
  s->bytes_alloc = 0;
  if (s->hscal) (void)hipHostFree(s->hscal);
  if (s->hstage) (void)hipHostFree(s->hstage);
  s->hscal = nullptr;
  s->hstage = nullptr;
}

// ---- allocation-free projection ------------------------------------------------
//
// pff_project_noalloc runs steps (a3)-(a5) on caller buffers for callers that
// cannot allocate device memory (graph capture, serving loops): its spectra
// and axis tables live in the library's static device array `scratch` (one
// per device, held until the process ends) instead of a solver's buffers.

struct NoAllocCtx {
  int nx = 0, ny = 0, nz = 0, dim = 0;
  GridDesc g{};
  AxisPlan plan[3]{};
  bool plan_any = false;
  hipStream_t stream = nullptr;
  // the launch configuration of a solver (pff_create's defaults)
  int x_rows = 64, spec_threads = 512, spec_tx = 8, axis_threads = 0, axis_tx = 16, xcd_remap = 1, zspec = 1, yreg = 0, fit_shapes = 1;
  GraphRec* rec = nullptr;             // launched directly
  size_t part_len = 0;                 // the projection has no reductions
  double* part0 = nullptr;
  double* part1 = nullptr;
  DevTables<double> td;
  DevTables<float> tf;
  cpx<double>* spec_d = nullptr;
  cpx<float>* spec_f = nullptr;
  template <typename T> const DevTables<T>& tables() const;
  template <typename T> cpx<T>* spec() const;
};
template <> const DevTables<double>& NoAllocCtx::tables<double>() const { return td; }
template <> const DevTables<float>& NoAllocCtx::tables<float>() const { return tf; }
template <> cpx<double>* NoAllocCtx::spec<double>() const { return spec_d; }
template <> cpx<float>* NoAllocCtx::spec<float>() const { return spec_f; }

// Per-axis tables of upload_tables (twiddles, rotated or standard symbol
// factors, q^2 with the Nyquist mode kept), formed on the device in double.
template <typename T>
__global__ void k_axis_tables(cpx<T>* __restrict__ tw, T* __restrict__ hs, T* __restrict__ hc, T* __restrict__ q2,
                              int n, int standard) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    double sn, cs;
    sincospi(-2.0 * double(j) / double(n), &sn, &cs);
    tw[j] = cpx<T>{T(cs), T(sn)};
    const int m = (2 * j < n) ? j : j - n;                 // signed frequency, Nyquist reads -n/2
    const bool nyq = n % 2 == 0 && 2 * j == n;
    double sh, ch;
    sincospi(double(m) / double(n), &sh, &ch);             // sin, cos of q/2
    const double q = 2.0 * 3.14159265358979323846 * double(m) / double(n);
    if (standard) {
      hs[j] = nyq ? T(0) : T(q);
      hc[j] = T(1);
    } else {
      hs[j] = T(sh);
      hc[j] = nyq ? T(0) : T(ch);
    }
    q2[j] = T(q * q);
  }
}

}  // namespace

// Scratch of the allocation-free entry point: its spectra (C+1 half spectra,
// at most kScratchBytes - kScratchTables bytes) and axis tables.  Host code
// never uses this name as an address: the per-device address comes from
// hipGetSymbolAddress.
namespace {
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr size_t kScratchTables = size_t(256) << 10;
}  // namespace
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

// Address of `scratch` on the current device, looked up once per device.
unsigned char* scratch_on_current_device() {
  int dev = 0;
  HC(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw Fail("device index out of range", PFF_ERR_DEVICE);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HC(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Fail("hipGetSymbolAddress returned no address for the scratch array", PFF_ERR_DEVICE);
    g_scratch_ptr[dev] = static_cast<unsigned char*>(p);
  }
  return g_scratch_ptr[dev];
}

template <typename T>
void noalloc_tables(NoAllocCtx& c, DevTables<T>& t, unsigned char* base, int standard) {
  const int ns[3] = {c.nx, c.ny, c.nz};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    unsigned char* p = base + off;
    off += (bytes + 255) / 256 * 256;
    if (off > kScratchTables) throw Fail("axis tables exceed the scratch table area", PFF_ERR_ARG);
    return p;
  };
  for (int a = 0; a < 3; ++a) {
    const int n = ns[a];
    t.tw[a] = reinterpret_cast<cpx<T>*>(take(n * sizeof(cpx<T>)));
    t.hs[a] = reinterpret_cast<T*>(take(n * sizeof(T)));
    t.hc[a] = reinterpret_cast<T*>(take(n * sizeof(T)));
    t.q2[a] = reinterpret_cast<T*>(take(n * sizeof(T)));
    k_axis_tables<T><<<(n + 255) / 256, 256, 0, c.stream>>>(t.tw[a], t.hs[a], t.hc[a], t.q2[a], n, standard);
    LAUNCH_CHECK();
  }
  t.fh = nullptr;
}

}  // namespace

// ================================================================== C ABI ====

extern "C" {

int pff_abi_version(void) { return PFF_ABI_VERSION; }

// text of the last failed pff_create on this thread (there is no handle then)
thread_local std::string g_create_error;

const char* pff_last_error(const pff_solver* s) {
  if (s) return s->err.c_str();
  return g_create_error.empty() ? "null handle" : g_create_error.c_str();
}

pff_status pff_create(const pff_grid* grid, const pff_phase* phases, int n_phases, const uint8_t* phase_id,
                      const uint8_t* crack_mask, const pff_params* params, const pff_allocator* allocator,
                      void* hip_stream, pff_solver** out) {
  if (!out) return PFF_ERR_ARG;
  *out = nullptr;
  if (!grid || !phases || !phase_id || !params) return PFF_ERR_ARG;
  if (n_phases < 1 || n_phases > kMaxPhases) return PFF_ERR_ARG;
  if (allocator && ((allocator->alloc == nullptr) != (allocator->free == nullptr))) return PFF_ERR_ARG;
  pff_solver* s = new (std::nothrow) pff_solver();
  if (!s) return PFF_ERR_OOM;
  if (allocator && allocator->alloc) s->allocator = *allocator;
  pff_status st = guarded(s, [&]() -> pff_status {
    s->nx = grid->nx;
    s->ny = grid->ny;
    s->nz = grid->nz;
    if (s->nx < 2 || s->ny < 2 || s->nz < 1 || s->nx > 512 || s->ny > 512 || s->nz > 512)
      throw Fail("grid sizes out of range", PFF_ERR_ARG);
    if (!make_plan(s->nx, s->plan[0]) || !make_plan(s->ny, s->plan[1]) || !make_plan(s->nz, s->plan[2]))
      throw Fail("grid sizes must be between 1 and 512", PFF_ERR_ARG);
    for (int a = 0; a < 3; ++a)
      for (int st = 0; st < s->plan[a].nstage; ++st) {
        const int R = s->plan[a].radix[st];
        if (R != 2 && R != 3 && R != 4 && R != 8) s->plan_any = true;
      }
    s->dim = s->nz == 1 ? 2 : 3;
    s->C = s->dim == 2 ? 3 : 6;
    s->nxh = s->nx / 2 + 1;
    s->N = (long long)s->nx * s->ny * s->nz;
    s->Nh = (long long)s->nxh * s->ny * s->nz;
    s->M = (long long)(s->C + 1) * s->N + 1;
    {
      const int nxm = s->nx % 2 == 0 ? s->nx / 2 : s->nxh;
      const long long Nm = (long long)nxm * s->ny * s->nz;
      s->g = GridDesc{s->nx, s->ny, s->nz, s->nxh, s->N, s->Nh, nxm, s->nx % 2 == 0 ? 1 : 0, Nm,
                      make_fastdiv((uint32_t)nxm)};
    }
    s->prm = *params;
    const pff_params& p = s->prm;
    if (!(p.l > 0) || !(p.k_resid >= 0) || !(p.delta_a > 0) || !(p.alpha > 0) || p.alpha > 1 ||
        !(p.newton_tol > 0) || !(p.krylov_rtol > 0) || p.newton_maxit < 1 || p.krylov_maxit < 1 ||
        (p.precision != PFF_PREC_FP64 && p.precision != PFF_PREC_MIXED) ||
        (p.split != PFF_SPLIT_SPECTRAL && p.split != PFF_SPLIT_NONE) ||
        (p.projection != PFF_PROJ_ROTATED && p.projection != PFF_PROJ_STANDARD) ||
        !(p.w_gamma >= 0) || !(p.w_load >= 0) || !std::isfinite(p.w_gamma) || !std::isfinite(p.w_load) ||
        !(p.resid_tol >= 0) || !std::isfinite(p.resid_tol))
      throw Fail("invalid solver parameters", PFF_ERR_ARG);
    if (p.control != PFF_CONTROL_LENGTH && p.control != PFF_CONTROL_DISSIPATION)
      throw Fail("invalid solver parameters", PFF_ERR_ARG);
    if ((p.gc_form != PFF_GC_POINTWISE && p.gc_form != PFF_GC_VARIATIONAL) ||
        (p.gc_form == PFF_GC_VARIATIONAL && p.control == PFF_CONTROL_DISSIPATION))
      throw Fail("invalid solver parameters", PFF_ERR_ARG);
    if (p.macro_bc != PFF_BC_STRAIN && p.macro_bc != PFF_BC_MIXED)
      throw Fail("invalid solver parameters", PFF_ERR_ARG);
    s->var = p.gc_form == PFF_GC_VARIATIONAL;
    s->dctl = p.control == PFF_CONTROL_DISSIPATION;
    if (p.w_gamma == 0.0 && p.w_load == 0.0) {
      s->wa = 1.0;                                    // crack-length control
      s->wE = 0.0;
    } else {
      s->wa = p.w_gamma;
      s->wE = p.w_load;
    }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        if (p.f[3 * i + j] != p.f[3 * j + i]) throw Fail("f must be symmetric", PFF_ERR_ARG);
    if (s->dim == 2 && (p.f[2] != 0 || p.f[5] != 0 || p.f[8] != 0))
      throw Fail("2D (plane strain) needs an in-plane f", PFF_ERR_ARG);
    const double r2 = std::sqrt(2.0);
    if (s->dim == 2) {
      s->fm[0] = p.f[0]; s->fm[1] = p.f[4]; s->fm[2] = r2 * p.f[1];
    } else {
      s->fm[0] = p.f[0]; s->fm[1] = p.f[4]; s->fm[2] = p.f[8];
      s->fm[3] = r2 * p.f[5]; s->fm[4] = r2 * p.f[2]; s->fm[5] = r2 * p.f[1];
    }
    if (p.macro_bc == PFF_BC_MIXED) {
      double nf = 0.0;
      for (int k = 0; k < 6; ++k) nf += s->fm[k] * s->fm[k];
      if (!(nf > 0)) throw Fail("mixed macroscopic conditions need f != 0", PFF_ERR_ARG);
      s->mixed_bc = 1;
      for (int k = 0; k < 6; ++k) s->fh[k] = s->fm[k] / std::sqrt(nf);
    }
    s->mat.nphase = n_phases;
    s->mat.iso = p.split == PFF_SPLIT_NONE ? 1 : 0;
    s->phases.assign(phases, phases + n_phases);
    for (int k = 0; k < n_phases; ++k) {
      const double E = phases[k].E, nu = phases[k].nu;
      if (!(E > 0) || !(nu > -1 && nu < 0.5) || !(phases[k].Gc > 0))
        throw Fail("invalid phase constants", PFF_ERR_ARG);
      s->mat.lam[k] = E * nu / ((1 + nu) * (1 - 2 * nu));
      s->mat.mu[k] = E / (2 * (1 + nu));
      s->mat.Gc[k] = phases[k].Gc;
    }
    {
      bool het = false;
      for (int k = 1; k < n_phases; ++k) het = het || phases[k].Gc != phases[0].Gc;
      // with one toughness the variational term is Gc times the (finite-
      // difference) Laplacian of the pipelines; otherwise the stencil kernel
      s->var_het = params->gc_form == PFF_GC_VARIATIONAL && het;
    }
    s->h_pid.assign(phase_id, phase_id + s->N);
    for (uint8_t v : s->h_pid)
      if (v >= n_phases) throw Fail("phase id out of range", PFF_ERR_ARG);
    s->h_mask.assign(s->N, 0);
    if (crack_mask) {
      for (long long i = 0; i < s->N; ++i) s->h_mask[i] = crack_mask[i] ? 1 : 0;
      s->has_mask = std::any_of(s->h_mask.begin(), s->h_mask.end(), [](uint8_t v) { return v != 0; });
    }
    s->stream = static_cast<hipStream_t>(hip_stream);
    const char* tr = std::getenv("PFF_TRACE");
    s->trace = tr && tr[0] == '1';
    s->ktrace = tr && tr[0] == '2';
    auto envi = [](const char* k, int d) {
      const char* v = std::getenv(k);
      return v ? std::atoi(v) : d;
    };
    s->axis_threads = envi("PFF_AXIS_THREADS", 0);
    s->spec_threads = envi("PFF_SPEC_THREADS", 512);
    s->axis_tx = envi("PFF_AXIS_TX", 16);
    s->spec_tx = envi("PFF_SPEC_TX", 8);
    s->x_rows = envi("PFF_X_ROWS", 64);
    s->xcd_remap = envi("PFF_XCD_REMAP", 1) != 0 ? 1 : 0;
    s->zspec = envi("PFF_ZSPEC", 1) != 0 ? 1 : 0;
    s->yreg = std::min(3, std::max(0, envi("PFF_YREG", 1)));
    s->fit_shapes = envi("PFF_FIT_SHAPES", 1) != 0 ? 1 : 0;
    s->max_substep_depth = std::min(8, std::max(0, envi("PFF_SUBSTEPS", 3)));
    s->fused = std::min(2, std::max(0, envi("PFF_FUSED", 1)));
    if (s->var_het) s->fused = std::min(s->fused, 1);   // the variational term needs the input before the pass
    {
      const char* v = std::getenv("PFF_INNER32");
      s->inner32 = v ? std::atof(v) : kInner32;
      if (!(s->inner32 > 0.0 && s->inner32 < 1.0)) s->inner32 = kInner32;
    }
    // device memory
    const long long N = s->N, M = s->M;
    const int C = s->C;
    s->pid = s->alloc<uint8_t>(N);
    s->mask = s->alloc<uint8_t>(N);
    HC(hipMemcpy(s->pid, s->h_pid.data(), N, hipMemcpyHostToDevice));
    HC(hipMemcpy(s->mask, s->h_mask.data(), N, hipMemcpyHostToDevice));
    s->eps_t = s->alloc<double>(C * N);
    s->eps_c = s->alloc<double>(C * N);
    s->phi = s->alloc<double>(N);
    s->phi_c = s->alloc<double>(N);
    s->phi_guess = s->alloc<double>(N);
    s->dmask = s->alloc<double>(N);
    s->Hn = s->alloc<double>(N);
    s->Hcur = s->alloc<double>(N);
    if (s->dim == 2) s->lap64 = s->alloc<double>(N);
    s->Edev = s->alloc<double>(4);
    const size_t nts = (size_t)(s->dim == 2 ? TsLayout<2>::COUNT : TsLayout<3>::COUNT) * N;
    s->ts64 = s->alloc<double>(nts);
    s->aux64 = s->alloc<double>(N);
    s->lgc64 = s->alloc<double>(N);
    for (int k = 0; k < kNumVec; ++k) s->kv64[k] = s->alloc<double>(M);
    if (s->mixed()) {
      s->ts32 = s->alloc<float>(nts);
      s->aux32 = s->alloc<float>(N);
      s->lgc32 = s->alloc<float>(N);
      for (int k = 0; k < kNumVec; ++k) s->kv32[k] = s->alloc<float>(M);
    }
    s->spec_d = s->alloc<cpx<double>>((size_t)(C + 1) * s->Nh);
    if (s->mixed()) s->spec_f = s->alloc<cpx<float>>((size_t)(C + 1) * s->Nh);
    s->part_len = std::max<size_t>(kRedBlocks, (size_t)s->ny * s->nz + 16);
    s->part0 = s->alloc<double>(s->part_len * kMaxRed);
    s->part1 = s->alloc<double>(s->part_len * kMaxRed);
    s->scal = s->alloc<double>(SC_COUNT);
    for (int k = 0; k < 4; ++k) s->cgv[k] = s->alloc<double>(N);
    HC(hipHostMalloc((void**)&s->hscal, SC_COUNT * sizeof(double), hipHostMallocDefault));
    HC(hipEventCreateWithFlags(&s->ev_scal, hipEventDisableTiming));
    HC(hipHostMalloc((void**)&s->hstage, 8 * sizeof(double), hipHostMallocDefault));
    upload_tables<double>(s, s->td);
    upload_tables<float>(s, s->tf);
    // stream-ordered: a solver created beside others running on their own
    // streams (the request server) does not wait for their work
    HC(hipMemsetAsync(s->eps_t, 0, C * N * sizeof(double), s->stream));
    HC(hipMemsetAsync(s->eps_c, 0, C * N * sizeof(double), s->stream));
    HC(hipMemsetAsync(s->phi, 0, N * sizeof(double), s->stream));
    HC(hipMemsetAsync(s->phi_c, 0, N * sizeof(double), s->stream));
    HC(hipMemsetAsync(s->Hn, 0, N * sizeof(double), s->stream));
    HC(hipMemsetAsync(s->Edev, 0, 4 * sizeof(double), s->stream));
    HC(hipMemsetAsync(s->scal, 0, SC_COUNT * sizeof(double), s->stream));
    HC(hipStreamSynchronize(s->stream));
    return PFF_OK;
  });
  if (st != PFF_OK) {
    g_create_error = "pff_create: " + s->err;
    destroy_buffers(s);
    delete s;
    return st;
  }
  g_create_error.clear();
  *out = s;
  return PFF_OK;
}

void pff_destroy(pff_solver* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  destroy_buffers(s);
  delete s;
}

pff_status pff_bootstrap(pff_solver* s, double* a0, double* E_s) {
  return guarded(s, [&]() -> pff_status {
    dispatch(s, [&](auto impl) {
      using I = decltype(impl);
      I::initial_damage(s, s->phi);
      // a0 = Gamma(phi0): a residual pass at eps = 0, E = 0, H = 0
      HC(hipMemsetAsync(s->eps_t, 0, s->C * s->N * sizeof(double), s->stream));
      HC(hipMemsetAsync(s->eps_c, 0, s->C * s->N * sizeof(double), s->stream));
      HC(hipMemsetAsync(s->Hn, 0, s->N * sizeof(double), s->stream));
      HC(hipMemsetAsync(s->Edev, 0, 4 * sizeof(double), s->stream));
      I::residual(s, 0.0, nullptr);
      sync_scal(s);
    });
    s->a = s->wa * s->hscal[s->dctl ? SC_DISS : SC_GAMMA];   // tau0 (E = 0)
    // predictor: bisection on the gradient-free homogeneous damage
    std::vector<double> psif(s->mat.nphase), cnt(s->mat.nphase, 0.0);
    for (int k = 0; k < s->mat.nphase; ++k) psif[k] = psi_plus_host(s->prm.f, s->mat.lam[k], s->mat.mu[k], s->dim, s->mat.iso);
    for (long long i = 0; i < s->N; ++i)
      if (!s->h_mask[i]) cnt[s->h_pid[i]] += 1.0;
    const double l = s->prm.l, da = s->prm.delta_a;
    auto loc = [&](double E, int k) {
      const double h = 2.0 * E * E * psif[k];
      return h / (s->mat.Gc[k] / l + h);
    };
    auto S = [&](double E) {      // control value gained by the homogeneous solution at E
      double acc = 0.0;
      for (int k = 0; k < s->mat.nphase; ++k) {
        const double p = loc(E, k);
        acc += cnt[k] * p * p * (s->dctl ? s->mat.Gc[k] : 1.0);
      }
      return s->wa * acc / (2.0 * l) + s->wE * E;
    };
    double lo = 0.0, hi = 1.0;
    while (S(hi) < da) {
      hi *= 2.0;
      if (hi > 1e12) throw Fail("predictor: crack-length increment not reachable", PFF_ERR_ARG);
    }
    for (int it = 0; it < kBisection; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (S(mid) < da) lo = mid;
      else hi = mid;
    }
    s->E_s = 0.5 * (lo + hi);
    Vec16 locm{};
    for (int k = 0; k < s->mat.nphase; ++k) locm.v[k] = loc(s->E_s, k);
    const int g = grid1(s->N);
    k_guess<<<g, kBlock, 0, s->stream>>>(s->phi_guess, s->phi, s->pid, s->mask, locm, s->N);
    LAUNCH_CHECK();
    HC(hipMemcpyAsync(s->phi_c, s->phi, s->N * sizeof(double), hipMemcpyDeviceToDevice, s->stream));
    HC(hipStreamSynchronize(s->stream));
    s->E = 0.0;
    s->n = 0;
    s->bootstrapped = true;
    s->ts_valid = false;
    if (a0) *a0 = s->a;
    if (E_s) *E_s = s->E_s;
    return PFF_OK;
  });
}

// One Newton solve of the increment from the committed state to the target
// a + delta (paper Algorithm 2); commits on convergence (count_inc: the
// increment counter advances), rolls back otherwise.
static pff_status step_once(pff_solver* s, double delta, bool count_inc, pff_increment_result* out) {
  {
    if (!s->bootstrapped) throw Fail("pff_step before pff_bootstrap/pff_set_state", PFF_ERR_STATE);
    const auto t0 = std::chrono::steady_clock::now();
    const long long ap0 = s->applies, ki0 = s->kiters;
    const double a_new = s->a + delta;
    const long long N = s->N;
    const int C = s->C;
    // Newton start
    if (s->n == 0 && s->E_s > 0.0) {
      HC(hipMemsetAsync(s->eps_t, 0, C * N * sizeof(double), s->stream));
      HC(hipMemcpyAsync(s->phi, s->phi_guess, N * sizeof(double), hipMemcpyDeviceToDevice, s->stream));
      HC(hipStreamSynchronize(s->stream));
      s->hstage[0] = s->E_s;
      HC(hipMemcpyAsync(s->Edev, s->hstage, sizeof(double), hipMemcpyHostToDevice, s->stream));
    } else {
      HC(hipMemcpyAsync(s->eps_t, s->eps_c, C * N * sizeof(double), hipMemcpyDeviceToDevice, s->stream));
      HC(hipMemcpyAsync(s->phi, s->phi_c, N * sizeof(double), hipMemcpyDeviceToDevice, s->stream));
      HC(hipStreamSynchronize(s->stream));
      s->hstage[0] = s->E;
      HC(hipMemcpyAsync(s->Edev, s->hstage, sizeof(double), hipMemcpyHostToDevice, s->stream));
    }
    int conv = 0, it = 0, stall = 0;
    double best_e = HUGE_VAL;
    double err[3] = {0, 0, 0};
    double res[2] = {0, 0};
    const bool trace = s->trace;
    const int fb0 = s->fallbacks;
    const int rf0 = s->refinements;
    const long long a64_0 = s->applies64;
    dispatch_dim(s, [&](auto dimc) {
      constexpr int DIM = decltype(dimc)::value;
      using I = Impl<DIM, double>;
      I::residual(s, a_new, nullptr);
      if (trace) {
        sync_scal(s);
        std::fprintf(stderr, "[pff] inc %d start |F1|=%.6e |F2|=%.6e F3=%.6e\n", s->n + 1,
                     std::sqrt(s->hscal[SC_F1]), std::sqrt(s->hscal[SC_F2]), s->hscal[SC_F3]);
      }
      for (it = 1; it <= s->prm.newton_maxit; ++it) {
        int kit = 0;
        double rr = 0;
        newton_linear_solve<DIM>(s, &kit, &rr);
        I::newton_update(s, I::vec(s, I::SOL), s->prm.alpha);
        I::residual(s, a_new, nullptr);
        sync_scal(s);
        const double* h = s->hscal;
        if (trace) {
          HC(hipMemcpy(s->hstage, s->Edev, sizeof(double), hipMemcpyDeviceToHost));
          std::fprintf(stderr,
                       "[pff] inc %d it %d krylov %d relres %.2e | E=%.12e |F1|=%.6e |F2|=%.6e F3=%.6e "
                       "|w|/|eps|=%.2e |dphi|/|phi|=%.2e\n",
                       s->n + 1, it, kit, rr, s->hstage[0], std::sqrt(h[SC_F1]), std::sqrt(h[SC_F2]),
                       h[SC_F3], std::sqrt(h[SC_NW] / h[SC_NEPS]), std::sqrt(h[SC_NDPHI] / h[SC_NPHI]));
        }
        err[0] = std::sqrt(h[SC_NW]) / std::sqrt(h[SC_NEPS]);
        err[1] = std::sqrt(h[SC_NDPHI]) / std::sqrt(h[SC_NPHI]);
        err[2] = std::fabs(h[SC_F3]) / std::fabs(a_new);
        // residual measures of the new state (parity-mode stop); a zero
        // numerator is zero whatever the scale
        auto rel = [](double num2, double den2) {
          return num2 == 0.0 ? 0.0 : (den2 > 0.0 ? std::sqrt(num2 / den2) : HUGE_VAL);
        };
        res[0] = rel(h[SC_F1], h[SC_NSIG]);
        res[1] = rel(h[SC_F2], h[SC_NH2]);
        const double e = std::max(err[0], std::max(err[1], err[2]));
        const bool rok = !(s->prm.resid_tol > 0.0) || std::max(res[0], res[1]) <= s->prm.resid_tol;
        if (e <= s->prm.newton_tol && rok) {
          conv = 1;
          break;
        }
        if (!std::isfinite(e)) break;
        // with sub-increments to fall back on, a Newton solve whose update
        // measure has not halved its best value for 12 iterations stops early
        // (the cycles of a failing increment repeat every few iterations)
        if (e < 0.5 * best_e) {
          best_e = e;
          stall = 0;
        } else if (++stall >= 12 && s->max_substep_depth > 0) {
          break;
        }
      }
    });
    if (it > s->prm.newton_maxit) it = s->prm.newton_maxit;
    const int g = grid1(N);
    if (out) {
      std::memset(out, 0, sizeof(*out));
      out->increment = s->n + 1;
      out->newton_iters = it;
      out->krylov_iters = (int)(s->kiters - ki0);
      out->applies = s->applies - ap0;
      out->applies_fp64 = s->applies64 - a64_0;
      out->fp64_fallbacks = s->fallbacks - fb0;
      out->refinements = s->refinements - rf0;
      out->converged = conv;
      out->target_a = a_new;
      for (int q = 0; q < 3; ++q) out->err[q] = err[q];
      out->resid[0] = res[0];
      out->resid[1] = res[1];
    }
    if (!conv) {
      // roll back to the committed increment
      HC(hipMemcpyAsync(s->eps_t, s->eps_c, C * N * sizeof(double), hipMemcpyDeviceToDevice, s->stream));
      HC(hipMemcpyAsync(s->phi, s->phi_c, N * sizeof(double), hipMemcpyDeviceToDevice, s->stream));
      HC(hipStreamSynchronize(s->stream));
      s->ts_valid = false;
      if (out) out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      return PFF_NOT_CONVERGED;
    }
    k_commit_history<<<g, kBlock, 0, s->stream>>>(s->Hn, s->Hcur, N);
    LAUNCH_CHECK();
    HC(hipMemcpyAsync(s->eps_c, s->eps_t, C * N * sizeof(double), hipMemcpyDeviceToDevice, s->stream));
    HC(hipMemcpyAsync(s->phi_c, s->phi, N * sizeof(double), hipMemcpyDeviceToDevice, s->stream));
    HC(hipMemcpyAsync(s->hstage, s->Edev, sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HC(hipStreamSynchronize(s->stream));
    const double Ecur = s->hstage[0];
    s->E = Ecur;
    s->a = a_new;
    if (count_inc) s->n += 1;
    s->ts_valid = false;
    if (out) {
      for (int q = 0; q < 6; ++q) out->sigma_M[q] = s->hscal[SC_SIG + q] / double(N);
      out->load_factor = Ecur;
      out->crack_length = s->hscal[SC_GAMMA];
      out->dissipation = s->hscal[SC_DISS];
      out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return PFF_OK;
  }
}

// Sub-increments: an increment whose Newton does not converge is retried as
// two half increments from the committed state, recursively down to
// delta_a / 2^max_depth (env PFF_SUBSTEPS, default 3; 0: off); each converged
// half commits its history, the last one advances the increment counter.
// (The paper takes fixed increments and notes that relaxation alpha < 1
// sometimes helps near developed cracks; on the 256^2 fibre composite the
// 62nd increment of delta_a = 2 cycles between four Newton iterates at any
// alpha in [0.5, 1], and two increments of 1 converge.)
namespace {

void add_counts(pff_increment_result& agg, const pff_increment_result& r) {
  agg.newton_iters += r.newton_iters;
  agg.krylov_iters += r.krylov_iters;
  agg.applies += r.applies;
  agg.applies_fp64 += r.applies_fp64;
  agg.fp64_fallbacks += r.fp64_fallbacks;
  agg.refinements += r.refinements;
}

bool substeps(pff_solver* s, double delta, int depth, bool last, pff_increment_result& agg,
              pff_increment_result& fin) {
  for (int h = 0; h < 2; ++h) {
    const bool final_half = last && h == 1;
    pff_increment_result r{};
    const pff_status st = step_once(s, 0.5 * delta, final_half, &r);
    add_counts(agg, r);
    if (st == PFF_OK) {
      if (final_half) fin = r;
      continue;
    }
    if (depth >= s->max_substep_depth) return false;
    if (!substeps(s, 0.5 * delta, depth + 1, final_half, agg, fin)) return false;
  }
  return true;
}

}  // namespace

pff_status pff_step(pff_solver* s, pff_increment_result* out) {
  return guarded(s, [&]() -> pff_status {
    const auto t0 = std::chrono::steady_clock::now();
    pff_increment_result first{};
    const pff_status st = step_once(s, s->prm.delta_a, true, &first);
    if (st == PFF_OK || s->max_substep_depth <= 0 || s->n == 0) {
      if (out) *out = first;
      return st;
    }
    // keep the committed state on the host, to restore it if the
    // sub-increments fail too (the contract of PFF_NOT_CONVERGED)
    const long long N = s->N;
    const int C = s->C;
    std::vector<double> eps(C * N), phi(N), Hn(N);
    HC(hipStreamSynchronize(s->stream));
    HC(hipMemcpy(eps.data(), s->eps_c, C * N * sizeof(double), hipMemcpyDeviceToHost));
    HC(hipMemcpy(phi.data(), s->phi_c, N * sizeof(double), hipMemcpyDeviceToHost));
    HC(hipMemcpy(Hn.data(), s->Hn, N * sizeof(double), hipMemcpyDeviceToHost));
    const double E0 = s->E, a0 = s->a;
    const int n0 = s->n;
    pff_increment_result agg = first, fin{};
    if (substeps(s, s->prm.delta_a, 1, true, agg, fin)) {
      fin.newton_iters = agg.newton_iters;
      fin.krylov_iters = agg.krylov_iters;
      fin.applies = agg.applies;
      fin.applies_fp64 = agg.applies_fp64;
      fin.fp64_fallbacks = agg.fp64_fallbacks;
      fin.refinements = agg.refinements;
      fin.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      if (out) *out = fin;
      return PFF_OK;
    }
    HC(hipMemcpy(s->eps_c, eps.data(), C * N * sizeof(double), hipMemcpyHostToDevice));
    HC(hipMemcpy(s->eps_t, eps.data(), C * N * sizeof(double), hipMemcpyHostToDevice));
    HC(hipMemcpy(s->phi_c, phi.data(), N * sizeof(double), hipMemcpyHostToDevice));
    HC(hipMemcpy(s->phi, phi.data(), N * sizeof(double), hipMemcpyHostToDevice));
    HC(hipMemcpy(s->Hn, Hn.data(), N * sizeof(double), hipMemcpyHostToDevice));
    double e2[2] = {E0, E0};
    HC(hipMemcpy(s->Edev, e2, 2 * sizeof(double), hipMemcpyHostToDevice));
    s->E = E0;
    s->a = a0;
    s->n = n0;
    s->ts_valid = false;
    if (out) {
      *out = first;
      out->newton_iters = agg.newton_iters;
      out->krylov_iters = agg.krylov_iters;
      out->applies = agg.applies;
      out->applies_fp64 = agg.applies_fp64;
      out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return PFF_NOT_CONVERGED;
  });
}

pff_status pff_effective_toughness(int n, const double* E, const double* sigma_M, const double* f,
                                   double volume, double L_g, double* work, double* gceff) {
  if (n < 0 || (n > 0 && (!E || !sigma_M)) || !f || !(volume > 0.0) || !(L_g > 0.0)) return PFF_ERR_ARG;
  // Sigma : f with sigma_M = (11, 22, 33, 23, 13, 12) and f a symmetric 3x3 tensor
  auto sf = [&](int k) {
    const double* q = sigma_M + 6 * (long long)k;
    return q[0] * f[0] + q[1] * f[4] + q[2] * f[8] + 2.0 * (q[3] * f[5] + q[4] * f[2] + q[5] * f[1]);
  };
  double W = 0.0, E0 = 0.0, S0 = 0.0;   // the path starts unloaded
  for (int k = 0; k < n; ++k) {
    const double S1 = sf(k);
    W += 0.5 * (S0 + S1) * (E[k] - E0);
    E0 = E[k];
    S0 = S1;
  }
  if (work) *work = W;
  if (gceff) *gceff = volume * W / L_g;
  return std::isfinite(W) ? PFF_OK : PFF_ERR_ARG;
}

pff_status pff_stagger_defaults(pff_stagger_params* p) {
  if (!p) return PFF_ERR_ARG;
  p->tol_mech = 1e-9;
  p->tol_sta = 1e-8;
  p->cg_rtol = 1e-11;
  p->max_stagger = 500;
  p->max_newton = 50;
  p->cg_maxit = 20000;
  return PFF_OK;
}

pff_status pff_stagger_step(pff_solver* s, double dE, const pff_stagger_params* params, pff_stagger_result* out) {
  return guarded(s, [&]() -> pff_status {
    if (!s->bootstrapped) throw Fail("pff_stagger_step before pff_bootstrap/pff_set_state", PFF_ERR_STATE);
    if (s->var) throw Fail("pff_stagger_step: the staggered scheme uses the pointwise toughness term", PFF_ERR_ARG);
    pff_stagger_params sp;
    pff_stagger_defaults(&sp);
    if (params) sp = *params;
    if (!(sp.tol_mech > 0.0) || !(sp.tol_sta > 0.0) || !(sp.cg_rtol > 0.0) || sp.max_stagger < 1 ||
        sp.max_newton < 1 || sp.cg_maxit < 1 || !std::isfinite(dE))
      throw Fail("pff_stagger_step: invalid parameters", PFF_ERR_ARG);
    const auto t0 = std::chrono::steady_clock::now();
    const long long N = s->N;
    const int C = s->C;
    const double E = s->E + dE;
    HC(hipMemcpyAsync(s->eps_t, s->eps_c, C * N * sizeof(double), hipMemcpyDeviceToDevice, s->stream));
    HC(hipMemcpyAsync(s->phi, s->phi_c, N * sizeof(double), hipMemcpyDeviceToDevice, s->stream));
    HC(hipStreamSynchronize(s->stream));
    s->hstage[0] = E;
    HC(hipMemcpyAsync(s->Edev, s->hstage, sizeof(double), hipMemcpyHostToDevice, s->stream));
    if (out) std::memset(out, 0, sizeof(*out));
    int conv = 0;
    dispatch_dim(s, [&](auto dimc) {
      constexpr int DIM = decltype(dimc)::value;
      conv = Impl<DIM, double>::stagger(s, sp, E, out);
    });
    if (out) {
      out->increment = s->n + 1;
      out->E = E;
    }
    if (!conv) {
      HC(hipMemcpyAsync(s->eps_t, s->eps_c, C * N * sizeof(double), hipMemcpyDeviceToDevice, s->stream));
      HC(hipMemcpyAsync(s->phi, s->phi_c, N * sizeof(double), hipMemcpyDeviceToDevice, s->stream));
      HC(hipStreamSynchronize(s->stream));
      s->ts_valid = false;
      if (out) out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      return PFF_NOT_CONVERGED;
    }
    const int g = grid1(N);
    k_commit_history<<<g, kBlock, 0, s->stream>>>(s->Hn, s->Hcur, N);
    LAUNCH_CHECK();
    HC(hipMemcpyAsync(s->eps_c, s->eps_t, C * N * sizeof(double), hipMemcpyDeviceToDevice, s->stream));
    HC(hipMemcpyAsync(s->phi_c, s->phi, N * sizeof(double), hipMemcpyDeviceToDevice, s->stream));
    HC(hipStreamSynchronize(s->stream));
    s->E = E;
    s->a = s->wa * s->hscal[s->dctl ? SC_DISS : SC_GAMMA] + s->wE * E;   // control value of this state
    s->n += 1;
    s->ts_valid = false;
    if (out) {
      for (int q = 0; q < 6; ++q) out->sigma_M[q] = s->hscal[SC_SIG + q] / double(N);
      out->crack_length = s->hscal[SC_GAMMA];
      out->dissipation = s->hscal[SC_DISS];
      out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return PFF_OK;
  });
}

pff_status pff_get_state(pff_solver* s, double* eps_total, double* phi, double* Hn, double* E, double* a) {
  return guarded(s, [&]() -> pff_status {
    const long long N = s->N;
    const int C = s->C;
    HC(hipStreamSynchronize(s->stream));
    if (eps_total) {
      HC(hipMemcpy(eps_total, s->eps_c, C * N * sizeof(double), hipMemcpyDeviceToHost));
      for (int k = 0; k < C; ++k)
        for (long long i = 0; i < N; ++i) eps_total[k * N + i] += s->fm[k] * s->E;
    }
    if (phi) HC(hipMemcpy(phi, s->phi_c, N * sizeof(double), hipMemcpyDeviceToHost));
    if (Hn) HC(hipMemcpy(Hn, s->Hn, N * sizeof(double), hipMemcpyDeviceToHost));
    if (E) *E = s->E;
    if (a) *a = s->a;
    return PFF_OK;
  });
}

pff_status pff_device_views(pff_solver* s, double** eps_tilde, double** phi, double** Hn) {
  return guarded(s, [&]() -> pff_status {
    if (eps_tilde) *eps_tilde = s->eps_c;
    if (phi) *phi = s->phi_c;
    if (Hn) *Hn = s->Hn;
    return PFF_OK;
  });
}

pff_status pff_set_state(pff_solver* s, const double* eps_tilde, const double* phi, const double* Hn, double E,
                         double a, int n) {
  return guarded(s, [&]() -> pff_status {
    if (!eps_tilde || !phi || !Hn || n < 0) throw Fail("pff_set_state: null buffer", PFF_ERR_ARG);
    const long long N = s->N;
    const int C = s->C;
    HC(hipStreamSynchronize(s->stream));
    HC(hipMemcpy(s->eps_c, eps_tilde, C * N * sizeof(double), hipMemcpyHostToDevice));
    HC(hipMemcpy(s->eps_t, eps_tilde, C * N * sizeof(double), hipMemcpyHostToDevice));
    HC(hipMemcpy(s->phi_c, phi, N * sizeof(double), hipMemcpyHostToDevice));
    HC(hipMemcpy(s->phi, phi, N * sizeof(double), hipMemcpyHostToDevice));
    HC(hipMemcpy(s->Hn, Hn, N * sizeof(double), hipMemcpyHostToDevice));
    double e2[2] = {E, E};
    HC(hipMemcpy(s->Edev, e2, 2 * sizeof(double), hipMemcpyHostToDevice));
    s->E = E;
    s->a = a;
    s->n = n;
    s->E_s = 0.0;
    s->bootstrapped = true;
    s->ts_valid = false;
    return PFF_OK;
  });
}

pff_status pff_residual(pff_solver* s, double a, double* F_dev, double* gamma, double* sigma_M,
                        double* dissipation) {
  return guarded(s, [&]() -> pff_status {
    dispatch(s, [&](auto impl) {
      using I = decltype(impl);
      I::residual(s, a, F_dev);
    });
    sync_scal(s);
    if (gamma) *gamma = s->hscal[SC_GAMMA];
    if (dissipation) *dissipation = s->hscal[SC_DISS];
    if (sigma_M)
      for (int q = 0; q < 6; ++q) sigma_M[q] = s->hscal[SC_SIG + q] / double(s->N);
    return PFF_OK;
  });
}

pff_status pff_apply_tangent(pff_solver* s, const void* v_dev, void* Jv_dev) {
  return guarded(s, [&]() -> pff_status {
    if (!v_dev || !Jv_dev || v_dev == Jv_dev) throw Fail("pff_apply_tangent: bad buffers", PFF_ERR_ARG);
    if (!s->ts_valid) throw Fail("pff_apply_tangent: no tangent state (call pff_residual)", PFF_ERR_STATE);
    dispatch(s, [&](auto impl) {
      using I = decltype(impl);
      using TW = typename std::remove_pointer<decltype(I::vec(s, 0))>::type;
      I::apply(s, static_cast<const TW*>(v_dev), static_cast<TW*>(Jv_dev));
    });
    return PFF_OK;
  });
}

pff_status pff_project(pff_solver* s, const void* in_dev, void* out_dev, int prec) {
  return guarded(s, [&]() -> pff_status {
    if (!in_dev || !out_dev || (prec != 0 && prec != 1)) throw Fail("pff_project: bad arguments", PFF_ERR_ARG);
    auto go = [&](auto tag, auto dimc) {
      using T = decltype(tag);
      constexpr int DIM = decltype(dimc)::value;
      typename ProjectPipe<T, DIM>::Args A;
      A.g = s->g;
      A.in = static_cast<const T*>(in_dev);
      A.out = static_cast<T*>(out_dev);
      A.tab = spec_tables<T>(s);
      int nblk = 0;
      if (std::is_same<T, float>::value && !s->spec_f) s->spec_f = s->alloc<cpx<float>>((size_t)(s->C + 1) * s->Nh);
      run_pipeline<ProjectPipe<T, DIM>>(s, A, nblk);
    };
    if (s->dim == 2) {
      if (prec == 0) go(double(), std::integral_constant<int, 2>());
      else go(float(), std::integral_constant<int, 2>());
    } else {
      if (prec == 0) go(double(), std::integral_constant<int, 3>());
      else go(float(), std::integral_constant<int, 3>());
    }
    HC(hipStreamSynchronize(s->stream));
    return PFF_OK;
  });
}

pff_status pff_project_noalloc(const pff_grid* grid, int projection, const void* in_dev, void* out_dev,
                               int prec, void* hip_stream) {
  if (!grid || !in_dev || !out_dev || in_dev == out_dev || (prec != 0 && prec != 1) ||
      (projection != PFF_PROJ_ROTATED && projection != PFF_PROJ_STANDARD))
    return PFF_ERR_ARG;
  NoAllocCtx c;
  c.nx = grid->nx;
  c.ny = grid->ny;
  c.nz = grid->nz;
  if (c.nx < 2 || c.ny < 2 || c.nz < 1 || c.nx > 512 || c.ny > 512 || c.nz > 512) return PFF_ERR_ARG;
  if (!make_plan(c.nx, c.plan[0]) || !make_plan(c.ny, c.plan[1]) || !make_plan(c.nz, c.plan[2]))
    return PFF_ERR_ARG;
  for (int a = 0; a < 3; ++a)
    for (int st = 0; st < c.plan[a].nstage; ++st) {
      const int R = c.plan[a].radix[st];
      if (R != 2 && R != 3 && R != 4 && R != 8) c.plan_any = true;
    }
  c.dim = c.nz == 1 ? 2 : 3;
  const int C = c.dim == 2 ? 3 : 6;
  const int nxh = c.nx / 2 + 1;
  const long long N = (long long)c.nx * c.ny * c.nz, Nh = (long long)nxh * c.ny * c.nz;
  const int nxm = c.nx % 2 == 0 ? c.nx / 2 : nxh;
  c.g = GridDesc{c.nx, c.ny, c.nz, nxh, N, Nh, nxm, c.nx % 2 == 0 ? 1 : 0, (long long)nxm * c.ny * c.nz,
                 make_fastdiv((uint32_t)nxm)};
  const size_t spec_bytes = (size_t)(C + 1) * Nh * (prec == 0 ? sizeof(cpx<double>) : sizeof(cpx<float>));
  if (spec_bytes > kScratchBytes - kScratchTables) return PFF_ERR_ARG;   // beyond the scratch array
  c.stream = static_cast<hipStream_t>(hip_stream);
  try {
    unsigned char* base = scratch_on_current_device();
    const int standard = projection == PFF_PROJ_STANDARD ? 1 : 0;
    auto go = [&](auto tag, auto dimc) {
      using T = decltype(tag);
      constexpr int DIM = decltype(dimc)::value;
      if constexpr (std::is_same<T, double>::value) {
        noalloc_tables<double>(c, c.td, base, standard);
        c.spec_d = reinterpret_cast<cpx<double>*>(base + kScratchTables);
      } else {
        noalloc_tables<float>(c, c.tf, base, standard);
        c.spec_f = reinterpret_cast<cpx<float>*>(base + kScratchTables);
      }
      typename ProjectPipe<T, DIM>::Args A;
      A.g = c.g;
      A.in = static_cast<const T*>(in_dev);
      A.out = static_cast<T*>(out_dev);
      const DevTables<T>& t = c.template tables<T>();
      for (int a = 0; a < 3; ++a) {
        A.tab.hs[a] = t.hs[a];
        A.tab.hc[a] = t.hc[a];
        A.tab.q2[a] = t.q2[a];
      }
      A.tab.invN = T(1.0 / double(N));
      A.tab.fh = nullptr;
      int nblk = 0;
      c.part_len = (size_t)c.ny * c.nz + 16;
      run_pipeline<ProjectPipe<T, DIM>>(&c, A, nblk);
    };
    if (c.dim == 2) {
      if (prec == 0) go(double(), std::integral_constant<int, 2>());
      else go(float(), std::integral_constant<int, 2>());
    } else {
      if (prec == 0) go(double(), std::integral_constant<int, 3>());
      else go(float(), std::integral_constant<int, 3>());
    }
  } catch (const Fail& e) {
    return e.code;
  } catch (const std::exception&) {
    return PFF_ERR_DEVICE;
  }
  return PFF_OK;
}

pff_status pff_krylov_solve(pff_solver* s, const void* b_dev, void* x_dev, double rtol, int maxit, int* iters,
                            double* relres) {
  return guarded(s, [&]() -> pff_status {
    if (!b_dev || !x_dev || !(rtol > 0) || maxit < 1) throw Fail("pff_krylov_solve: bad arguments", PFF_ERR_ARG);
    if (!s->ts_valid) throw Fail("pff_krylov_solve: no tangent state (call pff_residual)", PFF_ERR_STATE);
    int conv = 0;
    dispatch(s, [&](auto impl) {
      using I = decltype(impl);
      using TW = typename std::remove_pointer<decltype(I::vec(s, 0))>::type;
      conv = I::bicgstab(s, static_cast<const TW*>(b_dev), static_cast<TW*>(x_dev), rtol, maxit, iters, relres);
    });
    HC(hipStreamSynchronize(s->stream));
    return conv ? PFF_OK : PFF_NOT_CONVERGED;
  });
}

pff_status pff_timing(pff_solver* s, int every) {
  return guarded(s, [&]() -> pff_status {
    HC(hipStreamSynchronize(s->stream));
    timing_harvest(s);
    s->tim_every = every < 0 ? -every : every;
    s->tim_whole = every < 0;
    return PFF_OK;
  });
}

pff_status pff_timing_read(pff_solver* s, int kernel, long long* count, double* ms) {
  return guarded(s, [&]() -> pff_status {
    if (kernel < 0 || kernel >= kTimSlots) throw Fail("pff_timing_read: kernel id out of range", PFF_ERR_ARG);
    HC(hipStreamSynchronize(s->stream));
    timing_harvest(s);
    if (count) *count = s->tim_n[kernel];
    if (ms) *ms = s->tim_ms[kernel];
    return PFF_OK;
  });
}

pff_status pff_counters(pff_solver* s, long long* applies, long long* krylov_iters) {
  return guarded(s, [&]() -> pff_status {
    if (applies) *applies = s->applies;
    if (krylov_iters) *krylov_iters = s->kiters;
    return PFF_OK;
  });
}

pff_status pff_solver_bytes(pff_solver* s, size_t* bytes) {
  if (!s || !bytes) return PFF_ERR_ARG;
  *bytes = s->bytes_alloc;
  return PFF_OK;
}

pff_status pff_footprint_bytes(const pff_grid* grid, int precision, size_t* bytes) {
  if (!grid || !bytes || grid->nx < 1 || grid->ny < 1 || grid->nz < 1) return PFF_ERR_ARG;
  if (precision != PFF_PREC_FP64 && precision != PFF_PREC_MIXED) return PFF_ERR_ARG;
  const size_t nx = grid->nx, ny = grid->ny, nz = grid->nz;
  const size_t N = nx * ny * nz, dim = nz == 1 ? 2 : 3, C = dim == 2 ? 3 : 6;
  const size_t M = (C + 1) * N + 1, Nh = (nx / 2 + 1) * ny * nz;
  const size_t nts = (dim == 2 ? TsLayout<2>::COUNT : TsLayout<3>::COUNT) * N;
  const bool mixed = precision == PFF_PREC_MIXED;
  const size_t D = sizeof(double), F = sizeof(float);
  size_t b = 2 * N;                                   // phase ids, crack mask
  b += 2 * C * N * D;                                 // strain fluctuation, committed copy
  b += 6 * N * D;                                     // phi, committed phi, guess, mask, Hn, H
  if (dim == 2) b += N * D;                           // Laplacian of phi
  b += 4 * D;                                         // E
  b += nts * D + 2 * N * D + kNumVec * M * D;         // tangent state, aux, variational term, Krylov vectors
  if (mixed) b += nts * F + 2 * N * F + kNumVec * M * F;
  b += (C + 1) * Nh * 2 * D;                          // FP64 spectra
  if (mixed) b += (C + 1) * Nh * 2 * F;               // FP32 spectra
  const size_t part_len = std::max<size_t>(kRedBlocks, ny * nz + 16);
  b += 2 * part_len * kMaxRed * D + SC_COUNT * D + 4 * N * D;
  for (size_t n : {nx, ny, nz}) b += n * (2 * D + 3 * D) + n * (2 * F + 3 * F);   // FFT and spectral tables
  *bytes = b;
  return PFF_OK;
}

pff_status pff_save(pff_solver* s, void* buf, size_t* bytes) {
  return guarded(s, [&]() -> pff_status {
    if (!bytes) throw Fail("pff_save: bytes is NULL", PFF_ERR_ARG);
    const long long N = s->N;
    const int C = s->C;
    const size_t need = 64 + (size_t)(C + 2) * N * sizeof(double);
    if (!buf) {
      *bytes = need;
      return PFF_OK;
    }
    if (*bytes < need) throw Fail("pff_save: buffer too small", PFF_ERR_ARG);
    HC(hipStreamSynchronize(s->stream));
    unsigned char* b = static_cast<unsigned char*>(buf);
    std::memset(b, 0, 64);
    const int hdr[6] = {0x50464631, s->nx, s->ny, s->nz, s->n, s->bootstrapped ? 1 : 0};
    std::memcpy(b, hdr, sizeof(hdr));
    const double sc[3] = {s->E, s->a, s->E_s};
    std::memcpy(b + 32, sc, sizeof(sc));
    double* d = reinterpret_cast<double*>(b + 64);
    HC(hipMemcpy(d, s->eps_c, C * N * sizeof(double), hipMemcpyDeviceToHost));
    HC(hipMemcpy(d + C * N, s->phi_c, N * sizeof(double), hipMemcpyDeviceToHost));
    HC(hipMemcpy(d + (C + 1) * N, s->Hn, N * sizeof(double), hipMemcpyDeviceToHost));
    *bytes = need;
    return PFF_OK;
  });
}

pff_status pff_load(pff_solver* s, const void* buf, size_t bytes) {
  return guarded(s, [&]() -> pff_status {
    const long long N = s->N;
    const int C = s->C;
    const size_t need = 64 + (size_t)(C + 2) * N * sizeof(double);
    if (!buf || bytes < need) throw Fail("pff_load: buffer too small", PFF_ERR_ARG);
    const unsigned char* b = static_cast<const unsigned char*>(buf);
    int hdr[6];
    std::memcpy(hdr, b, sizeof(hdr));
    if (hdr[0] != 0x50464631 || hdr[1] != s->nx || hdr[2] != s->ny || hdr[3] != s->nz)
      throw Fail("pff_load: checkpoint does not match this grid", PFF_ERR_ARG);
    double sc[3];
    std::memcpy(sc, b + 32, sizeof(sc));
    const double* d = reinterpret_cast<const double*>(b + 64);
    HC(hipStreamSynchronize(s->stream));
    HC(hipMemcpy(s->eps_c, d, C * N * sizeof(double), hipMemcpyHostToDevice));
    HC(hipMemcpy(s->eps_t, d, C * N * sizeof(double), hipMemcpyHostToDevice));
    HC(hipMemcpy(s->phi_c, d + C * N, N * sizeof(double), hipMemcpyHostToDevice));
    HC(hipMemcpy(s->phi, d + C * N, N * sizeof(double), hipMemcpyHostToDevice));
    HC(hipMemcpy(s->Hn, d + (C + 1) * N, N * sizeof(double), hipMemcpyHostToDevice));
    s->n = hdr[4];
    s->bootstrapped = hdr[5] != 0;
    s->E = sc[0];
    s->a = sc[1];
    s->E_s = sc[2];
    s->ts_valid = false;
    if (s->n == 0 && s->bootstrapped) {
      // the first-increment guess is rebuilt by pff_bootstrap; resume only after an increment
      s->bootstrapped = false;
    }
    return PFF_OK;
  });
}

}  // extern "C"
