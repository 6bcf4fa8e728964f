"""Benchmark: crack-length increments of the MI355X phase-field FFT solver.

A step is one crack-length increment (paper Algorithm 2): constitutive
update, FP64 residual, BiCGSTAB on the matrix-free bordered tangent,
relaxed Newton updates and the history commit, i.e. every step of the hot
path.  `value` is the in-solver throughput in Mvoxel tangent-applies/s
(voxels x tangent applications / wall time of the K timed increments, all
inputs resident in HBM).  The roofline object covers the dominant FFT pass
kernel of the tangent apply, timed live with HIP events on the solver stream
(every 8th apply sampled); `cpu_baseline` times the CPU oracle's tangent
apply on a bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_NAMES = {0: "x-forward pass (R2C, tangent prologue)",
                1: "y pass (2D: forward, spectral stage, inverse)",
                2: "z pass (forward, spectral stage, inverse)",
                3: "y pass (inverse)",
                4: "x-inverse pass (C2R, tangent epilogue)"}


def kernel_bytes(shape, precision):
    """Algorithmic HBM bytes per launch of each tangent-apply pass kernel
    (compulsory reads + writes of that kernel, see the design notes)."""
    nz, ny, nx = shape
    N = nx * ny * nz
    c = 3 if nz == 1 else 6
    nf = c + 1
    nh = (nx // 2 + 1) * ny * nz
    T = 4 if precision == "mixed" else 8
    spec = nf * nh * 2 * T                       # all half spectra of one pass
    ts_fields = 6 if nz == 1 else 10          # strain frame, phi, Hs, r
    xf = (c + 1) * N * T + T + ts_fields * N * T + 2 * N + spec + N * T
    ax = 2 * spec
    xi = spec + N * T + 2 * N + (c + 1) * N * T
    if nz == 1:
        return {0: xf, 1: ax, 2: 0, 3: 0, 4: xi}
    return {0: xf, 1: ax, 2: ax, 3: ax, 4: xi}


def src_hash():
    h = hashlib.sha1()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2412_17445_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def load_traffic(workload, kernel_id, launches_bytes):
    """HBM traffic per launch from committed rocprofv3 counter summaries,
    only if they were taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_src_sha1") != src_hash():
        return None
    k = d.get("kernels", {}).get(str(kernel_id))
    return None if k is None else k.get("hbm_bytes_per_launch")


def cpu_baseline(prob, seconds=15.0):
    """Oracle tangent apply (NumPy FP64) on a frozen state of the workload."""
    import numpy as np

    from oracle import fourier as fo
    from oracle.system import System
    from synth import random_state, random_vector

    sysm = System(prob)
    eps, phi, Hn, E = random_state(sysm.shape, sysm.ncomp, 7, f_mandel=sysm.f, E=0.004)
    eps_t = fo.G_mandel(eps - sysm.fE(E))
    J = sysm.tangent(eps_t, phi, E, Hn)
    v = random_vector(sysm.N * (sysm.ncomp + 1) + 1, 8)
    J(v)
    n = 0
    w0, c0 = time.perf_counter(), time.process_time()
    while time.perf_counter() - w0 < seconds:
        J(v)
        n += 1
    wall = time.perf_counter() - w0
    cpu = time.process_time() - c0
    cores = max(1, int(round(cpu / wall)))
    return {"value": n * sysm.N / wall / 1e6, "unit": "Mvoxel-applies/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{n} oracle tangent applies (NumPy FP64) on a frozen seeded state of the "
                      f"{'x'.join(map(str, prob.shape[::-1]))} workload, {wall:.1f} s wall, "
                      f"host threads used ~{cpu / wall:.2f}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cfg1_256sq_fibres")
    ap.add_argument("--precision", default=None, help="override: fp64 or mixed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--timing-every", type=int, default=8)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs one RVE solve on one GPU; multi-GPU runs are not "
              "part of it (requests shard across GPUs with no communication).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2412_17445_amd import Solver
    from synth import problem_config

    prob = problem_config(args.workload)
    if args.precision:
        prob.precision = args.precision
    torch.cuda.set_device(0)
    s = Solver.from_problem(prob)
    s.bootstrap()
    for _ in range(args.warmup):
        out = s.step()
        if not out["converged"]:
            raise RuntimeError(f"warm-up increment did not converge: {out}")
    s.timing(args.timing_every)
    a0, _ = s.counters()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = []
    for _ in range(args.steps):
        outs.append(s.step())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    a1, _ = s.counters()
    if not all(o["converged"] for o in outs):
        raise RuntimeError("an increment in the timed region did not converge")
    elapsed = t1 - t0
    N = prob.nvox
    applies = a1 - a0
    value = applies * N / elapsed / 1e6

    tim = s.timing_read()
    kb = kernel_bytes(prob.shape, prob.precision)
    kern = {}
    for k in range(5):
        n, ms = tim[k]
        if n > 0 and kb[k] > 0:
            kern[k] = (ms / n, n, ms)
    dom = max(kern, key=lambda k: kern[k][2])
    avg_ms = kern[dom][0]
    achieved = kb[dom] / (avg_ms * 1e-3) / 1e9
    traffic = load_traffic(args.workload, dom, kb[dom])
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": KERNEL_NAMES[dom], "alg_bytes_per_launch": kb[dom],
                "avg_launch_us": round(avg_ms * 1e3, 2), "timed_launches": kern[dom][1]}
    apply_n, apply_ms = tim[5]
    line = {
        "metric": "Mvoxel tangent-applies/s",
        "value": round(value, 2),
        "unit": "Mvoxel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prob.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "grid": list(prob.shape[::-1]), "voxels": N,
                   "precision": prob.precision, "increments_timed": args.steps,
                   "tangent_applies": applies,
                   "newton_iters": sum(o["newton_iters"] for o in outs),
                   "krylov_iters": sum(o["krylov_iters"] for o in outs),
                   "apply_us_avg": round(apply_ms / max(apply_n, 1) * 1e3, 2),
                   "parallelism": "single GPU"},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
