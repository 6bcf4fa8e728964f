"""Benchmark: crack-length increments of the MI355X phase-field FFT solver.

A step is one crack-length increment (paper Algorithm 2): constitutive
update, FP64 residual, BiCGSTAB on the matrix-free bordered tangent,
relaxed Newton updates and the history commit, i.e. every step of the hot
path.  `value` is the in-solver throughput in Mvoxel tangent-applies/s
(voxels x tangent applications / wall time of the K timed increments, all
inputs resident in HBM).  The roofline object covers the tangent apply,
the unit of work of the metric: its algorithmic bytes (per voxel-apply:
read the input vector, write J v, read the compact tangent state, one
spectral round trip, the phase id) times the voxels, over the apply's
average duration (its five FFT pass kernels and the finisher), timed live
with HIP events on the solver stream (every 7th apply sampled).  The bare
apply leg times 1000 applies on the frozen state of the last increment
(median of 10 trials after 20 warm-ups), also for the other benchmark
grids.  `cpu_baseline` times the CPU oracle's tangent apply on the full
workload with every host core available to its FFTs.
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
BARE_WORKLOADS = ("crack2d_64", "fibres2d_256", "pores3d_64", "particles3d_128")


def alg_bytes_per_voxel(prob, precision):
    """Algorithmic HBM bytes of one voxel-apply of the bordered tangent:
    read the input (c+1 words), write J v (c+1), read the compact tangent
    state (strain c, phi, H, r: c+3), one spectral round trip (c+1 words
    each way), plus 1 byte of phase id on a heterogeneous cell: 22 words in
    2D (c = 3), 37 in 3D (c = 6)."""
    words = 22 if prob.shape[0] == 1 else 37
    T = 4 if precision == "mixed" else 8
    return words * T + (1 if len(prob.phases) > 1 else 0)
KERNEL_NAMES = {0: "x-forward pass (R2C, tangent prologue)",
                1: "y pass (2D: forward, spectral stage, inverse)",
                2: "z pass (forward, spectral stage, inverse)",
                3: "y pass (inverse)",
                4: "x-inverse pass (C2R, tangent epilogue)"}


def kernel_bytes(shape, precision, variant=0):
    """Algorithmic HBM bytes per launch of each tangent-apply pass kernel
    (the compulsory reads and writes of that kernel).  Variants 1-4 are the
    applies fused with BiCGSTAB steps: the x-inverse pass also reads the
    vector of its inner product (r_hat or s); in variants 3 and 4 the
    x-forward pass also forms the direction p (reads r, p, v, rewrites p) or
    s (reads r, v, writes s)."""
    nz, ny, nx = shape
    N = nx * ny * nz
    c = 3 if nz == 1 else 6
    nf = c + 1
    nh = (nx // 2 + 1) * ny * nz
    T = 4 if precision == "mixed" else 8
    spec = nf * nh * 2 * T                       # all half spectra of one pass
    ts_fields = 6 if nz == 1 else 10          # strain frame, phi, Hs, r
    V = (c + 1) * N * T                          # voxel part of one Krylov vector
    xf = V + T + ts_fields * N * T + 2 * N + spec + N * T
    ax = 2 * spec
    xi = spec + N * T + 2 * N + V
    if variant in (1, 2):
        xi += V
    elif variant == 3:
        xf += 3 * V
        xi += V
    elif variant == 4:
        xf += 2 * V
        xi += V
    if nz == 1:
        return {0: xf, 1: ax, 2: 0, 3: 0, 4: xi}
    return {0: xf, 1: ax, 2: ax, 3: ax, 4: xi}


def src_hash():
    h = hashlib.sha1()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2412_17445_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def load_traffic(workload):
    """HBM traffic (FETCH_SIZE + WRITE_SIZE, scaled by the plain-copy
    calibration) per apply, summed over the apply's kernels, from the
    committed rocprofv3 counter summary, only if it was taken on the current
    kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_src_sha1") != src_hash():
        return None
    return d.get("hbm_bytes_per_apply")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(prob, seconds=15.0):
    """Oracle tangent apply (NumPy FP64, scipy.fft) on a frozen seeded state
    of the whole workload, with os.cpu_count() FFT threads; the elementwise
    NumPy work is single-threaded."""
    from oracle import fourier as fo
    from oracle.system import System
    from synth import random_state, random_vector

    ncpu = os.cpu_count() or 1
    fo.FFT_WORKERS = ncpu
    sysm = System(prob)
    eps, phi, Hn, E = random_state(sysm.shape, sysm.ncomp, 7, f_mandel=sysm.f, E=0.004)
    eps_t = fo.G_mandel(eps - sysm.fE(E))
    J = sysm.tangent(eps_t, phi, E, Hn)
    v = random_vector(sysm.N * (sysm.ncomp + 1) + 1, 8)
    J(v)
    n = 0
    w0, c0 = time.perf_counter(), time.process_time()
    while time.perf_counter() - w0 < seconds or n < 2:
        J(v)
        n += 1
    wall = time.perf_counter() - w0
    cpu = time.process_time() - c0
    fo.FFT_WORKERS = 1
    return {"value": round(n * sysm.N / wall / 1e6, 4), "unit": "Mvoxel-applies/s",
            "cores": ncpu, "host_cpu_count": ncpu, "threads_busy_avg": round(cpu / wall, 2),
            "kind": "oracle",
            "sample": f"{n} oracle tangent applies (NumPy FP64, scipy.fft with {ncpu} workers) on a "
                      f"frozen seeded state of the whole {'x'.join(map(str, prob.shape[::-1]))} "
                      f"workload, {wall:.1f} s wall"}


def bare_apply(s, prob, precision, trials=10, n_applies=1000, warmup=20):
    """Bare tangent applies at the solver's current tangent state: median of
    `trials` timings of `n_applies` applies (HIP events on the solver stream,
    torch's current stream) after `warmup` applies."""
    import statistics

    import torch

    dt = torch.float32 if precision == "mixed" else torch.float64
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    v = torch.randn(s.M, dtype=dt, device="cuda", generator=g) * 1e-3
    out = torch.empty_like(v)
    for _ in range(warmup):
        s.apply(v, out)
    times = []
    for _ in range(trials):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n_applies):
            s.apply(v, out)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1) * 1e-3 / n_applies)
    t = statistics.median(times)
    b = alg_bytes_per_voxel(prob, precision)
    ach = b * prob.nvox / t / 1e9
    return {"apply_us": round(t * 1e6, 2), "mvoxel_applies_per_s": round(prob.nvox / t / 1e6, 1),
            "alg_bytes_per_voxel": b, "alg_GBs": round(ach, 1), "frac_of_hbm_peak": round(ach / HBM_PEAK_GBS, 4),
            "trials": trials, "applies_per_trial": n_applies, "spread_us": [round(min(times) * 1e6, 2),
                                                                            round(max(times) * 1e6, 2)]}


def bare_apply_leg(name):
    """Bootstrap and one increment of a benchmark grid, then bare applies at
    its committed state."""
    from paper_2412_17445_amd import Solver
    from synth import problem_config

    prob = problem_config(name)
    s = Solver.from_problem(prob)
    s.bootstrap()
    o = s.step()
    _, _, _, _, a = s.get_state()
    s.residual(a, want_F=False)
    r = bare_apply(s, prob, prob.precision)
    s.close()
    r.update(workload=name, grid=list(prob.shape[::-1]), precision=prob.precision,
             state=f"committed state of increment 1 (converged={o['converged']})")
    log(f"bare apply {name}: {r['apply_us']} us, {r['mvoxel_applies_per_s']} Mvoxel-applies/s, "
        f"frac {r['frac_of_hbm_peak']}")
    return r


def vs_oracle(prob, outs, s):
    """The benchmark's first increments against the oracle's stored ones (the
    oracle's parity-mode roots; the benchmark runs its own tolerances)."""
    import numpy as np

    path = os.path.join(ROOT, "tests", "golden", f"oracle_{prob.name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        g = json.load(fh)
    res = []
    for o, ref in zip(outs, g["increments"]):
        sig, sref = np.array(o["sigma_M"]), np.array(ref["sigma_M"])
        res.append({"increment": ref["increment"],
                    "E": float("%.3e" % (abs(o["E"] - ref["E"]) / abs(ref["E"]))),
                    "Gamma": float("%.3e" % (abs(o["Gamma"] - ref["Gamma"]) / abs(ref["Gamma"]))),
                    "sigma_M": float("%.3e" % (np.abs(sig - sref).max() / np.abs(sref).max()))})
    return res


def compare_fp64(prob, args, mixed_outs, mixed_s_per_step):
    """The same increments solved by the plain FP64 GPU solver: its time per
    increment and the largest relative difference of the per-increment
    outputs (load factor, crack length, macroscopic stress)."""
    import copy

    import numpy as np
    import torch

    from paper_2412_17445_amd import Solver

    p64 = copy.copy(prob)
    p64.precision = "fp64"
    log("plain FP64 solve of the same increments")
    s = Solver.from_problem(p64)
    s.bootstrap()
    d = {"E": 0.0, "Gamma": 0.0, "sigma_M": 0.0}
    t = []
    for i, ref in enumerate(mixed_outs):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        o = s.step()
        torch.cuda.synchronize()
        t.append(time.perf_counter() - t0)
        if not o["converged"]:
            raise RuntimeError(f"FP64 increment {i + 1} did not converge")
        log(f"fp64 increment {i + 1}: newton={o['newton_iters']} krylov={o['krylov_iters']} {t[-1]:.2f}s")
        d["E"] = max(d["E"], abs(ref["E"] - o["E"]) / abs(o["E"]))
        d["Gamma"] = max(d["Gamma"], abs(ref["Gamma"] - o["Gamma"]) / abs(o["Gamma"]))
        sm, so = np.array(ref["sigma_M"]), np.array(o["sigma_M"])
        d["sigma_M"] = max(d["sigma_M"], float(np.abs(sm - so).max() / np.abs(so).max()))
    s.close()
    timed = t[args.warmup:] or t
    fp64_s = sum(timed) / len(timed)
    return {"increments": len(mixed_outs), "fp64_ms_per_step": round(fp64_s * 1e3, 2),
            "mixed_ms_per_step": round(mixed_s_per_step * 1e3, 2),
            "fp64_time_over_mixed_time": round(fp64_s / mixed_s_per_step, 3),
            "fp64_first_increment_s": round(t[0], 3),
            "max_rel_diff": {k: float("%.3e" % v) for k, v in d.items()}}


def staggered_leg(prob, first):
    """The strain-controlled staggered scheme (Algorithm 1, FP64) from the
    bootstrap state to the load factor E1 of the first crack-length increment
    `first`: both schemes reach the same root there, so time and tangent
    applies compare the two controls on equal work."""
    import numpy as np

    from paper_2412_17445_amd import Solver

    s = Solver.from_problem(prob, precision="fp64")
    s.bootstrap()
    a0, _ = s.counters()
    o = s.stagger_step(first["E"])
    a1, _ = s.counters()
    s.close()
    log(f"staggered increment to E1: converged={o['converged']} stagger={o['stagger_iters']} "
        f"newton={o['newton_iters']} cg={o['cg_mech']}+{o['cg_helm']} {o['seconds']:.2f}s")
    sm, so = np.array(o["sigma_M"]), np.array(first["sigma_M"])
    return {"E": first["E"], "converged": o["converged"], "seconds": round(o["seconds"], 3),
            "stagger_iters": o["stagger_iters"], "newton_iters": o["newton_iters"],
            "cg_mech": o["cg_mech"], "cg_helm": o["cg_helm"], "tangent_applies": a1 - a0,
            "crack_control_applies": first["applies"],
            "crack_control_seconds": round(first["seconds"], 3),
            "rel_diff_Gamma": float("%.3e" % (abs(o["Gamma"] - first["Gamma"]) / abs(first["Gamma"]))),
            "rel_diff_sigma_M": float("%.3e" % (np.abs(sm - so).max() / np.abs(so).max()))}


def odd_grid_leg(args):
    """One crack-length increment on a grid whose length has prime factors
    above 3 (105 = 3 * 5 * 7, the paper's 3D grid): the pass kernels with
    generic-radix FFT stages.  Reports the in-solve apply time per voxel."""
    import torch

    from paper_2412_17445_amd import Solver
    from synth import problem_config

    prob = problem_config(args.odd_workload)
    s = Solver.from_problem(prob)
    s.bootstrap()
    w = s.step()
    log(f"{args.odd_workload} warm-up increment: converged={w['converged']} {w['seconds']:.2f}s")
    tim_warm = s.timing_read()
    s.timing(-args.timing_every)
    a0, _ = s.counters()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    o = s.step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    a1, _ = s.counters()
    tim = s.timing_read()
    whole = [v for sl, v in tim.items() if sl % 6 == 5]
    n_ap, ms_ap = sum(v[0] for v in whole), sum(v[1] for v in whole)
    s.close()
    log(f"{args.odd_workload} timed increment: converged={o['converged']} {dt:.2f}s")
    return {"workload": args.odd_workload, "grid": list(prob.shape[::-1]), "precision": prob.precision,
            "converged": o["converged"], "ms_per_increment": round(dt * 1e3, 2),
            "tangent_applies": a1 - a0,
            "mvoxel_applies_per_s": round((a1 - a0) * prob.nvox / dt / 1e6, 1),
            "apply_us_avg": round(ms_ap / max(n_ap, 1) * 1e3, 2),
            "apply_ns_per_voxel": round(ms_ap / max(n_ap, 1) * 1e6 / prob.nvox, 4)}


def mixed_bc_leg(prob, first):
    """The same workload under mixed macroscopic conditions (mean strain
    prescribed along f only, mean stress zero off f): one warm-up and one
    timed crack-length increment.  Reports its time and applies next to the
    strain-controlled increment, and the mean stress off f relative to its
    component along f (zero up to the Newton tolerance)."""
    import dataclasses

    import numpy as np
    import torch

    from paper_2412_17445_amd import Solver

    pm = dataclasses.replace(prob, name=prob.name + "_m", macro_bc="mixed")
    s = Solver.from_problem(pm)
    s.bootstrap()
    w = s.step()
    log(f"{pm.name} warm-up increment: converged={w['converged']} {w['seconds']:.2f}s")
    a0, _ = s.counters()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    o = s.step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    a1, _ = s.counters()
    s.close()
    log(f"{pm.name} timed increment: converged={o['converged']} {dt:.2f}s")
    f = np.asarray(pm.f, dtype=np.float64)
    sv = o["sigma_M"]
    S = np.array([[sv[0], sv[5], sv[4]], [sv[5], sv[1], sv[3]], [sv[4], sv[3], sv[2]]])
    if pm.dim == 2:                      # plane strain: sigma_zz is reported, not controlled
        S[2, 2] = 0.0
    fh = f / np.sqrt(np.sum(f * f))
    along = float(np.sum(fh * S))
    off = float(np.sqrt(np.sum((S - along * fh) ** 2)))
    return {"workload": pm.name, "converged": o["converged"], "timed_increment": 2,
            "ms_per_increment": round(dt * 1e3, 2), "tangent_applies": a1 - a0,
            "newton_iters": o["newton_iters"], "E_increment1": w["E"],
            "E_increment1_strain_control": first["E"], "sigma_off_f_over_along_f": off / abs(along)}


def serve_stream(args):
    """Seeded request stream (synth.stream) through the request server:
    Poisson arrivals, admission by footprint into slots, per-request latency
    (submission to last increment) and whole-stream throughput."""
    import numpy as np

    from paper_2412_17445_amd import Server, problem_kwargs
    from synth.stream import arrival_times, served_request

    log(f"served stream: {args.serve_requests} requests at {args.serve_rate}/s, "
        f"{args.serve_slots} slots, increments x{args.serve_inc_scale}")
    reqs = [served_request(k, args.serve_inc_scale) for k in range(args.serve_requests)]
    arr = arrival_times(len(reqs), args.serve_rate)
    srv = Server(int(args.serve_budget_gb * (1 << 30)), args.serve_slots)
    t0 = time.perf_counter()
    tickets = []
    for (prob, n), ta in zip(reqs, arr):
        dt = ta - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        tickets.append(srv.submit(n, **problem_kwargs(prob)))
    infos, applies_vox, incs, failed, alg_bytes = [], 0, 0, 0, 0
    # requests are collected in the order they finish, each logged as it completes
    pending = list(range(len(tickets)))
    while pending:
        finished = [k for k in pending if srv.wait(tickets[k], 0.0)]
        if not finished:
            srv.wait(tickets[pending[0]], 0.2)
            continue
        for k in finished:
            tk = tickets[k]
            info = srv.info(tk)
            res = srv.results(tk)
            infos.append(info)
            prob = reqs[k][0]
            n_all = sum(r["applies"] for r in res)
            n64 = sum(r["applies_fp64"] for r in res)
            applies_vox += n_all * prob.nvox
            # algorithmic bytes of every apply: the working-precision applies at
            # their width, the FP64 ones (refinement defects, fallbacks) at 8 bytes
            alg_bytes += ((n_all - n64) * alg_bytes_per_voxel(prob, prob.precision)
                          + n64 * alg_bytes_per_voxel(prob, "fp64")) * prob.nvox
            incs += len(res)
            failed += info["status"] != 0
            log(f"request {k}: {prob.notes}, {len(res)} increments, status {info['status']}, "
                f"latency {info['t_done'] - info['t_submit']:.2f}s")
        done = set(finished)
        pending = [k for k in pending if k not in done]
    makespan = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    lat = np.array([i["t_done"] - i["t_submit"] for i in infos])
    wait = np.array([i["t_admit"] - i["t_submit"] for i in infos])
    return {"requests": len(reqs), "failed": int(failed), "increments": int(incs),
            "latency_p50_s": round(float(np.percentile(lat, 50)), 3),
            "latency_p99_s": round(float(np.percentile(lat, 99)), 3),
            "latency_max_s": round(float(lat.max()), 3),
            "queue_wait_p50_s": round(float(np.percentile(wait, 50)), 3),
            "makespan_s": round(makespan, 3),
            "throughput_requests_per_s": round(len(reqs) / makespan, 3),
            "throughput_mvoxel_applies_per_s": round(applies_vox / makespan / 1e6, 1),
            "roofline": {"bound": "hbm", "achieved": round(alg_bytes / makespan / 1e9, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(alg_bytes / makespan / 1e9 / HBM_PEAK_GBS, 4),
                         "what": "algorithmic bytes of every tangent apply of the stream (22 words "
                                 "per voxel-apply in 2D, 37 in 3D, plus the phase byte) over the makespan"},
            "slots": args.serve_slots, "max_running": st["max_running"],
            "peak_bytes": st["peak_bytes"], "budget_bytes": st["budget"],
            "batched_inner_solves": {"chunks": st["batch_chunks"], "solves": st["batch_solves"],
                                     "iterations": st["batch_iterations"], "graphs": st["batch_graphs"],
                                     "max_batch": st["batch_max"], "mean_batch": round(st["batch_mean"], 3),
                                     "enabled": os.environ.get("PFF_SERVER_BATCH", "1") != "0"},
            "stream": f"synth.stream seeds 0..{len(reqs) - 1}, Poisson {args.serve_rate}/s, "
                      f"increments scaled by {args.serve_inc_scale}",
            "kind": ("the full 256-request served stream" if len(reqs) >= 256
                     else "a reduced served stream (smoke run of the serving path)")}


def fullrun_mode(prob, args):
    """The mixed-precision and the plain FP64 GPU solver over the workload's
    whole configured path (bootstrap and every increment): time per run and
    the largest relative difference per quantity over the increments."""
    import copy

    import numpy as np
    import torch

    from paper_2412_17445_amd import Solver

    n = prob.n_increments
    runs = {}
    for prec in ("mixed", "fp64"):
        p = copy.copy(prob)
        p.precision = prec
        s = Solver.from_problem(p)
        s.bootstrap()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rows = []
        for k in range(n):
            o = s.step()
            if not o["converged"]:
                log(f"{prec}: increment {k + 1} did not converge")
                break
            _, phi, _, _, _ = s.get_state()
            rows.append((o["E"], o["Gamma"], np.array(o["sigma_M"]), float(np.linalg.norm(phi)),
                         o["newton_iters"], o["krylov_iters"]))
            if (k + 1) % 10 == 0:
                log(f"{prec}: increment {k + 1}, {time.perf_counter() - t0:.1f}s")
        torch.cuda.synchronize()
        runs[prec] = (rows, time.perf_counter() - t0)
        s.close()
    (m, tm), (f, tf) = runs["mixed"], runs["fp64"]
    worst = {"E": 0.0, "Gamma": 0.0, "sigma_M": 0.0, "phi_norm": 0.0}
    for a, b in zip(m, f):
        worst["E"] = max(worst["E"], abs(a[0] - b[0]) / abs(b[0]))
        worst["Gamma"] = max(worst["Gamma"], abs(a[1] - b[1]) / abs(b[1]))
        worst["sigma_M"] = max(worst["sigma_M"], float(np.abs(a[2] - b[2]).max() / np.abs(b[2]).max()))
        worst["phi_norm"] = max(worst["phi_norm"], abs(a[3] - b[3]) / b[3])
    print(json.dumps({"mode": "fullrun", "workload": prob.name, "increments_configured": n,
                      "increments_mixed": len(m), "increments_fp64": len(f),
                      "seconds_mixed": round(tm, 2), "seconds_fp64": round(tf, 2),
                      "newton_mixed": sum(r[4] for r in m), "newton_fp64": sum(r[4] for r in f),
                      "max_rel_diff": {k: float("%.3e" % v) for k, v in worst.items()}}), flush=True)


def apply_mode(prob, args):
    """Tangent applies on a frozen synthetic state (for counter runs)."""
    import numpy as np
    import torch

    from paper_2412_17445_amd import Solver

    s = Solver.from_problem(prob)
    c = s.ncomp
    rng = np.random.default_rng(0)
    eps = rng.standard_normal((c,) + prob.shape) * 1e-3
    eps[1 if c == 3 else 2] += 4e-3
    phi = rng.uniform(0.0, 0.5, prob.shape)
    s.set_state(eps, phi, np.full(prob.shape, 1e-6), 4e-3, 1.0, n=1)
    s.residual(2.0, want_F=False)
    dt = torch.float32 if prob.precision == "mixed" else torch.float64
    v = torch.randn(s.M, dtype=dt, device="cuda") * 1e-3
    out = torch.empty_like(v)
    for _ in range(args.applies):
        s.apply(v, out)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "apply", "workload": args.workload, "applies": args.applies,
                      "alg_bytes_per_launch": kernel_bytes(prob.shape, prob.precision)}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="particles3d_128")
    ap.add_argument("--precision", default=None, help="override: fp64 or mixed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--timing-every", type=int, default=7,
                    help="sample every n-th apply (odd: the fused applies alternate modes)")
    ap.add_argument("--mode", default="solve", choices=["solve", "apply", "copy", "serve", "fullrun"],
                    help="solve: timed increments (default); apply: tangent applies on a frozen "
                         "state (profiling counters); copy: plain device copy of 256 MiB "
                         "(counter calibration); serve: the served request stream; fullrun: the "
                         "mixed and the plain FP64 solver over the workload's whole path")
    ap.add_argument("--applies", type=int, default=20)
    ap.add_argument("--no-compare", action="store_true",
                    help="mixed workloads: skip the plain-FP64 solve of the same increments")
    ap.add_argument("--no-serve", action="store_true", help="skip the served request stream")
    ap.add_argument("--no-stagger", action="store_true",
                    help="skip the staggered strain-controlled increment")
    ap.add_argument("--no-odd", action="store_true",
                    help="skip the increment on a grid with prime factors above 3")
    ap.add_argument("--odd-workload", default="pores3d_105")
    ap.add_argument("--no-bare-all", action="store_true",
                    help="skip the bare-apply timing of the other benchmark grids")
    ap.add_argument("--no-mixed-bc", action="store_true",
                    help="skip the increments under mixed macroscopic conditions")
    ap.add_argument("--serve-requests", type=int, default=16)
    ap.add_argument("--serve-rate", type=float, default=4.0, help="Poisson arrivals per second")
    ap.add_argument("--serve-inc-scale", type=float, default=0.1,
                    help="fraction of each request's 20-60 increments that is run")
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs one RVE solve on one GPU; multi-GPU runs are not "
              "part of it (requests shard across GPUs with no communication).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2412_17445_amd import Solver
    from synth import problem_config

    torch.cuda.set_device(0)
    if args.mode == "copy":
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "copy", "bytes_read_per_launch": src.numel() * 4,
                          "bytes_written_per_launch": dst.numel() * 4, "launches": 3}))
        return
    if args.mode == "serve":
        out = serve_stream(args)
        print(json.dumps({"metric": "RVE latency p50/p99 (served stream)", "value": out["latency_p50_s"],
                          "unit": "s", "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
                          "serving": out}), flush=True)
        return
    prob = problem_config(args.workload)
    if args.precision:
        prob.precision = args.precision
    if args.mode == "apply":
        apply_mode(prob, args)
        return
    if args.mode == "fullrun":
        fullrun_mode(prob, args)
        return
    log(f"workload {args.workload} {prob.shape[::-1]} {prob.precision}")
    s = Solver.from_problem(prob)
    s.bootstrap()
    log("bootstrap done")
    # per-pass events on the warm-up applies (the pass breakdown); the timed
    # region samples the whole apply only (two events, less perturbation)
    s.timing(args.timing_every)
    warm = []
    for i in range(args.warmup):
        out = s.step()
        warm.append(out)
        log(f"warm-up increment {i + 1}: converged={out['converged']} "
            f"newton={out['newton_iters']} krylov={out['krylov_iters']} {out['seconds']:.2f}s")
        if not out["converged"]:
            raise RuntimeError(f"warm-up increment did not converge: {out}")
    tim_warm = s.timing_read()
    s.timing(-args.timing_every)
    a0, _ = s.counters()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = []
    for i in range(args.steps):
        outs.append(s.step())
        log(f"timed increment {i + 1}: converged={outs[-1]['converged']} "
            f"newton={outs[-1]['newton_iters']} krylov={outs[-1]['krylov_iters']} "
            f"{outs[-1]['seconds']:.2f}s")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    a1, _ = s.counters()
    if not all(o["converged"] for o in outs):
        raise RuntimeError("an increment in the timed region did not converge")
    elapsed = t1 - t0
    N = prob.nvox
    applies = a1 - a0
    value = applies * N / elapsed / 1e6

    tim_all = s.timing_read()
    # the timed region's whole-apply samples
    tim = {k: (n - tim_warm.get(k, (0, 0.0))[0], ms - tim_warm.get(k, (0, 0.0))[1])
           for k, (n, ms) in tim_all.items()}
    prec_main = "mixed" if prob.precision == "mixed" else "fp64"
    main_groups = range(5, 10) if prec_main == "mixed" else range(0, 5)
    # whole apply (its five pass kernels and the finisher) over the sampled
    # applies of the working precision, every fused variant
    whole = [tim[6 * gp + 5] for gp in main_groups if tim.get(6 * gp + 5, (0, 0))[0] > 0]
    apply_n, apply_ms = sum(v[0] for v in whole), sum(v[1] for v in whole)
    apply_s = apply_ms * 1e-3 / apply_n
    bvox = alg_bytes_per_voxel(prob, prob.precision)
    achieved = bvox * N / apply_s / 1e9
    # per pass kernel: its own algorithmic bytes and time (secondary figures,
    # from the per-pass events of the warm-up increments)
    passes = {}
    for gp in main_groups:
        for k in range(5):
            if 6 * gp + k not in tim_warm:
                continue
            n, ms = tim_warm[6 * gp + k]
            b = kernel_bytes(prob.shape, prec_main, gp % 5)[k]
            if b <= 0:
                continue
            a = passes.setdefault(k, [0, 0.0, 0.0])
            a[0] += n
            a[1] += ms
            a[2] += n * b
    pass_out = {KERNEL_NAMES[k]: {"avg_us": round(ms / n * 1e3, 2), "own_bytes_per_launch": round(b / n),
                                  "own_GBs": round(b / n / (ms / n * 1e-3) / 1e9, 1)}
                for k, (n, ms, b) in sorted(passes.items())}
    traffic = load_traffic(args.workload)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "tangent apply (5 FFT pass kernels + finisher), "
                          + ("FP32" if prec_main == "mixed" else "FP64"),
                "alg_bytes_per_voxel_apply": bvox, "voxels_per_launch": N,
                "alg_bytes_per_launch": bvox * N, "avg_launch_us": round(apply_s * 1e6, 2),
                "timed_launches": apply_n,
                "timing": "HIP events around every sampled apply (two per apply) on the solver stream over "
                          "the timed region; passes: per-pass events over the warm-up increments",
                "traffic_over_alg": None if traffic is None else round(traffic / (bvox * N), 3),
                "passes": pass_out}
    by_mode = {"fp32": [0] * 5, "fp64": [0] * 5}
    for sl, (n, _) in tim_warm.items():
        if sl % 6 == 5:
            by_mode["fp32" if sl // 6 >= 5 else "fp64"][(sl // 6) % 5] += n
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
                   "fp64_applies": sum(o["applies_fp64"] for o in outs),
                   "fp64_refinements": sum(o["refinements"] for o in outs),
                   "fp64_fallback_solves": sum(o["fp64_fallbacks"] for o in outs),
                   "apply_us_avg": round(apply_s * 1e6, 2),
                   "sampled_applies_by_mode": by_mode,
                   "parallelism": "single GPU"},
        "roofline": roofline,
    }
    line["vs_oracle"] = vs_oracle(prob, warm + outs, s)
    # bare applies at the committed state of the last timed increment
    _, _, _, _, a_last = s.get_state()
    s.residual(a_last, want_F=False)
    line["bare_apply"] = bare_apply(s, prob, prob.precision)
    line["bare_apply"]["state"] = f"committed state of increment {args.warmup + args.steps}"
    log(f"bare apply: {line['bare_apply']}")
    if not args.no_bare_all:
        line["bare_apply_other_grids"] = [bare_apply_leg(w) for w in BARE_WORKLOADS if w != args.workload]
    if prob.precision == "mixed" and not args.no_compare:
        s.close()
        line["mixed_vs_fp64"] = compare_fp64(prob, args, warm + outs, elapsed / args.steps)
    if not args.no_stagger:
        first = (warm + outs)[0]
        line["staggered_vs_crack_control"] = staggered_leg(prob, first)
        if "mixed_vs_fp64" in line:
            line["staggered_vs_crack_control"]["crack_control_fp64_seconds"] = \
                line["mixed_vs_fp64"]["fp64_first_increment_s"]
    if not args.no_mixed_bc:
        line["mixed_bc"] = mixed_bc_leg(prob, (warm + outs)[0])
    if not args.no_odd:
        line["odd_grid"] = odd_grid_leg(args)
        line["odd_grid"]["apply_ns_per_voxel_main"] = round(
            line["config"]["apply_us_avg"] * 1e3 / N, 4)
    if not args.no_serve:
        line["serving"] = serve_stream(args)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
