"""Write the oracle's per-increment outputs used by the GPU increment-parity
tests.  Calls only `oracle/` and `synth/` (the seeded problem definitions).

    python tests/golden/make_oracle_runs.py CASE [CASE ...]

Each CASE writes tests/golden/oracle_<CASE>.json with the bootstrap values
(a0, E_s) and, per increment: E, Gamma, a, Sigma_M (11, 22, 33, 23, 13, 12),
||phi||, the dissipation D, the damage at sampled voxels, the residual
measures ||F1|| / ||sigma|| and ||F2|| / ||2H|| of the converged state,
Newton and Krylov iteration counts.  Runs use the parity-mode Newton stop
(residual measures <= RESID_TOL besides the update tolerance), so that the
stored increments are the roots of the discrete system to that residual and
not points a tolerance away from them.

Cases listed in STATES also write tests/golden/oracle_<CASE>_states.npz: the
committed state (strain fluctuation, damage, history, E, a) after the listed
increments, from which the GPU re-runs the next increment (re-seeded parity:
both sides take the same increment from the same state, so path drift along
a nearly neutral direction does not accumulate between them).

Full-size workloads take an inexact Newton: the Krylov tolerance of each
step is loose (KRYLOV_RTOL), which changes the iterates but not the root
that the residual stop pins.  tests/test_oracle_newton.py checks that the
inexact and the exact oracle Newton land on the same increment.
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import fourier  # noqa: E402
from oracle.newton import Solver  # noqa: E402
from synth import problem_config  # noqa: E402

# FFT threads of the oracle (the transforms of independent lines are split
# over the threads; the result does not depend on their number)
fourier.FFT_WORKERS = int(os.environ.get("ORACLE_FFT_WORKERS", "1"))

RESID_TOL = 1e-11
N_RANDOM_SAMPLES = 40      # damage sampled at seeded voxels ...
N_PEAK_SAMPLES = 24        # ... and at the most damaged voxels off the crack mask

CASES = {"tiny16": 4, "gc16": 4, "fib64": 4, "pore24": 3, "part24": 3, "crack2d_64": 30,
         "gc16_iso": 4, "part24_iso": 3, "gc16_std": 4, "gc16_w": 4,
         "crack2d_39": 4, "pore35": 1, "gc16_d": 4, "gc16_v": 4, "tiny16_v": 4,
         "gc16_m": 4, "tiny16_m": 4, "part12": 3, "part12_m": 3, "part24_m": 3,
         # full-size workloads (inexact Newton, see KRYLOV_RTOL)
         "fibres2d_256": 20, "pores3d_64": 3, "particles3d_128": 1}

# Krylov tolerance of the oracle's Newton steps where it differs from the
# problem's own (1e-10): loose inner solves for the full-size workloads
KRYLOV_RTOL = {"fibres2d_256": 1e-4, "pores3d_64": 1e-2, "particles3d_128": 1e-2}

# committed states stored for re-seeded parity: increments after which the
# state is written (0 = none)
STATES = {"part24_m": [1, 2], "part12_m": [1, 2]}


def sample_index(prob):
    rng = np.random.default_rng(20241217)
    return np.sort(rng.choice(prob.nvox, size=min(N_RANDOM_SAMPLES, prob.nvox), replace=False))


def run(case, n_inc):
    prob = problem_config(case)
    s = Solver(prob, rtol=KRYLOV_RTOL.get(case), resid_tol=RESID_TOL)
    t0 = time.time()
    boot = s.bootstrap()
    fixed = sample_index(prob)
    mask = np.zeros(prob.nvox, bool) if prob.mask is None else prob.mask.reshape(-1) != 0
    store = STATES.get(case, [])
    states = {}
    incs = []
    for _ in range(n_inc):
        o = s.step()
        if not o["converged"]:
            raise RuntimeError(f"{case}: oracle increment {len(incs) + 1} did not converge")
        sm = o["sigma_M"]
        phi = s.phi.reshape(-1)
        peak = np.argsort(np.where(mask, -np.inf, phi), kind="stable")[::-1][:N_PEAK_SAMPLES]
        idx = np.concatenate([fixed, np.sort(peak)])
        incs.append(dict(increment=o["increment"], E=o["E"], Gamma=o["Gamma"], a=o["a"],
                         sigma_M=[sm[0, 0], sm[1, 1], sm[2, 2], sm[1, 2], sm[0, 2], sm[0, 1]],
                         phi_norm=o["phi_norm"], dissipation=o["D"],
                         phi_index=[int(i) for i in idx], phi_samples=[float(phi[i]) for i in idx],
                         resid=[float(r) for r in o["resid"]],
                         newton_iters=o["newton_iters"], krylov_iters=o["krylov_iters"]))
        if o["increment"] in store:
            k = o["increment"]
            states[f"eps_t_{k}"] = s.eps_t.reshape(-1)
            states[f"phi_{k}"] = s.phi.reshape(-1)
            states[f"Hn_{k}"] = s.Hn.reshape(-1)
            states[f"E_{k}"] = np.array(s.E)
            states[f"a_{k}"] = np.array(s.a)
        brief = {k: v for k, v in incs[-1].items() if k not in ("phi_index", "phi_samples")}
        print(case, brief, f"{time.time() - t0:.0f}s", flush=True)
        with open(os.path.join(HERE, f"oracle_{case}.json"), "w") as fh:
            json.dump(dict(case=case, a0=boot["a0"], E_s=boot["E_s"], resid_tol=RESID_TOL,
                           krylov_rtol=s.rtol, increments=incs,
                           source="oracle/ (NumPy FP64), tests/golden/make_oracle_runs.py"),
                      fh, indent=1)
        if states:
            np.savez_compressed(os.path.join(HERE, f"oracle_{case}_states.npz"), **states)


if __name__ == "__main__":
    for c in sys.argv[1:] or list(CASES):
        run(c, CASES[c])
