"""Write the oracle's per-increment outputs used by the GPU increment-parity
tests.  Calls only `oracle/` and `synth/` (the seeded problem definitions).

    python tests/golden/make_oracle_runs.py CASE [CASE ...]

Each CASE writes tests/golden/oracle_<CASE>.json with the bootstrap values
(a0, E_s) and, per increment: E, Gamma, a, Sigma_M (11, 22, 33, 23, 13, 12),
||phi||, the dissipation D (runs written after it was added), Newton and
Krylov iteration counts.
"""

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.newton import Solver  # noqa: E402
from synth import problem_config  # noqa: E402

CASES = {"tiny16": 4, "gc16": 4, "fib64": 4, "pore24": 3, "part24": 3, "crack2d_64": 30,
         "gc16_iso": 4, "part24_iso": 3, "gc16_std": 4, "gc16_w": 4,
         "crack2d_39": 4, "pore35": 1, "gc16_d": 4, "gc16_v": 4, "tiny16_v": 4,
         "gc16_m": 4, "tiny16_m": 4, "part12": 3, "part12_m": 1}


def run(case, n_inc):
    prob = problem_config(case)
    s = Solver(prob)
    t0 = time.time()
    boot = s.bootstrap()
    incs = []
    for _ in range(n_inc):
        o = s.step()
        if not o["converged"]:
            raise RuntimeError(f"{case}: oracle increment {len(incs) + 1} did not converge")
        sm = o["sigma_M"]
        incs.append(dict(increment=o["increment"], E=o["E"], Gamma=o["Gamma"], a=o["a"],
                         sigma_M=[sm[0, 0], sm[1, 1], sm[2, 2], sm[1, 2], sm[0, 2], sm[0, 1]],
                         phi_norm=o["phi_norm"], dissipation=o["D"], newton_iters=o["newton_iters"],
                         krylov_iters=o["krylov_iters"]))
        print(case, incs[-1], f"{time.time() - t0:.0f}s", flush=True)
        with open(os.path.join(HERE, f"oracle_{case}.json"), "w") as fh:
            json.dump(dict(case=case, a0=boot["a0"], E_s=boot["E_s"], increments=incs,
                           source="oracle/ (NumPy FP64), tests/golden/make_oracle_runs.py"),
                      fh, indent=1)


if __name__ == "__main__":
    for c in sys.argv[1:] or list(CASES):
        run(c, CASES[c])
