"""Write the staggered (strain-controlled) oracle's per-increment outputs used
by the GPU parity tests of the staggered scheme.  Calls only `oracle/` and
`synth/` (the seeded problem definitions).

    python tests/golden/make_stagger_runs.py CASE [CASE ...]

Each CASE runs the load steps of STEPS from the bootstrap state and writes
tests/golden/stagger_<CASE>.json with, per increment: E, Gamma, Sigma_M
(11, 22, 33, 23, 13, 12), ||phi||, ||eps~||, phi at SAMPLES fixed voxels and
the stagger / Newton / CG counts.  "E1" in a step list stands for the load
factor of the first crack-length-controlled oracle increment of that case
(tests/golden/oracle_<CASE>.json), at which both schemes share a root.
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.staggered import StaggeredSolver  # noqa: E402
from synth import problem_config  # noqa: E402

STEPS = {"tiny16": ["E1", "E1"], "gc16": [3e-3, 3e-3, -2e-3], "crack2d_64": ["E1"],
         "pore24": ["E1"], "tiny16_m": ["E1", "E1"], "gc16_m": [3e-3, 3e-3, -2e-3]}
SAMPLES = 32


def sample_index(n_vox):
    return np.unique(np.linspace(0, n_vox - 1, SAMPLES).round().astype(np.int64))


def run(case):
    prob = problem_config(case)
    steps = STEPS[case]
    if "E1" in steps:
        with open(os.path.join(HERE, f"oracle_{case}.json")) as fh:
            E1 = json.load(fh)["increments"][0]["E"]
        steps = [E1 if d == "E1" else d for d in steps]
    st = StaggeredSolver(prob, dE=steps[0])
    idx = sample_index(st.phi.size)
    t0 = time.time()
    incs = []
    for dE in steps:
        st.dE = float(dE)
        o = st.step()
        sm = o["sigma_M"]
        incs.append(dict(increment=o["increment"], dE=float(dE), E=o["E"], Gamma=o["Gamma"],
                         sigma_M=[sm[0, 0], sm[1, 1], sm[2, 2], sm[1, 2], sm[0, 2], sm[0, 1]],
                         phi_norm=float(np.linalg.norm(st.phi)),
                         eps_norm=float(np.linalg.norm(st.eps_t)),
                         phi_samples=st.phi.ravel()[idx].tolist(),
                         stagger_iters=o["stagger_iters"], newton_iters=o["newton_iters"],
                         cg_mech=o["cg_mech"], cg_helm=o["cg_helm"]))
        print(case, {k: v for k, v in incs[-1].items() if k != "phi_samples"},
              f"{time.time() - t0:.0f}s", flush=True)
    with open(os.path.join(HERE, f"stagger_{case}.json"), "w") as fh:
        json.dump(dict(case=case, sample_index=idx.tolist(), increments=incs,
                       params=dict(tol_mech=st.tol_mech, tol_sta=st.tol_sta, cg_rtol=st.cg_rtol),
                       source="oracle/staggered.py (NumPy FP64), tests/golden/make_stagger_runs.py"),
                  fh, indent=1)


if __name__ == "__main__":
    for c in sys.argv[1:] or list(STEPS):
        run(c)
