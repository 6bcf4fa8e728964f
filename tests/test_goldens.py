"""The stored oracle goldens agree with the script that writes them
(tests/golden/make_oracle_runs.py, which calls only the oracle): every
listed case has its golden, with the listed number of increments in order,
written in parity mode; every stored increment is a root of eq.
`System_CrackLength` to that residual (||F1|| / ||sigma|| and ||F2|| / ||2H||)
and meets its control equation w_a Q + w_E E = a, the stored a being the
control target tau (Q = Gamma, or the dissipation D under dissipation
control, eq. `SystemDis`; Gamma = a under plain crack-length control,
Algorithm 2); the stored committed states are the listed ones.  Reads files
only (CPU)."""

import json
import os
import sys

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
sys.path.insert(0, GOLDEN)

import make_oracle_runs as mk  # noqa: E402
from synth import problem_config  # noqa: E402


@pytest.mark.parametrize("case", sorted(mk.CASES))
def test_golden_matches_its_generator(case):
    with open(os.path.join(GOLDEN, f"oracle_{case}.json")) as fh:
        g = json.load(fh)
    assert g["case"] == case
    assert g["resid_tol"] == mk.RESID_TOL
    incs = g["increments"]
    assert [i["increment"] for i in incs] == list(range(1, mk.CASES[case] + 1))
    prob = problem_config(case)
    wa, wE = prob.control_weights
    for i in incs:
        assert max(i["resid"]) <= mk.RESID_TOL, (i["increment"], i["resid"])
        Q = i["dissipation"] if prob.control == "dissipation" else i["Gamma"]
        assert abs(wa * Q + wE * i["E"] - i["a"]) <= 1e-8 * abs(i["a"]), (i["increment"], Q, i["a"])
        assert len(i["phi_index"]) == len(i["phi_samples"]) > 0
        assert len(i["sigma_M"]) == 6


@pytest.mark.parametrize("case", sorted(mk.STATES))
def test_stored_states_are_the_listed_ones(case):
    st = np.load(os.path.join(GOLDEN, f"oracle_{case}_states.npz"))
    stored = sorted(int(k[len("phi_"):]) for k in st.files if k.startswith("phi_"))
    assert stored == sorted(mk.STATES[case])
    with open(os.path.join(GOLDEN, f"oracle_{case}.json")) as fh:
        incs = {i["increment"]: i for i in json.load(fh)["increments"]}
    for k in stored:
        for name in ("eps_t", "phi", "Hn", "E", "a"):
            assert f"{name}_{k}" in st.files
        assert float(st[f"E_{k}"]) == incs[k]["E"]
        assert float(st[f"a_{k}"]) == incs[k]["a"]
        assert np.linalg.norm(st[f"phi_{k}"]) == pytest.approx(incs[k]["phi_norm"], rel=1e-14)
