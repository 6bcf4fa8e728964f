"""Pins of the staggered strain-controlled oracle (paper Algorithm 1).

* Homogeneous cell under uniaxial plane strain: the exact solution of every
  increment is uniform, eps = f E, phi = 2H / (Gc/l + 2H) with
  H = (lambda/2 + mu) E^2, sigma = g(phi) (lambda E, lambda E + 2 mu E,
  lambda E) (textbook linear elasticity, computed here).
* At the load factor of a converged crack-length-controlled increment, the
  staggered scheme (a different algorithm: alternating sub-problems at fixed
  strain) reaches the same root of G[sigma] = 0 and the Helmholtz equation.
* Unloading keeps the damage (history) and scales the stress down.
"""

import json
import os

import numpy as np
import pytest

from oracle.newton import Solver
from oracle.staggered import StaggeredSolver
from synth import problem_config
from synth.configs import Problem, _dyad


def test_homogeneous_uniaxial_closed_form():
    n = 8
    Ey, nu, Gc, l, k = 1.0, 0.3, 1e-3, 2.0, 1e-6
    prob = Problem(name="hom", shape=(1, n, n), phases=[(Ey, nu, Gc)],
                   phase_id=np.zeros((1, n, n), np.uint8), mask=None, f=_dyad(1, 1), l=l, k=k)
    lam = Ey * nu / ((1 + nu) * (1 - 2 * nu))
    mu = Ey / (2 * (1 + nu))
    st = StaggeredSolver(prob, dE=0.02)
    for _ in range(4):
        out = st.step()
        E = out["E"]
        H = (0.5 * lam + mu) * E * E
        phi = 2 * H / (Gc / l + 2 * H)
        g = (1 - phi) ** 2 + k
        assert np.abs(st.phi - phi).max() <= 1e-9 * phi
        sig = out["sigma_M"]
        assert abs(sig[0, 0] - g * lam * E) <= 1e-9 * abs(g * lam * E)
        assert abs(sig[1, 1] - g * (lam + 2 * mu) * E) <= 1e-9 * abs(g * (lam + 2 * mu) * E)
        assert abs(sig[2, 2] - g * lam * E) <= 1e-9 * abs(g * lam * E)
        assert abs(sig[0, 1]) <= 1e-12


def test_homogeneous_compression_damages_only_without_split():
    """Uniaxial plane-strain compression: the spectral split leaves no
    driving energy (all strain eigenvalues and the trace are <= 0), the
    isotropic model is driven by the whole psi0 = (lambda/2 + mu) E^2."""
    n = 8
    Ey, nu, Gc, l, k = 1.0, 0.3, 1e-3, 2.0, 1e-6
    lam = Ey * nu / ((1 + nu) * (1 - 2 * nu))
    mu = Ey / (2 * (1 + nu))
    for split in ("spectral", "none"):
        prob = Problem(name="hom", shape=(1, n, n), phases=[(Ey, nu, Gc)],
                       phase_id=np.zeros((1, n, n), np.uint8), mask=None, f=_dyad(1, 1), l=l, k=k,
                       split=split)
        st = StaggeredSolver(prob, dE=-0.02)
        out = st.step()
        E = out["E"]
        H = (0.5 * lam + mu) * E * E if split == "none" else 0.0
        phi = 2 * H / (Gc / l + 2 * H)
        g = (1 - phi) ** 2 + k
        assert np.abs(st.phi - phi).max() <= 1e-9 * max(phi, 1e-300)
        sig = out["sigma_M"]
        gs = g if split == "none" else 1.0
        assert abs(sig[1, 1] - gs * (lam + 2 * mu) * E) <= 1e-9 * abs((lam + 2 * mu) * E)
        assert abs(sig[0, 0] - gs * lam * E) <= 1e-9 * abs(lam * E)


@pytest.mark.parametrize("case", ["tiny16", "gc16"])
def test_reaches_the_crack_length_controlled_root(case):
    prob = problem_config(case)
    mono = Solver(prob)
    mono.bootstrap()
    ref = mono.step()
    stag = StaggeredSolver(prob, dE=ref["E"])
    out = stag.step()
    assert abs(out["Gamma"] - ref["Gamma"]) <= 1e-8 * ref["Gamma"]
    assert np.abs(stag.phi - mono.phi).max() <= 1e-7
    sm, so = out["sigma_M"], ref["sigma_M"]
    assert np.abs(sm - so).max() <= 1e-7 * np.abs(so).max()


def test_zero_load_is_the_bootstrap_state():
    prob = problem_config("tiny16")
    st = StaggeredSolver(prob, dE=0.0)
    phi0 = st.phi.copy()
    out = st.step()
    assert out["stagger_iters"] == 1 and out["newton_iters"] == 1
    assert np.abs(st.phi - phi0).max() <= 1e-9 and not st.eps_t.any()   # CG rtol 1e-11 vs 1e-14
    assert np.abs(out["sigma_M"]).max() == 0.0


def test_unloading_keeps_the_damage():
    prob = problem_config("gc16")
    st = StaggeredSolver(prob, dE=3e-3)
    st.step()
    st.step()
    phi_peak = st.phi.copy()
    st.dE = -2e-3
    out = st.step()
    assert np.abs(st.phi - phi_peak).max() <= 1e-9
    assert out["E"] == pytest.approx(4e-3)


def test_stored_increments_are_the_oracle_s():
    """tests/golden/stagger_gc16.json (used by the GPU tests) is what the
    committed oracle computes now."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "stagger_gc16.json")) as fh:
        g = json.load(fh)
    st = StaggeredSolver(problem_config("gc16"), dE=0.0, **g["params"])
    idx = np.array(g["sample_index"])
    for ref in g["increments"]:
        st.dE = ref["dE"]
        out = st.step()
        assert out["Gamma"] == pytest.approx(ref["Gamma"], rel=1e-12)
        assert out["stagger_iters"] == ref["stagger_iters"]
        assert out["newton_iters"] == ref["newton_iters"]
        assert np.abs(st.phi.ravel()[idx] - ref["phi_samples"]).max() <= 1e-12
