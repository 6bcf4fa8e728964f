"""Pins of the weighted control w_a Gamma + w_E E = tau (FFT analogue of the
paper's eq. FEMweights; (1, 0) is the crack-length control of eq.
System_CrackLength).

* Weights (0, 1) make the monolithic Newton a strain-controlled solver: it
  reaches the roots of the staggered scheme (Algorithm 1, a different
  algorithm on the same equations) at the same loads, and it starts an
  uncracked homogeneous cell from phi = 0 along the closed-form path.
* Mixed weights on the homogeneous cell: the increment satisfies the
  constraint with the closed-form damage phi(E) (root found by bisection of
  the scalar constraint, written out here).
* J v against central differences of the residual with mixed weights.
* Dissipation control (eq. SystemDis, last line): with homogeneous Gc it is
  crack-length control with the increment scaled by Gc; with two
  toughnesses every increment raises D = sum Gc gamma_f by exactly delta.
"""

import numpy as np
import pytest

from oracle.newton import Solver
from oracle.staggered import StaggeredSolver
from oracle.system import System
from synth import problem_config
from synth.configs import Problem, _dyad

EY, NU, GC, L, K = 1.0, 0.3, 1e-3, 2.0, 1e-6
LAM = EY * NU / ((1 + NU) * (1 - 2 * NU))
MU = EY / (2 * (1 + NU))


def homogeneous(weights, n=8, delta=0.01):
    return Problem(name="hom", shape=(1, n, n), phases=[(EY, NU, GC)],
                   phase_id=np.zeros((1, n, n), np.uint8), mask=None, f=_dyad(1, 1), l=L, k=K,
                   delta_a=delta, control_weights=weights)


def phi_of(E):
    H = (0.5 * LAM + MU) * E * E
    return 2 * H / (GC / L + 2 * H)


def test_strain_weights_follow_the_uncracked_homogeneous_path():
    s = Solver(homogeneous((0.0, 1.0)))
    boot = s.bootstrap()
    assert boot["a0"] == 0.0 and boot["E_s"] == pytest.approx(0.01, rel=1e-12)
    for i in range(1, 5):
        o = s.step()
        assert o["converged"]
        assert o["E"] == pytest.approx(0.01 * i, rel=1e-12)
        assert np.abs(s.phi - phi_of(o["E"])).max() <= 1e-9 * phi_of(o["E"])


def test_mixed_weights_satisfy_the_constraint_in_closed_form():
    n, wa, wE = 8, 0.5, 20.0
    s = Solver(homogeneous((wa, wE), n=n, delta=0.2))
    s.bootstrap()
    for i in range(1, 4):
        o = s.step()
        assert o["converged"]
        tau = 0.2 * i

        def c(E):                        # constraint of the homogeneous solution
            return wa * n * n * phi_of(E) ** 2 / (2 * L) + wE * E - tau

        lo, hi = 0.0, 1.0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            lo, hi = (mid, hi) if c(mid) < 0 else (lo, mid)
        assert o["E"] == pytest.approx(0.5 * (lo + hi), rel=1e-9)
        assert wa * o["Gamma"] + wE * o["E"] == pytest.approx(tau, rel=1e-9)


def test_strain_weights_reach_the_staggered_roots():
    prob = problem_config("gc16")
    prob.control_weights = (0.0, 1.0)
    prob.delta_a = 3e-3
    mono = Solver(prob)
    mono.bootstrap()
    stag = StaggeredSolver(problem_config("gc16"), dE=3e-3)
    for _ in range(2):
        m = mono.step()
        st = stag.step()
        assert m["converged"] and m["E"] == pytest.approx(st["E"], rel=1e-12)
        assert abs(m["Gamma"] - st["Gamma"]) <= 1e-8 * st["Gamma"]
        assert np.abs(mono.phi - stag.phi).max() <= 1e-7
        assert np.abs(m["sigma_M"] - st["sigma_M"]).max() <= 1e-7 * np.abs(st["sigma_M"]).max()


@pytest.mark.parametrize("weights", [(0.0, 1.0), (0.7, 3.0)])
def test_tangent_is_residual_derivative_with_weights(weights):
    prob = problem_config("gc16")
    prob.control_weights = weights
    sy = System(prob)
    rng = np.random.default_rng(4)
    eps_t = rng.standard_normal((sy.ncomp,) + sy.shape) * 1e-3
    from oracle import fourier as fo
    eps_t = fo.G_mandel(eps_t)
    phi = np.clip(rng.uniform(0, 0.6, sy.shape) + sy.m, 0, 1)
    E = 5e-3
    Hn = sy.point(eps_t + sy.fE(E), phi, np.zeros(sy.shape))["psi_p"] * 0.8
    J = sy.tangent(eps_t, phi, E, Hn)
    d_eps = fo.G_mandel(rng.standard_normal(eps_t.shape)) * 1e-2
    d_phi = rng.standard_normal(sy.shape) * 1e-2 * (1 - sy.m)
    dE = 1e-3
    Jv = J(sy.pack(d_eps, d_phi, dE))
    h = 1e-6

    def F(t):
        R = sy.residual(eps_t + t * d_eps, phi + t * d_phi, E + t * dE, Hn, 2.0)
        return sy.pack(R["F1"], R["F2"], R["F3"])

    fd = (F(h) - F(-h)) / (2 * h)
    assert abs(Jv[-1] - fd[-1]) <= 1e-7 * abs(fd[-1])
    assert np.abs(Jv[:-1] - fd[:-1]).max() <= 2e-5 * np.abs(fd[:-1]).max()


def test_dissipation_control_with_uniform_toughness_is_length_control():
    a = problem_config("tiny16")
    d = problem_config("tiny16_d")
    Gc = a.phases[0][2]
    assert d.delta_a == pytest.approx(Gc * a.delta_a)
    sa, sd = Solver(a), Solver(d)
    ba, bd = sa.bootstrap(), sd.bootstrap()
    assert bd["a0"] == pytest.approx(Gc * ba["a0"], rel=1e-13)
    assert bd["E_s"] == pytest.approx(ba["E_s"], rel=1e-12)
    for _ in range(2):
        oa, od = sa.step(), sd.step()
        assert od["E"] == pytest.approx(oa["E"], rel=1e-9)
        assert od["Gamma"] == pytest.approx(oa["Gamma"], rel=1e-9)
        assert od["D"] == pytest.approx(Gc * od["Gamma"], rel=1e-13)


def test_dissipation_control_with_two_toughnesses():
    prob = problem_config("gc16_d")
    s = Solver(prob)
    b = s.bootstrap()
    sy = s.sys
    D0 = b["a0"]
    assert D0 == pytest.approx(sy.dissipation(s.phi), rel=1e-13)
    length = Solver(problem_config("gc16"))
    length.bootstrap()
    for i in range(1, 3):
        o = s.step()
        assert o["converged"]
        assert o["D"] == pytest.approx(D0 + i * prob.delta_a, rel=1e-8)
        ol = length.step()
        assert abs(o["E"] - ol["E"]) > 1e-6 * ol["E"]          # a different control


def test_tangent_is_residual_derivative_under_dissipation_control():
    from oracle import fourier as fo
    prob = problem_config("gc16_d")
    sy = System(prob)
    rng = np.random.default_rng(6)
    eps_t = fo.G_mandel(rng.standard_normal((sy.ncomp,) + sy.shape) * 1e-3)
    phi = np.clip(rng.uniform(0, 0.6, sy.shape) + sy.m, 0, 1)
    E = 5e-3
    Hn = sy.point(eps_t + sy.fE(E), phi, np.zeros(sy.shape))["psi_p"] * 0.8
    J = sy.tangent(eps_t, phi, E, Hn)
    d_phi = rng.standard_normal(sy.shape) * 1e-2 * (1 - sy.m)
    Jv = J(sy.pack(np.zeros_like(eps_t), d_phi, 0.0))
    h = 1e-6

    def F3(t):
        return sy.residual(eps_t, phi + t * d_phi, E, Hn, 1.0)["F3"]

    fd = (F3(h) - F3(-h)) / (2 * h)
    assert abs(Jv[-1] - fd) <= 1e-7 * abs(fd)     # the row with Gc r instead is 2.5e-2 off
