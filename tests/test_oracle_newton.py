"""Newton-level pins of the oracle (paper Sec. 3.2, Algorithm 2).

* Brute force: a dense finite-difference-Jacobian Newton with LU (no analytic
  tangent, no Krylov solver) reaches the same increments as the
  Newton-BiCGSTAB oracle on a tiny grid.
* Symmetry: a centred crack in a homogeneous cell stays mirror-symmetric.
* Invariants of the path: Gamma(phi_n) = a_n, a and history non-decreasing,
  strain fluctuation zero-mean and compatible, damage within [0, 1] up to
  the AT2 overshoot.
"""

import numpy as np
import pytest

from oracle import brute
from oracle import fourier as fo
from oracle.newton import Solver
from synth import problem_config
from synth.microstructure import line_crack_mask


def tiny(n=12, crack=(4, 8), l=1.5, da=0.5):
    prob = problem_config("tiny16")
    prob.shape = (1, n, n)
    prob.phase_id = np.zeros(prob.shape, np.uint8)
    prob.mask = line_crack_mask(n, n, n // 2, crack[0], crack[1])
    prob.l, prob.delta_a = l, da
    return prob


def test_bruteforce_dense_newton_matches():
    prob = tiny()
    s = Solver(prob)
    s.bootstrap()
    ref = Solver(prob)
    ref.bootstrap()
    for n in range(2):
        a_new = ref.a + ref.delta_a
        start = ref.guess if n == 0 else (ref.eps_t, ref.phi, ref.E)
        eps_t, phi, E, info = brute.newton_dense(ref, *start, a_new)
        assert info["converged"]
        st = ref.sys.point(eps_t + ref.sys.fE(E), phi, ref.Hn)
        ref.Hn = np.maximum(st["psi_p"], ref.Hn)
        ref.eps_t, ref.phi, ref.E, ref.a = eps_t, phi, E, a_new
        out = s.step()
        assert out["converged"]
        assert abs(out["E"] - E) <= 1e-9 * abs(E)
        assert np.abs(s.phi - phi).max() <= 1e-9
        assert np.abs(s.eps_t - eps_t).max() <= 1e-9 * np.abs(eps_t).max()


def test_centred_crack_stays_symmetric():
    n = 32
    prob = tiny(n=n, crack=(12, 20), l=2.0, da=1.0)
    s = Solver(prob)
    s.bootstrap()
    for _ in range(2):
        assert s.step()["converged"]
    # symmetric up to the solver tolerances (Newton 1e-8, Krylov 1e-10)
    fx = lambda a: a[:, ::-1]                              # noqa: E731  x -> n-1-x
    fy = lambda a: np.roll(a[::-1, :], 1, axis=0)          # noqa: E731  y -> n-y
    phi = s.phi[0]
    for refl in (fx, fy):
        assert np.abs(phi - refl(phi)).max() < 1e-7
        for k, sign in ((0, 1.0), (1, 1.0), (2, -1.0)):    # eps_xy flips sign
            e = s.eps_t[k, 0]
            assert np.abs(e - sign * refl(e)).max() < 1e-7 * np.abs(e).max()


def test_path_invariants():
    prob = tiny(n=16, crack=(6, 10))
    s = Solver(prob)
    s.bootstrap()
    a_prev, H_prev = s.a, s.Hn.copy()
    for _ in range(4):
        out = s.step()
        assert out["converged"]
        assert abs(s.sys.gamma(s.phi) - s.a) <= 1e-8 * s.a
        assert s.a > a_prev
        assert np.all(s.Hn >= H_prev)
        assert abs(s.eps_t.mean(axis=(1, 2, 3))).max() < 1e-11 * np.abs(s.eps_t).max()
        comp = fo.G_mandel(s.eps_t)
        assert np.abs(comp - s.eps_t).max() <= 1e-9 * np.abs(s.eps_t).max()
        assert s.phi.min() > -1e-3 and s.phi.max() <= 1.0 + 1e-12
        a_prev, H_prev = s.a, s.Hn.copy()


@pytest.mark.parametrize("alpha", [1.0, 0.9])
def test_residual_stop_pins_the_root_whatever_the_krylov_tolerance(alpha):
    """With the parity-mode residual stop the increment is the root of the
    discrete system to the residual tolerance: an inexact Newton (Krylov
    tolerance 1e-3) lands on the same increments as the exact one (1e-10),
    with the linear convergence of a relaxed Newton (alpha = 0.9) too.  The
    full-size oracle runs use such inexact steps."""
    prob = tiny(n=16, crack=(6, 10))
    prob.alpha = alpha
    ex = Solver(prob, rtol=1e-10, resid_tol=1e-11)
    inx = Solver(prob, rtol=1e-3, resid_tol=1e-11)
    ex.bootstrap()
    inx.bootstrap()
    for _ in range(2):
        a, b = ex.step(), inx.step()
        assert a["converged"] and b["converged"]
        assert max(b["resid"]) <= 1e-11
        assert abs(a["E"] - b["E"]) <= 1e-10 * abs(a["E"])
        assert np.abs(ex.phi - inx.phi).max() <= 1e-10
        assert np.abs(ex.eps_t - inx.eps_t).max() <= 1e-10 * np.abs(ex.eps_t).max()
