"""Pins of the mixed macroscopic conditions (Sec. 2.3: the mean strain is
prescribed only along the loading direction f, the other macroscopic
components follow from zero mean stress), taken as the projection with
G(0) = P_f^perp (A -> A - fh (fh : A), fh = f / |f|).

* The projection: idempotent and self-adjoint (orthogonal) on random
  fields; its zero mode keeps exactly the part of the mean orthogonal to f;
  it equals the strain-controlled projection on every other mode.
* Homogeneous cell under uniaxial stress with the Miehe split, 2D (plane
  strain) and 3D: every crack-length increment equals the closed form
  (uniform phi from Gamma, H from the damage equation, lateral strain from
  zero lateral stress, E from H = psi+), and Sigma_M has zero lateral and
  shear components.  The isotropic model (no split) in 2D as well.
* Elastic laminate of two phases loaded across the layers' plane: each layer
  contracts freely, eps_xx = -lam/(lam + 2 mu) E, and Sigma_yy is the
  volume average of the layers' uniaxial plane-strain moduli.
* J v against central differences of the residual with mixed conditions, in
  2D with a crack and two phases and in 3D with particles.
* The staggered scheme (Algorithm 1) on the homogeneous cell: uniform damage
  at the root of the scalar fixed point phi(H(E, g(phi))), found by bisection.
* (f t uniform, -t) is a null direction of the bordered Jacobian under either
  condition, and the oracle's committed fluctuation has no mean along f.
* The stored mixed-condition runs are what the oracle computes now.
"""

import numpy as np
import pytest

from oracle import fourier as fo
from oracle.newton import Solver
from oracle.pointlaw import lame
from oracle.staggered import StaggeredSolver
from oracle.system import System
from synth import problem_config
from synth.configs import Problem, _dyad


def _sym_field(rng, shape):
    A = rng.standard_normal((3, 3) + shape)
    return 0.5 * (A + A.transpose(1, 0, 2, 3, 4))


@pytest.mark.parametrize("shape,f", [((1, 6, 8), _dyad(1, 1)),
                                     ((3, 4, 6), _dyad(2, 2) + 0.3 * (_dyad(0, 2) + _dyad(2, 0)))])
def test_projection_with_free_mean(shape, f):
    rng = np.random.default_rng(11)
    A, B = _sym_field(rng, shape), _sym_field(rng, shape)
    GA = fo.G_tensor(A, free_mean=f)
    GB = fo.G_tensor(B, free_mean=f)
    assert np.abs(fo.G_tensor(GA, free_mean=f) - GA).max() <= 1e-12 * np.abs(GA).max()
    # self-adjoint: <G A, B> = <A, G B>
    lhs, rhs = np.sum(GA * B), np.sum(A * GB)
    assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(A * GB))
    fh = f / np.sqrt(np.sum(f * f))
    mA = A.reshape(3, 3, -1).mean(axis=-1)
    mG = GA.reshape(3, 3, -1).mean(axis=-1)
    assert np.abs(mG - (mA - fh * np.sum(fh * mA))).max() <= 1e-13
    assert abs(np.sum(fh * mG)) <= 1e-13
    # fluctuations: the same as under a prescribed mean strain
    G0 = fo.G_tensor(A)
    assert np.abs((GA - mG[:, :, None, None, None]) - G0).max() <= 1e-13


def _uniaxial_path(prob, axis, nl, iso):
    """Closed-form increments of a homogeneous uncracked cell under uniaxial
    stress along `axis` (nl lateral axes carry zero stress)."""
    s = Solver(prob)
    s.bootstrap()
    E_mod, nu, Gc = prob.phases[0]
    lam, mu = lame(E_mod, nu)
    V = float(np.prod(prob.shape))
    l, k = prob.l, prob.k
    for n in range(1, 5):
        out = s.step()
        assert out["converged"]
        a = n * prob.delta_a
        phi = np.sqrt(2 * l * a / V)
        g = (1 - phi) ** 2 + k
        H = (Gc / l) * phi / (2 * (1 - phi))
        if iso:                       # sigma = g C eps: lateral strain independent of g
            c = -lam / (nl * lam + 2 * mu)
        else:                         # positive trace and axial strain degraded, lateral not
            c = -g * lam / (nl * g * lam + 2 * mu)
        tr = 1 + nl * c
        E = np.sqrt(H / (0.5 * lam * tr * tr + mu * (1 + (nl * c * c if iso else 0.0))))
        sig_ax = g * (lam * tr + 2 * mu) * E
        assert np.allclose(s.phi, phi, rtol=1e-9)
        assert abs(out["E"] - E) <= 1e-9 * E, (out["E"], E)
        S = np.asarray(out["sigma_M"])
        assert abs(S[axis, axis] - sig_ax) <= 1e-9 * sig_ax
        lateral = [i for i in range(3) if i != axis][:nl]
        for i in lateral:
            assert abs(S[i, i]) <= 1e-10 * sig_ax
        off = S - np.diag(np.diag(S))
        assert np.abs(off).max() <= 1e-10 * sig_ax
        if nl == 1:                   # plane strain: sigma_zz from the trace part
            assert abs(S[2, 2] - g * lam * tr * E) <= 1e-9 * sig_ax
        # the mean strain: E along f, c E on the lateral axes
        m_eps = s.eps_t.reshape(s.sys.ncomp, -1).mean(axis=-1)
        for j, i in enumerate(lateral):
            assert abs(m_eps[i] - c * out["E"]) <= 1e-9 * out["E"]
        assert np.abs(s.eps_t - m_eps.reshape((-1, 1, 1, 1))).max() <= 1e-12 * out["E"]


@pytest.mark.parametrize("shape,iso", [((1, 8, 8), False), ((2, 4, 6), False), ((1, 8, 8), True)])
def test_homogeneous_uniaxial_stress_path(shape, iso):
    prob = problem_config("tiny16_m")
    prob.shape = shape
    prob.phase_id = np.zeros(shape, np.uint8)
    prob.mask = None
    prob.split = "none" if iso else "spectral"
    if shape[0] > 1:
        prob.f = np.zeros((3, 3)); prob.f[2, 2] = 1.0
    prob.delta_a = 0.2
    axis = 1 if shape[0] == 1 else 2
    _uniaxial_path(prob, axis, 1 if shape[0] == 1 else 2, iso)


def test_elastic_laminate_under_uniaxial_stress():
    n = 12
    pid = np.zeros((1, n, n), np.uint8)
    pid[..., n // 3:] = 1                      # layers normal to x (x is the last axis)
    phases = [(1.0, 0.3, 1e-3), (4.0, 0.2, 1e-3)]
    prob = Problem(name="lam", shape=(1, n, n), phases=phases, phase_id=pid, mask=None,
                   f=_dyad(1, 1), l=2.0, k=1e-6, split="none", macro_bc="mixed")
    st = StaggeredSolver(prob, dE=1e-3)
    E = 1e-3
    phi = np.zeros(prob.shape)
    eps_t, _, _ = st.mechanical(np.zeros((3,) + prob.shape), phi, E)
    sy = st.sys
    eps = eps_t + sy.fE(E)
    lam, mu = sy.lam, sy.mu
    assert np.abs(eps[0] + lam / (lam + 2 * mu) * E).max() <= 1e-10 * E
    assert np.abs(eps[1] - E).max() <= 1e-12 * E
    assert np.abs(eps[2]).max() <= 1e-10 * E
    R = sy.residual(eps_t, phi, E, np.zeros(prob.shape), 0.0)
    S = R["sigma_M"]
    M = (1 + prob.k) * np.mean(4 * mu * (lam + mu) / (lam + 2 * mu))
    assert abs(S[1, 1] - M * E) <= 1e-10 * M * E
    assert abs(S[0, 0]) <= 1e-12 * M * E and abs(S[0, 1]) <= 1e-12 * M * E


@pytest.mark.parametrize("case", ["gc16_m", "part24_m"])
def test_tangent_is_residual_derivative_mixed(case):
    prob = problem_config(case)
    sy = System(prob)
    rng = np.random.default_rng(4)
    eps_t = sy.G_mandel(rng.standard_normal((sy.ncomp,) + sy.shape) * 1e-3)
    assert np.abs(eps_t.reshape(sy.ncomp, -1).mean(axis=-1)).max() > 1e-6   # a free mean strain
    phi = np.clip(rng.uniform(0, 0.6, sy.shape) + sy.m, 0, 1)
    E = 5e-3
    Hn = sy.point(eps_t + sy.fE(E), phi, np.zeros(sy.shape))["psi_p"] * 0.8
    J = sy.tangent(eps_t, phi, E, Hn)
    d_eps = sy.G_mandel(rng.standard_normal(eps_t.shape)) * 1e-2
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
    # the equilibrium rows keep a zero-mean part orthogonal to f only
    c = sy.ncomp
    mJ = Jv[: c * sy.N].reshape(c, -1).mean(axis=-1)
    assert abs(np.dot(mJ, sy.f)) <= 1e-12 * np.abs(Jv[: c * sy.N]).max()


def test_staggered_homogeneous_uniaxial_stress():
    """Algorithm 1 under mixed conditions on a homogeneous uncracked cell: at
    every load E the converged state is uniform, with phi the root of
    phi = 2H/(Gc/l + 2H), H = E^2 (lam/2 tr^2 + mu), tr = 1 + c(g),
    c(g) = -g lam/(g lam + 2 mu), g = (1 - phi)^2 + k (plane strain, f = e_y e_y),
    found here by bisection; stagger tolerance 1e-8."""
    n = 8
    prob = Problem(name="hom_m", shape=(1, n, n), phases=[(1.0, 0.3, 1e-3)],
                   phase_id=np.zeros((1, n, n), np.uint8), mask=None, f=_dyad(1, 1), l=2.0, k=1e-6,
                   macro_bc="mixed")
    lam, mu = lame(1.0, 0.3)
    Gc, l, k = 1e-3, 2.0, 1e-6
    st = StaggeredSolver(prob, dE=4e-3)

    def resid(phi, E):
        g = (1 - phi) ** 2 + k
        c = -g * lam / (g * lam + 2 * mu)
        H = E * E * (0.5 * lam * (1 + c) ** 2 + mu)
        return phi - 2 * H / (Gc / l + 2 * H)

    for _ in range(4):
        o = st.step()
        E = o["E"]
        lo, hi = 0.0, 1.0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if resid(mid, E) > 0:
                hi = mid
            else:
                lo = mid
        phi = 0.5 * (lo + hi)
        g = (1 - phi) ** 2 + k
        c = -g * lam / (g * lam + 2 * mu)
        assert np.abs(st.phi - phi).max() <= 1e-7 * phi, (st.phi.max(), phi)
        S = o["sigma_M"]
        sig = g * (lam * (1 + c) + 2 * mu) * E
        assert abs(S[1, 1] - sig) <= 1e-7 * sig
        # zero up to the mechanical Newton tolerance (1e-9 on the strain update)
        assert abs(S[0, 0]) <= 1e-8 * sig and abs(S[0, 1]) <= 1e-8 * sig
        m = st.eps_t.reshape(3, -1).mean(axis=-1)
        assert abs(m[0] - c * E) <= 1e-7 * E


@pytest.mark.parametrize("case", ["gc16", "gc16_m", "part24_m"])
def test_uniform_shift_along_f_is_a_null_direction(case):
    """(d eps~ = f t uniform, d E = -t) leaves eps = eps~ + f E unchanged, so
    the bordered Jacobian maps it to zero under either macroscopic condition;
    E is fixed only by asking the fluctuation to carry no mean along f, which
    the oracle's Newton enforces on every step."""
    prob = problem_config(case)
    sy = System(prob)
    rng = np.random.default_rng(8)
    eps_t = sy.G_mandel(rng.standard_normal((sy.ncomp,) + sy.shape) * 1e-3)
    phi = np.clip(rng.uniform(0, 0.6, sy.shape) + sy.m, 0, 1)
    E = 5e-3
    Hn = sy.point(eps_t + sy.fE(E), phi, np.zeros(sy.shape))["psi_p"] * 0.8
    J = sy.tangent(eps_t, phi, E, Hn)
    t = 1e-3
    n = sy.pack(np.broadcast_to(sy.fE(t), eps_t.shape), np.zeros(sy.shape), -t)
    Jn = J(n)
    ref = np.abs(J(sy.pack(sy.G_mandel(rng.standard_normal(eps_t.shape)) * t, np.zeros(sy.shape), 0.0))).max()
    assert np.abs(Jn).max() <= 1e-13 * ref


def test_committed_fluctuation_has_no_mean_along_f():
    s = Solver(problem_config("tiny16_m"))
    s.bootstrap()
    for _ in range(2):
        o = s.step()
        assert o["converged"]
        m = s.eps_t.reshape(s.sys.ncomp, -1).mean(axis=-1)
        assert abs(np.dot(m, s.sys.f)) <= 1e-15 * np.abs(s.eps_t).max()
        assert np.abs(m).max() > 1e-6 * o["E"]          # the free mean off f is there


@pytest.mark.parametrize("case", ["tiny16_m", "gc16_m"])
def test_stored_runs_are_what_the_oracle_computes(case):
    """tests/golden/oracle_<case>.json (used by the GPU tests) is what the
    oracle computes now, increment by increment (1e-9 relative: both stop on
    a Newton update below 1e-8)."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", f"oracle_{case}.json")) as fh:
        g = json.load(fh)
    s = Solver(problem_config(case))
    boot = s.bootstrap()
    assert abs(boot["a0"] - g["a0"]) <= 1e-12 * abs(g["a0"])
    for ref in g["increments"][:2]:
        o = s.step()
        assert o["converged"]
        assert abs(o["E"] - ref["E"]) <= 1e-9 * abs(ref["E"]), (o["E"], ref["E"])
        assert abs(o["Gamma"] - ref["Gamma"]) <= 1e-9 * abs(ref["Gamma"])
        sm = np.asarray(o["sigma_M"])
        sv = np.array([sm[0, 0], sm[1, 1], sm[2, 2], sm[1, 2], sm[0, 2], sm[0, 1]])
        assert np.abs(sv - np.asarray(ref["sigma_M"])).max() <= 1e-9 * np.abs(ref["sigma_M"]).max()
