"""Pins of the oracle's residual and tangent (paper Sec. 3.2, eqs.
`System_CrackLength`, `newGammaFourier`, `CrackLength_linearization`,
`Delta_history`).

The tangent action must equal the central difference of the residual
(a dropped or sign-flipped term of dF fails this), the constraint row must
be the gradient of Gamma, Gamma must equal the real-space sum of eq.
`CrackLenght` for band-limited fields, and the laminate solution must be the
closed-form piecewise-constant one.
"""

import numpy as np
import pytest

from oracle import fourier as fo
from oracle import krylov
from oracle.system import System
from synth import problem_config, random_state, random_vector
from synth.microstructure import laminate_x


def _state(sys, seed):
    eps, phi, Hn, E = random_state(sys.shape, sys.ncomp, seed, f_mandel=sys.f, E=0.01)
    eps_t = eps - sys.fE(E)
    eps_t = fo.G_mandel(eps_t)                  # a compatible fluctuation
    # keep the history away from the tie so the residual is smooth at the state
    st = sys.point(eps_t + sys.fE(E), phi, np.zeros(sys.shape))
    rng = np.random.default_rng(seed)
    Hn = st["psi_p"] * np.where(rng.uniform(size=sys.shape) < 0.5, 0.5, 1.5)
    if np.any(sys.m):
        phi = np.where(sys.m > 0, 1.0, phi)
    return eps_t, phi, E, Hn


@pytest.mark.parametrize("name,split", [("tiny16", "spectral"), ("fib64", "spectral"),
                                        ("pore24", "spectral"), ("part24", "spectral"),
                                        ("tiny16", "none"), ("part24", "none"),
                                        ("tiny16_std", "spectral"), ("part24_std", "spectral")])
def test_tangent_is_residual_derivative(name, split):
    prob = problem_config(name)
    prob.split = split
    if name == "fib64":
        prob.shape = (1, 32, 32)
        prob.phase_id = prob.phase_id[:, :32, :32]
        prob.mask = prob.mask[:, 16:48, 16:48]
    sys = System(prob)
    eps_t, phi, E, Hn = _state(sys, 7)
    a = 3.0
    J = sys.tangent(eps_t, phi, E, Hn)
    n = sys.N * (sys.ncomp + 1) + 1
    v = random_vector(n, 8)
    d_eps, d_phi, dE = sys.unpack(v)
    d_eps = fo.G_mandel(d_eps) * 1e-2
    d_phi = d_phi * 1e-2 * (1 - sys.m)
    dE = 1e-3
    v = sys.pack(d_eps, d_phi, dE)
    Jv = J(v)
    h = 1e-6

    def F(s):
        R = sys.residual(eps_t + s * d_eps, phi + s * d_phi, E + s * dE, Hn, a)
        return sys.pack(R["F1"], R["F2"], R["F3"])

    fd = (F(h) - F(-h)) / (2 * h)
    c, N = sys.ncomp, sys.N
    for blk in (slice(0, c * N), slice(c * N, (c + 1) * N), slice(-1, None)):
        ref = np.abs(fd[blk]).max()
        assert np.abs(Jv[blk] - fd[blk]).max() <= 2e-5 * ref


def test_constraint_row_is_gamma_gradient():
    sys = System(problem_config("tiny16"))
    rng = np.random.default_rng(3)
    phi = rng.uniform(0, 1, sys.shape)
    r = phi / sys.l - sys.l * fo.laplacian(phi)
    d = rng.standard_normal(sys.shape)
    h = 1e-6
    fd = (sys.gamma(phi + h * d) - sys.gamma(phi - h * d)) / (2 * h)
    assert abs(fd - np.sum(r * d)) <= 1e-8 * abs(fd)


def test_gamma_equals_real_space_sum_for_band_limited_field():
    """For a field with no Nyquist content the spectral gradient is exact, so
    Gamma = sum phi^2/(2l) + (l/2)|grad phi|^2 with the analytic gradient."""
    prob = problem_config("tiny16")
    prob.shape = (1, 16, 20)
    prob.phase_id = np.zeros(prob.shape, np.uint8)
    prob.mask = None
    sys = System(prob)
    y, x = np.meshgrid(np.arange(16), np.arange(20), indexing="ij")
    kx, ky = 2 * np.pi * 3 / 20, 2 * np.pi * 2 / 16
    phi = (0.3 + 0.2 * np.cos(kx * x + 0.4) + 0.1 * np.sin(ky * y - kx * x))[None]
    gx = (-0.2 * kx * np.sin(kx * x + 0.4) - 0.1 * kx * np.cos(ky * y - kx * x))[None]
    gy = (0.1 * ky * np.cos(ky * y - kx * x))[None]
    l = sys.l
    ref = np.sum(phi ** 2 / (2 * l) + 0.5 * l * (gx ** 2 + gy ** 2))
    assert abs(sys.gamma(phi) - ref) <= 1e-12 * ref


def test_homogeneous_uniform_state_is_equilibrated():
    """Homogeneous RVE, uniform damage: eps_tilde = 0 satisfies F1 = 0."""
    prob = problem_config("tiny16")
    prob.mask = None
    sys = System(prob)
    phi = 0.2 * np.ones(sys.shape)
    R = sys.residual(np.zeros((3,) + sys.shape), phi, 0.01, np.zeros(sys.shape), 1.0)
    assert np.abs(R["F1"]).max() < 1e-16
    s = R["state"]["sigma"]
    assert np.allclose(s, s[:, :, :1, :1, :1], rtol=1e-14)


def _laminate_closed_form(phases, frac, E):
    """Plane-strain laminate normal to x under E_M = E e_y (x) e_y:
    eps_yy = E everywhere, sigma_xx uniform, sigma_xy = 0, <eps_xx> = 0."""
    from oracle.pointlaw import lame
    lm = [lame(p[0], p[1]) for p in phases]
    num = sum(f * l / (l + 2 * m) for f, (l, m) in zip(frac, lm))
    den = sum(f / (l + 2 * m) for f, (l, m) in zip(frac, lm))
    S = E * num / den
    exx = [(S - l * E) / (l + 2 * m) for (l, m) in lm]
    return S, exx


@pytest.mark.parametrize("shape,scheme", [((1, 8, 24), "rotated"), ((1, 6, 21), "rotated"),
                                          ((1, 6, 21), "standard")])
def test_laminate_closed_form(shape, scheme):
    """Exact laminate solution.  With standard frequencies only on an odd grid:
    on an even one the Nyquist mode of the strain step is outside the range
    of the projection (xi = 0 there)."""
    prob = problem_config("tiny16")
    prob.projection = scheme
    prob.shape = shape
    prob.phases = [(1.0, 0.3, 1e-3), (5.0, 0.2, 1e-3)]
    prob.phase_id = laminate_x(shape[2], shape[1], shape[0], width=7, period=shape[2])
    prob.mask = None
    prob.k = 0.0
    sys = System(prob)
    E = 0.01
    phi = np.zeros(shape)
    J = sys.tangent(np.zeros((3,) + shape), phi, E, np.zeros(shape))
    R = sys.residual(np.zeros((3,) + shape), phi, E, np.zeros(shape), 1.0)
    c, N = 3, sys.N

    def mech(x):
        v = np.concatenate([x, np.zeros(N + 1)])
        return J(v)[: c * N]

    x, info = krylov.bicgstab(mech, -R["F1"].ravel(), rtol=1e-14, maxit=500)
    eps = x.reshape((c,) + shape) + sys.fE(E)
    frac = [np.mean(prob.phase_id == 0), np.mean(prob.phase_id == 1)]
    S, exx = _laminate_closed_form(prob.phases, frac, E)
    pid = prob.phase_id
    ref = np.where(pid == 0, exx[0], exx[1])
    assert np.allclose(eps[0], ref, rtol=1e-10, atol=1e-14)
    assert np.allclose(eps[1], E, rtol=1e-10)
    assert np.abs(eps[2]).max() < 1e-14
    st = sys.point(eps, phi, np.zeros(shape))
    assert np.allclose(st["sigma"][0, 0], S, rtol=1e-10)
