"""Closed-form pins of the oracle.

* Straight crack spanning the cell (paper Sec. 2.1 eq. `CrackLenght`, the
  Gamma-convergence statement): the masked damage-free Helmholtz solution is
  the discrete Green's function of (1/l - l Lap) normalised to 1 on the crack
  row, and Gamma / crack length = 1 / (2 G(0)); it tends to tanh(L/(2l)), the
  continuous periodic value, as l/h grows, with a leading O(h/l) excess
  2/(pi^2 l/h) from the frequencies the grid cannot hold.  G is summed directly as a cosine
  series here, with no FFT and no Krylov solver.
* Appendix A.1: the Fourier amplification factor of the sampled crack profile
  and the paper's least-squares coefficient a = 0.298 (golden fixture).
* Homogeneous diffuse damage (Sec. 2.3 eq. `SystemDis`, Sec. 3.1 eq.
  `Helm2`, eq. `CrackLenght`): one phase, no crack, uniaxial f; the uniform
  solution of every increment is known in closed form:
  phi = sqrt(2 l a / V), H = (Gc/l) phi / (2 (1 - phi)),
  E = sqrt(2 H / (lambda + 2 mu)), Sigma = g (lambda, lambda + 2 mu, lambda) E.
"""

import json
import os

import numpy as np
import pytest

from oracle import appendix
from oracle.newton import Solver
from oracle.pointlaw import lame
from synth import problem_config
from synth.microstructure import line_crack_mask

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def green_direct(N, l):
    """G(y) = (1/N) sum_m cos(q_m y) / (1/l + l q_m^2), q_m = 2 pi m / N."""
    m = np.arange(N)
    q = 2 * np.pi * np.where(m <= N // 2, m, m - N) / N
    y = np.arange(N)
    return np.array([np.sum(np.cos(q * yy) / (1 / l + l * q * q)) for yy in y]) / N


@pytest.mark.parametrize("N,nx,l", [(64, 8, 2.0), (65, 5, 2.0), (32, 6, 1.5), (48, 4, 2.5)])
def test_straight_crack_spanning_cell(N, nx, l):
    prob = problem_config("tiny16")
    prob.shape = (1, N, nx)
    prob.phase_id = np.zeros(prob.shape, np.uint8)
    y0 = N // 3
    prob.mask = line_crack_mask(nx, N, y0, 0, nx)
    prob.l = l
    s = Solver(prob)
    phi0, _ = s.initial_damage()
    G = green_direct(N, l)
    ref = np.roll(G / G[0], y0)[None, :, None] * np.ones(prob.shape)
    assert np.abs(phi0 - ref).max() < 1e-10
    gam = s.sys.gamma(phi0)
    assert abs(gam / nx - 1.0 / (2.0 * G[0])) < 1e-10


def test_straight_crack_known_values_and_limit():
    # Gamma per unit crack length: 1.1117 at l = 2h, 1.0877 at 2.5h, 1.1536 at 1.5h
    for N, l, val in [(64, 2.0, 1.1117), (256, 2.0, 1.1117), (64, 2.5, 1.0877), (64, 1.5, 1.1536)]:
        assert abs(1.0 / (2.0 * green_direct(N, l)[0]) - val) < 1e-4
    prob = problem_config("tiny16")
    N, nx, l = 128, 4, 16.0
    prob.shape = (1, N, nx)
    prob.phase_id = np.zeros(prob.shape, np.uint8)
    prob.mask = line_crack_mask(nx, N, 5, 0, nx)
    prob.l = l
    s = Solver(prob)
    phi0, _ = s.initial_damage()
    ratio = s.sys.gamma(phi0) / nx
    # continuum value tanh(L/(2l)) plus the truncated Fourier tail of the
    # Green's function, 2/(pi^2 (l/h)) to leading order
    assert abs((ratio - np.tanh(N / (2 * l))) * l - 2.0 / np.pi ** 2) < 5e-3


def test_appendix_amplification_factor_and_fit():
    with open(os.path.join(GOLDEN, "appendix_fit.json")) as fh:
        gold = json.load(fh)
    a, A = appendix.fit_a(np.linspace(1.0, 8.0, 29), N=gold["profile_N"])
    assert abs(a - gold["a_fft"]) < 2e-3
    assert a < gold["a_fem_bourdin"]
    # monotone decrease towards 1 as l/h grows
    vals = [appendix.amplification(v) for v in (1, 1.5, 2, 3, 4, 8)]
    assert all(x > y for x, y in zip(vals, vals[1:])) and vals[-1] > 1.0
    assert abs(vals[0] - 1.3005) < 1e-4 and abs(vals[2] - 1.1484) < 1e-4


def test_appendix_profile_exponent_reading():
    """The printed exponent |x|/(2l) gives Gamma = 1.25 per unit length in the
    continuum; exp(-|x|/l) gives exactly 1 (large-l sampled limit)."""
    N, l = 4097, 64.0
    assert abs(appendix.gamma_fourier(appendix.profile(N, l), l) - 1.0) < 5e-3
    assert abs(appendix.gamma_fourier(appendix.profile(N, 2 * l), l) - 1.25) < 5e-3


@pytest.mark.parametrize("shape", [(1, 8, 8), (2, 4, 6)])
def test_homogeneous_diffuse_damage_path(shape):
    prob = problem_config("tiny16")
    prob.shape = shape
    prob.phase_id = np.zeros(shape, np.uint8)
    prob.mask = None
    E_mod, nu, Gc = prob.phases[0]
    if shape[0] > 1:
        prob.f = np.zeros((3, 3)); prob.f[2, 2] = 1.0
    prob.delta_a = 0.2
    s = Solver(prob)
    s.bootstrap()
    lam, mu = lame(E_mod, nu)
    V = float(np.prod(shape))
    l, k = prob.l, prob.k
    axis = 1 if shape[0] == 1 else 2
    for n in range(1, 5):
        out = s.step()
        assert out["converged"]
        a = n * prob.delta_a
        phi = np.sqrt(2 * l * a / V)
        H = (Gc / l) * phi / (2 * (1 - phi))
        E = np.sqrt(2 * H / (lam + 2 * mu))
        g = (1 - phi) ** 2 + k
        sig = g * lam * E * np.ones(3)
        sig[axis] = g * (lam + 2 * mu) * E
        assert np.allclose(s.phi, phi, rtol=1e-9)
        assert abs(out["E"] - E) <= 1e-9 * E
        assert np.allclose(np.diag(out["sigma_M"]), sig, rtol=1e-9)
        assert np.abs(s.eps_t).max() < 1e-14
        assert np.allclose(s.Hn, H, rtol=1e-9)
