"""Pins of the oracle's point law (paper Sec. 2.1 eq. `PlusNegPsi`, `gFunct`;
Sec. 2.3 eq. `C_Calc`; eq. `history`, `Delta_history`).

Checks: degree-1 homogeneity (Euler identity C:eps = sigma), the tangent
against central differences of the stress, the stresses against central
differences of the energies, energy additivity psi+ + psi- = eps:C0:eps/2,
symmetry of C, and special cases that reduce to linear elasticity.
"""

import numpy as np
import pytest

from oracle import pointlaw as pl


def rand_sym(rng, n, scale=1e-2, plane=False):
    A = rng.standard_normal((n, 3, 3)) * scale
    A = 0.5 * (A + np.swapaxes(A, 1, 2))
    if plane:
        A[:, 2, :] = 0.0
        A[:, :, 2] = 0.0
    return np.moveaxis(A, 0, -1)                        # (3, 3, n)


def material(rng, n):
    E = rng.uniform(0.5, 10.0, n)
    nu = rng.uniform(0.1, 0.4, n)
    return pl.lame(E, nu)


def ev(eps, phi, Hn, lam, mu, k=1e-6, iso=False):
    return pl.evaluate(eps, phi, Hn, lam, mu, k, iso=iso)


@pytest.mark.parametrize("iso", [False, True])
@pytest.mark.parametrize("plane", [False, True])
def test_euler_identity(plane, iso):
    rng = np.random.default_rng(0)
    n = 500
    eps = rand_sym(rng, n, plane=plane)
    lam, mu = material(rng, n)
    phi = rng.uniform(0, 1, n)
    st = ev(eps, phi, np.zeros(n), lam, mu, iso=iso)
    Ce = pl.tangent_apply(st, eps)
    assert np.allclose(Ce, st["sigma"], atol=1e-15, rtol=1e-12)


@pytest.mark.parametrize("iso", [False, True])
@pytest.mark.parametrize("plane", [False, True])
def test_tangent_against_stress_differences(plane, iso):
    rng = np.random.default_rng(1)
    n = 400
    eps = rand_sym(rng, n, plane=plane)
    w = rand_sym(rng, n, plane=plane)
    lam, mu = material(rng, n)
    phi = rng.uniform(0, 1, n)
    st = ev(eps, phi, np.zeros(n), lam, mu, iso=iso)
    h = 1e-7
    sp = ev(eps + h * w, phi, np.zeros(n), lam, mu, iso=iso)["sigma"]
    sm = ev(eps - h * w, phi, np.zeros(n), lam, mu, iso=iso)["sigma"]
    fd = (sp - sm) / (2 * h)
    Cw = pl.tangent_apply(st, w)
    err = np.abs(fd - Cw).max(axis=(0, 1)) / np.abs(Cw).max(axis=(0, 1))
    # a handful of voxels may straddle a kink of the split within +-h
    assert np.mean(err < 1e-6) > 0.99


def test_stresses_are_energy_gradients():
    rng = np.random.default_rng(2)
    n = 300
    eps = rand_sym(rng, n)
    lam, mu = material(rng, n)
    st = ev(eps, np.zeros(n), np.zeros(n), lam, mu)
    h = 1e-7
    for (i, j) in [(0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (0, 2)]:
        d = np.zeros((3, 3, 1)); d[i, j] = d[j, i] = 1.0
        p = ev(eps + h * d, np.zeros(n), np.zeros(n), lam, mu)
        m = ev(eps - h * d, np.zeros(n), np.zeros(n), lam, mu)
        mult = 1.0 if i == j else 2.0
        for key, skey in (("psi_p", "sigma0p"), ("psi_m", "sigma0m")):
            fd = (p[key] - m[key]) / (2 * h)
            an = mult * st[skey][i, j]
            ok = np.abs(fd - an) <= 1e-6 * (np.abs(an) + 1e-6)
            assert np.mean(ok) > 0.99


def test_energy_split_adds_up():
    rng = np.random.default_rng(3)
    n = 300
    eps = rand_sym(rng, n)
    lam, mu = material(rng, n)
    st = ev(eps, np.zeros(n), np.zeros(n), lam, mu)
    tr = np.trace(eps)
    full = 0.5 * lam * tr ** 2 + mu * np.einsum("ij...,ij...->...", eps, eps)
    assert np.allclose(st["psi_p"] + st["psi_m"], full, rtol=1e-13, atol=1e-20)


def test_tangent_symmetric():
    rng = np.random.default_rng(4)
    n = 300
    eps = rand_sym(rng, n)
    lam, mu = material(rng, n)
    st = ev(eps, rng.uniform(0, 1, n), np.zeros(n), lam, mu)
    a, b = rand_sym(rng, n), rand_sym(rng, n)
    ab = np.einsum("ij...,ij...->...", a, pl.tangent_apply(st, b))
    ba = np.einsum("ij...,ij...->...", b, pl.tangent_apply(st, a))
    assert np.allclose(ab, ba, rtol=1e-12, atol=1e-20)


def test_undamaged_is_linear_elastic():
    """phi = 0, k = 0: g = 1, C = C0 and sigma = C0:eps whatever the split."""
    rng = np.random.default_rng(5)
    n = 200
    eps = rand_sym(rng, n)
    lam, mu = material(rng, n)
    st = ev(eps, np.zeros(n), np.zeros(n), lam, mu, k=0.0)
    tr = np.trace(eps)
    ref = lam * tr * np.eye(3)[:, :, None] + 2 * mu * eps
    assert np.allclose(st["sigma"], ref, rtol=1e-12, atol=1e-18)
    w = rand_sym(rng, n)
    refw = lam * np.trace(w) * np.eye(3)[:, :, None] + 2 * mu * w
    assert np.allclose(pl.tangent_apply(st, w), refw, rtol=1e-12, atol=1e-18)


def test_all_tensile_and_all_compressive():
    lam, mu = pl.lame(np.array([2.0, 2.0]), np.array([0.3, 0.3]))
    eps = np.zeros((3, 3, 2))
    eps[:, :, 0] = np.diag([1e-2, 2e-2, 3e-2])
    eps[:, :, 1] = -np.diag([1e-2, 2e-2, 3e-2])
    phi = np.array([0.5, 0.5])
    st = ev(eps, phi, np.zeros(2), lam, mu, k=0.0)
    g = 0.25
    s0 = lam[0] * 6e-2 * np.eye(3) + 2 * mu[0] * eps[:, :, 0]
    assert np.allclose(st["sigma"][:, :, 0], g * s0, rtol=1e-13)
    assert np.allclose(st["sigma"][:, :, 1], -s0, rtol=1e-13)
    assert st["psi_m"][0] == 0.0 and st["psi_p"][1] == 0.0


def test_repeated_eigenvalues_tangent():
    """eps = diag(a, a, b) with a > 0 > b: theta must stay finite and the
    tangent must match the stress difference quotient."""
    lam, mu = pl.lame(np.array([1.0]), np.array([0.3]))
    eps = np.diag([1e-2, 1e-2, -1.5e-2])[:, :, None]        # tr > 0: off the volumetric kink
    phi = np.array([0.3])
    st = ev(eps, phi, np.zeros(1), lam, mu)
    rng = np.random.default_rng(6)
    w = rand_sym(rng, 1)
    h = 1e-8
    fd = (ev(eps + h * w, phi, np.zeros(1), lam, mu)["sigma"]
          - ev(eps - h * w, phi, np.zeros(1), lam, mu)["sigma"]) / (2 * h)
    assert np.all(np.isfinite(st["theta"]))
    assert np.allclose(pl.tangent_apply(st, w), fd, rtol=1e-6, atol=1e-12)


def test_history_flag():
    lam, mu = pl.lame(np.array([1.0, 1.0, 1.0]), np.array([0.3, 0.3, 0.3]))
    eps = np.zeros((3, 3, 3))
    for v in range(3):
        eps[1, 1, v] = 1e-2
    st0 = ev(eps, np.zeros(3), np.zeros(3), lam, mu)
    psi = st0["psi_p"][0]
    Hn = np.array([0.5 * psi, psi, 2 * psi])
    st = ev(eps, np.zeros(3), Hn, lam, mu)
    assert list(st["chi"]) == [1.0, 1.0, 0.0]        # ties count as loading
    assert np.allclose(st["H"], [psi, psi, 2 * psi])


def test_isotropic_variant_is_degraded_linear_elasticity():
    """No split: sigma = g (lambda tr eps I + 2 mu eps) for any strain, and
    the driving energy is the whole psi0 = eps : C0 : eps / 2, also in
    compression, where the split model has no driving energy."""
    rng = np.random.default_rng(7)
    n = 300
    eps = rand_sym(rng, n)
    lam, mu = material(rng, n)
    phi = rng.uniform(0, 1, n)
    st = ev(eps, phi, np.zeros(n), lam, mu, iso=True)
    g = (1 - phi) ** 2 + 1e-6
    tr = np.einsum("ii...->...", eps)
    s0 = lam * tr * np.eye(3)[:, :, None] + 2 * mu * eps
    assert np.allclose(st["sigma"], g * s0, rtol=1e-12, atol=1e-17)
    psi0 = 0.5 * np.einsum("ij...,ij...->...", s0, eps)
    assert np.allclose(st["psi_p"], psi0, rtol=1e-12, atol=1e-20)
    comp = -np.abs(rand_sym(rng, 1))[:, :, 0]
    comp = np.diag(np.diag(comp))[:, :, None]                # all eigenvalues negative
    l1, m1 = np.array([1.0]), np.array([0.7])
    assert ev(comp, np.zeros(1), np.zeros(1), l1, m1)["psi_p"][0] == 0.0
    assert ev(comp, np.zeros(1), np.zeros(1), l1, m1, iso=True)["psi_p"][0] > 0.0
