"""Pins of the oracle's projection and Laplacian (paper Sec. 3.1, eq. `GFourier`
with Willot's rotated frequencies; eq. `LinearOpe_Helm`).

The compatible and equilibrated test fields are built in REAL space from the
rotated finite differences themselves (forward differences averaged over the
voxel faces), not from the oracle's Fourier symbols, so a wrong sign, axis or
half-angle in the oracle fails these tests.
"""

import numpy as np
import pytest

from oracle import fourier as fo

SHAPES = [(1, 16, 16), (1, 12, 18), (1, 15, 9), (6, 8, 10), (5, 7, 9), (8, 8, 8)]


def rot_diff(u, axis_xyz):
    """Rotated-scheme derivative of a scalar field u[z, y, x] along x/y/z:
    forward difference along the axis, averaged over the other axes' two
    neighbouring voxel layers (value at voxel corners)."""
    ax = {0: 2, 1: 1, 2: 0}[axis_xyz]
    d = np.roll(u, -1, axis=ax) - u
    for other in (0, 1, 2):
        if other == ax or u.shape[other] == 1:
            continue
        d = 0.5 * (d + np.roll(d, -1, axis=other))
    return d


def random_compatible(shape, rng):
    dim = 2 if shape[0] == 1 else 3
    u = [rng.standard_normal(shape) for _ in range(3)]
    eps = np.zeros((3, 3) + shape)
    for i in range(dim):
        for j in range(dim):
            eps[i, j] += 0.5 * rot_diff(u[i], j) + 0.5 * rot_diff(u[j], i)
    return eps


@pytest.mark.parametrize("scheme", ["rotated", "standard"])
@pytest.mark.parametrize("shape", SHAPES)
def test_projection_idempotent_symmetric(shape, scheme):
    n, zero = fo.direction(shape, scheme)
    c = 3 if shape[0] == 1 else 6
    basis = np.eye(c)
    cols = []
    for k in range(c):
        e = basis[k].reshape((c,) + (1,) * 3) * np.ones((c,) + shape)
        cols.append(fo.to_mandel(fo.project_hat(fo.to_tensor(e), n, zero), c))
    P = np.stack(cols, axis=1)                     # (c, c, nz, ny, nx)
    P = np.moveaxis(P, (0, 1), (-2, -1))
    assert np.allclose(P @ P, P, atol=1e-13)
    assert np.allclose(P, np.swapaxes(P, -1, -2), atol=1e-14)
    assert np.all(P[zero] == 0.0)
    # rank of the projector = space dimension where r != 0
    dim = 2 if shape[0] == 1 else 3
    tr = np.trace(P, axis1=-2, axis2=-1)
    assert np.allclose(tr[~zero], dim)


@pytest.mark.parametrize("shape", SHAPES)
def test_compatible_fields_preserved(shape):
    rng = np.random.default_rng(1)
    eps = random_compatible(shape, rng)
    out = fo.G_tensor(eps)
    scale = np.abs(eps).max()
    # (I - G) annihilates compatible fields, G keeps them
    assert np.abs(out - eps).max() <= 1e-12 * scale


@pytest.mark.parametrize("shape", SHAPES)
def test_equilibrated_fields_annihilated(shape):
    """Airy-type stress from rotated differences: divergence-free, so G = 0."""
    rng = np.random.default_rng(2)
    psi = rng.standard_normal(shape)
    D = rot_diff
    sig = np.zeros((3, 3) + shape)
    sig[0, 0] = D(D(psi, 1), 1)
    sig[1, 1] = D(D(psi, 0), 0)
    sig[0, 1] = sig[1, 0] = -D(D(psi, 0), 1)
    out = fo.G_tensor(sig)
    assert np.abs(out).max() <= 1e-12 * np.abs(sig).max()


def test_constant_annihilated():
    shape = (4, 6, 8)
    A = np.zeros((3, 3) + shape)
    A[0, 0] = 2.0
    A[1, 2] = A[2, 1] = -0.5
    assert np.abs(fo.G_tensor(A)).max() < 1e-15


def test_projection_matches_brute_force_lstsq():
    """Per-mode orthogonal projection onto sym(n (x) u): the oracle's closed
    form against a least-squares solve on the 6 Mandel components."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        nvec = rng.standard_normal(3)
        nvec /= np.linalg.norm(nvec)
        A = rng.standard_normal((3, 3)); A = A + A.T
        # basis of sym(n (x) u): columns for u = e_0, e_1, e_2
        B = np.stack([fo.to_mandel((np.outer(nvec, e) + np.outer(e, nvec))[:, :, None] / 2, 6)[:, 0]
                      for e in np.eye(3)], axis=1)
        a = fo.to_mandel(A[:, :, None], 6)[:, 0]
        coef, *_ = np.linalg.lstsq(B, a, rcond=None)
        ref = B @ coef
        got = fo.project_hat(A[:, :, None], nvec[:, None], np.array([False]))
        assert np.allclose(fo.to_mandel(got, 6)[:, 0], ref, atol=1e-13)


@pytest.mark.parametrize("N", [8, 9, 16])
def test_laplacian_of_cosine_modes(N):
    x = np.arange(N)
    for m in range(N // 2 + 1):
        q = 2 * np.pi * m / N
        u = np.cos(q * x)[None, None, :] * np.ones((1, 3, N))
        lap = fo.laplacian(u)
        assert np.allclose(lap, -q * q * u, atol=1e-12)
    # a mode along y and z too
    shape = (4, 6, N)
    z, y, xx = np.meshgrid(np.arange(4), np.arange(6), x, indexing="ij")
    u = np.sin(2 * np.pi * (z / 4 + 2 * y / 6 + xx / N))
    q2 = (2 * np.pi / 4) ** 2 + (4 * np.pi / 6) ** 2 + (2 * np.pi / N) ** 2
    assert np.allclose(fo.laplacian(u), -q2 * u, atol=1e-11)
    assert shape == u.shape


def test_nyquist_rotated_zero_modes():
    n, zero = fo.rotated_direction((1, 8, 8))
    # q = 0 and the (pi, pi) corner have r == 0; single-axis Nyquist does not
    assert zero[0, 0, 0] and zero[0, 4, 4]
    assert not zero[0, 0, 4] and not zero[0, 4, 0]
    assert np.allclose(np.abs(n[:, 0, 0, 4]), [1, 0, 0])


# ---- standard-frequency projection (eq. GFourier without the rotated scheme) ----

def plane_waves(shape, rng, nwave=4):
    """Random sums of plane waves below the Nyquist index, with their exact
    real-space derivatives (closed form, no FFT): returns (value, grad,
    hessian) callables over the voxel grid."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    pos = (x, y, z)
    waves = []
    for _ in range(nwave):
        k = [int(rng.integers(-((n - 1) // 2), (n - 1) // 2 + 1)) if n > 2 else 0 for n in (nx, ny, nz)]
        q = np.array([2 * np.pi * k[0] / nx, 2 * np.pi * k[1] / ny, 2 * np.pi * k[2] / nz])
        waves.append((q, rng.standard_normal(), rng.uniform(0, 2 * np.pi)))

    def phase(q, th):
        return q[0] * pos[0] + q[1] * pos[1] + q[2] * pos[2] + th

    def val():
        return sum(a * np.cos(phase(q, th)) for q, a, th in waves)

    def grad(i):
        return sum(-a * q[i] * np.sin(phase(q, th)) for q, a, th in waves)

    def hess(i, j):
        return sum(-a * q[i] * q[j] * np.cos(phase(q, th)) for q, a, th in waves)

    return val, grad, hess


@pytest.mark.parametrize("shape", [(1, 16, 16), (1, 12, 18), (1, 15, 9), (6, 8, 10), (5, 7, 9)])
def test_standard_projection_keeps_exact_symmetric_gradients(shape):
    rng = np.random.default_rng(11)
    dim = 2 if shape[0] == 1 else 3
    us = [plane_waves(shape, rng) for _ in range(3)]
    eps = np.zeros((3, 3) + shape)
    for i in range(dim):
        for j in range(dim):
            eps[i, j] = 0.5 * (us[i][1](j) + us[j][1](i))
    out = fo.G_tensor(eps, "standard")
    assert np.abs(out - eps).max() <= 1e-12 * np.abs(eps).max()
    # the rotated scheme does not keep them: the two schemes differ
    assert np.abs(fo.G_tensor(eps, "rotated") - eps).max() > 1e-3 * np.abs(eps).max()


@pytest.mark.parametrize("shape", [(1, 16, 16), (1, 15, 9), (6, 8, 10)])
def test_standard_projection_annihilates_exact_airy_stress(shape):
    rng = np.random.default_rng(12)
    _, _, H = plane_waves(shape, rng)
    sig = np.zeros((3, 3) + shape)
    sig[0, 0] = H(1, 1)
    sig[1, 1] = H(0, 0)
    sig[0, 1] = sig[1, 0] = -H(0, 1)
    assert np.abs(fo.G_tensor(sig, "standard")).max() <= 1e-12 * np.abs(sig).max()


def test_standard_projection_of_real_field_with_nyquist_content_is_real():
    """Reading: xi_j = 0 at an even axis' Nyquist index keeps the projected
    field real (either signed frequency there would not)."""
    rng = np.random.default_rng(13)
    shape = (4, 6, 8)
    A = rng.standard_normal((3, 3) + shape)
    A = 0.5 * (A + np.swapaxes(A, 0, 1))
    n, zero = fo.direction(shape, "standard")
    out = fo.ifftn(fo.project_hat(fo.fftn(A), n, zero))
    assert np.abs(out.imag).max() <= 1e-14 * np.abs(A).max()
    # modes whose non-zero indices are all Nyquist indices have xi = 0 and
    # are projected to 0, like the DC mode
    assert zero[0, 0, 4] and zero[2, 3, 4] and not zero[0, 1, 4]


def test_fft_bits_do_not_depend_on_the_thread_count(monkeypatch):
    """The library FFT splits independent lines over its threads, so the
    oracle's transforms and projection give the same bits for any
    FFT_WORKERS (the full-size goldens are written with several threads,
    the small ones with one)."""
    rng = np.random.default_rng(7)
    a = rng.standard_normal((3, 3, 6, 10, 12)) + 1j * rng.standard_normal((3, 3, 6, 10, 12))
    A = rng.standard_normal((3, 3, 6, 10, 12))
    A = A + A.transpose(1, 0, 2, 3, 4)
    monkeypatch.setattr(fo, "FFT_WORKERS", 1)
    f1, i1, g1 = fo.fftn(a), fo.ifftn(a), fo.G_tensor(A)
    monkeypatch.setattr(fo, "FFT_WORKERS", 4)
    f4, i4, g4 = fo.fftn(a), fo.ifftn(a), fo.G_tensor(A)
    assert np.array_equal(f1, f4) and np.array_equal(i1, i4) and np.array_equal(g1, g4)
