"""Discrete Fourier calculus on the periodic voxel grid (oracle).

Paper Sec. 3.1: fields are trigonometric polynomials on an nx*ny*nz grid; the
equilibrium residual uses the compatibility projection G (eq. `GFourier`)
built with Willot's rotated finite-difference frequencies, while the
Helmholtz/Laplacian terms use the standard frequencies (eq.
`LinearOpe_Helm`).

Readings taken here (the paper leaves them open):
* The projection is the orthogonal projection of a symmetric tensor onto the
  symmetric compatible fields sym(n (x) u):
      P(A) = (A n) (x) n + n (x) (A n) - (n . A n) n (x) n,
  which has the same kernel as the paper's G on symmetric stresses
  (both vanish iff A n = 0) and therefore gives the same Newton roots.
* Rotated frequencies: the rotated difference at voxel corners has symbol
  proportional to r_j = sin(q_j/2) prod_{m != j} cos(q_m/2); the common
  complex factor cancels in P, so n = r/|r|, and P = 0 where r = 0
  (q = 0 and modes with two or more Nyquist axes).  At an even axis' Nyquist
  index cos(q/2) is taken as exactly 0.
* Laplacian symbol -|q|^2 with q_j = 2 pi m_j / N_j and the Nyquist mode kept.
* Standard-frequency projection (the paper's eq. `GFourier` without the
  rotated scheme, `scheme="standard"`): n = xi/|xi| with xi_j = q_j, except
  that an even axis' Nyquist index contributes xi_j = 0.  The sign of the
  Nyquist frequency is undefined (m = N/2 and -N/2 alias), and taking either
  one would make the projected field complex; with xi_j = 0 the symbol is
  even in every m_j and the projection maps real fields to real fields.
* Mixed macroscopic conditions (Sec. 2.3 names them as the alternative to
  the prescribed macroscopic strain f E, done in FFT by stress control at
  the zero frequency): only the component of the mean strain along f is
  prescribed, and the mean stress must vanish on every direction Frobenius-
  orthogonal to f, so Sigma_M = s f.  In the Galerkin form this is the
  projection with G(0) = P_f^perp (A -> A - fh (fh : A), fh = f/|f|) instead
  of 0; the strain fluctuation then carries the free mean strain along
  P_f^perp, and the residual G[sigma] = 0 holds P_f^perp Sigma_M = 0.
Arrays are [z, y, x]; tensor index 0 <-> x, 1 <-> y, 2 <-> z.
"""

from __future__ import annotations

import numpy as np
import scipy.fft

# Mandel ordering of symmetric tensors (inner product = Frobenius product).
MANDEL3D = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))
MANDEL2D = ((0, 0), (1, 1), (0, 1))


def mandel_pairs(ncomp):
    return MANDEL2D if ncomp == 3 else MANDEL3D


def to_tensor(m):
    """Mandel vector field (c, ...) -> symmetric tensor field (3, 3, ...)."""
    c = m.shape[0]
    t = np.zeros((3, 3) + m.shape[1:], dtype=m.dtype)
    for k, (i, j) in enumerate(mandel_pairs(c)):
        if i == j:
            t[i, i] = m[k]
        else:
            t[i, j] = m[k] / np.sqrt(2.0)
            t[j, i] = m[k] / np.sqrt(2.0)
    return t


def to_mandel(t, ncomp):
    """Symmetric tensor field (3, 3, ...) -> Mandel vector field (c, ...)."""
    out = np.zeros((ncomp,) + t.shape[2:], dtype=t.dtype)
    for k, (i, j) in enumerate(mandel_pairs(ncomp)):
        out[k] = t[i, i] if i == j else np.sqrt(2.0) * 0.5 * (t[i, j] + t[j, i])
    return out


def standard_frequencies(shape):
    """q = (qx, qy, qz) broadcast to `shape`, q_j = 2 pi m_j / N_j, m_j in the
    usual FFT order (Nyquist index of an even axis reads m = -N/2)."""
    nz, ny, nx = shape
    qz = 2.0 * np.pi * np.fft.fftfreq(nz)[:, None, None]
    qy = 2.0 * np.pi * np.fft.fftfreq(ny)[None, :, None]
    qx = 2.0 * np.pi * np.fft.fftfreq(nx)[None, None, :]
    return [np.broadcast_to(q, shape) for q in (qx, qy, qz)]


def laplacian_symbol(shape):
    qx, qy, qz = standard_frequencies(shape)
    return -(qx * qx + qy * qy + qz * qz)


def _half_angle(n):
    m = np.fft.fftfreq(n) * n            # signed integer frequencies
    half = np.pi * m / n                 # q/2
    s = np.sin(half)
    c = np.cos(half)
    if n % 2 == 0:
        c[n // 2] = 0.0                  # Nyquist: cos(-pi/2) is exactly zero
    return s, c


def rotated_direction(shape):
    """Unit vectors n = r/|r| of the rotated scheme and the mask of r == 0."""
    nz, ny, nx = shape
    sx, cx = _half_angle(nx)
    sy, cy = _half_angle(ny)
    sz, cz = _half_angle(nz)
    sx, cx = sx[None, None, :], cx[None, None, :]
    sy, cy = sy[None, :, None], cy[None, :, None]
    sz, cz = sz[:, None, None], cz[:, None, None]
    rx = np.broadcast_to(sx * cy * cz, shape)
    ry = np.broadcast_to(cx * sy * cz, shape)
    rz = np.broadcast_to(cx * cy * sz, shape)
    r2 = rx * rx + ry * ry + rz * rz
    zero = r2 == 0.0
    inv = np.where(zero, 0.0, 1.0 / np.sqrt(np.where(zero, 1.0, r2)))
    n = np.stack([rx * inv, ry * inv, rz * inv])
    return n, zero


def standard_direction(shape):
    """Unit vectors n = xi/|xi| of the standard scheme and the mask of xi == 0."""
    nz, ny, nx = shape

    def axis(n_):
        q = 2.0 * np.pi * np.fft.fftfreq(n_)
        if n_ % 2 == 0:
            q[n_ // 2] = 0.0                # Nyquist: no signed frequency
        return q

    rx = np.broadcast_to(axis(nx)[None, None, :], shape)
    ry = np.broadcast_to(axis(ny)[None, :, None], shape)
    rz = np.broadcast_to(axis(nz)[:, None, None], shape)
    r2 = rx * rx + ry * ry + rz * rz
    zero = r2 == 0.0
    inv = np.where(zero, 0.0, 1.0 / np.sqrt(np.where(zero, 1.0, r2)))
    return np.stack([rx * inv, ry * inv, rz * inv]), zero


def direction(shape, scheme="rotated"):
    if scheme == "rotated":
        return rotated_direction(shape)
    if scheme == "standard":
        return standard_direction(shape)
    raise ValueError(scheme)


def project_hat(A_hat, n, zero):
    """P(A) = (A n) (x) n + n (x) (A n) - (n . A n) n (x) n, zero where r = 0."""
    An = np.einsum("ij...,j...->i...", A_hat, n)
    nAn = np.einsum("i...,i...->...", n, An)
    out = (np.einsum("i...,j...->ij...", An, n)
           + np.einsum("i...,j...->ij...", n, An)
           - nAn * np.einsum("i...,j...->ij...", n, n))
    out[:, :, zero] = 0.0
    return out


# Threads of the library FFT (scipy.fft `workers`).  The transforms give the
# same bits for any count; timing runs of the oracle on a many-core host
# raise it, everything else leaves it at 1.
FFT_WORKERS = 1


def fftn(a):
    return scipy.fft.fftn(a, axes=(-3, -2, -1), workers=FFT_WORKERS)


def ifftn(a):
    return scipy.fft.ifftn(a, axes=(-3, -2, -1), workers=FFT_WORKERS)


def G_tensor(A, scheme="rotated", free_mean=None):
    """Projection of a real symmetric tensor field A (3, 3, nz, ny, nx).
    free_mean: None (prescribed mean strain, G(0) = 0) or the 3x3 loading
    direction f of mixed macroscopic conditions (G(0) = P_f^perp)."""
    shape = A.shape[2:]
    n, zero = direction(shape, scheme)
    A_hat = fftn(A)
    out = project_hat(A_hat, n, zero)
    if free_mean is not None:
        fh = np.asarray(free_mean, dtype=np.float64)
        fh = fh / np.sqrt(np.sum(fh * fh))
        a0 = A_hat[:, :, 0, 0, 0]
        out[:, :, 0, 0, 0] = a0 - fh * np.sum(fh * a0)
    return ifftn(out).real


def G_mandel(m, scheme="rotated", free_mean=None):
    """Projection acting on a Mandel field (c, nz, ny, nx)."""
    return to_mandel(G_tensor(to_tensor(m), scheme, free_mean), m.shape[0])


def laplacian(phi):
    """Spectral Laplacian with standard frequencies, Nyquist kept."""
    return ifftn(laplacian_symbol(phi.shape) * fftn(phi)).real


def fd_laplacian_symbol(shape):
    """Symbol of the finite-difference Laplacian sum_j (u_{i+e_j} - 2 u_i +
    u_{i-e_j}): -sum_j 4 sin^2(q_j / 2)."""
    nz, ny, nx = shape
    out = np.zeros(shape)
    for n, sh in ((nx, (1, 1, nx)), (ny, (1, ny, 1)), (nz, (nz, 1, 1))):
        q = 2.0 * np.pi * np.fft.fftfreq(n)
        out = out - (4.0 * np.sin(q / 2.0) ** 2).reshape(sh)
    return out


def fd_laplacian(phi):
    return ifftn(fd_laplacian_symbol(phi.shape) * fftn(phi)).real


def face_average(k, axis_xyz):
    """k on the faces between voxel i and its upper neighbour along an axis:
    the arithmetic mean of the two voxels."""
    ax = {0: 2, 1: 1, 2: 0}[axis_xyz]
    return 0.5 * (k + np.roll(k, -1, axis=ax))


def div_k_grad(u, k):
    """Finite-difference div(k grad u) on the periodic grid (the variational
    form of the heterogeneous-toughness term): forward differences of u,
    times k on the faces (mean of the two voxels), backward differences of
    the fluxes.  Symmetric and negative semi-definite; with constant k it is
    k times the finite-difference Laplacian."""
    out = np.zeros(u.shape)
    for j in range(3):
        ax = {0: 2, 1: 1, 2: 0}[j]
        if u.shape[ax] == 1:
            continue
        flux = face_average(k, j) * (np.roll(u, -1, axis=ax) - u)
        out += flux - np.roll(flux, 1, axis=ax)
    return out
