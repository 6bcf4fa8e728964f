"""Pins of the variational toughness term l div(Gc grad phi) (the
heterogeneous-Gc alternative to the printed pointwise Gc l Lap phi), taken in
finite differences: forward differences of phi, Gc on the faces (mean of
the two voxels), backward differences of the fluxes; the crack density then
uses the same finite-difference Laplacian.

* Brute force: the three-point flux stencil written out with explicit
  periodic index loops on a small 3D grid.
* Constant toughness: k times the finite-difference Laplacian, whose symbol
  -sum 4 sin^2(q/2) is applied by FFT (an independent route); a plane wave
  is an eigenfunction with that eigenvalue (closed form).
* The operator is self-adjoint and negative semi-definite.
* J v against central differences of the residual with two toughnesses;
  Newton increments of the two-toughness cell converge, on a different
  path than the pointwise form's.
"""

import numpy as np
import pytest

from oracle import fourier as fo
from oracle.newton import Solver
from oracle.system import System
from synth import problem_config


def test_flux_stencil_by_brute_force():
    rng = np.random.default_rng(1)
    nz, ny, nx = 4, 5, 6
    u = rng.standard_normal((nz, ny, nx))
    k = rng.uniform(0.5, 2.0, (nz, ny, nx))
    ref = np.zeros_like(u)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                acc = 0.0
                for dz, dy, dx in ((0, 0, 1), (0, 1, 0), (1, 0, 0)):
                    up = ((z + dz) % nz, (y + dy) % ny, (x + dx) % nx)
                    dn = ((z - dz) % nz, (y - dy) % ny, (x - dx) % nx)
                    k_up = 0.5 * (k[z, y, x] + k[up])
                    k_dn = 0.5 * (k[z, y, x] + k[dn])
                    acc += k_up * (u[up] - u[z, y, x]) - k_dn * (u[z, y, x] - u[dn])
                ref[z, y, x] = acc
    assert np.abs(fo.div_k_grad(u, k) - ref).max() <= 1e-13


def test_constant_toughness_is_the_fd_laplacian():
    rng = np.random.default_rng(2)
    u = rng.standard_normal((6, 8, 10))
    assert np.abs(fo.div_k_grad(u, np.full(u.shape, 2.5)) - 2.5 * fo.fd_laplacian(u)).max() <= 1e-12
    ny, nx = 12, 10
    y = np.arange(ny)[None, :, None] * np.ones((1, ny, nx))
    q = 2 * np.pi * 5 / ny                                   # the Nyquist mode of y
    w = np.cos(q * y)
    assert np.abs(fo.div_k_grad(w, np.ones(w.shape)) - (-4 * np.sin(q / 2) ** 2) * w).max() <= 1e-14


def test_self_adjoint_and_negative():
    rng = np.random.default_rng(4)
    shape = (6, 8, 10)
    k = rng.uniform(0.5, 2.0, shape)
    u, w = rng.standard_normal(shape), rng.standard_normal(shape)
    Lu, Lw = fo.div_k_grad(u, k), fo.div_k_grad(w, k)
    assert abs(np.sum(w * Lu) - np.sum(u * Lw)) <= 1e-12 * np.sum(np.abs(u * Lw))
    assert np.sum(u * Lu) < 0.0
    assert np.abs(fo.div_k_grad(np.full(shape, 3.0), k)).max() <= 1e-14   # constants


def test_tangent_is_residual_derivative():
    prob = problem_config("gc16_v")
    sy = System(prob)
    rng = np.random.default_rng(6)
    eps_t = fo.G_mandel(rng.standard_normal((sy.ncomp,) + sy.shape) * 1e-3)
    phi = np.clip(rng.uniform(0, 0.6, sy.shape) + sy.m, 0, 1)
    E = 5e-3
    Hn = sy.point(eps_t + sy.fE(E), phi, np.zeros(sy.shape))["psi_p"] * 0.8
    J = sy.tangent(eps_t, phi, E, Hn)
    d_eps = fo.G_mandel(rng.standard_normal(eps_t.shape)) * 1e-2
    d_phi = rng.standard_normal(sy.shape) * 1e-2 * (1 - sy.m)
    Jv = J(sy.pack(d_eps, d_phi, 1e-3))
    h = 1e-6

    def F(t):
        R = sy.residual(eps_t + t * d_eps, phi + t * d_phi, E + t * 1e-3, Hn, 2.0)
        return sy.pack(R["F1"], R["F2"], R["F3"])

    fd = (F(h) - F(-h)) / (2 * h)
    c, N = sy.ncomp, sy.N
    for blk in (slice(c * N, (c + 1) * N), slice(-1, None)):
        assert np.abs(Jv[blk] - fd[blk]).max() <= 2e-5 * np.abs(fd[blk]).max()


def test_increments_converge_to_a_different_path():
    v = Solver(problem_config("gc16_v"))
    p = Solver(problem_config("gc16"))
    v.bootstrap()
    p.bootstrap()
    for _ in range(2):
        ov, op = v.step(), p.step()
        assert ov["converged"]
        assert abs(ov["E"] - op["E"]) > 1e-6 * op["E"]
        assert ov["Gamma"] == pytest.approx(ov["a"], rel=1e-8)
    from oracle.staggered import StaggeredSolver
    with pytest.raises(ValueError):
        StaggeredSolver(problem_config("gc16_v"), dE=1e-3)
