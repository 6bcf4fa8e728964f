"""GPU parity of the hot-path steps against the oracle (same seeded inputs).

Steps (a3)-(a5): projection + Laplacian through the FFT passes;
(a1)+(a8): constitutive update and FP64 residual; (a2)-(a6): tangent action;
(a7): BiCGSTAB.  Tolerances: FP64 1e-11 relative (FFT round-off grows like
log N eps), FP32 1e-5 relative.
"""

import numpy as np
import pytest

from oracle import fourier as fo
from oracle.system import System
from synth import problem_config, random_state, random_vector

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def gpu_solver(prob, **kw):
    from paper_2412_17445_amd import Solver
    return Solver.from_problem(prob, **kw)


def small_problem(name, shape=None, precision="fp64"):
    prob = problem_config(name)
    if shape is not None:
        prob.shape = shape
        rng = np.random.default_rng(5)
        prob.phase_id = (rng.uniform(size=shape) < 0.3).astype(np.uint8) if len(prob.phases) > 1 \
            else np.zeros(shape, np.uint8)
        if prob.mask is not None:
            m = np.zeros(shape, np.uint8)
            m[shape[0] // 2, shape[1] // 2, shape[2] // 4: shape[2] // 2] = 1
            prob.mask = m
    prob.precision = precision
    return prob


SHAPES = [("tiny16", None), ("tiny16", (1, 12, 18)), ("fib64", None), ("pore24", None),
          ("part24", (12, 18, 16)), ("part24", (9, 8, 6))]

# z lengths 32, 64 and 128 take the z pass with register-resident end stages;
# odd x lengths (no Nyquist plane) and other radices on x and y included
ZSPEC_SHAPES = [("part24", (32, 12, 10)), ("pore24", (64, 6, 10)), ("part24", (128, 4, 6)),
                ("part24", (32, 8, 9)), ("part24", (32, 7, 13))]


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300)


# lengths with prime factors above 3 (generic-radix FFT stages): 5, 7, 11,
# 13, 17, 31, and the paper's 39 = 3 * 13 and 77 = 7 * 11
ODD_SHAPES = [("tiny16", (1, 15, 20)), ("tiny16", (1, 13, 11)), ("tiny16", (1, 39, 39)),
              ("tiny16", (1, 31, 17)), ("tiny16", (1, 14, 77)), ("part24", (5, 7, 10)),
              ("part24", (7, 11, 13)), ("pore24", (10, 14, 35))]

STD_SHAPES = [("tiny16_std", None), ("tiny16_std", (1, 12, 18)), ("tiny16_std", (1, 18, 9)),
              ("part24_std", (12, 18, 16)), ("part24_std", (9, 8, 6))]


@pytest.mark.parametrize("name,shape", SHAPES + STD_SHAPES + ODD_SHAPES + ZSPEC_SHAPES +
                         [("part24_std", (64, 8, 6))])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_projection_and_laplacian(name, shape, prec):
    prob = small_problem(name, shape)
    s = gpu_solver(prob)
    c = 3 if prob.shape[0] == 1 else 6
    rng = np.random.default_rng(1)
    x = rng.standard_normal((c + 1,) + tuple(prob.shape))
    dt = torch.float64 if prec == "fp64" else torch.float32
    out = s.project(torch.tensor(x.reshape(-1), dtype=dt, device="cuda")).double().cpu().numpy()
    out = out.reshape(x.shape)
    refG = fo.G_mandel(x[:c], prob.projection)
    refL = fo.laplacian(x[c])
    tol = 1e-12 if prec == "fp64" else 2e-6
    assert rel(out[:c], refG) < tol
    assert rel(out[c], refL) < tol


@pytest.mark.parametrize("name,shape", SHAPES + ZSPEC_SHAPES)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_projection_of_nearly_equilibrated_field_stays_compatible(name, shape, prec):
    """G of a field that is mostly divergence-free (the residual near a root:
    sigma is nearly equilibrated, G sigma is small) must still be compatible
    to round-off of the small result, not of the large input.  A C2R pass that
    lets the imaginary round-off of the DC / Nyquist bins of one field leak
    into its packed partner breaks this at eps * |x| and leaves the Newton
    right-hand side outside the range of the tangent."""
    prob = small_problem(name, shape)
    s = gpu_solver(prob)
    c = 3 if prob.shape[0] == 1 else 6
    rng = np.random.default_rng(7)
    r1 = rng.standard_normal((c,) + tuple(prob.shape))
    r2 = rng.standard_normal((c,) + tuple(prob.shape))
    small = 1e-10 if prec == "fp64" else 1e-4
    x = np.zeros((c + 1,) + tuple(prob.shape))
    x[:c] = (r1 - fo.G_mandel(r1)) + small * fo.G_mandel(r2)
    dt = torch.float64 if prec == "fp64" else torch.float32
    y = s.project(torch.tensor(x.reshape(-1), dtype=dt, device="cuda"))
    # compatibility of the output, measured with the same GPU projection
    # (equal to the oracle's to 1e-12 / 2e-6 by the test above): G y = y
    y2 = s.project(y.clone()).double().cpu().numpy().reshape(x.shape)[:c]
    y = y.double().cpu().numpy().reshape(x.shape)[:c]
    incompat = np.linalg.norm(y - y2) / np.linalg.norm(y)
    assert incompat < (1e-12 if prec == "fp64" else 1e-5), incompat


def test_newton_solve_on_own_residual_near_root():
    """Near a root the Newton right-hand side is small; the GPU's own FP64
    residual must still be solvable to the Krylov tolerance (as the oracle's
    is).  Oracle Newton iterations bring the 16^2 case close to its first
    root; the GPU then solves J dq = -F with its own F."""
    from oracle import krylov
    from oracle.newton import Solver as OracleSolver
    prob = problem_config("tiny16")
    o = OracleSolver(prob)
    o.bootstrap()
    sy = o.sys
    eps_t, phi, E = o.guess
    a_new = o.a + o.delta_a
    for _ in range(5):
        R = sy.residual(eps_t, phi, E, o.Hn, a_new)
        J = sy.tangent(eps_t, phi, E, o.Hn)
        dx, _ = krylov.bicgstab(J, -sy.pack(R["F1"], R["F2"], R["F3"]), rtol=1e-10, maxit=5000)
        de, dp, dE = sy.unpack(dx)
        eps_t, phi, E = eps_t + de, phi + (1 - sy.m) * dp, E + dE
    s = gpu_solver(prob, precision="fp64")
    s.bootstrap()
    s.set_state(eps_t, phi, o.Hn, E, o.a, 0)
    F, _, _, _ = s.residual(a_new)
    assert float(F.abs().max()) < 1e-9          # close to the root
    x, it, rr, ok = s.krylov_solve(F.neg(), rtol=1e-10, maxit=2000)
    assert ok and rr <= 1e-10, (it, rr)
    s.close()


def _frozen_state(sysm, seed):
    eps, phi, Hn, E = random_state(sysm.shape, sysm.ncomp, seed, f_mandel=sysm.f, E=0.01)
    eps_t = fo.G_mandel(eps - sysm.fE(E))
    st = sysm.point(eps_t + sysm.fE(E), phi, np.zeros(sysm.shape))
    rng = np.random.default_rng(seed + 1)
    Hn = st["psi_p"] * np.where(rng.uniform(size=sysm.shape) < 0.5, 0.7, 1.3)
    phi = np.where(sysm.m > 0, 1.0, phi)
    return eps_t, phi, E, Hn


@pytest.mark.parametrize("name,shape", SHAPES + [("gc16_iso", None), ("part24_iso", (12, 18, 16)),
                                              ("tiny16_std", (1, 12, 18)), ("part24_std", (12, 18, 16)),
                                              ("gc16_w", None), ("part24_w", (9, 8, 6)),
                                              ("tiny16", (1, 15, 20)), ("tiny16", (1, 39, 39)),
                                              ("part24", (5, 7, 10)), ("part24", (7, 11, 13)),
                                              ("gc16_d", None), ("part24_d", (9, 8, 6)),
                                              ("tiny16_v", None), ("gc16_v", None), ("part24_v", (9, 8, 6)),
                                              ("part24_v", (12, 18, 16))] + ZSPEC_SHAPES +
                         [("part24_iso", (32, 8, 9)), ("part24_std", (64, 8, 6)), ("part24_d", (32, 12, 10))])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_residual_and_tangent(name, shape, precision):
    prob = small_problem(name, shape, precision)
    sysm = System(prob)
    eps_t, phi, E, Hn = _frozen_state(sysm, 3)
    a = 2.5
    s = gpu_solver(prob)
    s.set_state(eps_t, phi, Hn, E, a - 1.0, n=1)
    F, gam, sig, dis = s.residual(a)
    R = sysm.residual(eps_t, phi, E, Hn, a)
    F = F.cpu().numpy()
    c, N = sysm.ncomp, sysm.N
    assert rel(F[: c * N], R["F1"].ravel()) < 1e-11
    assert rel(F[c * N:(c + 1) * N], R["F2"].ravel()) < 1e-11
    assert abs(F[-1] - R["F3"]) <= 1e-12 * abs(R["Gamma"])
    assert abs(gam - R["Gamma"]) <= 1e-12 * abs(R["Gamma"])
    D = sysm.dissipation(phi)
    assert abs(dis - D) <= 1e-12 * abs(D)
    sM = R["sigma_M"]
    ref_sig = [sM[0, 0], sM[1, 1], sM[2, 2], sM[1, 2], sM[0, 2], sM[0, 1]]
    assert rel(sig, ref_sig) < 1e-12
    # tangent action on a seeded vector
    v = random_vector(sysm.N * (c + 1) + 1, 9) * 1e-3
    J = sysm.tangent(eps_t, phi, E, Hn)
    ref = J(v)
    dt = torch.float32 if precision == "mixed" else torch.float64
    Jv = s.apply(torch.tensor(v, dtype=dt, device="cuda")).double().cpu().numpy()
    tol = 1e-11 if precision == "fp64" else 2e-5
    for blk in (slice(0, c * N), slice(c * N, (c + 1) * N)):
        assert rel(Jv[blk], ref[blk]) < tol
    r = phi / sysm.l - sysm.l * fo.laplacian(phi)
    if sysm.dctl:
        Gc = sysm.Gc
        r = Gc * phi / sysm.l - 0.5 * sysm.l * (Gc * fo.laplacian(phi) + fo.laplacian(Gc * phi))
    scale = sysm.wa * np.sum(np.abs(r * (1 - sysm.m) * v[c * N:(c + 1) * N].reshape(sysm.shape))) \
        + sysm.wE * abs(v[-1])
    assert abs(Jv[-1] - ref[-1]) <= tol * scale
    s.close()


@pytest.mark.parametrize("name", ["tiny16", "pore24"])
def test_krylov_solve(name):
    prob = small_problem(name)
    sysm = System(prob)
    eps_t, phi, E, Hn = _frozen_state(sysm, 4)
    s = gpu_solver(prob)
    s.set_state(eps_t, phi, Hn, E, 1.0, n=1)
    F, _, _, _ = s.residual(2.0)
    b = -F
    x, it, rr, ok = s.krylov_solve(b, rtol=1e-10, maxit=3000)
    assert ok and rr <= 1e-10
    J = sysm.tangent(eps_t, phi, E, Hn)
    xr = x.cpu().numpy()
    bb = b.cpu().numpy()
    assert np.linalg.norm(J(xr) - bb) <= 1e-8 * np.linalg.norm(bb)
    s.close()
