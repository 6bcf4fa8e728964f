"""Dense finite-difference-Jacobian Newton for tiny grids (oracle pin).

Same residual, same start and same relaxed update as `newton.Solver`, but
every Newton system is assembled column by column from central differences
of the residual (no analytic tangent, no Krylov solver) and solved by LU.
Because the equilibrium rows only see compatible strains, the strain rows are
completed with (I - G) eps_tilde, whose Jacobian is nonsingular on the
incompatible complement; at every iterate eps_tilde is compatible, so this
extra term is zero and the Newton step is the one of the bordered system.
"""

from __future__ import annotations

import numpy as np

from . import fourier as fo
from .newton import Solver


def full_residual(sys, x, Hn, a):
    eps_t, phi, E = sys.unpack(x)
    R = sys.residual(eps_t, phi, E, Hn, a)
    F1 = R["F1"] + (eps_t - sys.G_mandel(eps_t))
    m = sys.m
    F2 = R["F2"] + m * (phi - 1.0) * (1.0 if np.any(m) else 0.0)
    return sys.pack(F1, F2, R["F3"])


def fd_jacobian(sys, x, Hn, a, h=1e-7):
    n = x.size
    J = np.empty((n, n))
    for j in range(n):
        step = h * max(1.0, abs(x[j]))
        xp = x.copy(); xp[j] += step
        xm = x.copy(); xm[j] -= step
        J[:, j] = (full_residual(sys, xp, Hn, a) - full_residual(sys, xm, Hn, a)) / (2 * step)
    return J


def newton_dense(solver: Solver, eps_t, phi, E, a, maxit=None, tol=None):
    sys = solver.sys
    maxit = solver.maxit if maxit is None else maxit
    tol = solver.tol if tol is None else tol
    x = sys.pack(eps_t, phi, E)
    for it in range(1, maxit + 1):
        F = full_residual(sys, x, solver.Hn, a)
        J = fd_jacobian(sys, x, solver.Hn, a)
        dx = np.linalg.solve(J, -F)
        d_eps, d_phi, dE = sys.unpack(dx)
        d_phi = (1 - sys.m) * d_phi
        w = d_eps + sys.fE(dE)
        x = x + solver.alpha * sys.pack(d_eps, d_phi, dE)
        eps_t, phi, E = sys.unpack(x)
        eps = eps_t + sys.fE(E)
        errs = (np.linalg.norm(w) / np.linalg.norm(eps),
                np.linalg.norm(d_phi) / np.linalg.norm(phi),
                abs(sys.gamma(phi) - a) / abs(a))
        if max(errs) <= tol:
            return eps_t, phi, E, dict(converged=True, newton_iters=it)
    return eps_t, phi, E, dict(converged=False, newton_iters=maxit)
