"""Strain-controlled implicit staggered scheme (oracle).

Test infrastructure only: imported by tests/ and by bench.py's CPU baseline,
never by the product path.

Paper Sec. 3.1 and Algorithm 1.  Per increment the magnitude of the
prescribed macroscopic strain is raised by a fixed step, E <- E + dE, and
stagger iterations alternate two sub-problems until the fields settle:

* mechanical problem at the damage of the last stagger iteration: Newton on
  G[sigma(f E + eps~, phi)] = 0, each step solving G[C_i : d eps~] =
  -G[sigma_i] (eq. `LinearOpe_Mech`) by conjugate gradients, with C_i the
  degraded split stiffness at eps_i; it stops when
  max|d eps~| / ||f E|| < tol_mech (eq. `errors_strain`, first line);
* history H = max(psi0(+)(eps), H_n) of the converged strain (eq. `history`);
* Helmholtz problem (Gc/l + 2H) phi - Gc l Lap phi = 2H (eq.
  `LinearOpe_Helm`, with the sign reading of the monolithic system) by
  conjugate gradients;

until max(||eps_s - eps_{s-1}|| / ||eps_s||, ||phi_s - phi_{s-1}|| / ||phi_s||)
< tol_sta (eq. `errors_strain`, last line).  H_n is committed after the
increment.

Readings:
* ||f E|| is the Frobenius norm of the prescribed mean strain (Mandel
  components), the norm of the mean strain in eq. `errors_strain`.
* With heterogeneous Gc the Helmholtz equation is divided by Gc(x) > 0
  before CG: (1/l + 2H/Gc) phi - l Lap phi = 2H/Gc has the same solution
  and a symmetric positive definite operator.
* The crack mask is a Dirichlet condition, phi = m + (1 - m) u with u = 0 on
  the mask (as in the bootstrap of the monolithic oracle).
* CG on the mechanical operator starts from 0; its iterates stay in the
  range of G (compatible strain fields).
* The start state is the monolithic oracle's bootstrap damage phi0
  (the damage-free profile around the crack mask), eps~ = 0, E = 0, H = 0.
* A relative error whose numerator is zero is zero, also over a zero norm
  (the unloaded state E = 0, eps = 0 is then converged at once).
"""

from __future__ import annotations

import numpy as np

from . import fourier as fo
from . import krylov
from .newton import Solver as _Monolithic
from .system import System


def _rel(num, den):
    """num / den, with 0 / x = 0 for any x (the error of an unchanged field)."""
    if num == 0.0:
        return 0.0
    return num / den if den > 0.0 else np.inf


class StaggeredSolver:
    def __init__(self, prob, dE, tol_mech=1e-9, tol_sta=1e-8, cg_rtol=1e-11, max_stagger=500,
                 max_newton=50, cg_maxit=20000):
        self.sys = System(prob)
        s = self.sys
        if s.var:
            raise ValueError("the staggered oracle uses the pointwise toughness term")
        self.dE = float(dE)
        self.tol_mech, self.tol_sta = tol_mech, tol_sta
        self.cg_rtol, self.cg_maxit = cg_rtol, cg_maxit
        self.max_stagger, self.max_newton = max_stagger, max_newton
        self.eps_t = np.zeros((s.ncomp,) + s.shape)
        self.phi = _Monolithic(prob).initial_damage()[0]
        self.E = 0.0
        self.Hn = np.zeros(s.shape)
        self.n = 0

    # -- sub-problems -----------------------------------------------------------
    def mechanical(self, eps_t, phi, E):
        """Newton + CG on G[sigma(f E + eps~, phi)] = 0 at fixed phi."""
        s = self.sys
        c, N = s.ncomp, s.N
        zeros = np.zeros(N + 1)
        nf = float(np.linalg.norm(s.f)) * abs(E)
        cg_total = 0
        for it in range(1, self.max_newton + 1):
            R = s.residual(eps_t, phi, E, self.Hn, 0.0)
            J = s.tangent(eps_t, phi, E, self.Hn)
            op = lambda v: J(np.concatenate([v, zeros]))[: c * N]        # noqa: E731
            d, info = krylov.cg(op, -R["F1"].ravel(), rtol=self.cg_rtol, maxit=self.cg_maxit)
            cg_total += info["iters"]
            d = d.reshape((c,) + s.shape)
            eps_t = eps_t + d
            if nf == 0.0 or np.abs(d).max() / nf < self.tol_mech:
                return eps_t, it, cg_total
        raise RuntimeError("staggered oracle: mechanical Newton did not converge")

    def helmholtz(self, H):
        """(1/l + 2H/Gc) phi - l Lap phi = 2H/Gc off the mask, phi = 1 on it."""
        s = self.sys
        l, m = s.l, s.m
        a = 1.0 / l + 2.0 * H / s.Gc
        B = lambda u: a * u - l * fo.laplacian(u)                          # noqa: E731
        op = lambda x: ((1 - m) * B((1 - m) * x.reshape(s.shape))).ravel()  # noqa: E731
        rhs = ((1 - m) * (2.0 * H / s.Gc - B(m))).ravel()
        u, info = krylov.cg(op, rhs, rtol=self.cg_rtol, maxit=self.cg_maxit)
        return m + (1 - m) * u.reshape(s.shape), info["iters"]

    # -- one increment (Algorithm 1) --------------------------------------------
    def step(self):
        s = self.sys
        E = self.E + self.dE
        eps_t, phi = self.eps_t.copy(), self.phi.copy()
        newton, cgm, cgh = 0, 0, 0
        for st in range(1, self.max_stagger + 1):
            eps_new, it, k = self.mechanical(eps_t, phi, E)
            newton += it
            cgm += k
            psi_p = s.point(eps_new + s.fE(E), phi, self.Hn)["psi_p"]
            H = np.maximum(psi_p, self.Hn)
            phi_new, k = self.helmholtz(H)
            cgh += k
            eps_full = eps_new + s.fE(E)
            err = max(_rel(np.linalg.norm(eps_new - eps_t), np.linalg.norm(eps_full)),
                      _rel(np.linalg.norm(phi_new - phi), np.linalg.norm(phi_new)))
            eps_t, phi = eps_new, phi_new
            if err < self.tol_sta:
                break
        else:
            raise RuntimeError("staggered oracle: stagger iterations did not converge")
        st_final = s.point(eps_t + s.fE(E), phi, self.Hn)
        self.Hn = np.maximum(st_final["psi_p"], self.Hn)
        self.eps_t, self.phi, self.E = eps_t, phi, E
        self.n += 1
        return dict(increment=self.n, E=E, Gamma=s.gamma(phi),
                    sigma_M=st_final["sigma"].reshape(3, 3, -1).mean(axis=-1),
                    stagger_iters=st, newton_iters=newton, cg_mech=cgm, cg_helm=cgh)
