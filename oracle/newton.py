"""Monolithic Newton with crack-length control (oracle).

Paper Sec. 3.2 and Algorithm 2: per increment the prescribed crack length is
raised by a constant step (the linear ramp of Sec. 2.3), Newton starts from
the last converged fields, each iteration solves dF(q; dq) = -F(q)
(eq. `LinearSyst_CrackCont`) with BiCGSTAB and takes the relaxed update
q += alpha dq; the history is committed after convergence.

Readings (see also `system`):
* Convergence (eq. `errors_crack`, whose first term is garbled): the largest
  of ||d eps_tilde + f dE|| / ||eps||, ||d phi|| / ||phi|| and
  |Gamma - a| / a, all taken after the update, must drop to `tol`.
* Krylov start x0 = 0 (keeps the strain update compatible), stop at
  ||r|| <= rtol ||b||.
* Bootstrap (the paper starts from E = 0, phi = 0, where the bordered
  Jacobian is singular): with an initial-crack mask, phi0 solves the
  damage-free Helmholtz problem (1/l - l Lap) phi = 0 off the mask with
  phi = 1 on it (CG), and a0 = Gamma(phi0); without a mask phi0 = 0, a0 = 0.
  The first increment starts from the gradient-free homogeneous solution:
  E_s is the bisection root of sum_x (1-m) phi_loc(E)^2 / (2l) = delta_a
  with phi_loc = 2 psi0(+)(f E) / (Gc/l + 2 psi0(+)(f E)), using
  psi0(+)(f E) = E^2 psi0(+)(f); the guess is eps = f E_s,
  phi = max(phi0, (1-m) phi_loc(E_s)), E = E_s > 0.
* Weighted control (FFT analogue of eq. `FEMweights`): the constraint is
  w_a Gamma + w_E E = tau with tau raised by `delta_a` per increment; the
  weights (1, 0) give crack-length control, (0, 1) monolithic strain
  control, which can start an uncracked cell from phi = 0.  tau0 =
  w_a Gamma(phi0), the convergence measure is |w_a Gamma + w_E E - tau| /
  |tau|, and the predictor solves w_a S(E) + w_E E = delta_a.
* Dissipation control (eq. `SystemDis`, last line): Gamma is replaced by
  D = integral of Gc gamma_f in the constraint, its row (r -> Gc r), tau0
  and the predictor (S weighted by Gc).
* Parity mode (`resid_tol` > 0): besides the update measures of eq.
  `errors_crack`, Newton also requires the residual of eq.
  `System_CrackLength` at the new state to be small, ||F1|| / ||sigma|| <=
  resid_tol and ||F2|| / ||2H|| <= resid_tol (norms over all voxels, sigma
  and F1 in the Mandel components of the strain unknowns).  The update
  measure alone leaves a linearly converging iteration (relaxation
  alpha < 1) as far from the root as its last step; the residual stop pins
  the root itself, whatever the Krylov tolerance of the steps, so two
  implementations that both meet it agree to the conditioning of the root.
"""

from __future__ import annotations

import numpy as np

from . import fourier as fo
from . import krylov
from .system import System

BISECTION_STEPS = 100


class Solver:
    def __init__(self, prob, tol=None, rtol=None, kmaxit=None, alpha=None, maxit=None,
                 resid_tol=0.0):
        self.sys = System(prob)
        self.resid_tol = float(resid_tol)
        s = self.sys
        self.tol = prob.newton_tol if tol is None else tol
        self.rtol = prob.krylov_rtol if rtol is None else rtol
        self.kmaxit = prob.krylov_maxit if kmaxit is None else kmaxit
        self.alpha = prob.alpha if alpha is None else alpha
        self.maxit = prob.newton_maxit if maxit is None else maxit
        self.delta_a = float(prob.delta_a)
        self.eps_t = np.zeros((s.ncomp,) + s.shape)
        self.phi = np.zeros(s.shape)
        self.E = 0.0
        self.Hn = np.zeros(s.shape)
        self.a = 0.0
        self.n = 0
        self.history = []

    # -- bootstrap ------------------------------------------------------------
    def initial_damage(self):
        s = self.sys
        if not np.any(s.m):
            return np.zeros(s.shape), {"iters": 0}
        l, m = s.l, s.m
        B = lambda u: u / l - l * s.lap(u)                       # noqa: E731
        op = lambda x: ((1 - m) * B((1 - m) * x.reshape(s.shape))).ravel()  # noqa: E731
        rhs = (-(1 - m) * B(m)).ravel()
        u, info = krylov.cg(op, rhs, rtol=1e-14, maxit=20000)
        return m + (1 - m) * u.reshape(s.shape), info

    def psi_f(self):
        """psi0(+) of the unit loading strain f, per voxel (degree-2 scaling)."""
        s = self.sys
        st = s.point(s.fE(1.0) * np.ones((s.ncomp,) + s.shape), np.zeros(s.shape),
                     np.zeros(s.shape))
        return st["psi_p"]

    def local_damage(self, E, psif):
        s = self.sys
        h = 2.0 * E * E * psif
        return h / (s.Gc / s.l + h)

    def predictor(self, delta_a):
        s = self.sys
        psif = self.psi_f()
        gw = s.Gc if s.dctl else 1.0
        S0 = lambda E: float(np.sum(gw * (1 - s.m) * self.local_damage(E, psif) ** 2)) / (2 * s.l)  # noqa: E731
        S = lambda E: s.wa * S0(E) + s.wE * E                                   # noqa: E731
        lo, hi = 0.0, 1.0
        while S(hi) < delta_a:
            hi *= 2.0
            if hi > 1e12:
                raise RuntimeError("predictor: crack-length increment not reachable")
        for _ in range(BISECTION_STEPS):
            mid = 0.5 * (lo + hi)
            if S(mid) < delta_a:
                lo = mid
            else:
                hi = mid
        return 0.5 * (lo + hi), psif

    def bootstrap(self):
        s = self.sys
        phi0, _ = self.initial_damage()
        self.phi = phi0
        self.a = s.wa * s.controlled(phi0)
        Es, psif = self.predictor(self.delta_a)
        self.guess = (np.zeros_like(self.eps_t),
                      np.maximum(phi0, (1 - s.m) * self.local_damage(Es, psif)), Es)
        return dict(a0=self.a, E_s=Es)

    # -- Newton -----------------------------------------------------------------
    def compatible(self, x):
        """The Krylov vector x with its strain block replaced by its projection
        onto compatible fields (eq. `GFourier`)."""
        s = self.sys
        d_eps, d_phi, dE = s.unpack(x)
        return s.pack(s.G_mandel(d_eps), d_phi, dE)

    def residual_measures(self, R):
        """(||F1|| / ||sigma||, ||F2|| / ||2H||) of a residual evaluation; a
        zero numerator counts as zero whatever the scale."""
        s = self.sys
        sig = np.linalg.norm(fo.to_mandel(R["state"]["sigma"], s.ncomp))
        h2 = 2.0 * np.linalg.norm(R["state"]["H"])
        f1, f2 = np.linalg.norm(R["F1"]), np.linalg.norm(R["F2"])
        rel = lambda num, den: 0.0 if num == 0.0 else (num / den if den > 0.0 else np.inf)  # noqa: E731
        return rel(f1, sig), rel(f2, h2)

    def newton(self, eps_t, phi, E, a):
        s = self.sys
        kit = 0
        applies = 0
        err = np.inf
        errs = (np.inf, np.inf, np.inf)
        res = (np.inf, np.inf)
        R = s.residual(eps_t, phi, E, self.Hn, a)
        for it in range(1, self.maxit + 1):
            rhs = -s.pack(R["F1"], R["F2"], R["F3"])
            J = s.tangent(eps_t, phi, E, self.Hn)
            # Newton on compatible strains: the strain unknown is a compatible
            # fluctuation (Sec. 3.1), so the Krylov operator is J applied to
            # the compatible part of its argument, and the step is that part.
            # G[sigma] = 0 does not see an incompatible strain, so J alone has
            # near-null directions made of incompatible strain coupled with
            # damage and E wherever the history is at a tie (every warm start),
            # which a Krylov solve can pick up.  Under mixed macroscopic
            # conditions the projection also keeps the mean strain off f, so
            # that E alone sets the mean along f: (f t, -t) is a null direction
            # of the bordered system (eps = eps~ + f E is unchanged).
            JP = lambda v: J(self.compatible(v))                        # noqa: E731
            dx, info = krylov.bicgstab(JP, rhs, rtol=self.rtol, maxit=self.kmaxit)
            kit += info["iters"]
            applies += info["applies"]
            d_eps, d_phi, dE = s.unpack(self.compatible(dx))
            d_phi = (1 - s.m) * d_phi
            w = d_eps + s.fE(dE)
            eps_t = eps_t + self.alpha * d_eps
            phi = phi + self.alpha * d_phi
            E = E + self.alpha * dE
            eps = eps_t + s.fE(E)
            q = s.controlled(phi)
            errs = (np.linalg.norm(w) / np.linalg.norm(eps),
                    np.linalg.norm(d_phi) / np.linalg.norm(phi),
                    abs(s.wa * q + s.wE * E - a) / abs(a))
            err = max(errs)
            R = s.residual(eps_t, phi, E, self.Hn, a)
            res = self.residual_measures(R)
            if err <= self.tol and (self.resid_tol <= 0.0 or max(res) <= self.resid_tol):
                return eps_t, phi, E, dict(converged=True, newton_iters=it,
                                           krylov_iters=kit, applies=applies,
                                           err=errs, resid=res)
        return eps_t, phi, E, dict(converged=False, newton_iters=self.maxit,
                                   krylov_iters=kit, applies=applies, err=errs, resid=res)

    def step(self):
        """One crack-length increment; returns the per-increment outputs."""
        s = self.sys
        a_new = self.a + self.delta_a
        if self.n == 0:
            eps_t, phi, E = self.guess
        else:
            eps_t, phi, E = self.eps_t, self.phi, self.E
        eps_t, phi, E, info = self.newton(eps_t, phi, E, a_new)
        if not info["converged"]:
            info["increment"] = self.n + 1
            return info                       # state left at the last converged increment
        st = s.point(eps_t + s.fE(E), phi, self.Hn)
        self.Hn = np.maximum(st["psi_p"], self.Hn)
        self.eps_t, self.phi, self.E, self.a = eps_t, phi, E, a_new
        self.n += 1
        out = dict(info)
        out.update(increment=self.n, E=E, Gamma=s.gamma(phi), a=a_new, D=s.dissipation(phi),
                   sigma_M=st["sigma"].reshape(3, 3, -1).mean(axis=-1),
                   phi_norm=float(np.linalg.norm(phi)))
        self.history.append(out)
        return out
