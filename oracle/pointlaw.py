"""Constitutive point law of the phase-field model (oracle).

Paper Sec. 2.1 (eqs. `Emec`, `PlusNegPsi`, `gFunct`), Sec. 2.3 (eq.
`C_Calc`), Sec. 3.1 (eq. `history`) and Sec. 3.2 (eq. `Delta_history`):

* spectral split of the strain: eps(+/-) = sum_a <zeta_a>(+/-) e_a (x) e_a,
* psi0(+/-) = lambda/2 <tr eps>(+/-)^2 + mu eps(+/-) : eps(+/-),
* sigma0(+/-) = d psi0(+/-) / d eps = lambda <tr eps>(+/-) I + 2 mu eps(+/-),
* degradation g(phi) = (1 - phi)^2 + k   (read with +k: the printed -k makes
  the fully broken stiffness negative),
* sigma = g sigma0(+) + sigma0(-),
* tangent C = g d2psi0(+) + d2psi0(-), applied to a strain w as
      C:w = lambda [ (g-1) Theta(tr eps) + 1 ] tr(w) I
            + 2 mu [ w + (g-1) P(+):w ],
  with P(+) = d eps(+) / d eps, which in the eigenbasis multiplies the
  component (a, b) by theta_ab: Theta(zeta_a) on the diagonal, the divided
  difference (<zeta_a>+ - <zeta_b>+)/(zeta_a - zeta_b) when the two
  eigenvalues lie on different sides of zero, and Theta(zeta_a) otherwise
  (which is the exact limit there, so no division by a small difference),
* history H = max(psi0(+), Hn), active flag chi = [psi0(+) >= Hn]: a tie
  takes the loading-side derivative.  (With ties inactive the bordered
  Jacobian is singular at the warm start of every increment, where the
  committed history equals psi0(+) wherever it was active, so no strain
  reaches the damage rows while the constraint row still asks for damage.)
Theta(x) = 1 for x > 0 and 0 otherwise.  Plane strain (2D) is the 3x3
problem with zero out-of-plane strain.

Isotropic variant (`iso=True`, Sec. 5.4: no split, the whole elastic energy
psi0 = psi0(+) + psi0(-) is degraded): sigma = g sigma0, C = g C0, and
psi0 takes the place of psi0(+) as the history driver (H = max(psi0, Hn))
and sigma0 the place of sigma0(+) in d sigma / d phi.  The returned keys keep
their names: psi_p is the driving energy and sigma0p the degraded stress part.
"""

from __future__ import annotations

import numpy as np


def lame(E, nu):
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def heaviside(x):
    return (x > 0.0).astype(np.float64)


def evaluate(eps_t, phi, Hn, lam, mu, k, iso=False):
    """Point law on a tensor field eps_t (3, 3, ...) with per-voxel lam, mu.

    Returns a dict with sigma, sigma0p, psi_p, psi_m, H, chi, g and the
    eigen-decomposition used by `tangent_apply`.
    """
    E = np.moveaxis(eps_t, (0, 1), (-2, -1))            # (..., 3, 3)
    zeta, vec = np.linalg.eigh(E)                        # ascending eigenvalues
    tr = np.trace(E, axis1=-2, axis2=-1)
    trp, trm = np.maximum(tr, 0.0), np.minimum(tr, 0.0)
    zp, zm = np.maximum(zeta, 0.0), np.minimum(zeta, 0.0)
    vecT = np.swapaxes(vec, -1, -2)
    epsp = (vec * zp[..., None, :]) @ vecT
    epsm = (vec * zm[..., None, :]) @ vecT
    psi_p = 0.5 * lam * trp ** 2 + mu * np.einsum("...ij,...ij->...", epsp, epsp)
    psi_m = 0.5 * lam * trm ** 2 + mu * np.einsum("...ij,...ij->...", epsm, epsm)
    I = np.eye(3)
    s0p = (lam * trp)[..., None, None] * I + 2.0 * mu[..., None, None] * epsp
    s0m = (lam * trm)[..., None, None] * I + 2.0 * mu[..., None, None] * epsm
    g = (1.0 - phi) ** 2 + k
    if iso:                                  # the whole energy is degraded
        psi_p, psi_m = psi_p + psi_m, np.zeros_like(psi_m)
        s0p, s0m = s0p + s0m, np.zeros_like(s0m)
    sigma = g[..., None, None] * s0p + s0m
    H = np.maximum(psi_p, Hn)
    chi = (psi_p >= Hn).astype(np.float64)
    # theta_ab of the derivative of the positive part
    ta = heaviside(zeta)
    za, zb = zeta[..., :, None], zeta[..., None, :]
    pa, pb = zp[..., :, None], zp[..., None, :]
    differ = ta[..., :, None] != ta[..., None, :]
    denom = np.where(differ, za - zb, 1.0)
    theta = np.where(differ, (pa - pb) / denom,
                     np.broadcast_to(ta[..., :, None], differ.shape))
    trflag = heaviside(tr)
    if iso:                                  # P(+) = identity, Theta(tr) = 1: C = g C0
        theta = np.ones_like(theta)
        trflag = np.ones_like(trflag)
    back = lambda t: np.moveaxis(t, (-2, -1), (0, 1))   # noqa: E731
    return dict(sigma=back(sigma), sigma0p=back(s0p), sigma0m=back(s0m),
                psi_p=psi_p, psi_m=psi_m, H=H, chi=chi, g=g, tr=tr, trflag=trflag,
                vec=vec, theta=theta, lam=lam, mu=mu)


def tangent_apply(st, w_t):
    """C:w for a tensor field w_t (3, 3, ...), C at the evaluated state `st`."""
    W = np.moveaxis(w_t, (0, 1), (-2, -1))
    vec, theta = st["vec"], st["theta"]
    vecT = np.swapaxes(vec, -1, -2)
    Wp = vecT @ W @ vec                              # components in the eigenbasis
    PpW = vec @ (theta * Wp) @ vecT
    g, lam, mu = st["g"], st["lam"], st["mu"]
    trw = np.trace(W, axis1=-2, axis2=-1)
    coef = lam * ((g - 1.0) * st["trflag"] + 1.0) * trw
    out = coef[..., None, None] * np.eye(3) + 2.0 * mu[..., None, None] * (
        W + (g - 1.0)[..., None, None] * PpW)
    return np.moveaxis(out, (-2, -1), (0, 1))
