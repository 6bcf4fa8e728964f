"""Residual and tangent action of the crack-length-controlled system (oracle).

Paper Sec. 3.2: unknowns q = (eps_tilde, phi, E) with macroscopic strain
E_M = f E (Sec. 2.3, eq. `SystemDis`); residual eq. `System_CrackLength`,
crack functional eq. `CrackLenght` evaluated spectrally (eq.
`newGammaFourier`), tangent action eq. `CrackLength_linearization` with the
history derivative of eq. `Delta_history`.

Readings (the paper is silent, garbled or inconsistent):
* Signs: the Fourier symbol xi stands for the derivative i q, so the
  Helmholtz operator is (Gc/l + 2H) phi - Gc l Lap(phi) (SPD), consistent
  with the derivative of the crack density (eq. `gamFunct`).
* Gc(x) multiplies the Laplacian pointwise, as printed.
* Length control: F3 = Gamma - a (the paper's dissipation form with one
  homogeneous Gc only rescales it); its exact derivative is
  r = phi/l - l Lap(phi).
* Gamma = sum_x [phi^2/(2l) - (l/2) phi Lap(phi)] (discrete Parseval form of
  eq. `CrackLenght`, Nyquist energy kept), so that r is its exact gradient.
* An initial crack is a Dirichlet mask m (phi = 1 there): the phase-field
  rows of masked voxels become the identity and their increments are
  excluded from all couplings.
* H = max(psi0(+)(eps), Hn) with Hn the last converged history.
Fields: Mandel strain (c, nz, ny, nx), c = 3 in 2D plane strain, 6 in 3D.
"""

from __future__ import annotations

import numpy as np

from . import fourier as fo
from . import pointlaw as pl


class System:
    """Fixed data of one RVE problem (grid, phases, mask, l, k, f)."""

    def __init__(self, prob):
        self.prob = prob
        self.shape = tuple(prob.shape)
        self.ncomp = 3 if self.shape[0] == 1 else 6
        self.N = int(np.prod(self.shape))
        pid = np.asarray(prob.phase_id, dtype=np.int64).reshape(self.shape)
        E = np.array([p[0] for p in prob.phases], dtype=np.float64)[pid]
        nu = np.array([p[1] for p in prob.phases], dtype=np.float64)[pid]
        self.Gc = np.array([p[2] for p in prob.phases], dtype=np.float64)[pid]
        self.lam, self.mu = pl.lame(E, nu)
        self.m = (np.zeros(self.shape) if prob.mask is None
                  else np.asarray(prob.mask, dtype=np.float64).reshape(self.shape))
        self.l = float(prob.l)
        self.k = float(prob.k)
        self.iso = getattr(prob, "split", "spectral") == "none"
        self.scheme = getattr(prob, "projection", "rotated")
        # control F3 = w_a Gamma + w_E E - tau (eq. `FEMweights`, FFT analogue);
        # (1, 0) is the crack-length control of eq. `System_CrackLength`
        self.wa, self.wE = (float(w) for w in getattr(prob, "control_weights", (1.0, 0.0)))
        # controlled quantity: the crack length Gamma (eq. `System_CrackLength`) or
        # the dissipation D = integral of Gc gamma_f (eq. `SystemDis`, last line);
        # the two coincide up to the factor Gc for homogeneous toughness
        self.dctl = getattr(prob, "control", "length") == "dissipation"
        # heterogeneous toughness in the damage equation: the printed Gc l Lap phi
        # (pointwise Gc) or the variational l div(Gc grad phi)
        self.var = getattr(prob, "gc_form", "pointwise") == "variational"
        if self.var and self.dctl:
            raise ValueError("the variational toughness term is built for crack-length control only")
        self.f = fo.to_mandel(np.asarray(prob.f, dtype=np.float64)[:, :, None, None, None],
                              self.ncomp)[:, 0, 0, 0]
        # macroscopic conditions: "strain" (mean strain f E, Sec. 2.3) or
        # "mixed" (mean strain prescribed along f only, mean stress zero on the
        # directions orthogonal to f; the zero mode of G projects onto them)
        self.bc = getattr(prob, "macro_bc", "strain")
        if self.bc not in ("strain", "mixed"):
            raise ValueError(self.bc)
        self.free_mean = (np.asarray(prob.f, dtype=np.float64) if self.bc == "mixed" else None)

    def G(self, A):
        """The compatibility projection of the problem on a tensor field."""
        return fo.G_tensor(A, self.scheme, self.free_mean)

    def G_mandel(self, m):
        return fo.G_mandel(m, self.scheme, self.free_mean)

    def lap(self, u):
        """The Laplacian of the crack functional.  With the variational
        toughness term the crack density uses the same finite differences as
        div(Gc grad phi) (symbol -sum 4 sin^2(q/2)); otherwise the spectral
        Laplacian with the Nyquist mode kept."""
        return fo.fd_laplacian(u) if self.var else fo.laplacian(u)

    # -- helpers -----------------------------------------------------------
    def fE(self, E):
        return self.f.reshape((self.ncomp, 1, 1, 1)) * E

    def point(self, eps, phi, Hn):
        return pl.evaluate(fo.to_tensor(eps), phi, Hn, self.lam, self.mu, self.k, iso=self.iso)

    def gamma(self, phi):
        """Crack length/area Gamma(phi) (eq. `CrackLenght`, spectral form)."""
        l = self.l
        return float(np.sum(phi * phi / (2.0 * l) - 0.5 * l * phi * self.lap(phi)))

    def controlled(self, phi):
        """The controlled quantity: Gamma, or D for dissipation control."""
        return self.dissipation(phi) if self.dctl else self.gamma(phi)

    def dissipation(self, phi):
        """D = integral of Gc gamma_f (eq. `JaviGc`, middle form; unit voxels),
        gamma_f in the spectral form of `gamma`."""
        l = self.l
        return float(np.sum(self.Gc * (phi * phi / (2.0 * l) - 0.5 * l * phi * self.lap(phi))))

    # -- residual (eq. System_CrackLength) ---------------------------------
    def residual(self, eps_t, phi, E, Hn, a):
        eps = eps_t + self.fE(E)
        st = self.point(eps, phi, Hn)
        F1 = fo.to_mandel(self.G(st["sigma"]), self.ncomp)
        lap = self.lap(phi)
        l, Gc, H = self.l, self.Gc, st["H"]
        gterm = l * fo.div_k_grad(phi, Gc) if self.var else Gc * l * lap
        F2 = (1.0 - self.m) * ((Gc / l + 2.0 * H) * phi - gterm - 2.0 * H)
        dens = phi * phi / (2.0 * l) - 0.5 * l * phi * lap
        gam = float(np.sum(dens))
        Q = float(np.sum(Gc * dens)) if self.dctl else gam
        F3 = self.wa * Q + self.wE * E - a
        sig_mean = st["sigma"].reshape(3, 3, -1).mean(axis=-1)
        return dict(F1=F1, F2=F2, F3=F3, Gamma=gam, sigma_M=sig_mean, state=st,
                    r=phi / l - l * lap)

    # -- tangent action (eq. CrackLength_linearization) --------------------
    def tangent(self, eps_t, phi, E, Hn):
        """Return a function v -> J v on flat vectors [d_eps_t, d_phi, dE]."""
        eps = eps_t + self.fE(E)
        st = self.point(eps, phi, Hn)
        l, Gc, m = self.l, self.Gc, self.m
        b = -2.0 * (1.0 - phi) * st["sigma0p"]          # d sigma / d phi
        A = Gc / l + 2.0 * st["H"]
        r = phi / l - l * self.lap(phi)
        # gradient of the controlled quantity: dGamma/dphi = r; with dissipation
        # control dD/dphi = Gc phi/l - (l/2) (Gc Lap phi + Lap(Gc phi)) (the
        # Laplacian is symmetric, Gc is not constant)
        rq = (Gc * phi / l - 0.5 * l * (Gc * fo.laplacian(phi) + fo.laplacian(Gc * phi))
              if self.dctl else r)
        c, shp = self.ncomp, self.shape

        def apply(v):
            d_eps = v[: c * self.N].reshape((c,) + shp)
            d_phi = v[c * self.N: (c + 1) * self.N].reshape(shp)
            dE = v[-1]
            w = fo.to_tensor(d_eps + self.fE(dE))
            dphi_f = (1.0 - m) * d_phi
            tau = pl.tangent_apply(st, w) + b * dphi_f
            J1 = fo.to_mandel(self.G(tau), c)
            bw = np.einsum("ij...,ij...->...", b, w)
            gterm = l * fo.div_k_grad(dphi_f, Gc) if self.var else Gc * l * fo.laplacian(dphi_f)
            J2 = (1.0 - m) * (st["chi"] * bw + A * dphi_f - gterm) + m * d_phi
            J3 = self.wa * np.sum(rq * dphi_f) + self.wE * dE
            return np.concatenate([J1.ravel(), J2.ravel(), [J3]])

        return apply

    # -- flat-vector packing ----------------------------------------------
    def pack(self, F1, F2, F3):
        return np.concatenate([np.ravel(F1), np.ravel(F2), [F3]])

    def unpack(self, x):
        c, N = self.ncomp, self.N
        return (x[: c * N].reshape((c,) + self.shape),
                x[c * N: (c + 1) * N].reshape(self.shape), float(x[-1]))
