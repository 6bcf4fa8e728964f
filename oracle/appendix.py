"""Fourier amplification factor of the crack functional (oracle).

Paper Appendix A.1: the regularised crack profile across a straight crack is
sampled on N voxels of a periodic line, its crack functional Gamma_x is
evaluated from the discrete Fourier coefficients (derivative symbol
i 2 pi k / L), and the ratio to the exact unit value defines the
amplification factor A(l/h); a least-squares fit of 1 + a/(l/h) gives the
paper's a.

Readings: the printed profile exponent |x - a|/(2 l) does not minimise the
functional of eq. `CrackLenght` (it gives Gamma = 1.25 per unit length); the
minimiser exp(-|x - a|/l), whose exact Gamma is 1, is used.  The garbled
bracket of eqs. `AP2_Int1`/`AP2_Int3` is read as
    Gamma_x = (h/N) sum_k |phi_k|^2 [1/(2l) + (l/2)(2 pi k / L)^2],
with the frequencies k in the symmetric range (Nyquist kept for even N).
"""

from __future__ import annotations

import numpy as np


def profile(N, l, h=1.0, centre=0.0):
    x = (np.arange(N) * h) - centre
    L = N * h
    d = np.abs((x + 0.5 * L) % L - 0.5 * L)       # periodic distance to the centre
    return np.exp(-d / l)


def gamma_fourier(phi, l, h=1.0):
    N = phi.size
    L = N * h
    ph = np.fft.fft(phi)
    k = np.fft.fftfreq(N) * N
    q = 2.0 * np.pi * k / L
    return float((h / N) * np.sum(np.abs(ph) ** 2 * (1.0 / (2.0 * l) + 0.5 * l * q * q)))


def amplification(l_over_h, N=257):
    return gamma_fourier(profile(N, float(l_over_h)), float(l_over_h))


def fit_a(l_values, N=257):
    """Least-squares a of A(l/h) = 1 + a / (l/h)."""
    x = 1.0 / np.asarray(l_values, dtype=np.float64)
    A = np.array([amplification(v, N) for v in l_values])
    return float(np.dot(x, A - 1.0) / np.dot(x, x)), A
