"""Seeded random states and Krylov vectors for single-operator parity tests.

Smooth random fields are made by box-averaging white noise a few times on the
periodic grid (a plain moving average, no spectral arithmetic), so that they
have the spatial correlation of a real solution without depending on any
operator of the method.
"""

from __future__ import annotations

import numpy as np


def smooth_field(shape, rng, passes=3):
    a = rng.standard_normal(shape)
    for _ in range(passes):
        b = a.copy()
        for ax in range(len(shape)):
            if shape[ax] > 1:
                b = b + np.roll(a, 1, axis=ax) + np.roll(a, -1, axis=ax)
        a = b / (1.0 + 2.0 * sum(1 for s in shape if s > 1))
    return a / (np.abs(a).max() + 1e-300)


def random_state(shape, ncomp, seed, strain_scale=0.01, f_mandel=None, E=None):
    """A frozen Newton state: total strain (Mandel, ncomp x shape), damage in
    [0, 0.9], committed history >= 0 and the load factor.

    The strain is f*E plus a smooth fluctuation of relative size 0.3, mixing
    signs so that both branches of the strain split occur.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    if E is None:
        E = strain_scale
    eps = np.stack([smooth_field(shape, rng) for _ in range(ncomp)]) * (0.3 * strain_scale)
    if f_mandel is not None:
        eps = eps + np.asarray(f_mandel).reshape((ncomp,) + (1,) * len(shape)) * E
    phi = 0.45 * (1.0 + smooth_field(shape, rng))
    phi = np.clip(phi, 0.0, 0.9)
    Hn = 0.5 * (strain_scale ** 2) * np.abs(smooth_field(shape, rng))
    return eps, phi, Hn, float(E)


def random_vector(n, seed, scale=1.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(n) * scale
