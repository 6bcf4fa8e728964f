"""Effective toughness from the macroscopic response (oracle).

Test infrastructure only: imported by tests/, never by the product path.

Paper Sec. 2.4, eq. `JaviGc`: once the crack has crossed the cell the
elastic energy is gone and the external work equals the energy of the
created crack, so G_Ceff = (1/L_g) * (work), with the work the area under
the macroscopic curve, the integral of Sigma_M : f dE.

Readings:
* The printed right-hand side is a work per unit volume; it is multiplied by
  the cell volume (N unit voxels) to match the middle form, an energy.
* The integral follows the path in its order, from the unloaded state
  (E = 0, Sigma = 0), by the trapezoidal rule over the converged increments;
  segments where E decreases (snap-backs) count negative.
* L_g is a caller input: the cell length across the crack path, less the
  initial crack where the path starts from one (the crack length developed,
  as in the Griffith panel study of Sec. 5.2).
"""

from __future__ import annotations

import numpy as np


def contract(sigma, f):
    """Sigma : f for a 3x3 tensor or the 6-vector (11, 22, 33, 23, 13, 12)."""
    s = np.asarray(sigma, dtype=np.float64)
    if s.shape == (6,):
        s = np.array([[s[0], s[5], s[4]], [s[5], s[1], s[3]], [s[4], s[3], s[2]]])
    return float(np.sum(s * np.asarray(f, dtype=np.float64)))


def work_integral(E, sigma, f):
    """Area under the macroscopic curve: integral of Sigma : f dE along the path."""
    e_prev, s_prev, w = 0.0, 0.0, 0.0
    for e, sig in zip(E, sigma):
        s = contract(sig, f)
        w += 0.5 * (s + s_prev) * (float(e) - e_prev)
        e_prev, s_prev = float(e), s
    return w


def effective_toughness(E, sigma, f, volume, L_g):
    """G_Ceff = volume * work / L_g (eq. `JaviGc`)."""
    return volume * work_integral(E, sigma, f) / L_g
