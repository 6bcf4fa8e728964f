"""Seeded stream of RVE requests for the request server.

Each request is drawn from its own seed.
- Half are 2D fibre composites: 128^2 to 512^2 voxels, 20-45% random
  sequential adsorption disks of radius 4-12, fibre/matrix stiffness contrast
  5-20, transverse tension.
- Half are 3D cubes: 32^3 to 96^3, 10-25% non-overlapping spheres of radius
  3-8, either pores (stiffness 1e-6 of the matrix) or stiff particles
  (contrast 5-20), uniaxial tension.
- All requests: l = 1.5-2.5 voxels, 20-60 crack-length increments, mixed
  precision.

Arrivals form a Poisson process.  Grid sizes are products of 2s and 3s, and
inclusion membership is the periodic voxel-centre test of
`synth.microstructure`.
"""

from __future__ import annotations

import numpy as np

from .configs import Problem, _dyad

SIZES_2D = (128, 192, 256, 384, 512)
SIZES_3D = (32, 48, 64, 96)


def _disks(n, radius, gap, fraction, rng, max_tries=200000):
    """Periodic RSA of equal disks (vectorised rejection test)."""
    pid = np.zeros((n, n), np.uint8)
    cx = np.empty(0)
    cy = np.empty(0)
    dmin2 = (2.0 * radius + gap) ** 2
    ax = np.arange(n) + 0.5
    covered = 0
    tries = 0
    while covered < fraction * n * n:
        tries += 1
        if tries > max_tries:
            break
        x, y = rng.uniform(0, n, size=2)
        if cx.size:
            dx = np.abs(cx - x)
            dx = np.minimum(dx, n - dx)
            dy = np.abs(cy - y)
            dy = np.minimum(dy, n - dy)
            if np.any(dx * dx + dy * dy < dmin2):
                continue
        cx, cy = np.append(cx, x), np.append(cy, y)
        ix = np.arange(int(np.floor(x - radius - 1)), int(np.ceil(x + radius + 1)) + 1) % n
        iy = np.arange(int(np.floor(y - radius - 1)), int(np.ceil(y + radius + 1)) + 1) % n
        ddx = np.abs(ax[ix] - x)
        ddx = np.minimum(ddx, n - ddx)
        ddy = np.abs(ax[iy] - y)
        ddy = np.minimum(ddy, n - ddy)
        inside = (ddy[:, None] ** 2 + ddx[None, :] ** 2) <= radius * radius
        sub = np.ix_(iy, ix)
        block = pid[sub]
        covered += int((inside & (block == 0)).sum())
        block[inside] = 1
        pid[sub] = block
    return pid[None]


def _spheres(n, rmin, rmax, fraction, rng, gap=1.0, max_tries=200000):
    """Periodic non-overlapping spheres (vectorised rejection test)."""
    pid = np.zeros((n, n, n), np.uint8)
    cen = np.empty((0, 3))
    rad = np.empty(0)
    ax = np.arange(n) + 0.5
    covered = 0
    tries = 0
    while covered < fraction * n ** 3:
        tries += 1
        if tries > max_tries:
            break
        r = rng.uniform(rmin, rmax)
        c = rng.uniform(0, n, size=3)
        if rad.size:
            d = np.abs(cen - c)
            d = np.minimum(d, n - d)
            if np.any((d * d).sum(axis=1) < (r + rad + gap) ** 2):
                continue
        cen = np.vstack([cen, c])
        rad = np.append(rad, r)
        idx = [np.arange(int(np.floor(c[k] - r - 1)), int(np.ceil(c[k] + r + 1)) + 1) % n
               for k in range(3)]
        dd = []
        for k in range(3):
            t = np.abs(ax[idx[k]] - c[k])
            dd.append(np.minimum(t, n - t) ** 2)
        inside = (dd[2][:, None, None] + dd[1][None, :, None] + dd[0][None, None, :]) <= r * r
        sub = np.ix_(idx[2], idx[1], idx[0])
        block = pid[sub]
        covered += int((inside & (block == 0)).sum())
        block[inside] = 1
        pid[sub] = block
    return pid


def served_request(seed, inc_scale=1.0):
    """(Problem, number of increments) of request `seed`."""
    rng = np.random.Generator(np.random.PCG64(1000003 + seed))
    l = float(rng.uniform(1.5, 2.5))
    contrast = float(rng.uniform(5.0, 20.0))
    n_inc = max(1, int(round(int(rng.integers(20, 61)) * inc_scale)))
    if rng.random() < 0.5:
        n = int(rng.choice(SIZES_2D))
        radius = int(rng.integers(4, 13))
        frac = float(rng.uniform(0.20, 0.45))
        pid = _disks(n, radius, 2.0, frac, rng)
        prob = Problem(
            name=f"request{seed}", shape=(1, n, n),
            phases=[(1.0, 0.35, 1e-3), (contrast, 0.2, 1e-2)], phase_id=pid, mask=None,
            f=_dyad(1, 1), l=l, delta_a=2.0, n_increments=n_inc, alpha=1.0,
            precision="mixed", krylov_rtol=1e-5,
            notes=f"2D {n}^2 fibres r={radius} {frac:.2f} contrast {contrast:.1f}")
    else:
        n = int(rng.choice(SIZES_3D))
        frac = float(rng.uniform(0.10, 0.25))
        rmax = min(8.0, n / 6.0)
        pid = _spheres(n, min(3.0, rmax), rmax, frac, rng)
        pores = rng.random() < 0.5
        phases = ([(1.0, 0.3, 1e-3), (1e-6, 0.3, 1e-3)] if pores
                  else [(1.0, 0.3, 1e-3), (contrast, 0.2, 5e-3)])
        prob = Problem(
            name=f"request{seed}", shape=(n, n, n), phases=phases, phase_id=pid, mask=None,
            f=_dyad(2, 2), l=l, delta_a=4.0, n_increments=n_inc, alpha=0.9,
            precision="mixed", krylov_rtol=1e-5,
            notes=f"3D {n}^3 {'pores' if pores else 'particles'} {frac:.2f}")
    return prob, n_inc


def arrival_times(n_requests, rate, seed=0):
    """Poisson arrivals (seconds from the start), `rate` requests per second."""
    rng = np.random.Generator(np.random.PCG64(77 + seed))
    return np.cumsum(rng.exponential(1.0 / rate, size=n_requests))
