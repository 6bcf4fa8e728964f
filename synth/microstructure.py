"""Seeded voxel microstructures and initial-crack masks.

Arrays are indexed [z, y, x] (x fastest in memory); a 2D grid has nz == 1.
Membership of a voxel in an inclusion is decided by its centre, with periodic
minimum-image distances, the way the paper's periodic RVEs are built (random
sequential adsorption of fibres for the composites of Sec. 5.1/5.2, random
spherical voids for the porous RVE of Sec. 5.3).
"""

from __future__ import annotations

import numpy as np


def _periodic_d2(coords, centre, lengths):
    d2 = np.zeros(coords[0].shape, dtype=np.float64)
    for c, x0, L in zip(coords, centre, lengths):
        d = np.abs(c - x0)
        d = np.minimum(d, L - d)
        d2 = d2 + d * d
    return d2


def _min_image(a, b, L):
    d = np.abs(a - b)
    return np.minimum(d, L - d)


def disks_rsa(nx, ny, radius, min_gap, target_fraction, seed, max_tries=200000):
    """Random sequential adsorption of equal disks on a periodic nx*ny grid.

    Disks of `radius` voxels are inserted at uniform random centres; a new disk
    is rejected if its centre distance to any accepted disk is below
    2*radius + min_gap.  Insertion stops once the voxel fraction covered by
    disks reaches `target_fraction`.  Returns uint8 phase ids (1 = disk) of
    shape (1, ny, nx) and the list of centres.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    yy, xx = np.meshgrid(np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    pid = np.zeros((ny, nx), dtype=np.uint8)
    centres = []
    dmin = 2.0 * radius + min_gap
    tries = 0
    while pid.mean() < target_fraction:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("RSA jammed before reaching the target fraction")
        cx, cy = rng.uniform(0, nx), rng.uniform(0, ny)
        ok = True
        for (ax, ay) in centres:
            dx = _min_image(cx, ax, nx)
            dy = _min_image(cy, ay, ny)
            if dx * dx + dy * dy < dmin * dmin:
                ok = False
                break
        if not ok:
            continue
        centres.append((cx, cy))
        d2 = _periodic_d2((xx, yy), (cx, cy), (nx, ny))
        pid[d2 <= radius * radius] = 1
    return pid[None, :, :], centres


def spheres_random(n, rmin, rmax, target_fraction, seed, gap=1.0, fixed_radius=None,
                   max_tries=400000):
    """Non-overlapping random spheres in a periodic n^3 cube.

    Radii are uniform in [rmin, rmax] (or all equal to `fixed_radius`); a
    sphere is rejected when its centre distance to an accepted one is below
    r_i + r_j + gap.  Insertion stops when the covered voxel fraction reaches
    `target_fraction`.  Returns uint8 ids (1 = sphere) of shape (n, n, n).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    ax = np.arange(n) + 0.5
    zz, yy, xx = np.meshgrid(ax, ax, ax, indexing="ij")
    pid = np.zeros((n, n, n), dtype=np.uint8)
    spheres = []
    tries = 0
    covered = 0
    while covered < target_fraction * pid.size:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("sphere packing jammed before reaching the target")
        r = fixed_radius if fixed_radius is not None else rng.uniform(rmin, rmax)
        c = rng.uniform(0, n, size=3)
        ok = True
        for (s, rs) in spheres:
            d = _min_image(c, s, n)
            if np.dot(d, d) < (r + rs + gap) ** 2:
                ok = False
                break
        if not ok:
            continue
        spheres.append((c, r))
        # only touch a bounding box around the sphere (periodic wrap)
        lo = np.floor(c - r - 1).astype(int)
        hi = np.ceil(c + r + 1).astype(int)
        iz = np.arange(lo[2], hi[2] + 1) % n
        iy = np.arange(lo[1], hi[1] + 1) % n
        ix = np.arange(lo[0], hi[0] + 1) % n
        sub = np.ix_(iz, iy, ix)
        d2 = _periodic_d2((xx[sub], yy[sub], zz[sub]), c, (n, n, n))
        block = pid[sub]
        newly = (d2 <= r * r) & (block == 0)
        covered += int(newly.sum())
        block[d2 <= r * r] = 1
        pid[sub] = block
    return pid, spheres


def line_crack_mask(nx, ny, y, x0, x1):
    """Crack mask of one voxel row: voxels (x, y) with x0 <= x < x1."""
    m = np.zeros((1, ny, nx), dtype=np.uint8)
    m[0, y, x0:x1] = 1
    return m


def penny_crack_mask(n, z, cx, cy, radius):
    """Penny-shaped crack mask in the plane z: (x - cx)^2 + (y - cy)^2 <= R^2."""
    m = np.zeros((n, n, n), dtype=np.uint8)
    yy, xx = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    m[z] = (((xx - cx) ** 2 + (yy - cy) ** 2) <= radius * radius).astype(np.uint8)
    return m


def laminate_x(nx, ny, nz, width, period):
    """Layers normal to x: phase 1 where (x mod period) < width."""
    pid = np.zeros((nz, ny, nx), dtype=np.uint8)
    x = np.arange(nx)
    pid[:, :, (x % period) < width] = 1
    return pid
