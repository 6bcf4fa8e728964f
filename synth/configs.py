"""Problem definitions of the benchmark workloads and of small parity cases.

A problem is the paper's statement of the RVE problem (Sec. 2.3 and Sec. 3.2):
a periodic voxel grid with a phase per voxel, per-phase Young modulus,
Poisson ratio and toughness Gc (as in Table 2), the length scale l, the
loading-direction tensor f (Table 1), the crack-length increment per step and
the solver controls.  The values themselves are synthetic stand-ins for the
paper's figure-only geometries (the fibre composite, porous and 3D cases of
Sec. 5); voxel units throughout (h = 1).
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

from .microstructure import (
    disks_rsa,
    line_crack_mask,
    penny_crack_mask,
    spheres_random,
)


def _dyad(a, b):
    t = np.zeros((3, 3))
    t[a, b] += 0.5
    t[b, a] += 0.5
    return t


@dataclass
class Problem:
    name: str
    shape: Tuple[int, int, int]          # (nz, ny, nx); nz == 1 means 2D plane strain
    phases: List[Tuple[float, float, float]]  # (E, nu, Gc) per phase id
    phase_id: np.ndarray                 # uint8, shape `shape`
    mask: Optional[np.ndarray]           # uint8 crack mask (phi == 1 there) or None
    f: np.ndarray                        # 3x3 symmetric loading direction
    l: float = 2.0
    k: float = 1e-6
    delta_a: float = 1.0
    n_increments: int = 10
    alpha: float = 1.0
    newton_tol: float = 1e-8
    newton_maxit: int = 50
    krylov_rtol: float = 1e-10
    krylov_maxit: int = 5000
    precision: str = "fp64"              # "fp64" or "mixed"
    split: str = "spectral"              # "spectral" (Miehe split) or "none" (isotropic degradation)
    projection: str = "rotated"          # "rotated" (Willot) or "standard" frequencies in G
    control_weights: Tuple[float, float] = (1.0, 0.0)   # (w_a, w_E): F3 = w_a Gamma + w_E E - tau
    control: str = "length"              # controlled quantity: "length" (Gamma) or "dissipation" (D)
    gc_form: str = "pointwise"           # "pointwise" Gc l Lap phi or "variational" l div(Gc grad phi)
    macro_bc: str = "strain"             # "strain" (mean strain f E) or "mixed" (stress-free off f)
    notes: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def dim(self) -> int:
        return 2 if self.shape[0] == 1 else 3

    @property
    def nvox(self) -> int:
        return int(np.prod(self.shape))


CONFIG_NAMES = ("crack2d_64", "fibres2d_256", "pores3d_64",
                "particles3d_128")


def problem_config(name: str) -> Problem:
    """Return the seeded problem called `name` (benchmark or parity case).
    Suffixes: "_iso" gives the same problem with the isotropic (no split)
    degradation of Sec. 5.4, "_std" with the standard-frequency projection,
    "_w" with the weighted control 0.7 Gamma + 3 E, "_d" with dissipation
    control (increment delta_a times the smallest Gc), "_v" with the
    variational toughness term l div(Gc grad phi), "_m" with mixed
    macroscopic conditions (mean stress zero off the loading direction)."""
    if name.endswith("_m"):
        prob = problem_config(name[:-2])
        prob.name, prob.macro_bc = name, "mixed"
        prob.notes = (prob.notes + "; " if prob.notes else "") + "mixed macroscopic conditions"
        return prob
    if name.endswith("_v"):
        prob = problem_config(name[:-2])
        prob.name, prob.gc_form = name, "variational"
        prob.notes = (prob.notes + "; " if prob.notes else "") + "variational toughness term"
        return prob
    if name.endswith("_d"):
        prob = problem_config(name[:-2])
        prob.name, prob.control = name, "dissipation"
        prob.delta_a = prob.delta_a * min(ph[2] for ph in prob.phases)
        prob.notes = (prob.notes + "; " if prob.notes else "") + "dissipation control"
        return prob
    if name.endswith("_w"):
        prob = problem_config(name[:-2])
        prob.name, prob.control_weights = name, (0.7, 3.0)
        prob.notes = (prob.notes + "; " if prob.notes else "") + "weighted control 0.7 Gamma + 3 E"
        return prob
    if name.endswith("_std"):
        prob = problem_config(name[:-4])
        prob.name, prob.projection = name, "standard"
        prob.notes = (prob.notes + "; " if prob.notes else "") + "standard-frequency projection"
        return prob
    if name.endswith("_iso"):
        prob = problem_config(name[:-4])
        prob.name, prob.split = name, "none"
        prob.notes = (prob.notes + "; " if prob.notes else "") + "isotropic degradation (no split)"
        return prob
    if name == "crack2d_64":
        n = 64
        return Problem(
            name=name, shape=(1, n, n), phases=[(1.0, 0.3, 1e-3)],
            phase_id=np.zeros((1, n, n), np.uint8),
            mask=line_crack_mask(n, n, 32, 24, 40), f=_dyad(1, 1), l=2.0,
            delta_a=1.0, n_increments=30, alpha=1.0, newton_tol=1e-8,
            notes="homogeneous 64^2, centred 16-voxel crack, uniaxial yy")
    if name == "fibres2d_256":
        n = 256
        pid, _ = disks_rsa(n, n, radius=8, min_gap=2, target_fraction=0.30, seed=2)
        return Problem(
            name=name, shape=(1, n, n),
            phases=[(1.0, 0.35, 1e-3), (10.0, 0.2, 1e-2)], phase_id=pid, mask=None,
            f=_dyad(1, 1), l=2.0, delta_a=2.0, n_increments=100, alpha=1.0,
            notes="256^2 fibre composite, 30% RSA disks r=8 gap 2, transverse tension")
    if name == "pores3d_64":
        n = 64
        pid, _ = spheres_random(n, 3.0, 6.0, 0.15, seed=3, gap=1.0)
        return Problem(
            name=name, shape=(n, n, n),
            phases=[(1.0, 0.3, 1e-3), (1e-6, 0.3, 1e-3)], phase_id=pid, mask=None,
            f=_dyad(2, 2), l=1.5, delta_a=4.0, n_increments=60, alpha=0.9,
            precision="mixed", krylov_rtol=1e-5,
            notes="64^3 porous, 15% spherical pores r~U[3,6]")
    if name == "pores3d_105":
        # stand-in for the paper's 3D porous case (Sec. 5.5: 105^3 voxels,
        # 8 random spherical voids, 20% porosity); 105 = 3 * 5 * 7 takes
        # generic radix-5 and radix-7 FFT stages
        n = 105
        pid, _ = spheres_random(n, 0.0, 0.0, 0.199, seed=5, gap=2.0, fixed_radius=19.05)
        return Problem(
            name=name, shape=(n, n, n),
            phases=[(1.0, 0.3, 1e-3), (1e-6, 0.3, 1e-3)], phase_id=pid, mask=None,
            f=_dyad(2, 2), l=1.5, delta_a=8.0, n_increments=40, alpha=0.9,
            precision="mixed", krylov_rtol=1e-5,
            notes="105^3 porous, 8 spherical voids r=19.05, ~20%")
    if name == "particles3d_128":
        n = 128
        pid, _ = spheres_random(n, 6.0, 6.0, 0.25, seed=4, gap=1.0, fixed_radius=6.0)
        f = _dyad(2, 2) + 0.3 * (2.0 * _dyad(0, 2))
        return Problem(
            name=name, shape=(n, n, n),
            phases=[(1.0, 0.3, 1e-3), (8.0, 0.2, 5e-3)], phase_id=pid,
            mask=penny_crack_mask(n, 64, 64, 64, 10), f=f, l=2.0, delta_a=8.0,
            n_increments=80, alpha=0.9, precision="mixed", krylov_rtol=1e-5,
            notes="128^3 particle composite 25%, penny crack R=10, eps_zz:eps_xz=1:0.3")
    # ---- small parity cases ------------------------------------------------
    if name == "tiny16":
        n = 16
        return Problem(
            name=name, shape=(1, n, n), phases=[(1.0, 0.3, 1e-3)],
            phase_id=np.zeros((1, n, n), np.uint8),
            mask=line_crack_mask(n, n, 8, 6, 10), f=_dyad(1, 1), l=1.5,
            delta_a=0.5, n_increments=4)
    if name == "crack2d_39":
        # one of the paper's grid sizes (Sec. 5.1 uses 39^2, 77^2, 155^2):
        # 39 = 3 * 13 takes a generic radix-13 FFT stage
        n = 39
        return Problem(
            name=name, shape=(1, n, n), phases=[(1.0, 0.3, 1e-3)],
            phase_id=np.zeros((1, n, n), np.uint8),
            mask=line_crack_mask(n, n, 19, 14, 25), f=_dyad(1, 1), l=2.0,
            delta_a=1.0, n_increments=4,
            notes="homogeneous 39^2, centred 11-voxel crack, uniaxial yy")
    if name == "pore35":
        # 35 = 5 * 7: radix-5 and radix-7 stages on all three axes
        n = 35
        pid, _ = spheres_random(n, 3.0, 4.5, 0.12, seed=14, gap=1.0)
        return Problem(
            name=name, shape=(n, n, n),
            phases=[(1.0, 0.3, 1e-3), (1e-6, 0.3, 1e-3)], phase_id=pid, mask=None,
            f=_dyad(2, 2), l=1.5, delta_a=2.0, n_increments=2, alpha=0.9)
    if name == "gc16":
        n = 16
        pid = np.zeros((1, n, n), np.uint8)
        pid[..., n // 2:] = 1
        return Problem(
            name=name, shape=(1, n, n), phases=[(1.0, 0.3, 3e-3), (1.0, 0.3, 1e-3)],
            phase_id=pid, mask=line_crack_mask(n, n, 8, 6, 10), f=_dyad(1, 1), l=1.5,
            delta_a=0.5, n_increments=4,
            notes="16^2, centred crack between a tough (x < 8) and a weak half: one tip grows")
    if name == "fib64":
        n = 64
        pid, _ = disks_rsa(n, n, radius=5, min_gap=2, target_fraction=0.25, seed=11)
        return Problem(
            name=name, shape=(1, n, n),
            phases=[(1.0, 0.35, 1e-3), (10.0, 0.2, 1e-2)], phase_id=pid,
            mask=line_crack_mask(n, n, 32, 28, 36), f=_dyad(1, 1), l=2.0,
            delta_a=1.0, n_increments=5)
    if name == "pore24":
        n = 24
        pid, _ = spheres_random(n, 2.5, 4.0, 0.12, seed=12, gap=1.0)
        return Problem(
            name=name, shape=(n, n, n),
            phases=[(1.0, 0.3, 1e-3), (1e-6, 0.3, 1e-3)], phase_id=pid, mask=None,
            f=_dyad(2, 2), l=1.5, delta_a=2.0, n_increments=3, alpha=0.9)
    if name == "part12":                 # the part24 recipe on a 12^3 cell (a quick 3D parity case)
        n = 12
        pid, _ = spheres_random(n, 2.0, 2.0, 0.15, seed=13, gap=1.0, fixed_radius=2.0)
        f = _dyad(2, 2) + 0.3 * (2.0 * _dyad(0, 2))
        return Problem(
            name=name, shape=(n, n, n),
            phases=[(1.0, 0.3, 1e-3), (8.0, 0.2, 5e-3)], phase_id=pid,
            mask=penny_crack_mask(n, 6, 6, 6, 2), f=f, l=1.5, delta_a=1.0,
            n_increments=3, alpha=0.9)
    if name == "part24":
        n = 24
        pid, _ = spheres_random(n, 3.0, 3.0, 0.15, seed=13, gap=1.0, fixed_radius=3.0)
        f = _dyad(2, 2) + 0.3 * (2.0 * _dyad(0, 2))
        return Problem(
            name=name, shape=(n, n, n),
            phases=[(1.0, 0.3, 1e-3), (8.0, 0.2, 5e-3)], phase_id=pid,
            mask=penny_crack_mask(n, 12, 12, 12, 3), f=f, l=2.0, delta_a=2.0,
            n_increments=3, alpha=0.9)
    raise KeyError(name)
