"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This package holds only input generation: voxel microstructures (phase ids),
initial-crack masks, the problem definitions of the benchmark workloads and
seeded random states/vectors for parity tests.  It contains none of the
method's arithmetic (no projection, no constitutive law, no solver), so that
the oracle and the GPU path can both draw identical inputs from it without
sharing any computation.
"""

from .microstructure import (  # noqa: F401
    disks_rsa,
    spheres_random,
    line_crack_mask,
    penny_crack_mask,
    laminate_x,
)
from .configs import Problem, problem_config, CONFIG_NAMES  # noqa: F401
from .states import random_state, random_vector, smooth_field  # noqa: F401
