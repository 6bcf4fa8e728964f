"""MI355X-native crack-length-controlled phase-field FFT solver.

The compute path is the HIP library libpff.so (C ABI in include/pff.h);
this package only builds it and marshals arguments to it.
"""

from ._lib import load as load_library  # noqa: F401
from .solver import (PffError, Server, Solver, effective_toughness, footprint_bytes,  # noqa: F401
                     problem_kwargs)

__all__ = ["Solver", "Server", "PffError", "effective_toughness", "footprint_bytes", "problem_kwargs",
           "load_library"]
