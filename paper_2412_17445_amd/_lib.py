"""ctypes binding of libpff.so (argument marshalling only).

Every function keeps the C name and signature of include/pff.h.  Loading
fails loudly when the library has not been built: there is no fallback.
"""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; PFF_LIB_PATH points at another build of the same ABI
# (side-by-side timing of two builds)
LIB_PATH = os.environ.get("PFF_LIB_PATH") or os.path.join(HERE, "libpff.so")

PFF_OK, PFF_NOT_CONVERGED, PFF_QUEUED = 0, 1, 2
PFF_ERR_ARG, PFF_ERR_OOM, PFF_ERR_DEVICE, PFF_ERR_STATE = -1, -2, -3, -4
PFF_PREC_FP64, PFF_PREC_MIXED = 0, 1
PFF_SPLIT_SPECTRAL, PFF_SPLIT_NONE = 0, 1
PFF_PROJ_ROTATED, PFF_PROJ_STANDARD = 0, 1
PFF_CONTROL_LENGTH, PFF_CONTROL_DISSIPATION = 0, 1
PFF_GC_POINTWISE, PFF_GC_VARIATIONAL = 0, 1
PFF_BC_STRAIN, PFF_BC_MIXED = 0, 1


class pff_grid(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int)]


class pff_phase(C.Structure):
    _fields_ = [("E", C.c_double), ("nu", C.c_double), ("Gc", C.c_double)]


class pff_params(C.Structure):
    _fields_ = [("l", C.c_double), ("k_resid", C.c_double), ("f", C.c_double * 9),
                ("delta_a", C.c_double), ("alpha", C.c_double), ("newton_tol", C.c_double),
                ("krylov_rtol", C.c_double), ("newton_maxit", C.c_int),
                ("krylov_maxit", C.c_int), ("precision", C.c_int), ("split", C.c_int),
                ("projection", C.c_int), ("control", C.c_int), ("gc_form", C.c_int), ("w_gamma", C.c_double),
                ("w_load", C.c_double), ("macro_bc", C.c_int), ("resid_tol", C.c_double)]


class pff_increment_result(C.Structure):
    _fields_ = [("increment", C.c_int), ("newton_iters", C.c_int), ("krylov_iters", C.c_int),
                ("converged", C.c_int), ("applies", C.c_longlong), ("applies_fp64", C.c_longlong),
                ("fp64_fallbacks", C.c_int), ("refinements", C.c_int), ("sigma_M", C.c_double * 6),
                ("load_factor", C.c_double), ("crack_length", C.c_double),
                ("target_a", C.c_double), ("err", C.c_double * 3), ("seconds", C.c_double),
                ("dissipation", C.c_double), ("resid", C.c_double * 2)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p)


class pff_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


class pff_stagger_params(C.Structure):
    _fields_ = [("tol_mech", C.c_double), ("tol_sta", C.c_double), ("cg_rtol", C.c_double),
                ("max_stagger", C.c_int), ("max_newton", C.c_int), ("cg_maxit", C.c_int)]


class pff_stagger_result(C.Structure):
    _fields_ = [("increment", C.c_int), ("converged", C.c_int), ("stagger_iters", C.c_int),
                ("newton_iters", C.c_int), ("cg_mech", C.c_longlong), ("cg_helm", C.c_longlong),
                ("E", C.c_double), ("crack_length", C.c_double), ("sigma_M", C.c_double * 6),
                ("err", C.c_double), ("seconds", C.c_double), ("dissipation", C.c_double)]


class pff_request_info(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("state", C.c_int), ("status", C.c_int),
                ("n_done", C.c_int), ("slot", C.c_int), ("footprint", C.c_size_t),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double),
                ("a0", C.c_double), ("E_s", C.c_double)]


class pff_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_longlong), ("completed", C.c_longlong),
                ("queued", C.c_longlong), ("running", C.c_longlong),
                ("max_running", C.c_longlong), ("slots", C.c_int), ("reserved", C.c_int),
                ("budget", C.c_size_t), ("bytes_in_use", C.c_size_t),
                ("peak_bytes", C.c_size_t), ("clock", C.c_double), ("batch_chunks", C.c_longlong),
                ("batch_solves", C.c_longlong), ("batch_iterations", C.c_longlong),
                ("batch_graphs", C.c_longlong), ("batch_max", C.c_int), ("reserved2", C.c_int),
                ("batch_mean", C.c_double)]


EXPORTS = {
    "pff_abi_version": (C.c_int, []),
    "pff_create": (C.c_int, [C.POINTER(pff_grid), C.POINTER(pff_phase), C.c_int, C.c_void_p,
                             C.c_void_p, C.POINTER(pff_params), C.POINTER(pff_allocator), C.c_void_p,
                             C.POINTER(C.c_void_p)]),
    "pff_bootstrap": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "pff_step": (C.c_int, [C.c_void_p, C.POINTER(pff_increment_result)]),
    "pff_effective_toughness": (C.c_int, [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                          C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "pff_stagger_defaults": (C.c_int, [C.POINTER(pff_stagger_params)]),
    "pff_stagger_step": (C.c_int, [C.c_void_p, C.c_double, C.POINTER(pff_stagger_params),
                                   C.POINTER(pff_stagger_result)]),
    "pff_get_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "pff_device_views": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                   C.POINTER(C.c_void_p)]),
    "pff_set_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                C.c_double, C.c_int]),
    "pff_residual": (C.c_int, [C.c_void_p, C.c_double, C.c_void_p, C.POINTER(C.c_double),
                               C.c_void_p, C.POINTER(C.c_double)]),
    "pff_apply_tangent": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "pff_project": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "pff_project_noalloc": (C.c_int, [C.POINTER(pff_grid), C.c_int, C.c_void_p, C.c_void_p, C.c_int,
                                      C.c_void_p]),
    "pff_krylov_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int,
                                   C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    "pff_timing": (C.c_int, [C.c_void_p, C.c_int]),
    "pff_timing_read": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_longlong),
                                  C.POINTER(C.c_double)]),
    "pff_counters": (C.c_int, [C.c_void_p, C.POINTER(C.c_longlong), C.POINTER(C.c_longlong)]),
    "pff_save": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_size_t)]),
    "pff_load": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "pff_last_error": (C.c_char_p, [C.c_void_p]),
    "pff_destroy": (None, [C.c_void_p]),
    "pff_solver_bytes": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "pff_footprint_bytes": (C.c_int, [C.POINTER(pff_grid), C.c_int, C.POINTER(C.c_size_t)]),
    "pff_server_create": (C.c_int, [C.c_size_t, C.c_int, C.POINTER(pff_allocator), C.POINTER(C.c_void_p)]),
    "pff_server_submit": (C.c_int, [C.c_void_p, C.POINTER(pff_grid), C.POINTER(pff_phase), C.c_int,
                                    C.c_void_p, C.c_void_p, C.POINTER(pff_params), C.c_int,
                                    C.POINTER(C.c_uint64)]),
    "pff_server_wait": (C.c_int, [C.c_void_p, C.c_uint64, C.c_double]),
    "pff_server_info": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(pff_request_info)]),
    "pff_server_results": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(pff_increment_result),
                                     C.c_int, C.POINTER(C.c_int)]),
    "pff_server_release": (C.c_int, [C.c_void_p, C.c_uint64]),
    "pff_server_get_stats": (C.c_int, [C.c_void_p, C.POINTER(pff_server_stats)]),
    "pff_server_last_error": (C.c_char_p, [C.c_void_p]),
    "pff_server_destroy": (None, [C.c_void_p]),
}

_lib = None


def load():
    """Load libpff.so and bind every exported function (raises if missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() or "
                           "python -m paper_2412_17445_amd.build")
    # PyTorch ships its own HIP runtime (same soname as the system one, but
    # loaded by file name).  Importing torch first makes the library bind to
    # that runtime; loaded the other way round, the process would hold two
    # HIP runtimes, and the second to initialise finds no device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
