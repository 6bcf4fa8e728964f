"""Host-side checks of the C ABI (no GPU needed).

The library must load, export every function that include/pff.h declares
with the binding's names, and reject invalid arguments before touching the
device.
"""

import ctypes as C
import os
import re

import pytest

from paper_2412_17445_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pff.h")

pytestmark = pytest.mark.skipif(not os.path.exists(L.LIB_PATH),
                                reason="libpff.so not built (run __graft_entry__.build())")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pff_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(L.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = L.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert lib.pff_abi_version() == 4


def test_struct_layouts():
    assert C.sizeof(L.pff_grid) == 12
    assert C.sizeof(L.pff_phase) == 24
    # 2 doubles + f[9] + 4 doubles, 7 ints (+ padding), 2 doubles, macro_bc (+ padding), resid_tol
    assert C.sizeof(L.pff_params) == 8 * (2 + 9 + 4) + 4 * 7 + 4 + 8 * 2 + 4 + 4 + 8
    assert C.sizeof(L.pff_increment_result) == 4 * 4 + 8 * 2 + 4 * 2 + 8 * (6 + 3 + 3 + 2 + 2)
    assert C.sizeof(L.pff_allocator) == 3 * 8


STRUCTS = ["pff_grid", "pff_phase", "pff_params", "pff_increment_result", "pff_stagger_params",
           "pff_stagger_result", "pff_request_info", "pff_server_stats", "pff_allocator"]


def test_ctypes_layouts_match_the_c_compiler(tmp_path):
    """sizeof and every field offset of the header's structs, as gcc lays
    them out, equal the ctypes mirrors of the binding."""
    import shutil
    import subprocess
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pff.h"', "int main(void) {"]
    want = []
    for name in STRUCTS:
        cls = getattr(L, name)
        lines.append(f'  printf("%zu\\n", sizeof({name}));')
        want.append(C.sizeof(cls))
        for fname, _ in cls._fields_:
            lines.append(f'  printf("%zu\\n", offsetof({name}, {fname}));')
            want.append(getattr(cls, fname).offset)
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", inc, str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    assert got == want


def _params(**kw):
    p = L.pff_params()
    p.l, p.k_resid, p.delta_a, p.alpha = 2.0, 1e-6, 1.0, 1.0
    p.newton_tol, p.krylov_rtol, p.newton_maxit, p.krylov_maxit = 1e-8, 1e-10, 50, 100
    p.f[4] = 1.0
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _create(grid, phases, pid, params):
    lib = L.load()
    h = C.c_void_p()
    ph = (L.pff_phase * len(phases))(*phases)
    st = lib.pff_create(C.byref(grid), ph, len(phases), pid, None, C.byref(params), None, None,
                        C.byref(h))
    return st, h


def test_invalid_arguments_rejected_before_device_work():
    lib = L.load()
    h = C.c_void_p()
    assert lib.pff_create(None, None, 0, None, None, None, None, None, C.byref(h)) == L.PFF_ERR_ARG
    pid = (C.c_ubyte * 64)()
    ok_phase = [L.pff_phase(1.0, 0.3, 1e-3)]
    # grid lengths above the 512 limit of the FFT tiles, and below the minimum
    big = (C.c_ubyte * (1024 * 8))()
    st, h = _create(L.pff_grid(1024, 8, 1), ok_phase, big, _params())
    assert st == L.PFF_ERR_ARG and not h.value
    st, h = _create(L.pff_grid(1, 8, 1), ok_phase, pid, _params())
    assert st == L.PFF_ERR_ARG and not h.value
    # unknown model and control options
    for opt in ("split", "projection", "control", "precision", "gc_form", "macro_bc"):
        st, h = _create(L.pff_grid(8, 8, 1), ok_phase, pid, _params(**{opt: 7}))
        assert st == L.PFF_ERR_ARG, opt
    st, h = _create(L.pff_grid(8, 8, 1), ok_phase, pid, _params(w_gamma=-1.0))
    assert st == L.PFF_ERR_ARG
    for bad in (-1e-11, float("nan"), float("inf")):   # parity-mode residual tolerance
        st, h = _create(L.pff_grid(8, 8, 1), ok_phase, pid, _params(resid_tol=bad))
        assert st == L.PFF_ERR_ARG, bad
    # an allocator with only one of its two functions
    half = L.pff_allocator(L.ALLOC_FN(lambda n, c: None), L.FREE_FN(), None)
    ph = (L.pff_phase * 1)(*ok_phase)
    st = lib.pff_create(C.byref(L.pff_grid(8, 8, 1)), ph, 1, pid, None, C.byref(_params()), C.byref(half),
                        None, C.byref(h))
    assert st == L.PFF_ERR_ARG and not h.value
    assert lib.pff_server_create(1 << 20, 1, C.byref(half), C.byref(h)) == L.PFF_ERR_ARG
    st, h = _create(L.pff_grid(8, 8, 1), ok_phase, pid, _params(gc_form=1, control=1))
    assert st == L.PFF_ERR_ARG                    # variational term with dissipation control
    p = _params(macro_bc=1)
    for i in range(9):
        p.f[i] = 0.0
    st, h = _create(L.pff_grid(8, 8, 1), ok_phase, pid, p)
    assert st == L.PFF_ERR_ARG                    # mixed conditions without a loading direction
    # too many phases
    st, h = _create(L.pff_grid(8, 8, 1), ok_phase * 17, pid, _params())
    assert st == L.PFF_ERR_ARG
    # relaxation out of range
    st, h = _create(L.pff_grid(8, 8, 1), ok_phase, pid, _params(alpha=1.5))
    assert st == L.PFF_ERR_ARG
    # asymmetric f
    p = _params()
    p.f[1] = 0.5
    st, h = _create(L.pff_grid(8, 8, 1), ok_phase, pid, p)
    assert st == L.PFF_ERR_ARG
    # 2D with out-of-plane loading
    p = _params()
    p.f[8] = 1.0
    st, h = _create(L.pff_grid(8, 8, 1), ok_phase, pid, p)
    assert st == L.PFF_ERR_ARG
    # null handle calls
    assert lib.pff_step(None, None) == L.PFF_ERR_ARG
    assert lib.pff_device_views(None, None, None, None) == L.PFF_ERR_ARG
    assert lib.pff_last_error(None).startswith(b"pff_create")   # the last failed create on this thread
    lib.pff_destroy(None)
