"""pff_project_noalloc (no device allocation, scratch in a static device
array) against the existing entry point pff_project of a solver on the same
grid: the same C+1 seeded fields in, the projection G of the strain fields
and the Laplacian of the last field out, element by element (FP64 1e-12,
FP32 2e-6 relative to the largest output).  Two calls in a row on each
precision, the second on a smaller grid, so the shared scratch array is
reused with a different layout; also the size limit (host-side rejection)."""

import ctypes as C

import numpy as np
import pytest

from synth import problem_config

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _solver(shape, standard):
    from paper_2412_17445_amd import Solver
    prob = problem_config("part24" if shape[0] > 1 else "gc16")
    nz, ny, nx = shape
    return Solver(shape, [(1.0, 0.3, 1e-3)], np.zeros(shape, np.uint8), None, prob.f, 2.0,
                  projection="standard" if standard else "rotated")


def _noalloc(shape, x, standard):
    from paper_2412_17445_amd import _lib as L
    nz, ny, nx = shape
    out = torch.full_like(x, float("nan"))
    st = L.load().pff_project_noalloc(C.byref(L.pff_grid(nx, ny, nz)), 1 if standard else 0, x.data_ptr(),
                                      out.data_ptr(), 1 if x.dtype == torch.float32 else 0,
                                      C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, st
    return out


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("shapes,standard", [(((24, 24, 24), (12, 18, 16)), False),
                                             (((1, 64, 64), (1, 18, 12)), False),
                                             (((20, 18, 16), (9, 8, 6)), True),
                                             (((1, 39, 39), (1, 11, 13)), False)])
def test_noalloc_projection_equals_pff_project(shapes, standard, dtype):
    dt = getattr(torch, dtype)
    tol = 1e-12 if dtype == "float64" else 2e-6
    for k, shape in enumerate(shapes):
        s = _solver(shape, standard)
        c = s.ncomp
        g = torch.Generator(device="cuda")
        g.manual_seed(100 + k)
        x = torch.randn((c + 1) * s.N, dtype=dt, device="cuda", generator=g)
        ref = s.project(x)
        got = _noalloc(shape, x, standard)
        torch.cuda.synchronize()
        err = (got - ref).abs().max().item() / ref.abs().max().item()
        print(shape, dtype, "standard" if standard else "rotated", "rel err %.2e" % err, flush=True)
        assert err <= tol, (shape, err)
        s.close()


def test_noalloc_rejects_grids_beyond_the_scratch():
    from paper_2412_17445_amd import _lib as L
    x = torch.zeros(16, dtype=torch.float64, device="cuda")
    y = torch.zeros(16, dtype=torch.float64, device="cuda")
    lib = L.load()
    # 128^3 in double needs 7 * 65 * 128 * 128 complex doubles (119 MB) > 64 MiB
    assert lib.pff_project_noalloc(C.byref(L.pff_grid(128, 128, 128)), 0, x.data_ptr(), y.data_ptr(), 0,
                                   None) == L.PFF_ERR_ARG
    assert lib.pff_project_noalloc(C.byref(L.pff_grid(8, 8, 1)), 0, x.data_ptr(), x.data_ptr(), 0,
                                   None) == L.PFF_ERR_ARG
    assert lib.pff_project_noalloc(None, 0, x.data_ptr(), y.data_ptr(), 0, None) == L.PFF_ERR_ARG
    assert lib.pff_project_noalloc(C.byref(L.pff_grid(8, 8, 1)), 3, x.data_ptr(), y.data_ptr(), 0,
                                   None) == L.PFF_ERR_ARG
