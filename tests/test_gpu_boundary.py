"""The boundary's memory contract, through the C ABI on the GPU.

* Every device buffer of a solver comes from the caller's allocator: with
  PyTorch's caching allocator behind pff_allocator, the bytes the library
  requests equal pff_solver_bytes and pff_footprint_bytes, and the solver's
  fields count in torch.cuda.memory_allocated(); destroying the solver hands
  every block back.
* pff_device_views lends the committed state: after an increment the
  borrowed eps_tilde / phi / Hn memory holds exactly what pff_get_state
  copies out (eps_tilde plus f E is the total strain it reports).
* With the library's own hipMalloc (allocator NULL) the results are the
  same bits.
"""

import ctypes as C

import numpy as np
import pytest

from synth import problem_config

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _d2h(ptr, n):
    """Copy n doubles from a device address to the host (hipMemcpy through
    torch's untyped storage is not available for a foreign pointer)."""
    hip = C.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    hip.hipMemcpy.restype = C.c_int
    out = np.empty(n)
    assert hip.hipMemcpy(out.ctypes.data, ptr, n * 8, 2) == 0      # hipMemcpyDeviceToHost
    return out


@pytest.mark.parametrize("case,precision", [("tiny16", "fp64"), ("pore24", "mixed")])
def test_allocator_receives_every_buffer(case, precision):
    from paper_2412_17445_amd import Solver, footprint_bytes
    from paper_2412_17445_amd.solver import TorchAllocator
    prob = problem_config(case)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    alloc = TorchAllocator(torch.cuda.current_stream())
    s = Solver.from_problem(prob, precision=precision, allocator=alloc)
    nbytes = s.device_bytes()
    assert alloc.requested == nbytes
    assert nbytes == footprint_bytes(prob.shape, precision)
    assert alloc.bytes_live() == nbytes
    assert torch.cuda.memory_allocated() - base >= nbytes
    s.bootstrap()
    s.step()
    s.close()
    assert alloc.bytes_live() == 0
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base


def test_device_views_alias_the_committed_state():
    from paper_2412_17445_amd import Solver
    prob = problem_config("tiny16")
    res = {}
    for kind in ("torch", "hip"):
        s = Solver.from_problem(prob, allocator=kind)
        s.bootstrap()
        out = s.step()
        assert out["converged"]
        eps, phi, Hn, E, a = s.get_state()
        pe, pp, ph = s.device_views()
        c, N = s.ncomp, s.N
        eps_t = _d2h(pe, c * N).reshape(eps.shape)
        fm = np.array([prob.f[0, 0], prob.f[1, 1], np.sqrt(2.0) * prob.f[0, 1]])
        assert np.array_equal(eps_t + fm.reshape((c, 1, 1, 1)) * E, eps)
        assert np.array_equal(_d2h(pp, N).reshape(phi.shape), phi)
        assert np.array_equal(_d2h(ph, N).reshape(Hn.shape), Hn)
        res[kind] = (out["E"], phi.copy())
        s.close()
    assert res["torch"][0] == res["hip"][0]
    assert np.array_equal(res["torch"][1], res["hip"][1])
