"""Python wrapper of the C ABI (marshalling only; all compute is in libpff.so).

PyTorch provides device memory and the HIP stream: tensors handed to the
library are HIP device buffers, and the solver queues its work on the
stream that was current when it was created.
"""

from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L


class PffError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"pff status {status}: {msg}")
        self.status = status


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device: the solver runs only on the GPU")
    return torch


def marshal_problem(shape, phases, phase_id, mask, f, l, k=1e-6, delta_a=1.0, alpha=1.0,
                    newton_tol=1e-8, krylov_rtol=1e-10, newton_maxit=50, krylov_maxit=5000,
                    precision="fp64", split="spectral", projection="rotated",
                    control_weights=(1.0, 0.0), control="length", gc_form="pointwise",
                    macro_bc="strain", resid_tol=0.0):
    """C structs and host arrays of one RVE problem (pff_create's inputs).
    split: "spectral" (Miehe split) or "none" (isotropic degradation);
    projection: "rotated" (Willot) or "standard" frequencies in G;
    control_weights: (w_a, w_E) of the controlled quantity w_a Q + w_E E;
    control: Q is "length" (Gamma) or "dissipation" (sum of Gc gamma_f);
    gc_form: "pointwise" Gc l Lap phi or "variational" l div(Gc grad phi);
    macro_bc: "strain" (mean strain f E) or "mixed" (mean strain prescribed
    along f only, mean stress zero on the directions orthogonal to f);
    resid_tol: parity-mode residual stop of Newton (0 = off)."""
    if macro_bc not in ("strain", "mixed"):
        raise ValueError("macro_bc must be 'strain' or 'mixed'")
    if gc_form not in ("pointwise", "variational"):
        raise ValueError("gc_form must be 'pointwise' or 'variational'")
    if control not in ("length", "dissipation"):
        raise ValueError("control must be 'length' or 'dissipation'")
    if split not in ("spectral", "none"):
        raise ValueError("split must be 'spectral' or 'none'")
    if projection not in ("rotated", "standard"):
        raise ValueError("projection must be 'rotated' or 'standard'")
    nz, ny, nx = shape
    grid = L.pff_grid(nx, ny, nz)
    ph = (L.pff_phase * len(phases))(*[L.pff_phase(*map(float, p)) for p in phases])
    pid = np.ascontiguousarray(np.asarray(phase_id, dtype=np.uint8).reshape(-1))
    if pid.size != nx * ny * nz:
        raise ValueError("phase_id does not match the grid")
    msk = None if mask is None else np.ascontiguousarray(np.asarray(mask, dtype=np.uint8).reshape(-1))
    prm = L.pff_params()
    prm.l, prm.k_resid = float(l), float(k)
    fa = np.asarray(f, dtype=np.float64).reshape(-1)
    for i in range(9):
        prm.f[i] = float(fa[i])
    prm.delta_a, prm.alpha = float(delta_a), float(alpha)
    prm.newton_tol, prm.krylov_rtol = float(newton_tol), float(krylov_rtol)
    prm.newton_maxit, prm.krylov_maxit = int(newton_maxit), int(krylov_maxit)
    prm.precision = L.PFF_PREC_MIXED if precision == "mixed" else L.PFF_PREC_FP64
    prm.split = L.PFF_SPLIT_NONE if split == "none" else L.PFF_SPLIT_SPECTRAL
    prm.projection = L.PFF_PROJ_STANDARD if projection == "standard" else L.PFF_PROJ_ROTATED
    prm.w_gamma, prm.w_load = (float(w) for w in control_weights)
    prm.control = L.PFF_CONTROL_DISSIPATION if control == "dissipation" else L.PFF_CONTROL_LENGTH
    prm.gc_form = L.PFF_GC_VARIATIONAL if gc_form == "variational" else L.PFF_GC_POINTWISE
    prm.macro_bc = L.PFF_BC_MIXED if macro_bc == "mixed" else L.PFF_BC_STRAIN
    prm.resid_tol = float(resid_tol)
    return grid, ph, pid, msk, prm


def problem_kwargs(prob, **over):
    kw = dict(shape=prob.shape, phases=prob.phases, phase_id=prob.phase_id, mask=prob.mask,
              f=prob.f, l=prob.l, k=prob.k, delta_a=prob.delta_a, alpha=prob.alpha,
              newton_tol=prob.newton_tol, krylov_rtol=prob.krylov_rtol,
              newton_maxit=prob.newton_maxit, krylov_maxit=prob.krylov_maxit,
              precision=prob.precision, split=getattr(prob, "split", "spectral"),
              projection=getattr(prob, "projection", "rotated"),
              control_weights=getattr(prob, "control_weights", (1.0, 0.0)),
              control=getattr(prob, "control", "length"),
              gc_form=getattr(prob, "gc_form", "pointwise"),
              macro_bc=getattr(prob, "macro_bc", "strain"))
    kw.update(over)
    return kw


def _result_dict(r):
    return dict(increment=r.increment, newton_iters=r.newton_iters, krylov_iters=r.krylov_iters,
                converged=bool(r.converged), applies=r.applies, applies_fp64=r.applies_fp64,
                fp64_fallbacks=r.fp64_fallbacks, refinements=r.refinements,
                sigma_M=list(r.sigma_M), E=r.load_factor, Gamma=r.crack_length,
                a=r.target_a, err=list(r.err), seconds=r.seconds, dissipation=r.dissipation,
                resid=list(r.resid))


class TorchAllocator:
    """pff_allocator backed by PyTorch's caching allocator on the current
    device: the library's device buffers are torch allocations and count in
    torch.cuda.memory_allocated().  Keeps the C callbacks alive; the blocks
    are associated with `stream` (the library synchronises its stream before
    freeing).  `requested` sums the bytes the library asked for."""

    def __init__(self, stream=None):
        torch = _torch()
        self._torch = torch
        self.device = torch.cuda.current_device()
        self.stream = stream
        self.requested = 0
        self.live = {}

        def _alloc(nbytes, ctx):
            try:
                ptr = self._torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
            except Exception:                   # out of memory: the library reports PFF_ERR_OOM
                return None
            self.live[ptr] = int(nbytes)
            self.requested += int(nbytes)
            return ptr

        def _free(ptr, nbytes, ctx):
            self.live.pop(ptr, None)
            cuda = getattr(self._torch, "cuda", None)
            if cuda is None:                    # interpreter shutdown: the process returns the memory
                return
            cuda.caching_allocator_delete(ptr)

        self._alloc = L.ALLOC_FN(_alloc)
        self._free = L.FREE_FN(_free)
        self.struct = L.pff_allocator(self._alloc, self._free, None)

    def bytes_live(self):
        return sum(self.live.values())


class Solver:
    """One RVE solve.  `precision` is "fp64" or "mixed"."""

    def __init__(self, shape, phases, phase_id, mask, f, l, k=1e-6, delta_a=1.0, alpha=1.0,
                 newton_tol=1e-8, krylov_rtol=1e-10, newton_maxit=50, krylov_maxit=5000,
                 precision="fp64", split="spectral", projection="rotated",
                 control_weights=(1.0, 0.0), control="length", gc_form="pointwise",
                 macro_bc="strain", resid_tol=0.0, stream=None, allocator="torch"):
        """allocator: "torch" (device buffers from torch's caching allocator,
        the default), "hip" (the library's own hipMalloc) or a TorchAllocator."""
        torch = _torch()
        self.lib = L.load()
        nz, ny, nx = shape
        self.shape = (nz, ny, nx)
        self.N = nx * ny * nz
        self.ncomp = 3 if nz == 1 else 6
        self.M = (self.ncomp + 1) * self.N + 1
        self.mixed = precision == "mixed"
        self.wdtype = torch.float32 if self.mixed else torch.float64
        grid, ph, pid, msk, prm = marshal_problem(
            shape, phases, phase_id, mask, f, l, k=k, delta_a=delta_a, alpha=alpha,
            newton_tol=newton_tol, krylov_rtol=krylov_rtol, newton_maxit=newton_maxit,
            krylov_maxit=krylov_maxit, precision=precision, split=split, projection=projection,
            control_weights=control_weights, control=control, gc_form=gc_form,
            macro_bc=macro_bc, resid_tol=resid_tol)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self._stream = stream
        if allocator == "torch":
            allocator = TorchAllocator(torch.cuda.current_stream())
        elif allocator == "hip":
            allocator = None
        self.allocator = allocator
        h = C.c_void_p()
        st = self.lib.pff_create(C.byref(grid), ph, len(phases), pid.ctypes.data,
                                 None if msk is None else msk.ctypes.data, C.byref(prm),
                                 None if allocator is None else C.byref(allocator.struct),
                                 C.c_void_p(stream), C.byref(h))
        if st != L.PFF_OK:
            msg = self.lib.pff_last_error(None)
            raise PffError(st, msg.decode() if msg else "pff_create failed")
        self.h = h

    @classmethod
    def from_problem(cls, prob, **over):
        kw = dict(k=prob.k, delta_a=prob.delta_a, alpha=prob.alpha, newton_tol=prob.newton_tol,
                  krylov_rtol=prob.krylov_rtol, newton_maxit=prob.newton_maxit,
                  krylov_maxit=prob.krylov_maxit, precision=prob.precision,
                  split=getattr(prob, "split", "spectral"),
                  projection=getattr(prob, "projection", "rotated"),
                  control_weights=getattr(prob, "control_weights", (1.0, 0.0)),
                  control=getattr(prob, "control", "length"),
                  gc_form=getattr(prob, "gc_form", "pointwise"),
                  macro_bc=getattr(prob, "macro_bc", "strain"))
        kw.update(over)
        return cls(prob.shape, prob.phases, prob.phase_id, prob.mask, prob.f, prob.l, **kw)

    def device_views(self):
        """Borrowed device pointers (eps_tilde, phi, Hn) of the committed state."""
        e, p, h = C.c_void_p(), C.c_void_p(), C.c_void_p()
        self._check(self.lib.pff_device_views(self.h, C.byref(e), C.byref(p), C.byref(h)),
                    "pff_device_views")
        return e.value, p.value, h.value

    # -- helpers ------------------------------------------------------------
    def _check(self, st, what):
        if st < 0:
            msg = self.lib.pff_last_error(self.h)
            raise PffError(st, f"{what}: {msg.decode() if msg else ''}")
        return st

    def close(self):
        if getattr(self, "h", None):
            self.lib.pff_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- solver -------------------------------------------------------------
    def bootstrap(self):
        a0, es = C.c_double(), C.c_double()
        self._check(self.lib.pff_bootstrap(self.h, C.byref(a0), C.byref(es)), "pff_bootstrap")
        return a0.value, es.value

    def step(self):
        r = L.pff_increment_result()
        st = self._check(self.lib.pff_step(self.h, C.byref(r)), "pff_step")
        out = _result_dict(r)
        out["status"] = st
        return out

    def stagger_step(self, dE, **params):
        """One strain-controlled increment of the staggered scheme (load E += dE).
        Keyword overrides of the defaults: tol_mech, tol_sta, cg_rtol,
        max_stagger, max_newton, cg_maxit."""
        p = L.pff_stagger_params()
        self._check(self.lib.pff_stagger_defaults(C.byref(p)), "pff_stagger_defaults")
        for k, v in params.items():
            if not hasattr(p, k):
                raise TypeError(f"unknown staggered-scheme parameter {k}")
            setattr(p, k, v)
        r = L.pff_stagger_result()
        st = self._check(self.lib.pff_stagger_step(self.h, float(dE), C.byref(p), C.byref(r)),
                         "pff_stagger_step")
        return dict(increment=r.increment, converged=bool(r.converged), stagger_iters=r.stagger_iters,
                    newton_iters=r.newton_iters, cg_mech=r.cg_mech, cg_helm=r.cg_helm, E=r.E,
                    Gamma=r.crack_length, sigma_M=list(r.sigma_M), err=r.err, seconds=r.seconds,
                    dissipation=r.dissipation, status=st)

    def device_bytes(self):
        b = C.c_size_t()
        self._check(self.lib.pff_solver_bytes(self.h, C.byref(b)), "pff_solver_bytes")
        return b.value

    def get_state(self):
        c, N = self.ncomp, self.N
        eps = np.empty(c * N)
        phi = np.empty(N)
        Hn = np.empty(N)
        E, a = C.c_double(), C.c_double()
        self._check(self.lib.pff_get_state(self.h, eps.ctypes.data, phi.ctypes.data,
                                           Hn.ctypes.data, C.byref(E), C.byref(a)),
                    "pff_get_state")
        return (eps.reshape((c,) + self.shape), phi.reshape(self.shape),
                Hn.reshape(self.shape), E.value, a.value)

    def set_state(self, eps_tilde, phi, Hn, E, a, n=1):
        e = np.ascontiguousarray(eps_tilde, dtype=np.float64).reshape(-1)
        p = np.ascontiguousarray(phi, dtype=np.float64).reshape(-1)
        h = np.ascontiguousarray(Hn, dtype=np.float64).reshape(-1)
        self._check(self.lib.pff_set_state(self.h, e.ctypes.data, p.ctypes.data, h.ctypes.data,
                                           float(E), float(a), int(n)), "pff_set_state")

    def residual(self, a, want_F=True):
        """(F on the device or None, Gamma, Sigma_M, dissipation) at the current state."""
        torch = _torch()
        F = torch.empty(self.M, dtype=torch.float64, device="cuda") if want_F else None
        gam, dis = C.c_double(), C.c_double()
        sig = (C.c_double * 6)()
        self._check(self.lib.pff_residual(self.h, float(a), None if F is None else F.data_ptr(),
                                          C.byref(gam), sig, C.byref(dis)), "pff_residual")
        return F, gam.value, list(sig), dis.value

    def apply(self, v, out=None):
        torch = _torch()
        if v.dtype != self.wdtype or v.numel() != self.M or not v.is_cuda:
            raise ValueError("v must be a contiguous device vector of the working precision")
        v = v.contiguous()
        if out is None:
            out = torch.empty_like(v)
        self._check(self.lib.pff_apply_tangent(self.h, v.data_ptr(), out.data_ptr()),
                    "pff_apply_tangent")
        return out

    def project(self, x):
        torch = _torch()
        prec = 1 if x.dtype == torch.float32 else 0
        x = x.contiguous()
        out = torch.empty_like(x)
        self._check(self.lib.pff_project(self.h, x.data_ptr(), out.data_ptr(), prec), "pff_project")
        return out

    def krylov_solve(self, b, rtol=1e-10, maxit=5000):
        torch = _torch()
        b = b.contiguous()
        x = torch.empty_like(b)
        it, rr = C.c_int(), C.c_double()
        st = self._check(self.lib.pff_krylov_solve(self.h, b.data_ptr(), x.data_ptr(), float(rtol),
                                                   int(maxit), C.byref(it), C.byref(rr)),
                         "pff_krylov_solve")
        return x, it.value, rr.value, st == L.PFF_OK

    def timing(self, every):
        """Sample every `every`-th tangent apply's pass kernels with HIP events
        (every < 0: every |every|-th apply, the whole apply only)."""
        self._check(self.lib.pff_timing(self.h, int(every)), "pff_timing")

    def timing_read(self):
        """{slot: (launches, ms)} for every slot with timed launches (see
        pff_timing_read: slot = 6 * (5 * fp32 + variant) + kernel)."""
        out = {}
        for k in range(60):
            n, ms = C.c_longlong(), C.c_double()
            self._check(self.lib.pff_timing_read(self.h, k, C.byref(n), C.byref(ms)), "pff_timing_read")
            if n.value:
                out[k] = (n.value, ms.value)
        return out

    def counters(self):
        a, k = C.c_longlong(), C.c_longlong()
        self._check(self.lib.pff_counters(self.h, C.byref(a), C.byref(k)), "pff_counters")
        return a.value, k.value

    def save(self):
        n = C.c_size_t()
        self._check(self.lib.pff_save(self.h, None, C.byref(n)), "pff_save")
        buf = (C.c_ubyte * n.value)()
        self._check(self.lib.pff_save(self.h, buf, C.byref(n)), "pff_save")
        return bytes(buf)

    def load(self, data):
        buf = (C.c_ubyte * len(data)).from_buffer_copy(data)
        self._check(self.lib.pff_load(self.h, buf, len(data)), "pff_load")


def effective_toughness(E, sigma_M, f, volume, L_g):
    """(work, G_Ceff) of a macroscopic path: E[k] and sigma_M[k] (11, 22, 33,
    23, 13, 12) per increment in path order, f the 3x3 loading tensor
    (pff_effective_toughness, host only)."""
    E = np.ascontiguousarray(E, dtype=np.float64).reshape(-1)
    S = np.ascontiguousarray(sigma_M, dtype=np.float64).reshape(-1)
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
    if S.size != 6 * E.size or f.size != 9:
        raise ValueError("sigma_M must hold 6 values per path point and f 9 values")
    w, g = C.c_double(), C.c_double()
    st = L.load().pff_effective_toughness(E.size, E.ctypes.data, S.ctypes.data, f.ctypes.data,
                                          float(volume), float(L_g), C.byref(w), C.byref(g))
    if st != L.PFF_OK:
        raise PffError(st, "pff_effective_toughness: invalid arguments")
    return w.value, g.value


def footprint_bytes(shape, precision):
    """Device bytes of a solver of this grid (host-side estimate, no GPU)."""
    nz, ny, nx = shape
    lib = L.load()
    b = C.c_size_t()
    st = lib.pff_footprint_bytes(C.byref(L.pff_grid(nx, ny, nz)),
                                 L.PFF_PREC_MIXED if precision == "mixed" else L.PFF_PREC_FP64,
                                 C.byref(b))
    if st != L.PFF_OK:
        raise PffError(st, "pff_footprint_bytes")
    return b.value


class Server:
    """Request server of the C ABI: RVE solves admitted by memory footprint
    into `slots` concurrent slots on the current device."""

    def __init__(self, budget_bytes, slots, allocator=None):
        """allocator: None (hipMalloc) or a TorchAllocator (its callbacks
        run on the server's worker threads)."""
        _torch()
        self.lib = L.load()
        self.allocator = allocator
        h = C.c_void_p()
        st = self.lib.pff_server_create(int(budget_bytes), int(slots),
                                        None if allocator is None else C.byref(allocator.struct),
                                        C.byref(h))
        if st != L.PFF_OK:
            raise PffError(st, "pff_server_create")
        self.h = h

    def submit(self, n_increments, **problem):
        grid, ph, pid, msk, prm = marshal_problem(**problem)
        t = C.c_uint64()
        st = self.lib.pff_server_submit(self.h, C.byref(grid), ph, len(ph), pid.ctypes.data,
                                        None if msk is None else msk.ctypes.data, C.byref(prm),
                                        int(n_increments), C.byref(t))
        if st != L.PFF_OK:
            raise PffError(st, (self.lib.pff_server_last_error(self.h) or b"").decode())
        return t.value

    def wait(self, ticket, timeout=-1.0):
        st = self.lib.pff_server_wait(self.h, C.c_uint64(ticket), float(timeout))
        if st < 0:
            raise PffError(st, "pff_server_wait")
        return st == L.PFF_OK

    def info(self, ticket):
        i = L.pff_request_info()
        st = self.lib.pff_server_info(self.h, C.c_uint64(ticket), C.byref(i))
        if st != L.PFF_OK:
            raise PffError(st, "pff_server_info")
        return {k: getattr(i, k) for k, _ in L.pff_request_info._fields_}

    def results(self, ticket):
        n = C.c_int()
        st = self.lib.pff_server_results(self.h, C.c_uint64(ticket), None, 0, C.byref(n))
        if st != L.PFF_OK:
            raise PffError(st, "pff_server_results")
        arr = (L.pff_increment_result * max(n.value, 1))()
        st = self.lib.pff_server_results(self.h, C.c_uint64(ticket), arr, n.value, C.byref(n))
        if st != L.PFF_OK:
            raise PffError(st, "pff_server_results")
        return [_result_dict(arr[k]) for k in range(n.value)]

    def last_error(self):
        msg = self.lib.pff_server_last_error(self.h)
        return msg.decode() if msg else ""

    def release(self, ticket):
        st = self.lib.pff_server_release(self.h, C.c_uint64(ticket))
        if st != L.PFF_OK:
            raise PffError(st, "pff_server_release")

    def stats(self):
        s = L.pff_server_stats()
        st = self.lib.pff_server_get_stats(self.h, C.byref(s))
        if st != L.PFF_OK:
            raise PffError(st, "pff_server_get_stats")
        return {k: getattr(s, k) for k, _ in L.pff_server_stats._fields_}

    def close(self):
        if getattr(self, "h", None):
            self.lib.pff_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
