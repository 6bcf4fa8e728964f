"""Plain Krylov solvers (oracle).

Paper Sec. 3.2: the bordered Newton system is non-symmetric and is solved
with the bi-conjugate gradient stabilised method (van der Vorst's BiCGSTAB);
Sec. 3.1 uses conjugate gradients for the symmetric Helmholtz problem.
Start x0 = 0, stop at ||r|| <= rtol ||b|| on the TRUE residual b - A x.
Within one run the iterate with the smallest recursive residual is kept, and
the run stops early when the residual exceeds DIVERGED * ||b|| or a scalar
breaks down (zero or not finite).  When a run ends, b - A x of its best
iterate is evaluated; if it misses the tolerance (the recursive residual of
BiCGSTAB drifts from the true one after large intermediate iterates), a new
run starts from that iterate.  Near Newton convergence the right-hand side is
small and the drift can otherwise return a step that is pure noise.

Reading: the shadow residual is r_hat = r0 + (||r0|| / sqrt(n)) s with s a
fixed +-1 sequence.  With r_hat = r0 the method breaks down at the first
step of every warm-started increment: the right-hand side is then the
constraint entry alone and the crack-length row does not see the load-factor
column, so (r_hat, A r0) = 0.  s_i is the sign bit of the i-th output of the
splitmix64 generator (Steele, Lea & Flood 2014) started from SHADOW_SEED.
"""

from __future__ import annotations

import numpy as np


SHADOW_SEED = 0x5EED
DIVERGED = 1e8
MAX_CYCLES = 8


def splitmix64_signs(n, seed=SHADOW_SEED):
    """s_i = +1 if bit 63 of splitmix64 output i (i = 0, 1, ...) is set, else -1."""
    with np.errstate(over="ignore"):
        state = np.uint64(seed) + (np.arange(n, dtype=np.uint64) + np.uint64(1)) \
            * np.uint64(0x9E3779B97F4A7C15)
        z = state
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return np.where((z >> np.uint64(63)) == np.uint64(1), 1.0, -1.0)


def _bicgstab_cycle(apply, b, x, r, bnorm, rtol, maxit, info):
    """One BiCGSTAB run from iterate x with residual r = b - A x.  Returns the
    iterate with the smallest recursive residual and that residual."""
    rnorm = float(np.linalg.norm(r))
    rhat = r + (rnorm / np.sqrt(b.size)) * splitmix64_signs(b.size)
    rho_old = alpha = omega = 1.0
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    x_best, res_best = x.copy(), rnorm
    for it in range(1, maxit + 1):
        rho = float(np.dot(rhat, r))
        if rho == 0.0 or not np.isfinite(rho):
            break
        beta = (rho / rho_old) * (alpha / omega) if it > 1 else 0.0
        p = r + beta * (p - omega * v)
        v = apply(p)
        rv = float(np.dot(rhat, v))
        if rv == 0.0 or not np.isfinite(rv):
            break
        alpha = rho / rv
        s = r - alpha * v
        t = apply(s)
        info["applies"] += 2
        tt = float(np.dot(t, t))
        if tt == 0.0 or not np.isfinite(tt):
            break
        omega = float(np.dot(t, s)) / tt
        x = x + alpha * p + omega * s
        r = s - omega * t
        rho_old = rho
        res = float(np.linalg.norm(r))
        info["iters"] += 1
        if res < res_best:
            x_best, res_best = x.copy(), res
        if res <= rtol * bnorm:
            break
        if omega == 0.0 or not np.isfinite(res) or res > DIVERGED * bnorm:
            break
    return x_best


def bicgstab(apply, b, rtol=1e-10, maxit=5000):
    """BiCGSTAB with a true-residual check: when a run stops, b - A x of its
    best iterate is computed; if it misses rtol ||b||, the method restarts
    from that iterate (at most MAX_CYCLES runs, maxit iterations in total)."""
    x = np.zeros_like(b)
    bnorm = float(np.linalg.norm(b))
    info = dict(iters=0, converged=bnorm == 0.0, applies=0, resid=0.0, cycles=0)
    if bnorm == 0.0:
        return x, info
    r = b.copy()
    for cycle in range(MAX_CYCLES):
        info["cycles"] = cycle + 1
        x = _bicgstab_cycle(apply, b, x, r, bnorm, rtol, maxit - info["iters"], info)
        r = b - apply(x)
        info["applies"] += 1
        res = float(np.linalg.norm(r))
        info["resid"] = res / bnorm
        if res <= rtol * bnorm:
            info["converged"] = True
            break
        if info["iters"] >= maxit:
            break
    return x, info


def cg(apply, b, rtol=1e-12, maxit=5000):
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = float(np.dot(r, r))
    bnorm = np.sqrt(rr)
    info = dict(iters=0, converged=bnorm == 0.0)
    if bnorm == 0.0:
        return x, info
    for it in range(1, maxit + 1):
        Ap = apply(p)
        a = rr / float(np.dot(p, Ap))
        x = x + a * p
        r = r - a * Ap
        rr_new = float(np.dot(r, r))
        info["iters"] = it
        if np.sqrt(rr_new) <= rtol * bnorm:
            info["converged"] = True
            break
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, info
