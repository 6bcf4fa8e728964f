// Vector kernels of the Krylov and Newton loops.
//
// BiCGSTAB (van der Vorst) for the non-symmetric bordered Newton system
// (paper Sec. 3.2); vectors are in the apply precision TW, every inner
// product is accumulated in FP64 per thread, then per block, then over
// blocks in a fixed order (bitwise reproducible).  Scalars live on the
// device in `ks` so that no host round trip sits between the vector steps.
#pragma once

#include "common.hpp"

namespace pff {

enum KrylovScalar {
  KS_RHO = 0, KS_RHO_OLD, KS_ALPHA, KS_OMEGA, KS_BETA, KS_RR, KS_BNORM, KS_FLAG,
  KS_RV, KS_TS, KS_TT, KS_RNORM, KS_TRUE, KS_ULAST,
  // device-side run control of the batched solves (k_fin_rr_b): stop flag
  // (non-zero: every later kernel of this solve returns at once), reason,
  // iteration count, current and best iterate buffers, best residual,
  // rtol ||b|| and the iteration cap
  KS_STOP, KS_REASON, KS_ITER, KS_CUR, KS_BEST, KS_RESBEST, KS_RTOLB, KS_MAXIT,
  KS_COUNT
};

// reasons a batched run stops (KS_REASON)
enum { KR_CONVERGED = 1, KR_BREAKDOWN = 2, KR_OTHER = 3, KR_MAXIT = 4 };

constexpr int kRedBlocks = 1024;   // upper bound on the blocks of a vector reduction

__host__ __device__ inline int red_blocks(long long M) {
  long long b = (M + (long long)kBlock * 8 - 1) / ((long long)kBlock * 8);
  if (b < 1) b = 1;
  if (b > kRedBlocks) b = kRedBlocks;
  return (int)b;
}

// splitmix64 (Steele, Lea & Flood 2014): output number i of the stream
// started at `seed` is mix(seed + (i+1) * golden).
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <int ND>
__device__ __forceinline__ void write_partials(double (&acc)[ND], double* partials) {
  __shared__ double lds[ND * kBlock];
  block_reduce<ND>(acc, lds);
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < ND; ++q) partials[(long long)q * gridDim.x + blockIdx.x] = acc[q];
}

// partials of up to three inner products (a_q, b_q)
template <typename T, int ND>
__global__ void __launch_bounds__(kBlock) k_dots(const T* __restrict__ a0, const T* __restrict__ b0,
                                                 const T* __restrict__ a1, const T* __restrict__ b1,
                                                 const T* __restrict__ a2, const T* __restrict__ b2,
                                                 long long M, double* __restrict__ partials) {
  double acc[ND];
#pragma unroll
  for (int q = 0; q < ND; ++q) acc[q] = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < M;
       i += (long long)gridDim.x * blockDim.x) {
    acc[0] += double(a0[i]) * double(b0[i]);
    if (ND > 1) acc[1] += double(a1[i]) * double(b1[i]);
    if (ND > 2) acc[2] += double(a2[i]) * double(b2[i]);
  }
  write_partials<ND>(acc, partials);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_copy(T* __restrict__ dst, const T* __restrict__ src, long long M) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < M;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_fill(T* __restrict__ dst, T val, long long M) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < M;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = val;
}

// BiCGSTAB start: x = 0, r = b, p = v = 0, partial of (b, b)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_bicg_init(const T* __restrict__ b, T* __restrict__ x,
                                                      T* __restrict__ r, T* __restrict__ p,
                                                      T* __restrict__ v, long long M,
                                                      double* __restrict__ partials) {
  double acc[1] = {0.0};
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < M;
       i += (long long)gridDim.x * blockDim.x) {
    const T bi = b[i];
    x[i] = T(0);
    r[i] = bi;
    p[i] = T(0);
    v[i] = T(0);
    acc[0] += double(bi) * double(bi);
  }
  write_partials<1>(acc, partials);
}

// shadow residual r_hat = r0 + (||r0|| / sqrt(M)) s_i, and partial of (r_hat, r0)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_bicg_shadow(const T* __restrict__ r, T* __restrict__ rhat,
                                                        const double* __restrict__ ks, uint64_t seed,
                                                        long long M, double* __restrict__ partials) {
  const double scale = ks[KS_RNORM] / sqrt(double(M));
  double acc[1] = {0.0};
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < M;
       i += (long long)gridDim.x * blockDim.x) {
    const double s = (splitmix64_at(seed, (uint64_t)i) >> 63) ? 1.0 : -1.0;
    const T h = T(double(r[i]) + scale * s);
    rhat[i] = h;
    acc[0] += double(h) * double(r[i]);
  }
  write_partials<1>(acc, partials);
}

// 16-byte packets for the streaming BiCGSTAB updates (float4 / double2):
// one load or store instruction per lane moves 16 bytes.  The Krylov vectors
// are separate device allocations (256-byte aligned); any other pointer
// that is not 16-byte aligned takes the element loop.
template <typename T> struct Packet;
template <> struct Packet<float> { using V = float4; static constexpr int W = 4; };
template <> struct Packet<double> { using V = double2; static constexpr int W = 2; };
template <typename T> struct Lanes { T v[Packet<T>::W]; };

template <typename T> __device__ __forceinline__ Lanes<T> pk_load(const T* p, long long j) {
  const typename Packet<T>::V q = reinterpret_cast<const typename Packet<T>::V*>(p)[j];
  Lanes<T> o;
  __builtin_memcpy(&o, &q, sizeof(o));
  return o;
}
template <typename T> __device__ __forceinline__ void pk_store(T* p, long long j, const Lanes<T>& o) {
  typename Packet<T>::V q;
  __builtin_memcpy(&q, &o, sizeof(q));
  reinterpret_cast<typename Packet<T>::V*>(p)[j] = q;
}
__device__ __forceinline__ bool aligned16(const void* a, const void* b = nullptr, const void* c = nullptr,
                                          const void* d = nullptr, const void* e = nullptr,
                                          const void* f = nullptr, const void* g = nullptr) {
  return ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b) | reinterpret_cast<uintptr_t>(c) |
           reinterpret_cast<uintptr_t>(d) | reinterpret_cast<uintptr_t>(e) | reinterpret_cast<uintptr_t>(f) |
           reinterpret_cast<uintptr_t>(g)) & 15) == 0;
}

// p = r + beta (p - omega v)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_bicg_p(T* __restrict__ p, const T* __restrict__ r,
                                                   const T* __restrict__ v, const double* __restrict__ ks,
                                                   long long M) {
  const T beta = T(ks[KS_BETA]), omega = T(ks[KS_OMEGA]);
  constexpr int W = Packet<T>::W;
  const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  long long i0 = 0;
  if (aligned16(p, r, v)) {
    const long long nv = M / W;
    for (long long j = tid; j < nv; j += stride) {
      const Lanes<T> rr = pk_load(r, j), pp = pk_load(p, j), vv = pk_load(v, j);
      Lanes<T> o;
#pragma unroll
      for (int w = 0; w < W; ++w) o.v[w] = rr.v[w] + beta * (pp.v[w] - omega * vv.v[w]);
      pk_store(p, j, o);
    }
    i0 = nv * W;
  }
  for (long long i = i0 + tid; i < M; i += stride) p[i] = r[i] + beta * (p[i] - omega * v[i]);
}

// s = r - alpha v
template <typename T>
__global__ void __launch_bounds__(kBlock) k_bicg_s(T* __restrict__ s, const T* __restrict__ r,
                                                   const T* __restrict__ v, const double* __restrict__ ks,
                                                   long long M) {
  const T alpha = T(ks[KS_ALPHA]);
  constexpr int W = Packet<T>::W;
  const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  long long i0 = 0;
  if (aligned16(s, r, v)) {
    const long long nv = M / W;
    for (long long j = tid; j < nv; j += stride) {
      const Lanes<T> rr = pk_load(r, j), vv = pk_load(v, j);
      Lanes<T> o;
#pragma unroll
      for (int w = 0; w < W; ++w) o.v[w] = rr.v[w] - alpha * vv.v[w];
      pk_store(s, j, o);
    }
    i0 = nv * W;
  }
  for (long long i = i0 + tid; i < M; i += stride) s[i] = r[i] - alpha * v[i];
}

// x_next = x + alpha p + omega s ; r = s - omega t ; partials (r, r), (r_hat, r)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_bicg_xr(T* __restrict__ xn, const T* __restrict__ x,
                                                    const T* __restrict__ p, const T* __restrict__ s,
                                                    const T* __restrict__ t, T* __restrict__ r,
                                                    const T* __restrict__ rhat,
                                                    const double* __restrict__ ks, long long M,
                                                    double* __restrict__ partials) {
  const T alpha = T(ks[KS_ALPHA]), omega = T(ks[KS_OMEGA]);
  constexpr int W = Packet<T>::W;
  const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  double acc[2] = {0.0, 0.0};
  long long i0 = 0;
  if (aligned16(xn, x, p, s, t, r, rhat)) {
    const long long nv = M / W;
    for (long long j = tid; j < nv; j += stride) {
      const Lanes<T> xx = pk_load(x, j), pp = pk_load(p, j), ss = pk_load(s, j), tt = pk_load(t, j),
                     hh = pk_load(rhat, j);
      Lanes<T> xo, ro;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        xo.v[w] = xx.v[w] + alpha * pp.v[w] + omega * ss.v[w];
        const T ri = ss.v[w] - omega * tt.v[w];
        ro.v[w] = ri;
        acc[0] += double(ri) * double(ri);
        acc[1] += double(hh.v[w]) * double(ri);
      }
      pk_store(xn, j, xo);
      pk_store(r, j, ro);
    }
    i0 = nv * W;
  }
  for (long long i = i0 + tid; i < M; i += stride) {
    const T si = s[i];
    xn[i] = x[i] + alpha * p[i] + omega * si;
    const T ri = si - omega * t[i];
    r[i] = ri;
    acc[0] += double(ri) * double(ri);
    acc[1] += double(rhat[i]) * double(ri);
  }
  write_partials<2>(acc, partials);
}

// ---- scalar finalisers (run by one thread after the fixed-order reduction)

struct FinStore {   // copy totals to dst[0..n)
  struct Args { double* dst; int n; };
  __device__ static void run(const Args& F, const double* tot) {
    for (int q = 0; q < F.n; ++q) F.dst[q] = tot[q];
  }
};

struct FinBnorm {   // ||b|| -> ks, initial scalars
  struct Args { double* ks; };
  __device__ static void run(const Args& F, const double* tot) {
    double* ks = F.ks;
    ks[KS_BNORM] = sqrt(tot[0]);
    ks[KS_RNORM] = sqrt(tot[0]);
    ks[KS_RR] = tot[0];
    ks[KS_RHO_OLD] = 1.0;
    ks[KS_ALPHA] = 1.0;
    ks[KS_OMEGA] = 1.0;
    ks[KS_BETA] = 0.0;
    ks[KS_FLAG] = 0.0;
  }
};

struct FinRestart {  // true residual of the best iterate; scalars of a new run
  struct Args { double* ks; };
  __device__ static void run(const Args& F, const double* tot) {
    double* ks = F.ks;
    ks[KS_TRUE] = sqrt(tot[0]);
    ks[KS_RNORM] = sqrt(tot[0]);
    ks[KS_RR] = tot[0];
    ks[KS_RHO_OLD] = 1.0;
    ks[KS_ALPHA] = 1.0;
    ks[KS_OMEGA] = 1.0;
    ks[KS_BETA] = 0.0;
    ks[KS_FLAG] = 0.0;
  }
};

// r = b - t (t = A x), partial of (r, r); p = v = 0 for a new run
template <typename T>
__global__ void __launch_bounds__(kBlock) k_true_resid(T* __restrict__ r, const T* __restrict__ b,
                                                       const T* __restrict__ t, T* __restrict__ p,
                                                       T* __restrict__ v, long long M,
                                                       double* __restrict__ partials) {
  double acc[1] = {0.0};
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < M;
       i += (long long)gridDim.x * blockDim.x) {
    const T ri = b[i] - t[i];
    r[i] = ri;
    p[i] = T(0);
    v[i] = T(0);
    acc[0] += double(ri) * double(ri);
  }
  write_partials<1>(acc, partials);
}

struct FinRho0 {    // rho = (r_hat, r0)
  struct Args { double* ks; };
  __device__ static void run(const Args& F, const double* tot) { F.ks[KS_RHO] = tot[0]; }
};

struct FinAlpha {   // alpha = rho / (r_hat, v)
  struct Args { double* ks; };
  __device__ static void run(const Args& F, const double* tot) {
    double* ks = F.ks;
    const double rv = tot[0];
    ks[KS_RV] = rv;
    if (rv == 0.0 || !isfinite(rv)) {
      ks[KS_FLAG] = 1.0;
      ks[KS_ALPHA] = 0.0;
    } else {
      ks[KS_ALPHA] = ks[KS_RHO] / rv;
    }
  }
};

struct FinOmega {   // omega = (t, s) / (t, t)
  struct Args { double* ks; };
  __device__ static void run(const Args& F, const double* tot) {
    double* ks = F.ks;
    ks[KS_TS] = tot[0];
    ks[KS_TT] = tot[1];
    if (tot[1] == 0.0 || !isfinite(tot[1])) {
      ks[KS_FLAG] = 2.0;
      ks[KS_OMEGA] = 0.0;
    } else {
      ks[KS_OMEGA] = tot[0] / tot[1];
    }
  }
};

struct FinRR {      // ||r||^2 and the next rho, beta
  struct Args { double* ks; };
  __device__ static void run(const Args& F, const double* tot) {
    double* ks = F.ks;
    ks[KS_RR] = tot[0];
    const double rho_new = tot[1];
    const double rho = ks[KS_RHO];
    ks[KS_RHO_OLD] = rho;
    ks[KS_RHO] = rho_new;
    const double om = ks[KS_OMEGA];
    if (rho_new == 0.0 || !isfinite(rho_new) || rho == 0.0 || om == 0.0) {
      if (ks[KS_FLAG] == 0.0) ks[KS_FLAG] = 3.0;
      ks[KS_BETA] = 0.0;
    } else {
      ks[KS_BETA] = (rho_new / rho) * (ks[KS_ALPHA] / om);
    }
  }
};

// Finisher of a fused tangent apply (mode 1 or 2): fixed-order totals of the
// prologue partials (the border row J3) and of the epilogue partials (the
// voxel part of the inner products); writes J u and the updated vector at
// their trailing entries, adds the trailing terms to the inner products and
// forms alpha (mode 1) or omega (mode 2) with the breakdown flags.
// vout_last and dv_last are the same entry in mode 2, and in_last may be
// either of them (no __restrict__).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fin_fused(const double* __restrict__ part0,
                                                      const double* __restrict__ part1, int nblk, int mode,
                                                      int pro, T* Jv_last, T* vout_last, const T* dv_last,
                                                      const T* in_last, double wa, double wE, double* ks) {
  __shared__ double tot[3];
  const double* const src[3] = {part0, part1, part1 + nblk};
  block_slot_sums<3>(src, mode == 1 ? 2 : 3, nblk, tot);
  if (threadIdx.x != 0) return;
  // border row J3 = w_a (r, d phi) + w_E dE, dE the trailing entry of the input
  const double din = pro ? ks[KS_ULAST] : double(*in_last);
  const T j3 = T(wa * tot[0] + wE * din);
  // mode 1 pairs J u with r_hat; mode 2 with u itself, whose trailing entry
  // the prologue formed (pro) or the caller holds in dv
  T dlast;
  if (pro) {
    const T ulast = T(ks[KS_ULAST]);
    dlast = mode == 1 ? *dv_last : ulast;
    *vout_last = ulast;
  } else {
    dlast = *dv_last;
  }
  *Jv_last = j3;
  if (mode == 1) {
    const double rv = tot[1] + double(dlast) * double(j3);
    ks[KS_RV] = rv;
    if (rv == 0.0 || !isfinite(rv)) {
      ks[KS_FLAG] = 1.0;
      ks[KS_ALPHA] = 0.0;
    } else {
      ks[KS_ALPHA] = ks[KS_RHO] / rv;
    }
  } else {
    const double ts = tot[1] + double(j3) * double(dlast);
    const double tt = tot[2] + double(j3) * double(j3);
    ks[KS_TS] = ts;
    ks[KS_TT] = tt;
    if (tt == 0.0 || !isfinite(tt)) {
      ks[KS_FLAG] = 2.0;
      ks[KS_OMEGA] = 0.0;
    } else {
      ks[KS_OMEGA] = ts / tt;
    }
  }
}

template <typename T>
struct FinLast {    // border row: J3 = w_a (r, d phi) + w_E dE into the trailing entry
  struct Args { T* dst; double wa, wE; const T* vlast; };
  __device__ static void run(const Args& F, const double* tot) {
    *F.dst = T(F.wa * tot[0] + F.wE * double(*F.vlast));
  }
};

// ---- batched BiCGSTAB (one solve per RVE of a size class, blockIdx.y) ------
//
// Every RVE of the batch runs its own iteration with its own scalars; the
// arithmetic of each RVE is that of the kernels above, so a solve gives the
// same bits alone and in a batch.  A stopped solve (KS_STOP) returns at the
// top of every kernel, so a fixed chunk of iterations can be queued (or
// replayed from a graph) without the host deciding between iterations.

template <typename T> struct KryEntry {
  T* x[3];            // iterate buffers: current, best and the next one rotate
  T* r;
  const T* rhat;
  T* p;
  T* v;
  T* s;
  T* t;
  double* ks;         // Krylov scalars of this solve
  double* part;       // partials of the vector reductions
  double* part0;      // partials of the apply prologue (border row)
  double* part1;      // partials of the apply epilogue (inner products)
  double wa, wE;      // control weights of the border row
};

__device__ __forceinline__ int kry_next(const double* ks) {
  const int cur = int(ks[KS_CUR]), best = int(ks[KS_BEST]);
  int nxt = 0;
  while (nxt == cur || nxt == best) ++nxt;
  return nxt;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_bicg_p_b(const KryEntry<T>* __restrict__ E, long long M) {
  const KryEntry<T>& e = E[blockIdx.y];
  if (e.ks[KS_STOP] != 0.0) return;
  const T beta = T(e.ks[KS_BETA]), omega = T(e.ks[KS_OMEGA]);
  T* __restrict__ p = e.p;
  const T* __restrict__ r = e.r;
  const T* __restrict__ v = e.v;
  constexpr int W = Packet<T>::W;
  const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  long long i0 = 0;
  if (aligned16(p, r, v)) {
    const long long nv = M / W;
    for (long long j = tid; j < nv; j += stride) {
      const Lanes<T> rr = pk_load(r, j), pp = pk_load(p, j), vv = pk_load(v, j);
      Lanes<T> o;
#pragma unroll
      for (int w = 0; w < W; ++w) o.v[w] = rr.v[w] + beta * (pp.v[w] - omega * vv.v[w]);
      pk_store(p, j, o);
    }
    i0 = nv * W;
  }
  for (long long i = i0 + tid; i < M; i += stride) p[i] = r[i] + beta * (p[i] - omega * v[i]);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_bicg_s_b(const KryEntry<T>* __restrict__ E, long long M) {
  const KryEntry<T>& e = E[blockIdx.y];
  if (e.ks[KS_STOP] != 0.0) return;
  const T alpha = T(e.ks[KS_ALPHA]);
  T* __restrict__ sv = e.s;
  const T* __restrict__ r = e.r;
  const T* __restrict__ v = e.v;
  constexpr int W = Packet<T>::W;
  const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  long long i0 = 0;
  if (aligned16(sv, r, v)) {
    const long long nv = M / W;
    for (long long j = tid; j < nv; j += stride) {
      const Lanes<T> rr = pk_load(r, j), vv = pk_load(v, j);
      Lanes<T> o;
#pragma unroll
      for (int w = 0; w < W; ++w) o.v[w] = rr.v[w] - alpha * vv.v[w];
      pk_store(sv, j, o);
    }
    i0 = nv * W;
  }
  for (long long i = i0 + tid; i < M; i += stride) sv[i] = r[i] - alpha * v[i];
}

// x[next] = x[cur] + alpha p + omega s ; r = s - omega t ; partials (r, r), (r_hat, r)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_bicg_xr_b(const KryEntry<T>* __restrict__ E, long long M) {
  const KryEntry<T>& e = E[blockIdx.y];
  if (e.ks[KS_STOP] != 0.0) return;
  const T alpha = T(e.ks[KS_ALPHA]), omega = T(e.ks[KS_OMEGA]);
  T* __restrict__ xn = e.x[kry_next(e.ks)];
  const T* __restrict__ x = e.x[int(e.ks[KS_CUR])];
  const T* __restrict__ p = e.p;
  const T* __restrict__ s = e.s;
  const T* __restrict__ t = e.t;
  T* __restrict__ r = e.r;
  const T* __restrict__ rhat = e.rhat;
  constexpr int W = Packet<T>::W;
  const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  double acc[2] = {0.0, 0.0};
  long long i0 = 0;
  if (aligned16(xn, x, p, s, t, r, rhat)) {
    const long long nv = M / W;
    for (long long j = tid; j < nv; j += stride) {
      const Lanes<T> xx = pk_load(x, j), pp = pk_load(p, j), ss = pk_load(s, j), tt = pk_load(t, j),
                     hh = pk_load(rhat, j);
      Lanes<T> xo, ro;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        xo.v[w] = xx.v[w] + alpha * pp.v[w] + omega * ss.v[w];
        const T ri = ss.v[w] - omega * tt.v[w];
        ro.v[w] = ri;
        acc[0] += double(ri) * double(ri);
        acc[1] += double(hh.v[w]) * double(ri);
      }
      pk_store(xn, j, xo);
      pk_store(r, j, ro);
    }
    i0 = nv * W;
  }
  for (long long i = i0 + tid; i < M; i += stride) {
    const T si = s[i];
    xn[i] = x[i] + alpha * p[i] + omega * si;
    const T ri = si - omega * t[i];
    r[i] = ri;
    acc[0] += double(ri) * double(ri);
    acc[1] += double(rhat[i]) * double(ri);
  }
  __shared__ double lds[2 * kBlock];
  block_reduce<2>(acc, lds);
  if (threadIdx.x == 0) {
    e.part[blockIdx.x] = acc[0];
    e.part[gridDim.x + blockIdx.x] = acc[1];
  }
}

// finisher of the fused applies, one block per RVE (blockIdx.x): mode 1 is
// v = J p with (r_hat, v), mode 2 t = J s with (t, s), (t, t); as k_fin_fused
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fin_fused_b(const KryEntry<T>* __restrict__ E, int nblk, int mode,
                                                        long long last) {
  const KryEntry<T>& e = E[blockIdx.x];
  double* ks = e.ks;
  if (ks[KS_STOP] != 0.0) return;
  __shared__ double tot[3];
  const double* const src[3] = {e.part0, e.part1, e.part1 + nblk};
  block_slot_sums<3>(src, mode == 1 ? 2 : 3, nblk, tot);
  if (threadIdx.x != 0) return;
  const T* in = mode == 1 ? e.p : e.s;
  T* Jv = mode == 1 ? e.v : e.t;
  const T* dv = mode == 1 ? e.rhat : e.s;
  const T j3 = T(e.wa * tot[0] + e.wE * double(in[last]));
  const T dlast = dv[last];
  Jv[last] = j3;
  if (mode == 1) {
    const double rv = tot[1] + double(dlast) * double(j3);
    ks[KS_RV] = rv;
    if (rv == 0.0 || !isfinite(rv)) {
      ks[KS_FLAG] = 1.0;
      ks[KS_ALPHA] = 0.0;
    } else {
      ks[KS_ALPHA] = ks[KS_RHO] / rv;
    }
  } else {
    const double ts = tot[1] + double(j3) * double(dlast);
    const double tt = tot[2] + double(j3) * double(j3);
    ks[KS_TS] = ts;
    ks[KS_TT] = tt;
    if (tt == 0.0 || !isfinite(tt)) {
      ks[KS_FLAG] = 2.0;
      ks[KS_OMEGA] = 0.0;
    } else {
      ks[KS_OMEGA] = ts / tt;
    }
  }
}

// end of a batched iteration, one block per RVE: ||r||^2, the next rho and
// beta (as FinRR), then the run control of the host loop: a breakdown
// before the update (flag 1, 2) stops without adopting the new iterate;
// otherwise the new iterate becomes current, the best is tracked, and the
// run stops on convergence (||r|| <= rtol ||b||), on any other breakdown,
// divergence or non-finite residual, or at the iteration cap.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_fin_rr_b(const KryEntry<T>* __restrict__ E, int nb, double diverged) {
  const KryEntry<T>& e = E[blockIdx.x];
  double* ks = e.ks;
  if (ks[KS_STOP] != 0.0) return;
  __shared__ double tot[2];
  const double* const src[2] = {e.part, e.part + nb};
  block_slot_sums<2>(src, 2, nb, tot);
  if (threadIdx.x != 0) return;
  FinRR::run(FinRR::Args{ks}, tot);
  const double flag = ks[KS_FLAG];
  if (flag == 1.0 || flag == 2.0) {
    ks[KS_STOP] = 1.0;
    ks[KS_REASON] = KR_BREAKDOWN;
    return;
  }
  ks[KS_ITER] += 1.0;
  const int nxt = kry_next(ks);
  ks[KS_CUR] = nxt;
  const double res = sqrt(ks[KS_RR]);
  if (res < ks[KS_RESBEST]) {
    ks[KS_BEST] = nxt;
    ks[KS_RESBEST] = res;
  }
  int reason = 0;
  if (res <= ks[KS_RTOLB]) reason = KR_CONVERGED;
  else if (flag != 0.0 || !isfinite(res) || res > diverged * ks[KS_BNORM]) reason = KR_OTHER;
  else if (ks[KS_ITER] >= ks[KS_MAXIT]) reason = KR_MAXIT;
  if (reason) {
    ks[KS_STOP] = 1.0;
    ks[KS_REASON] = reason;
  }
}

// run control of a batched solve at the start of a run (one thread): the
// first run starts from x = 0 with the best residual ||b|| (resbest < 0),
// a later one from the best iterate `cur` with its true residual.  rtol ||b||
// is formed from ||b|| on the device; b = 0 is solved at once.
__global__ void k_ks_run_start(double* ks, double iter, double cur, double resbest, double rtol, double maxit) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const double bnorm = ks[KS_BNORM];
    ks[KS_STOP] = bnorm == 0.0 ? 1.0 : 0.0;
    ks[KS_REASON] = bnorm == 0.0 ? double(KR_CONVERGED) : 0.0;
    ks[KS_ITER] = iter;
    ks[KS_CUR] = cur;
    ks[KS_BEST] = cur;
    ks[KS_RESBEST] = resbest < 0.0 ? bnorm : resbest;
    ks[KS_RTOLB] = rtol * bnorm;
    ks[KS_MAXIT] = maxit;
  }
}

// stop flag, reason, iteration count and best iterate of every solve of a
// batch -> out[4 b ...]
template <typename T>
__global__ void k_gather_run(const KryEntry<T>* __restrict__ E, int B, double* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) {
    out[4 * b] = E[b].ks[KS_STOP];
    out[4 * b + 1] = E[b].ks[KS_REASON];
    out[4 * b + 2] = E[b].ks[KS_ITER];
    out[4 * b + 3] = E[b].ks[KS_BEST];
  }
}

}  // namespace pff
