// Common device types and helpers for the phase-field FFT solver kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fastdiv.hpp"

namespace pff {

constexpr int kBlock = 256;          // threads per workgroup of vector kernels (4 wavefronts)
// threads per workgroup of the FFT pass kernels (at most 8 LDS elements per
// thread).  512 for both precisions: FP32 x-pass tiles of 32 KB let three to
// four blocks share a CU, so one block's loads overlap another's transform
// (1024-thread, 64 KB blocks left the x-forward pass latency-bound in the
// solve: 89 us against 55 us per launch at 128^3).
template <typename T> struct FftThreads { static constexpr int value = 512; };

// The LDS tiles of the x passes are padded by one element every 32: their
// Stockham stages write outputs at strides of R * Ns elements of contiguous
// rows, which without the pad fall on few banks (measured: 2.3 bank-conflict
// cycles per LDS instruction, halved by the pad, and the x-inverse pass's
// LDS wait cycles halved).  The interleaved tiles of the y/z passes are not
// padded: their columns already spread the banks, and the extra index
// arithmetic cost more than it saved there.
__host__ __device__ __forceinline__ int lpad(int i) { return i + (i >> 5); }
template <bool PAD> __host__ __device__ __forceinline__ int lidx(int i) { return PAD ? lpad(i) : i; }
__host__ __device__ __forceinline__ long long lds_padded(long long n) { return n + (n >> 5) + 1; }
constexpr int kMaxPhases = 16;
constexpr int kMaxRed = 12;          // reduction slots per pass
constexpr int kMaxStages = 10;

// Totals of NQ slots of per-block partials (slot q at src[q], nblk entries;
// the first nq slots are summed) by one block of kBlock threads, in a fixed
// order: every thread adds a strided subset of all slots at once, each
// wavefront combines its 64 lanes by an xor butterfly (lane 0's sum is
// taken), and the wavefront sums are added in order.  tot: nq doubles.
template <int NQ>
__device__ __forceinline__ void block_slot_sums(const double* const (&src)[NQ], int nq, int nblk,
                                                double* tot) {
  __shared__ double wsum[NQ][kBlock / 64];
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kBlock) {
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      if (q < nq) acc[q] += src[q][b];
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    if (q < nq) {
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) acc[q] += __shfl_xor(acc[q], o, 64);
      if (lane == 0) wsum[q][w] = acc[q];
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < nq) {
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) t += wsum[threadIdx.x][i];
    tot[threadIdx.x] = t;
  }
  __syncthreads();
}

template <typename T> struct cpx { T x, y; };

template <typename T> __device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T> __device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) {
  return {a.x + b.x, a.y + b.y};
}
template <typename T> __device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) {
  return {a.x - b.x, a.y - b.y};
}
template <typename T> __device__ __forceinline__ cpx<T> cconj(cpx<T> a) { return {a.x, -a.y}; }
// multiply by s*i (s = +1 or -1)
template <typename T, int S> __device__ __forceinline__ cpx<T> mul_si(cpx<T> a) {
  return S > 0 ? cpx<T>{-a.y, a.x} : cpx<T>{a.y, -a.x};
}

// One FFT axis: length n = prod(radix), twiddles tw[k] = exp(-2 pi i k / n).
// Per stage st (Stockham, Ns = product of the earlier radices) the
// reciprocal divisors of n / radix[st] and of Ns, and of n itself.
struct AxisPlan {
  int n;
  int nstage;
  int radix[kMaxStages];
  FastDiv dn;
  FastDiv dnb[kMaxStages], dns[kMaxStages];
};

// Per-phase material constants (Lame lambda, mu and toughness Gc).
struct Material {
  int nphase;
  int iso;       // 1: isotropic degradation (no split): sigma = g sigma0, C = g C0, psi0 drives H
  double lam[kMaxPhases], mu[kMaxPhases], Gc[kMaxPhases];
};

// Small per-component constant vector passed by value (e.g. f in Mandel form).
struct Vec16 {
  double v[16];
};

// Geometry of the voxel grid and of the x-halved spectrum.
// Half spectrum of one field (Nh points): a main block [z][y][kx], kx in
// [0, nxm), with row pitch nxm (= nx/2 for even nx: 128-byte aligned rows for
// the benchmark sizes), followed, for even nx, by the Nyquist plane
// kx = nx/2 stored as [z][y].
struct GridDesc {
  int nx, ny, nz, nxh;   // nxh = nx/2 + 1
  long long N, Nh;       // voxels, half-spectrum points per field
  int nxm, nyq;          // main-block columns; 1 if the Nyquist plane exists
  long long Nm;          // points of the main block (nz ny nxm)
  FastDiv dnxm;          // division by nxm
};

// Deterministic block reduction of NR double accumulators; thread 0 of the
// block ends with the totals.  Fixed pairing order -> bitwise reproducible.
template <int NR, int BS = kBlock>
__device__ __forceinline__ void block_reduce(double (&v)[NR], double* lds /* NR*BS */) {
  const int t = threadIdx.x;
#pragma unroll
  for (int q = 0; q < NR; ++q) lds[q * BS + t] = v[q];
  __syncthreads();
  for (int s = BS / 2; s > 0; s >>= 1) {
    if (t < s) {
#pragma unroll
      for (int q = 0; q < NR; ++q) lds[q * BS + t] += lds[q * BS + t + s];
    }
    __syncthreads();
  }
  if (t == 0) {
#pragma unroll
    for (int q = 0; q < NR; ++q) v[q] = lds[q * BS];
  }
  __syncthreads();
}

}  // namespace pff
