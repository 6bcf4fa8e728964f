// FFT pass kernels with fused point-wise stages.
//
// A multi-dimensional real FFT round trip is split into axis passes over a
// half spectrum stored per field as [z][y][kx], kx in [0, nx/2]:
//   k_xfwd : per row (y, z): a "prologue" computes NF real values per voxel,
//            pairs of fields are packed as one complex sequence, transformed
//            along x in LDS and unpacked into two half spectra;
//   k_axis : complex FFT along y or z for a tile of consecutive kx columns
//            (coalesced loads), optionally followed by the point-wise
//            "spectral" stage and the inverse transform along the same axis
//            (the last axis of the forward transform);
//   k_xinv : per row: the half spectra of two fields are packed into one
//            Hermitian-extended complex sequence, inverse-transformed along x
//            and an "epilogue" consumes the NF real values per voxel.
// A Pipe class supplies the fields, the point-wise stages and the
// per-block reductions (summed in a fixed order by k_reduce).
#pragma once

#include "common.hpp"
#include "fft.hpp"
#include "pointlaw.hpp"

namespace pff {

template <typename T> struct SpecTables {
  const T* hs[3];   // sin(q/2) per axis (x, y, z), indexed by mode index
  const T* hc[3];   // cos(q/2), exactly 0 at an even axis' Nyquist index
  const T* q2[3];   // q^2 (standard frequencies, Nyquist kept)
  T invN;
};

// Max LDS elements per thread of the in-place FFT (64 KB per block).
template <typename T> struct FftCap { static constexpr int MAXE = 8; };

template <class P>
__global__ void __launch_bounds__(FftThreads<typename P::real>::value) k_xfwd(const typename P::Args A, const AxisPlan pl,
                                                 const cpx<typename P::real>* __restrict__ tw_g,
                                                 cpx<typename P::real>* __restrict__ spec,
                                                 int rows_per_block, double* __restrict__ partials) {
  using T = typename P::real;
  constexpr int NF = P::NF;
  constexpr int NP = (NF + 1) / 2;
  constexpr int NR = P::NRED_PRO;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int nx = A.g.nx, nxh = A.g.nxh;
  const long long nrows = (long long)A.g.ny * A.g.nz;
  const int RB = rows_per_block;
  const int seq = RB * NP * nx;
  cpx<T>* bufa = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tw = bufa + seq;
  for (int t = threadIdx.x; t < nx; t += blockDim.x) tw[t] = tw_g[t];
  const long long row0 = (long long)blockIdx.x * RB;
  double red[NR > 0 ? NR : 1];
#pragma unroll
  for (int q = 0; q < (NR > 0 ? NR : 1); ++q) red[q] = 0.0;
  for (int idx = threadIdx.x; idx < RB * nx; idx += blockDim.x) {
    const int r = idx / nx, x = idx - r * nx;
    const long long row = row0 + r;
    T vals[2 * NP];
#pragma unroll
    for (int f = 0; f < 2 * NP; ++f) vals[f] = T(0);
    if (row < nrows) P::prologue(A, x + (long long)nx * row, vals, red);
#pragma unroll
    for (int p = 0; p < NP; ++p) bufa[(r * NP + p) * nx + x] = cpx<T>{vals[2 * p], vals[2 * p + 1]};
  }
  __syncthreads();
  fft_lds<T, -1, FftCap<T>::MAXE>(bufa, RB * NP, 0, pl, tw);
  const cpx<T>* res = bufa;
  const long long Nh = A.g.Nh;
  for (int idx = threadIdx.x; idx < RB * NP * nxh; idx += blockDim.x) {
    const int k = idx % nxh;
    const int rest = idx / nxh;
    const int p = rest % NP, r = rest / NP;
    const long long row = row0 + r;
    if (row >= nrows) continue;
    const cpx<T> Z = res[(r * NP + p) * nx + k];
    const cpx<T> Zm = res[(r * NP + p) * nx + (k == 0 ? 0 : nx - k)];
    // X_a = (Z + conj Zm)/2, X_b = (Z - conj Zm)/(2i)
    const cpx<T> Xa = {T(0.5) * (Z.x + Zm.x), T(0.5) * (Z.y - Zm.y)};
    const cpx<T> Xb = {T(0.5) * (Z.y + Zm.y), T(-0.5) * (Z.x - Zm.x)};
    const long long o = k + (long long)nxh * row;
    spec[(2 * p) * Nh + o] = Xa;
    if (2 * p + 1 < NF) spec[(2 * p + 1) * Nh + o] = Xb;
  }
  if constexpr (NR > 0) {
    __syncthreads();
    block_reduce<NR, FftThreads<T>::value>(red, reinterpret_cast<double*>(smem_raw));
    if (threadIdx.x == 0)
      for (int q = 0; q < NR; ++q) partials[(long long)q * gridDim.x + blockIdx.x] = red[q];
  }
}

// Complex FFT along y (axis 1) or z (axis 2) for a tile of TX consecutive
// kx columns, one index of the remaining axis (blockIdx.y) and a group of
// NFB fields (blockIdx.z).  With SPECTRAL (NFB = NF) the point-wise spectral
// stage and the inverse transform along the same axis follow.
template <class P, int S, bool SPECTRAL>
__global__ void __launch_bounds__(FftThreads<typename P::real>::value) k_axis(const typename P::Args A, const AxisPlan pl,
                                                 const cpx<typename P::real>* __restrict__ tw_g,
                                                 cpx<typename P::real>* __restrict__ spec, int axis,
                                                 int ltx, int NFB) {
  using T = typename P::real;
  constexpr int NF = P::NF;
  constexpr int MAXE = FftCap<T>::MAXE;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n = pl.n;
  const int TX = 1 << ltx;
  const int nxh = A.g.nxh, ny = A.g.ny;
  const long long Nh = A.g.Nh;
  const int kx0 = blockIdx.x * TX;
  const int o = blockIdx.y;                       // z for the y pass, y for the z pass
  const int f0 = blockIdx.z * NFB;
  const int nfb = (f0 + NFB <= NF) ? NFB : NF - f0;
  const long long stride = axis == 1 ? (long long)nxh : (long long)nxh * ny;
  const long long base = axis == 1 ? (long long)nxh * ny * o : (long long)nxh * o;
  const int seq = nfb * n * TX;
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tw = buf + NFB * n * TX;
  for (int t = threadIdx.x; t < n; t += blockDim.x) tw[t] = tw_g[t];
  for (int idx = threadIdx.x; idx < seq; idx += blockDim.x) {
    const int t = idx & (TX - 1);
    const int rest = idx >> ltx;                  // = f*n + j
    const int j = rest % n, f = rest / n;
    const int kx = kx0 + t;
    cpx<T> val = {T(0), T(0)};
    if (kx < nxh) val = spec[(f0 + f) * Nh + base + kx + stride * j];
    buf[idx] = val;
  }
  __syncthreads();
  fft_lds<T, S, MAXE>(buf, nfb, ltx, pl, tw);
  if constexpr (SPECTRAL) {
    for (int idx = threadIdx.x; idx < TX * n; idx += blockDim.x) {
      const int t = idx & (TX - 1), j = idx >> ltx;
      const int kx = kx0 + t;
      if (kx >= nxh) continue;
      cpx<T> v[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) v[f] = buf[(f * n + j) * TX + t];
      if (axis == 1) P::spectral(A, kx, j, 0, v);
      else P::spectral(A, kx, o, j, v);
#pragma unroll
      for (int f = 0; f < NF; ++f) buf[(f * n + j) * TX + t] = v[f];
    }
    __syncthreads();
    fft_lds<T, -S, MAXE>(buf, nfb, ltx, pl, tw);
  }
  for (int idx = threadIdx.x; idx < seq; idx += blockDim.x) {
    const int t = idx & (TX - 1);
    const int rest = idx >> ltx;
    const int j = rest % n, f = rest / n;
    const int kx = kx0 + t;
    if (kx < nxh) spec[(f0 + f) * Nh + base + kx + stride * j] = buf[idx];
  }
}

template <class P>
__global__ void __launch_bounds__(FftThreads<typename P::real>::value) k_xinv(const typename P::Args A, const AxisPlan pl,
                                                 const cpx<typename P::real>* __restrict__ tw_g,
                                                 const cpx<typename P::real>* __restrict__ spec,
                                                 int rows_per_block, double* __restrict__ partials) {
  using T = typename P::real;
  constexpr int NF = P::NF;
  constexpr int NP = (NF + 1) / 2;
  constexpr int NR = P::NRED_EPI;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int nx = A.g.nx, nxh = A.g.nxh;
  const long long nrows = (long long)A.g.ny * A.g.nz;
  const long long Nh = A.g.Nh;
  const int RB = rows_per_block;
  const int seq = RB * NP * nx;
  cpx<T>* bufa = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tw = bufa + seq;
  for (int t = threadIdx.x; t < nx; t += blockDim.x) tw[t] = tw_g[t];
  const long long row0 = (long long)blockIdx.x * RB;
  for (int idx = threadIdx.x; idx < seq; idx += blockDim.x) {
    const int x = idx % nx;
    const int rest = idx / nx;
    const int p = rest % NP, r = rest / NP;
    const long long row = row0 + r;
    cpx<T> Z = {T(0), T(0)};
    if (row < nrows) {
      const bool mirror = x > nx / 2;
      const int k = mirror ? nx - x : x;
      const long long o = k + (long long)nxh * row;
      cpx<T> a = spec[(2 * p) * Nh + o];
      cpx<T> b = (2 * p + 1 < NF) ? spec[(2 * p + 1) * Nh + o] : cpx<T>{T(0), T(0)};
      if (mirror) {
        a.y = -a.y;
        b.y = -b.y;
      }
      if (k == 0 || 2 * k == nx) {
        // DC and Nyquist bins of a real field are real: their imaginary parts
        // are round-off that would otherwise leak into the partner field of
        // the pair (a + i b).  Dropping them gives the real part of the full
        // inverse transform.
        a.y = T(0);
        b.y = T(0);
      }
      Z = cpx<T>{a.x - b.y, a.y + b.x};   // a + i b
    }
    bufa[(r * NP + p) * nx + x] = Z;
  }
  __syncthreads();
  fft_lds<T, 1, FftCap<T>::MAXE>(bufa, RB * NP, 0, pl, tw);
  const cpx<T>* res = bufa;
  double red[NR > 0 ? NR : 1];
#pragma unroll
  for (int q = 0; q < (NR > 0 ? NR : 1); ++q) red[q] = 0.0;
  for (int idx = threadIdx.x; idx < RB * nx; idx += blockDim.x) {
    const int r = idx / nx, x = idx - r * nx;
    const long long row = row0 + r;
    if (row >= nrows) continue;
    T vals[2 * NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const cpx<T> z = res[(r * NP + p) * nx + x];
      vals[2 * p] = z.x;
      vals[2 * p + 1] = z.y;
    }
    P::epilogue(A, x + (long long)nx * row, vals, red);
  }
  if constexpr (NR > 0) {
    __syncthreads();
    block_reduce<NR, FftThreads<T>::value>(red, reinterpret_cast<double*>(smem_raw));
    if (threadIdx.x == 0)
      for (int q = 0; q < NR; ++q) partials[(long long)q * gridDim.x + blockIdx.x] = red[q];
  }
}

// ---- spectral stage shared by the pipes -------------------------------------

// P(A) = (A n) n + n (A n) - (n.A n) n n on a real Mandel vector (in place).
template <typename T, int D>
__device__ __forceinline__ void project_mandel(T* a, const T (&n)[3]) {
  if constexpr (D == 2) {
    const T r = Consts<T>::rs2;
    const T A00 = a[0], A11 = a[1], A01 = r * a[2];
    const T An0 = A00 * n[0] + A01 * n[1];
    const T An1 = A01 * n[0] + A11 * n[1];
    const T nAn = n[0] * An0 + n[1] * An1;
    a[0] = T(2) * An0 * n[0] - nAn * n[0] * n[0];
    a[1] = T(2) * An1 * n[1] - nAn * n[1] * n[1];
    a[2] = Consts<T>::s2 * (An0 * n[1] + n[0] * An1 - nAn * n[0] * n[1]);
  } else {
    T W[3][3];
    mandel_to_tensor<T, 3>(a, W);
    T An[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) An[i] = W[i][0] * n[0] + W[i][1] * n[1] + W[i][2] * n[2];
    const T nAn = n[0] * An[0] + n[1] * An[1] + n[2] * An[2];
    T O[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) O[i][j] = An[i] * n[j] + n[i] * An[j] - nAn * n[i] * n[j];
    tensor_to_mandel<T, 3>(O, a);
  }
}

// vals[0..C-1]: projected with the rotated-scheme direction; vals[C]:
// multiplied by the Laplacian symbol; everything scaled by 1/N.
template <typename T, int DIM, int C, bool HAS_LAP>
__device__ __forceinline__ void spectral_proj_lap(const SpecTables<T>& tb, int kx, int ky, int kz,
                                                  cpx<T>* vals) {
  const T sx = tb.hs[0][kx], cx = tb.hc[0][kx];
  const T sy = tb.hs[1][ky], cy = tb.hc[1][ky];
  T sz = T(0), cz = T(1);
  if constexpr (DIM == 3) {
    sz = tb.hs[2][kz];
    cz = tb.hc[2][kz];
  }
  T n[3] = {sx * cy * cz, cx * sy * cz, cx * cy * sz};
  const T r2 = n[0] * n[0] + n[1] * n[1] + n[2] * n[2];
  if (C > 0) {
    if (r2 == T(0)) {
#pragma unroll
      for (int k = 0; k < C; ++k) vals[k] = cpx<T>{T(0), T(0)};
    } else {
      const T s = T(1) / sqrt(r2);
      n[0] *= s; n[1] *= s; n[2] *= s;
      T re[C > 0 ? C : 1], im[C > 0 ? C : 1];
#pragma unroll
      for (int k = 0; k < C; ++k) { re[k] = vals[k].x; im[k] = vals[k].y; }
      project_mandel<T, (DIM == 2 ? 2 : 3)>(re, n);
      project_mandel<T, (DIM == 2 ? 2 : 3)>(im, n);
#pragma unroll
      for (int k = 0; k < C; ++k) vals[k] = cpx<T>{re[k] * tb.invN, im[k] * tb.invN};
    }
  }
  if constexpr (HAS_LAP) {
    T q2 = tb.q2[0][kx] + tb.q2[1][ky];
    if constexpr (DIM == 3) q2 += tb.q2[2][kz];
    const T L = -q2 * tb.invN;
    vals[C] = cpx<T>{L * vals[C].x, L * vals[C].y};
  }
}

// Fixed-order reduction of per-block partials; Fin consumes the totals.
template <class Fin>
__global__ void __launch_bounds__(kBlock) k_reduce(const double* __restrict__ partials, int nblk,
                                                   int nslot, const typename Fin::Args F) {
  __shared__ double lds[kBlock];
  __shared__ double tot[kMaxRed];
  for (int q = 0; q < nslot; ++q) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) acc += partials[(long long)q * nblk + b];
    lds[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) tot[q] = lds[0];
    __syncthreads();
  }
  if (threadIdx.x == 0) Fin::run(F, tot);
}

}  // namespace pff
