// FFT pass kernels with fused point-wise stages.
//
// A multi-dimensional real FFT round trip is split into axis passes over a
// half spectrum stored per field as a main block [z][y][kx], kx < nxm, and
// (even nx) the Nyquist plane kx = nx/2 as [z][y] (see GridDesc):
//   k_xfwd : per row (y, z): a "prologue" computes NF real values per voxel,
//            pairs of fields are packed as one complex sequence, transformed
//            along x in LDS and unpacked into two half spectra;
//   k_axis : complex FFT along y or z for a tile of consecutive kx columns
//            (aligned 128-byte row segments) or of the Nyquist plane,
//            optionally followed by the point-wise
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
  const T* hs[3];   // sin(q/2) per axis (x, y, z), indexed by mode index (standard scheme: q)
  const T* hc[3];   // cos(q/2), exactly 0 at an even axis' Nyquist index (standard scheme: 1)
  const T* q2[3];   // q^2 (standard frequencies, Nyquist kept)
  T invN;
  const T* fh;      // f / |f| in Mandel components: the zero mode projects onto
                    // its complement (mixed macroscopic conditions); null: G(0) = 0
};

// Max LDS elements per thread of the in-place FFT (64 KB per block).
template <typename T> struct FftCap { static constexpr int MAXE = 8; };

// One RVE of a batched launch: its pipe arguments, half spectra, partial-sum
// buffers and the stop flag of its Krylov solve (non-zero: every block of
// this RVE returns at once).  A batched launch adds one grid dimension over
// the entries; an unbatched one passes a null batch and its own arguments.
// Pipes whose kernels take batched launches (the others compile without
// the batched branch).
template <class P> struct Batchable : std::false_type {};

template <class P> struct BatchEntry {
  typename P::Args A;
  cpx<typename P::real>* spec;
  double* part0;
  double* part1;
  const double* stop;
};

// rows_per_block rows of x per block (blockIdx.x).  BATCHED: one RVE of the
// batch per blockIdx.y, its arguments, spectra and partials from its entry
// (a separate instantiation: the unbatched kernel is the plain code).
template <class P, bool ANY, bool BATCHED = false>
__global__ void __launch_bounds__(FftThreads<typename P::real>::value) k_xfwd(const typename P::Args A_in, const AxisPlan pl,
                                                 const cpx<typename P::real>* __restrict__ tw_g,
                                                 cpx<typename P::real>* __restrict__ spec_in,
                                                 int rows_per_block, double* __restrict__ partials_in,
                                                 const BatchEntry<P>* __restrict__ batch) {
  using T = typename P::real;
  const BatchEntry<P>* e = nullptr;
  if constexpr (BATCHED) {
    e = &batch[blockIdx.y];
    if (e->stop && *e->stop != 0.0) return;
  }
  const typename P::Args& A = BATCHED ? e->A : A_in;
  cpx<T>* __restrict__ spec = BATCHED ? e->spec : spec_in;
  double* __restrict__ partials = BATCHED ? e->part0 : partials_in;
  constexpr int NF = P::NF;
  constexpr int NP = (NF + 1) / 2;
  constexpr int NR = P::NRED_PRO;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int nx = A.g.nx, nxh = A.g.nxh;
  const long long nrows = (long long)A.g.ny * A.g.nz;
  const int RB = rows_per_block;
  const int seq = RB * NP * nx;
  cpx<T>* bufa = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tw = bufa + lds_padded(seq);
  for (int t = threadIdx.x; t < nx; t += blockDim.x) tw[t] = tw_g[t];
  const long long row0 = (long long)blockIdx.x * RB;
  double red[NR > 0 ? NR : 1];
#pragma unroll
  for (int q = 0; q < (NR > 0 ? NR : 1); ++q) red[q] = 0.0;
  for (int idx = threadIdx.x; idx < RB * nx; idx += blockDim.x) {
    const int r = (int)fdiv((uint32_t)idx, pl.dn), x = idx - r * nx;
    const long long row = row0 + r;
    T vals[2 * NP];
#pragma unroll
    for (int f = 0; f < 2 * NP; ++f) vals[f] = T(0);
    if (row < nrows) P::prologue(A, x + (long long)nx * row, vals, red);
#pragma unroll
    for (int p = 0; p < NP; ++p) bufa[lpad((r * NP + p) * nx + x)] = cpx<T>{vals[2 * p], vals[2 * p + 1]};
  }
  __syncthreads();
  fft_lds<T, -1, FftCap<T>::MAXE, ANY, true>(bufa, RB * NP, 0, pl, tw);
  const cpx<T>* res = bufa;
  const long long Nh = A.g.Nh;
  const int nxm = A.g.nxm;
  const int nrow_here = (int)((nrows - row0) < RB ? (nrows - row0) : RB);
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    cpx<T>* sa = spec + (long long)(2 * p) * Nh;
    cpx<T>* sb = spec + (long long)(2 * p + 1) * Nh;
    // main block: the rows of this block are contiguous with pitch nxm
    for (int idx = threadIdx.x; idx < nrow_here * nxm; idx += blockDim.x) {
      const int r = (int)fdiv((uint32_t)idx, A.g.dnxm);
      const int k = idx - r * nxm;
      const cpx<T> Z = res[lpad((r * NP + p) * nx + k)];
      const cpx<T> Zm = res[lpad((r * NP + p) * nx + (k == 0 ? 0 : nx - k))];
      // X_a = (Z + conj Zm)/2, X_b = (Z - conj Zm)/(2i)
      const long long o = row0 * nxm + idx;
      sa[o] = cpx<T>{T(0.5) * (Z.x + Zm.x), T(0.5) * (Z.y - Zm.y)};
      if (2 * p + 1 < NF) sb[o] = cpx<T>{T(0.5) * (Z.y + Zm.y), T(-0.5) * (Z.x - Zm.x)};
    }
    // Nyquist plane (even nx): one value per row
    if (A.g.nyq) {
      for (int r = threadIdx.x; r < nrow_here; r += blockDim.x) {
        const cpx<T> Z = res[lpad((r * NP + p) * nx + nx / 2)];
        const long long o = A.g.Nm + row0 + r;
        sa[o] = cpx<T>{Z.x, T(0)};
        if (2 * p + 1 < NF) sb[o] = cpx<T>{Z.y, T(0)};
      }
    }
  }
  if constexpr (NR > 0) {
    __syncthreads();
    block_reduce<NR, FftThreads<T>::value>(red, reinterpret_cast<double*>(smem_raw));
    if (threadIdx.x == 0)
      for (int q = 0; q < NR; ++q) partials[(long long)q * gridDim.x + blockIdx.x] = red[q];
  }
}

constexpr int kXcds = 8;   // MI355X: workgroups are dispatched round-robin over 8 XCDs

// Complex FFT along y (axis 1) or z (axis 2) for one tile and a group of NFB
// fields (blockIdx.z).  Tiles (blockIdx.x, blockIdx.y):
//   main block: TX consecutive kx columns (one 128-byte row segment for
//   TX * sizeof(complex) = 128) at z = blockIdx.y (y pass) or y = blockIdx.y
//   (z pass);
//   Nyquist plane (blockIdx.x = number of main tiles, even nx only): TX
//   consecutive z (y pass: pencils of [z][y] along y) or TX consecutive y
//   (z pass) starting at blockIdx.y * TX; blocks past the plane exit.
// With SPECTRAL (NFB = NF) the point-wise spectral stage and the inverse
// transform along the same axis follow.  With remap, consecutive tiles are
// given to workgroups on the same XCD, so that two tiles sharing 128-byte
// lines meet in that XCD's L2.
template <class P, int S, bool SPECTRAL, bool ANY>
__device__ __forceinline__ void axis_body(const typename P::Args A, const AxisPlan pl,
                                          const cpx<typename P::real>* __restrict__ tw_g,
                                          cpx<typename P::real>* __restrict__ spec, int axis, int ltx, int NFB,
                                          int remap, int fg) {
  using T = typename P::real;
  constexpr int NF = P::NF;
  constexpr int MAXE = FftCap<T>::MAXE;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const GridDesc& g = A.g;
  const int n = pl.n;
  const int TX = 1 << ltx;
  int bx = blockIdx.x, by = blockIdx.y;
  if (remap) {
    const int nb = gridDim.x * gridDim.y;
    const int per = nb / kXcds;
    int b = blockIdx.y * gridDim.x + blockIdx.x;
    if (b < per * kXcds) b = (b % kXcds) * per + b / kXcds;
    bx = b % gridDim.x;
    by = b / gridDim.x;
  }
  const int nkt = (g.nxm + TX - 1) >> ltx;
  // element (j, t) of a field at off0 + j * js + t * ts, valid for t < tc;
  // its mode (kx, ky, kz) = (kxb + t kxs, ., .) with j on the pass axis
  long long off0;
  int js, ts, tc, kxb, kxs, kb, ks;   // kb + t ks: the index of the third axis
  if (bx < nkt) {
    const int kx0 = bx << ltx;
    tc = min(TX, g.nxm - kx0);
    ts = 1;
    kxb = kx0;
    kxs = 1;
    kb = by;
    ks = 0;
    if (axis == 1) {
      off0 = (long long)by * g.ny * g.nxm + kx0;
      js = g.nxm;
    } else {
      off0 = (long long)by * g.nxm + kx0;
      js = g.ny * g.nxm;
    }
  } else {
    kxb = g.nx / 2;
    kxs = 0;
    const int q0 = by << ltx;
    const int lim = axis == 1 ? g.nz : g.ny;
    if (q0 >= lim) return;
    tc = min(TX, lim - q0);
    kb = q0;
    ks = 1;
    if (axis == 1) {
      off0 = g.Nm + (long long)q0 * g.ny;
      js = 1;
      ts = g.ny;
    } else {
      off0 = g.Nm + q0;
      js = g.ny;
      ts = 1;
    }
  }
  const int f0 = fg * NFB;
  const int nfb = (f0 + NFB <= NF) ? NFB : NF - f0;
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tw = buf + NFB * n * TX;
  for (int t = threadIdx.x; t < n; t += blockDim.x) tw[t] = tw_g[t];
  const int per_field = n << ltx;
  for (int f = 0; f < nfb; ++f) {
    const cpx<T>* src = spec + (long long)(f0 + f) * g.Nh + off0;
    for (int i2 = threadIdx.x; i2 < per_field; i2 += blockDim.x) {
      const int t = i2 & (TX - 1), j = i2 >> ltx;
      cpx<T> val = {T(0), T(0)};
      if (t < tc) val = src[j * js + t * ts];
      buf[f * per_field + i2] = val;
    }
  }
  __syncthreads();
  fft_lds<T, S, MAXE, ANY, false>(buf, nfb, ltx, pl, tw);
  if constexpr (SPECTRAL) {
    for (int idx = threadIdx.x; idx < per_field; idx += blockDim.x) {
      const int t = idx & (TX - 1), j = idx >> ltx;
      if (t >= tc) continue;
      const int kx = kxb + t * kxs, kq = kb + t * ks;
      cpx<T> v[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) v[f] = buf[f * per_field + idx];
      if (axis == 1) P::spectral(A, kx, j, kq, v);
      else P::spectral(A, kx, kq, j, v);
#pragma unroll
      for (int f = 0; f < NF; ++f) buf[f * per_field + idx] = v[f];
    }
    __syncthreads();
    fft_lds<T, -S, MAXE, ANY, false>(buf, nfb, ltx, pl, tw);
  }
  for (int f = 0; f < nfb; ++f) {
    cpx<T>* dst = spec + (long long)(f0 + f) * g.Nh + off0;
    for (int i2 = threadIdx.x; i2 < per_field; i2 += blockDim.x) {
      const int t = i2 & (TX - 1), j = i2 >> ltx;
      if (t < tc) dst[j * js + t * ts] = buf[f * per_field + i2];
    }
  }
}

// The last axis of a 3D round trip (z) for lengths N = 32, 64, 128 as one
// pass with the first and the last radix stage in registers: N = RA * 4,
//   forward stage A (radix RA, span 1): loaded straight from the spectra,
//                 written to LDS;
//   forward stage B (radix 4, span RA), the spectral stage on the four modes
//                 kz = j2 + r RA of the item (all NF fields at once) and the
//                 inverse stage B' (radix 4, span 1), which reads exactly the
//                 outputs of stage B: all in registers, one LDS read and one
//                 LDS write;
//   inverse stage A' (radix RA, span 4): read from LDS, stored straight to
//                 the spectra.
// Each element crosses the LDS twice per direction instead of once per
// radix stage plus the staging copies.  Tiles as in k_axis (axis 2): TX
// consecutive kx columns of the main block at one y, or TX consecutive y of
// the Nyquist plane; RA * TX threads.  The tile is padded by one element
// every 32.  (A second padding for the inverse exchange, eight every 32,
// removes the 4-way bank conflicts of the stage-B' writes at N = 128, but
// the larger tile made the pass slower, 39.7 against 38.7 us.)
template <class P, int N, int TX> struct ZspecLds {
  static constexpr long long E = (long long)P::NF * N * TX;
  static constexpr long long ELEMS = E + (E >> 5) + 1;   // the padded tile (lds_padded), then N twiddles
};
// field groups of NFB fields on blockIdx.z
template <class P, int S, bool SPECTRAL, bool ANY>
__global__ void __launch_bounds__(FftThreads<typename P::real>::value) k_axis(const typename P::Args A, const AxisPlan pl,
                                                 const cpx<typename P::real>* __restrict__ tw_g,
                                                 cpx<typename P::real>* __restrict__ spec, int axis,
                                                 int ltx, int NFB, int remap) {
  axis_body<P, S, SPECTRAL, ANY>(A, pl, tw_g, spec, axis, ltx, NFB, remap, blockIdx.z);
}

// batched launch: blockIdx.z = RVE * NG + group, NG = ceil(NF / NFB)
template <class P, int S, bool SPECTRAL, bool ANY>
__global__ void __launch_bounds__(FftThreads<typename P::real>::value) k_axis_b(const BatchEntry<P>* __restrict__ batch,
                                                   const AxisPlan pl,
                                                   const cpx<typename P::real>* __restrict__ tw_g, int axis,
                                                   int ltx, int NFB, int remap) {
  const int ng = (P::NF + NFB - 1) / NFB;
  const BatchEntry<P>& e = batch[blockIdx.z / ng];
  if (e.stop && *e.stop != 0.0) return;
  axis_body<P, S, SPECTRAL, ANY>(e.A, pl, tw_g, e.spec, axis, ltx, NFB, remap, blockIdx.z % ng);
}

template <class P, int N, int TX>
__device__ __forceinline__ void zspec_body(const typename P::Args A, const cpx<typename P::real>* __restrict__ tw_g,
                                           cpx<typename P::real>* __restrict__ spec, int remap) {
  using T = typename P::real;
  constexpr int NF = P::NF;
  constexpr int RA = N / 4;
  constexpr int NT = RA * TX;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const GridDesc& g = A.g;
  int bx = blockIdx.x, by = blockIdx.y;
  if (remap) {
    const int nb = gridDim.x * gridDim.y;
    const int per = nb / kXcds;
    int b = blockIdx.y * gridDim.x + blockIdx.x;
    if (b < per * kXcds) b = (b % kXcds) * per + b / kXcds;
    bx = b % gridDim.x;
    by = b / gridDim.x;
  }
  const int nkt = (g.nxm + TX - 1) / TX;
  long long off0;
  int js, ts, tc, kxb, kxs, kb, ks;
  if (bx < nkt) {
    const int kx0 = bx * TX;
    tc = min(TX, g.nxm - kx0);
    ts = 1;
    kxb = kx0;
    kxs = 1;
    kb = by;
    ks = 0;
    off0 = (long long)by * g.nxm + kx0;
    js = g.ny * g.nxm;
  } else {
    kxb = g.nx / 2;
    kxs = 0;
    const int q0 = by * TX;
    if (q0 >= g.ny) return;
    tc = min(TX, g.ny - q0);
    kb = q0;
    ks = 1;
    off0 = g.Nm + q0;
    js = g.ny;
    ts = 1;
  }
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tw = buf + ZspecLds<P, N, TX>::ELEMS;
  for (int t = threadIdx.x; t < N; t += NT) tw[t] = tw_g[t];
  auto L = [](int f, int pos, int t) { return lpad((f * N + pos) * TX + t); };
  // forward stage A
  for (int item = threadIdx.x; item < NF * 4 * TX; item += NT) {
    const int t = item % TX, j = (item / TX) % 4, f = item / (4 * TX);
    const cpx<T>* src = spec + (long long)f * g.Nh + off0 + (long long)t * ts;
    cpx<T> v[RA];
#pragma unroll
    for (int r = 0; r < RA; ++r) v[r] = t < tc ? src[(long long)(j + 4 * r) * js] : cpx<T>{T(0), T(0)};
    dft_pow2<T, -1, RA>(v);
#pragma unroll
    for (int m = 0; m < RA; ++m) buf[L(f, j * RA + m, t)] = v[m];
  }
  __syncthreads();
  {
    const int t = threadIdx.x % TX, j2 = threadIdx.x / TX;
    cpx<T> v[NF][4];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
#pragma unroll
      for (int r = 0; r < 4; ++r) v[f][r] = buf[L(f, j2 + r * RA, t)];
#pragma unroll
      for (int r = 1; r < 4; ++r) v[f][r] = cmul(v[f][r], tw[r * j2]);
      dft4<T, -1>(v[f]);
    }
    if (t < tc) {
      const int kx = kxb + t * kxs, ky = kb + t * ks;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        cpx<T> vals[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) vals[f] = v[f][r];
        P::spectral(A, kx, ky, j2 + r * RA, vals);
#pragma unroll
        for (int f = 0; f < NF; ++f) v[f][r] = vals[f];
      }
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) dft4<T, 1>(v[f]);
    __syncthreads();      // every stage-B read is done before the stage-B' writes
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int r = 0; r < 4; ++r) buf[L(f, j2 * 4 + r, t)] = v[f][r];
  }
  __syncthreads();
  // inverse stage A'
  for (int item = threadIdx.x; item < NF * 4 * TX; item += NT) {
    const int t = item % TX, j = (item / TX) % 4, f = item / (4 * TX);
    cpx<T> v[RA];
#pragma unroll
    for (int r = 0; r < RA; ++r) v[r] = buf[L(f, j + 4 * r, t)];
#pragma unroll
    for (int r = 1; r < RA; ++r) {
      cpx<T> w = tw[r * j];
      w.y = -w.y;
      v[r] = cmul(v[r], w);
    }
    dft_pow2<T, 1, RA>(v);
    if (t < tc) {
      cpx<T>* dst = spec + (long long)f * g.Nh + off0 + (long long)t * ts;
#pragma unroll
      for (int m = 0; m < RA; ++m) dst[(long long)(j + 4 * m) * js] = v[m];
    }
  }
}

template <class P, int N, int TX>
__global__ void __launch_bounds__(N / 4 * TX) k_zspec(const typename P::Args A,
                                                     const cpx<typename P::real>* __restrict__ tw_g,
                                                     cpx<typename P::real>* __restrict__ spec, int remap) {
  zspec_body<P, N, TX>(A, tw_g, spec, remap);
}

// batched launch: RVE blockIdx.z
template <class P, int N, int TX>
__global__ void __launch_bounds__(N / 4 * TX) k_zspec_b(const BatchEntry<P>* __restrict__ batch,
                                                       const cpx<typename P::real>* __restrict__ tw_g, int remap) {
  const BatchEntry<P>& e = batch[blockIdx.z];
  if (e.stop && *e.stop != 0.0) return;
  zspec_body<P, N, TX>(e.A, tw_g, e.spec, remap);
}

// The y passes of a 3D round trip for lengths N = 32, 64, 128 with the first
// and the last radix stage in registers, N = RA * 4 (decimation in time):
//   stage A (radix RA over the rows j + 4 r, j < 4): loaded straight from the
//           spectra, written to LDS as Y_j[m];
//   stage B (radix 4 over j, twiddles w^(j m)): read from LDS and stored
//           straight to the spectra at rows m + RA q (natural order).
// Each element crosses the LDS once instead of once per radix stage plus the
// staging copies.  S = -1 forward, +1 inverse (conjugate twiddles, no
// scaling: the x-inverse pass scales).  Tiles as in k_axis (axis 1): TX
// consecutive kx columns of the main block at one z, or TX consecutive z of
// the Nyquist plane; one field per block (blockIdx.z); 4 * TX threads, each
// holding one radix-RA transform in stage A.
template <class T, int N, int TX> struct YregLds {
  static constexpr int E = N * TX;
  static constexpr int ELEMS = E + (E >> 5) + 1;   // the padded tile, then N twiddles
};

template <class T, int N, int TX, int S>
__device__ __forceinline__ void yreg_body(const GridDesc& g, const cpx<T>* __restrict__ tw_g,
                                          cpx<T>* __restrict__ spec, int field, int bx, int by) {
  constexpr int RA = N / 4;
  constexpr int NT = 4 * TX;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int nkt = (g.nxm + TX - 1) / TX;
  long long off0;
  int js, ts, tc;
  if (bx < nkt) {
    const int kx0 = bx * TX;
    tc = min(TX, g.nxm - kx0);
    off0 = (long long)by * g.ny * g.nxm + kx0;
    js = g.nxm;
    ts = 1;
  } else {
    const int q0 = by * TX;
    if (q0 >= g.nz) return;
    tc = min(TX, g.nz - q0);
    off0 = g.Nm + (long long)q0 * g.ny;
    js = 1;
    ts = g.ny;
  }
  cpx<T>* buf = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tw = buf + YregLds<T, N, TX>::ELEMS;
  for (int t = threadIdx.x; t < N; t += NT) tw[t] = tw_g[t];
  cpx<T>* base = spec + (long long)field * g.Nh + off0;
  {
    const int t = threadIdx.x % TX, j = threadIdx.x / TX;
    const cpx<T>* src = base + (long long)t * ts;
    cpx<T> v[RA];
#pragma unroll
    for (int r = 0; r < RA; ++r) v[r] = t < tc ? src[(long long)(j + 4 * r) * js] : cpx<T>{T(0), T(0)};
    dft_pow2<T, S, RA>(v);
#pragma unroll
    for (int m = 0; m < RA; ++m) buf[lpad((j * RA + m) * TX + t)] = v[m];
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < RA / 4; ++it) {
    const int item = it * NT + threadIdx.x;
    const int t = item % TX, m = item / TX;
    cpx<T> v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = buf[lpad((j * RA + m) * TX + t)];
#pragma unroll
    for (int j = 1; j < 4; ++j) {
      cpx<T> w = tw[j * m];
      if constexpr (S > 0) w.y = -w.y;
      v[j] = cmul(v[j], w);
    }
    dft4<T, S>(v);
    if (t < tc) {
      cpx<T>* dst = base + (long long)t * ts;
#pragma unroll
      for (int q = 0; q < 4; ++q) dst[(long long)(m + RA * q) * js] = v[q];
    }
  }
}

template <class P, int N, int TX, int S>
__global__ void __launch_bounds__(4 * TX) k_yreg(const typename P::Args A,
                                                 const cpx<typename P::real>* __restrict__ tw_g,
                                                 cpx<typename P::real>* __restrict__ spec) {
  yreg_body<typename P::real, N, TX, S>(A.g, tw_g, spec, blockIdx.z, blockIdx.x, blockIdx.y);
}

// batched launch: blockIdx.z = RVE * NF + field
template <class P, int N, int TX, int S>
__global__ void __launch_bounds__(4 * TX) k_yreg_b(const BatchEntry<P>* __restrict__ batch,
                                                   const cpx<typename P::real>* __restrict__ tw_g) {
  const BatchEntry<P>& e = batch[blockIdx.z / P::NF];
  if (e.stop && *e.stop != 0.0) return;
  yreg_body<typename P::real, N, TX, S>(e.A.g, tw_g, e.spec, blockIdx.z % P::NF, blockIdx.x, blockIdx.y);
}

// BATCHED: one RVE of the batch per blockIdx.y (as k_xfwd)
template <class P, bool ANY, bool BATCHED = false>
__global__ void __launch_bounds__(FftThreads<typename P::real>::value) k_xinv(const typename P::Args A_in, const AxisPlan pl,
                                                 const cpx<typename P::real>* __restrict__ tw_g,
                                                 const cpx<typename P::real>* __restrict__ spec_in,
                                                 int rows_per_block, double* __restrict__ partials_in,
                                                 const BatchEntry<P>* __restrict__ batch) {
  using T = typename P::real;
  const BatchEntry<P>* e = nullptr;
  if constexpr (BATCHED) {
    e = &batch[blockIdx.y];
    if (e->stop && *e->stop != 0.0) return;
  }
  const typename P::Args& A = BATCHED ? e->A : A_in;
  const cpx<T>* __restrict__ spec = BATCHED ? e->spec : spec_in;
  double* __restrict__ partials = BATCHED ? e->part1 : partials_in;
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
  cpx<T>* tw = bufa + lds_padded(seq);
  for (int t = threadIdx.x; t < nx; t += blockDim.x) tw[t] = tw_g[t];
  const long long row0 = (long long)blockIdx.x * RB;
  const int nxm = A.g.nxm;
  const int nrow_here = (int)((nrows - row0) < RB ? (nrows - row0) : RB);
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const cpx<T>* sa = spec + (long long)(2 * p) * Nh;
    const cpx<T>* sb = spec + (long long)(2 * p + 1) * Nh;
    for (int idx = threadIdx.x; idx < RB * nx; idx += blockDim.x) {
      const int r = (int)fdiv((uint32_t)idx, pl.dn);
      const int x = idx - r * nx;
      cpx<T> Z = {T(0), T(0)};
      if (r < nrow_here) {
        const bool mirror = x > nx / 2;
        const int k = mirror ? nx - x : x;
        const long long o = k < nxm ? (row0 + r) * nxm + k : A.g.Nm + row0 + r;
        cpx<T> a = sa[o];
        cpx<T> b = (2 * p + 1 < NF) ? sb[o] : cpx<T>{T(0), T(0)};
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
      bufa[lpad((r * NP + p) * nx + x)] = Z;
    }
  }
  __syncthreads();
  fft_lds<T, 1, FftCap<T>::MAXE, ANY, true>(bufa, RB * NP, 0, pl, tw);
  const cpx<T>* res = bufa;
  double red[NR > 0 ? NR : 1];
#pragma unroll
  for (int q = 0; q < (NR > 0 ? NR : 1); ++q) red[q] = 0.0;
  for (int idx = threadIdx.x; idx < RB * nx; idx += blockDim.x) {
    const int r = (int)fdiv((uint32_t)idx, pl.dn), x = idx - r * nx;
    const long long row = row0 + r;
    if (row >= nrows) continue;
    T vals[2 * NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const cpx<T> z = res[lpad((r * NP + p) * nx + x)];
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
      if (tb.fh && kx == 0 && ky == 0 && (DIM == 2 || kz == 0)) {
        // mean of the field under mixed macroscopic conditions: keep the
        // part orthogonal to f (the mean is real)
        T d = T(0);
#pragma unroll
        for (int k = 0; k < C; ++k) d += tb.fh[k] * vals[k].x;
#pragma unroll
        for (int k = 0; k < C; ++k) vals[k] = cpx<T>{(vals[k].x - d * tb.fh[k]) * tb.invN, T(0)};
      } else {
#pragma unroll
        for (int k = 0; k < C; ++k) vals[k] = cpx<T>{T(0), T(0)};
      }
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
  __shared__ double tot[kMaxRed];
  const double* src[kMaxRed];
#pragma unroll
  for (int q = 0; q < kMaxRed; ++q) src[q] = partials + (long long)(q < nslot ? q : 0) * nblk;
  block_slot_sums<kMaxRed>(src, nslot, nblk, tot);
  if (threadIdx.x == 0) Fin::run(F, tot);
}

}  // namespace pff
