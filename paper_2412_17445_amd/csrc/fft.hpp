// Batched mixed-radix Stockham FFT over sequences held in LDS.
//
// Decimation-in-time Stockham autosort (no bit reversal): with Ns the
// product of the radices already applied, butterfly j of a radix-R stage
// reads the R inputs j + r*n/R, multiplies input r by w_{Ns*R}^{r*(j mod Ns)},
// applies an R-point DFT and writes output r to (j div Ns)*Ns*R + j mod Ns +
// r*Ns.  Radices 2, 3, 4 and 8 cover every length 2^a 3^b.  S = -1 is the
// forward transform (exp(-2 pi i jk/n), the numpy convention), S = +1 the
// unnormalised inverse.  The caller scales by 1/N elsewhere.
//
// Layout: element j of sequence q, interleaved column t, sits at
// (q*n + j)*TX + t.  TX = 1 gives contiguous sequences (x passes); TX > 1
// interleaves TX columns so that a strided-axis tile is loaded and stored
// with TX contiguous values per row and consecutive threads touch
// consecutive columns.  Stages run in place: each thread first reads all
// inputs of its butterflies into registers, then (after a barrier) writes
// the outputs, so one LDS buffer suffices.  A thread handles at most MAXE/R
// butterflies per stage: the caller guarantees nseq*TX*n <= MAXE*blockDim.
#pragma once

#include "common.hpp"

namespace pff {

template <typename T, int S> __device__ __forceinline__ void dft2(cpx<T>* v) {
  cpx<T> a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <typename T, int S> __device__ __forceinline__ void dft3(cpx<T>* v) {
  const T h = T(0.86602540378443864676372317075294);  // sqrt(3)/2
  cpx<T> t = cadd(v[1], v[2]);
  cpx<T> u = csub(v[1], v[2]);
  cpx<T> a0 = v[0];
  v[0] = cadd(a0, t);
  cpx<T> m = {a0.x - T(0.5) * t.x, a0.y - T(0.5) * t.y};
  cpx<T> nn = mul_si<T, S>(cpx<T>{h * u.x, h * u.y});
  v[1] = cadd(m, nn);
  v[2] = csub(m, nn);
}

template <typename T, int S> __device__ __forceinline__ void dft4(cpx<T>* v) {
  cpx<T> t0 = cadd(v[0], v[2]);
  cpx<T> t1 = csub(v[0], v[2]);
  cpx<T> t2 = cadd(v[1], v[3]);
  cpx<T> t3 = mul_si<T, S>(csub(v[1], v[3]));
  v[0] = cadd(t0, t2);
  v[2] = csub(t0, t2);
  v[1] = cadd(t1, t3);
  v[3] = csub(t1, t3);
}

template <typename T, int S> __device__ __forceinline__ void dft8(cpx<T>* v) {
  const T r2 = T(0.70710678118654752440084436210485);
  cpx<T> e[4] = {v[0], v[2], v[4], v[6]};
  cpx<T> o[4] = {v[1], v[3], v[5], v[7]};
  dft4<T, S>(e);
  dft4<T, S>(o);
  // w8^k = exp(S 2 pi i k / 8)
  cpx<T> o1 = {r2 * (o[1].x - T(S) * o[1].y), r2 * (o[1].y + T(S) * o[1].x)};   // (1 + S i)/sqrt2
  cpx<T> o2 = mul_si<T, S>(o[2]);                                                 // S i
  cpx<T> o3 = {r2 * (-o[3].x - T(S) * o[3].y), r2 * (-o[3].y + T(S) * o[3].x)}; // (-1 + S i)/sqrt2
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], o1);
  v[5] = csub(e[1], o1);
  v[2] = cadd(e[2], o2);
  v[6] = csub(e[2], o2);
  v[3] = cadd(e[3], o3);
  v[7] = csub(e[3], o3);
}

template <typename T, int S, int R> __device__ __forceinline__ void dftR(cpx<T>* v) {
  if constexpr (R == 2) dft2<T, S>(v);
  else if constexpr (R == 3) dft3<T, S>(v);
  else if constexpr (R == 4) dft4<T, S>(v);
  else dft8<T, S>(v);
}

template <typename T, int S, int R, int MAXE>
__device__ __forceinline__ void stockham_stage(cpx<T>* buf, int n, int Ns, int nseq, int ltx,
                                               const cpx<T>* tw) {
  constexpr int MB = (MAXE + R - 1) / R;        // butterflies per thread
  const int TX = 1 << ltx;
  const int nb = n / R;
  const int total = (nb * nseq) << ltx;
  const int twstep = n / (Ns * R);
  cpx<T> v[MB][R];
#pragma unroll
  for (int q = 0; q < MB; ++q) {
    const int idx = threadIdx.x + q * blockDim.x;
    if (idx < total) {
      const int t = idx & (TX - 1);
      const int rest = idx >> ltx;
      const int s = rest / nb;
      const int j = rest - s * nb;
      const int base_in = (s * n + j) * TX + t;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = buf[base_in + r * nb * TX];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MB; ++q) {
    const int idx = threadIdx.x + q * blockDim.x;
    if (idx < total) {
      const int t = idx & (TX - 1);
      const int rest = idx >> ltx;
      const int s = rest / nb;
      const int j = rest - s * nb;
      const int kk = j % Ns;
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cpx<T> w = tw[r * kk * twstep];
          if (S > 0) w.y = -w.y;
          v[q][r] = cmul(v[q][r], w);
        }
      }
      dftR<T, S, R>(v[q]);
      // output base (j div Ns) * Ns * R + j mod Ns
      const int base_out = (s * n + (j - kk) * R + kk) * TX + t;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[base_out + r * Ns * TX] = v[q][r];
    }
  }
  __syncthreads();
}

// In-place transform of nseq sequences (times TX = 2^ltx interleaved
// columns) of length pl.n held in buf; tw is the LDS twiddle table
// exp(-2 pi i k/n).
// Must be called by every thread of the block; ends with a barrier.
template <typename T, int S, int MAXE>
__device__ void fft_lds(cpx<T>* buf, int nseq, int ltx, const AxisPlan& pl, const cpx<T>* tw) {
  int Ns = 1;
  for (int st = 0; st < pl.nstage; ++st) {
    const int R = pl.radix[st];
    if (R == 8) stockham_stage<T, S, 8, MAXE>(buf, pl.n, Ns, nseq, ltx, tw);
    else if (R == 4) stockham_stage<T, S, 4, MAXE>(buf, pl.n, Ns, nseq, ltx, tw);
    else if (R == 3) stockham_stage<T, S, 3, MAXE>(buf, pl.n, Ns, nseq, ltx, tw);
    else stockham_stage<T, S, 2, MAXE>(buf, pl.n, Ns, nseq, ltx, tw);
    Ns *= R;
  }
}

}  // namespace pff
