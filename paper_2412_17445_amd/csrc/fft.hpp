// Batched mixed-radix Stockham FFT over sequences held in LDS.
//
// Decimation-in-time Stockham autosort (no bit reversal): with Ns the
// product of the radices already applied, butterfly j of a radix-R stage
// reads the R inputs j + r*n/R, multiplies input r by w_{Ns*R}^{r*(j mod Ns)},
// applies an R-point DFT and writes output r to (j div Ns)*Ns*R + j mod Ns +
// r*Ns.  Radices 2, 3, 4 and 8 cover every length 2^a 3^b.  S = -1 is the
// forward transform (exp(-2 pi i jk/n), the numpy convention), S = +1 the
// unnormalised inverse.  The caller scales by 1/N elsewhere.
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

template <typename T, int S, int R>
__device__ __forceinline__ void stockham_stage(const cpx<T>* __restrict__ src, cpx<T>* __restrict__ dst,
                                               int n, int Ns, int ntr, const cpx<T>* tw) {
  const int nb = n / R;
  const int total = nb * ntr;
  const int twstep = n / (Ns * R);
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int b = t / nb;
    const int j = t - b * nb;
    const cpx<T>* s = src + b * n;
    cpx<T>* d = dst + b * n;
    const int k = j % Ns;
    cpx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = s[j + r * nb];
    if (Ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        cpx<T> w = tw[r * k * twstep];
        if (S > 0) w.y = -w.y;
        v[r] = cmul(v[r], w);
      }
    }
    dftR<T, S, R>(v);
    const int base = (j - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) d[base + r * Ns] = v[r];
  }
}

// Transforms `ntr` sequences of length pl.n stored at a + b*n; b is scratch
// of the same size.  Returns the buffer that holds the result.  Must be
// called by every thread of the block; ends with a barrier.
template <typename T, int S>
__device__ cpx<T>* fft_lds(cpx<T>* a, cpx<T>* b, int ntr, const AxisPlan& pl, const cpx<T>* tw) {
  int Ns = 1;
  for (int st = 0; st < pl.nstage; ++st) {
    const int R = pl.radix[st];
    if (R == 8) stockham_stage<T, S, 8>(a, b, pl.n, Ns, ntr, tw);
    else if (R == 4) stockham_stage<T, S, 4>(a, b, pl.n, Ns, ntr, tw);
    else if (R == 3) stockham_stage<T, S, 3>(a, b, pl.n, Ns, ntr, tw);
    else stockham_stage<T, S, 2>(a, b, pl.n, Ns, ntr, tw);
    __syncthreads();
    cpx<T>* tmp = a;
    a = b;
    b = tmp;
    Ns *= R;
  }
  return a;
}

}  // namespace pff
