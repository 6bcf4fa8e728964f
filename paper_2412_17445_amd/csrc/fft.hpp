// Batched mixed-radix Stockham FFT over sequences held in LDS.
//
// Decimation-in-time Stockham autosort (no bit reversal): with Ns the
// product of the radices already applied, butterfly j of a radix-R stage
// reads the R inputs j + r*n/R, multiplies input r by w_{Ns*R}^{r*(j mod Ns)},
// applies an R-point DFT and writes output r to (j div Ns)*Ns*R + j mod Ns +
// r*Ns.  Radices 2, 3, 4, 8 and the odd primes 5, 7, 11, 13 have unrolled
// butterflies; every other prime factor p of the length runs a stage of
// radix p in which each item computes one output element from its p inputs
// (O(p) work per element), so any length up to the tile limit is covered.  S = -1 is the
// forward transform (exp(-2 pi i jk/n), the numpy convention), S = +1 the
// unnormalised inverse.  The caller scales by 1/N elsewhere.
//
// Layout: element j of sequence q, interleaved column t, sits at
// lidx<PAD>((q*n + j)*TX + t) (one pad element every 32, common.hpp).  TX = 1 gives contiguous sequences (x passes); TX > 1
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

// cos and sin of 2 pi j / P for the odd prime radices with unrolled butterflies
__host__ __device__ constexpr double odd_cos(int P, int j) {
  // j = 1 .. (P-1)/2
  if (P == 5) { constexpr double t[] = {0.30901699437494745, -0.8090169943749473}; return t[j - 1]; }
  if (P == 7) { constexpr double t[] = {0.6234898018587336, -0.22252093395631434, -0.900968867902419}; return t[j - 1]; }
  if (P == 11) { constexpr double t[] = {0.8412535328311812, 0.41541501300188644, -0.142314838273285, -0.654860733945285, -0.9594929736144974}; return t[j - 1]; }
  if (P == 13) { constexpr double t[] = {0.8854560256532099, 0.5680647467311559, 0.120536680255323, -0.35460488704253545, -0.7485107481711012, -0.970941817426052}; return t[j - 1]; }
  return 0.0;
}
__host__ __device__ constexpr double odd_sin(int P, int j) {
  // j = 1 .. (P-1)/2
  if (P == 5) { constexpr double t[] = {0.9510565162951535, 0.5877852522924732}; return t[j - 1]; }
  if (P == 7) { constexpr double t[] = {0.7818314824680298, 0.9749279121818236, 0.43388373911755823}; return t[j - 1]; }
  if (P == 11) { constexpr double t[] = {0.5406408174555976, 0.9096319953545183, 0.9898214418809328, 0.7557495743542583, 0.28173255684142967}; return t[j - 1]; }
  if (P == 13) { constexpr double t[] = {0.4647231720437685, 0.8229838658936564, 0.992708874098054, 0.9350162426854148, 0.6631226582407952, 0.23931566428755768}; return t[j - 1]; }
  return 0.0;
}

// P-point DFT for odd prime P, pairing inputs j and P - j:
//   y_k     = x_0 + sum_j [cos(2 pi jk/P) (x_j + x_{P-j}) + S i sin(2 pi jk/P) (x_j - x_{P-j})]
//   y_{P-k} = the same with -S i,   j, k = 1 .. (P-1)/2.
template <typename T, int S, int P> __device__ __forceinline__ void dft_odd(cpx<T>* v) {
  constexpr int H = (P - 1) / 2;
  cpx<T> a[H], b[H];
  const cpx<T> x0 = v[0];
  cpx<T> y0 = x0;
#pragma unroll
  for (int j = 1; j <= H; ++j) {
    a[j - 1] = cadd(v[j], v[P - j]);
    b[j - 1] = csub(v[j], v[P - j]);
    y0 = cadd(y0, a[j - 1]);
  }
#pragma unroll
  for (int k = 1; k <= H; ++k) {
    cpx<T> re = x0, im = {T(0), T(0)};
#pragma unroll
    for (int j = 1; j <= H; ++j) {
      const int m = (j * k) % P;
      const int idx = m <= H ? m : P - m;
      const T c = T(odd_cos(P, idx));
      const T sn = T(m <= H ? odd_sin(P, idx) : -odd_sin(P, idx));
      re = {re.x + c * a[j - 1].x, re.y + c * a[j - 1].y};
      im = {im.x + sn * b[j - 1].x, im.y + sn * b[j - 1].y};
    }
    const cpx<T> t = mul_si<T, S>(im);
    v[k] = cadd(re, t);
    v[P - k] = csub(re, t);
  }
  v[0] = y0;
}

// cos(2 pi k / 32) for k = 0..8 (the first quadrant); the other angles of the
// radix-16/32 butterflies follow by symmetry.
__host__ __device__ constexpr double cos32_q(int k) {
  constexpr double t[9] = {1.0, 0.98078528040323044913, 0.92387953251128675613, 0.83146961230254523708,
                           0.70710678118654752440, 0.55557023301960222474, 0.38268343236508977173,
                           0.19509032201612826785, 0.0};
  return t[k];
}
__host__ __device__ constexpr double cos32(int k) {
  k &= 31;
  return k <= 8 ? cos32_q(k) : k <= 16 ? -cos32_q(16 - k) : k <= 24 ? -cos32_q(k - 16) : cos32_q(32 - k);
}
__host__ __device__ constexpr double sin32(int k) { return cos32(k + 24); }   // sin x = cos(x - pi/2)

// R-point DFT (R a power of two up to 32) in registers, natural order in
// and out: v[m] <- sum_r v[r] exp(S 2 pi i r m / R).  Radix-2 decimation in
// time over the radix-8/4/2 butterflies, with compile-time twiddles.
template <typename T, int S, int R> __device__ __forceinline__ void dft_pow2(cpx<T>* v) {
  if constexpr (R == 1) {
  } else if constexpr (R == 2) {
    dft2<T, S>(v);
  } else if constexpr (R == 4) {
    dft4<T, S>(v);
  } else if constexpr (R == 8) {
    dft8<T, S>(v);
  } else {
    static_assert(R == 16 || R == 32, "radix");
    constexpr int H = R / 2;
    cpx<T> e[H], o[H];
#pragma unroll
    for (int k = 0; k < H; ++k) {
      e[k] = v[2 * k];
      o[k] = v[2 * k + 1];
    }
    dft_pow2<T, S, H>(e);
    dft_pow2<T, S, H>(o);
#pragma unroll
    for (int k = 0; k < H; ++k) {
      const int m = k * (32 / R);
      const cpx<T> w = {T(cos32(m)), T(S) * T(sin32(m))};
      const cpx<T> t = cmul(o[k], w);
      v[k] = cadd(e[k], t);
      v[k + H] = csub(e[k], t);
    }
  }
}

template <typename T, int S, int R> __device__ __forceinline__ void dftR(cpx<T>* v) {
  if constexpr (R == 2) dft2<T, S>(v);
  else if constexpr (R == 3) dft3<T, S>(v);
  else if constexpr (R == 4) dft4<T, S>(v);
  else if constexpr (R == 8) dft8<T, S>(v);
  else dft_odd<T, S, R>(v);
}

template <typename T, int S, int R, int MAXE, bool PAD>
__device__ __forceinline__ void stockham_stage(cpx<T>* buf, int n, int Ns, int nseq, int ltx,
                                               const cpx<T>* tw, const FastDiv& dnb, const FastDiv& dns) {
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
      const int s = (int)fdiv((uint32_t)rest, dnb);
      const int j = rest - s * nb;
      const int base_in = (s * n + j) * TX + t;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = buf[lidx<PAD>(base_in + r * nb * TX)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MB; ++q) {
    const int idx = threadIdx.x + q * blockDim.x;
    if (idx < total) {
      const int t = idx & (TX - 1);
      const int rest = idx >> ltx;
      const int s = (int)fdiv((uint32_t)rest, dnb);
      const int j = rest - s * nb;
      const int kk = j - (int)fdiv((uint32_t)j, dns) * Ns;
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
      for (int r = 0; r < R; ++r) buf[lidx<PAD>(base_out + r * Ns * TX)] = v[q][r];
    }
  }
  __syncthreads();
}

// Stage of any radix R, one output element per item: output o of the stage
// (o = (j div Ns) Ns R + j mod Ns + r Ns) sums its R inputs j + m n/R times
// w_{Ns R}^{m (j mod Ns)} w_R^{m r}, one table lookup per term (both factors
// are powers of w_n: tw[(m (j mod Ns) n/(Ns R) + (m r mod R) n/R) mod n]).
// All items read before the barrier and write their own element after it.
template <typename T, int S, int MAXE, bool PAD>
__device__ __forceinline__ void stockham_stage_any(cpx<T>* buf, int n, int R, int Ns, int nseq, int ltx,
                                                const cpx<T>* tw) {
  const int TX = 1 << ltx;
  const int total = (n * nseq) << ltx;
  const int nb = n / R;
  const int twstep = n / (Ns * R);
  cpx<T> out[MAXE];
#pragma unroll
  for (int q = 0; q < MAXE; ++q) {
    const int idx = threadIdx.x + q * blockDim.x;
    if (idx < total) {
      const int t = idx & (TX - 1);
      const int rest = idx >> ltx;
      const int sq = rest / n;
      const int o = rest - sq * n;                  // output position in the sequence
      const int kk = o % Ns;
      const int r = (o / Ns) % R;
      const int j = (o / (Ns * R)) * Ns + kk;       // butterfly index
      const int in0 = (sq * n + j) * TX + t;
      const int d1 = kk * twstep;                   // m kk twstep < n for every m < R
      const int d2 = r * nb;                        // (m r mod R) nb = m r nb mod n
      int e1 = 0, e2 = 0;
      cpx<T> acc = {T(0), T(0)};
      for (int m = 0; m < R; ++m) {
        int e = e1 + e2;
        if (e >= n) e -= n;
        cpx<T> w = tw[e];
        if (S > 0) w.y = -w.y;
        acc = cadd(acc, cmul(buf[lidx<PAD>(in0 + m * nb * TX)], w));
        e1 += d1;
        e2 += d2;
        if (e2 >= n) e2 -= n;
      }
      out[q] = acc;
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXE; ++q) {
    const int idx = threadIdx.x + q * blockDim.x;
    if (idx < total) buf[lidx<PAD>(idx)] = out[q];     // element idx is the item's own output
  }
  __syncthreads();
}

// ---- lengths known at compile time ----------------------------------------
// The radix sequence of factor23 (8s, then one 4 or 2, then 3s), as constexpr.
constexpr int c_pow2(int n) { return n % 2 == 0 ? 1 + c_pow2(n / 2) : 0; }
constexpr int c_pow3(int n) { return n % 3 == 0 ? 1 + c_pow3(n / 3) : 0; }
constexpr int c_nstage(int n) {
  return c_pow2(n) / 3 + (c_pow2(n) % 3 != 0 ? 1 : 0) + c_pow3(n);
}
constexpr int c_radix(int n, int st) {
  return st < c_pow2(n) / 3 ? 8
       : (c_pow2(n) % 3 != 0 && st == c_pow2(n) / 3) ? (c_pow2(n) % 3 == 2 ? 4 : 2)
       : 3;
}

// Stage with compile-time length N, radix R and span NS: all strides of the
// index arithmetic are constants (shifts for powers of two).
template <typename T, int S, int N, int R, int NS, int MAXE, bool PAD>
__device__ __forceinline__ void stockham_stage_c(cpx<T>* buf, int nseq, int ltx, const cpx<T>* tw) {
  constexpr int MB = (MAXE + R - 1) / R;
  constexpr int NB = N / R;
  constexpr int TWS = N / (NS * R);
  const int TX = 1 << ltx;
  const int total = (NB * nseq) << ltx;
  cpx<T> v[MB][R];
#pragma unroll
  for (int q = 0; q < MB; ++q) {
    const int idx = threadIdx.x + q * blockDim.x;
    if (idx < total) {
      const int t = idx & (TX - 1);
      const int rest = idx >> ltx;
      const int s = rest / NB;
      const int j = rest - s * NB;
      const int base_in = ((s * N + j) << ltx) + t;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = buf[lidx<PAD>(base_in + ((r * NB) << ltx))];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MB; ++q) {
    const int idx = threadIdx.x + q * blockDim.x;
    if (idx < total) {
      const int t = idx & (TX - 1);
      const int rest = idx >> ltx;
      const int s = rest / NB;
      const int j = rest - s * NB;
      const int kk = j % NS;
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cpx<T> w = tw[r * kk * TWS];
          if (S > 0) w.y = -w.y;
          v[q][r] = cmul(v[q][r], w);
        }
      }
      dftR<T, S, R>(v[q]);
      const int base_out = ((s * N + (j - kk) * R + kk) << ltx) + t;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[lidx<PAD>(base_out + ((r * NS) << ltx))] = v[q][r];
    }
  }
  __syncthreads();
}

template <typename T, int S, int N, int ST, int NS, int MAXE, bool PAD>
__device__ __forceinline__ void fft_c(cpx<T>* buf, int nseq, int ltx, const cpx<T>* tw) {
  if constexpr (ST < c_nstage(N)) {
    constexpr int R = c_radix(N, ST);
    stockham_stage_c<T, S, N, R, NS, MAXE, PAD>(buf, nseq, ltx, tw);
    fft_c<T, S, N, ST + 1, NS * R, MAXE, PAD>(buf, nseq, ltx, tw);
  }
}

// In-place transform of nseq sequences (times TX = 2^ltx interleaved
// columns) of length pl.n held in buf; tw is the LDS twiddle table
// exp(-2 pi i k/n).  Lengths 32..512 (powers of two) take the compile-time
// path, every other length the generic one.
// Must be called by every thread of the block; ends with a barrier.
// ANY: the kernel may meet radices other than 2, 3, 4 and 8 (generic stage
// compiled in).  PAD: the tile is padded (lidx).  Kernels of 2^a 3^b grids are instantiated without it, so the
// generic stage's registers do not count against their occupancy.
template <typename T, int S, int MAXE, bool ANY, bool PAD>
__device__ void fft_lds(cpx<T>* buf, int nseq, int ltx, const AxisPlan& pl, const cpx<T>* tw) {
  switch (pl.n) {
    case 32: fft_c<T, S, 32, 0, 1, MAXE, PAD>(buf, nseq, ltx, tw); return;
    case 64: fft_c<T, S, 64, 0, 1, MAXE, PAD>(buf, nseq, ltx, tw); return;
    case 128: fft_c<T, S, 128, 0, 1, MAXE, PAD>(buf, nseq, ltx, tw); return;
    case 256: fft_c<T, S, 256, 0, 1, MAXE, PAD>(buf, nseq, ltx, tw); return;
    case 512: fft_c<T, S, 512, 0, 1, MAXE, PAD>(buf, nseq, ltx, tw); return;
    default: break;
  }
  int Ns = 1;
  for (int st = 0; st < pl.nstage; ++st) {
    const int R = pl.radix[st];
    const FastDiv& a = pl.dnb[st];
    const FastDiv& b = pl.dns[st];
    if (R == 8) stockham_stage<T, S, 8, MAXE, PAD>(buf, pl.n, Ns, nseq, ltx, tw, a, b);
    else if (R == 4) stockham_stage<T, S, 4, MAXE, PAD>(buf, pl.n, Ns, nseq, ltx, tw, a, b);
    else if (R == 3) stockham_stage<T, S, 3, MAXE, PAD>(buf, pl.n, Ns, nseq, ltx, tw, a, b);
    else if (R == 2) stockham_stage<T, S, 2, MAXE, PAD>(buf, pl.n, Ns, nseq, ltx, tw, a, b);
    else if constexpr (ANY) {
      if (R == 5) stockham_stage<T, S, 5, MAXE, PAD>(buf, pl.n, Ns, nseq, ltx, tw, a, b);
      else if (R == 7) stockham_stage<T, S, 7, MAXE, PAD>(buf, pl.n, Ns, nseq, ltx, tw, a, b);
      else if (R == 11) stockham_stage<T, S, 11, MAXE, PAD>(buf, pl.n, Ns, nseq, ltx, tw, a, b);
      else if (R == 13) stockham_stage<T, S, 13, MAXE, PAD>(buf, pl.n, Ns, nseq, ltx, tw, a, b);
      else stockham_stage_any<T, S, MAXE, PAD>(buf, pl.n, R, Ns, nseq, ltx, tw);
    }
    Ns *= R;
  }
}

}  // namespace pff
