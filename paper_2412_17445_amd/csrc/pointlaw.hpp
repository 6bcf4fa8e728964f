// Per-voxel constitutive law of the phase-field model (device side).
//
// Paper Sec. 2.1 (eqs. Emec, PlusNegPsi, gFunct), Sec. 2.3 (eq. C_Calc),
// Sec. 3.1 (eq. history) and Sec. 3.2 (eq. Delta_history):
//   eps(+/-) = sum_a <zeta_a>(+/-) e_a e_a,
//   psi0(+/-) = lambda/2 <tr eps>(+/-)^2 + mu eps(+/-):eps(+/-),
//   sigma0(+/-) = lambda <tr eps>(+/-) I + 2 mu eps(+/-),
//   g = (1 - phi)^2 + k,  sigma = g sigma0(+) + sigma0(-),
//   C:w = lambda [(g-1) Theta(tr eps) + 1] tr(w) I + 2 mu [w + (g-1) P(+):w],
// where P(+):w multiplies the eigenbasis component (a,b) of w by theta_ab:
// Theta(zeta_a) when zeta_a and zeta_b lie on the same side of zero (the
// exact limit, no division), else the divided difference
// (<zeta_a>+ - <zeta_b>+)/(zeta_a - zeta_b).  Theta(0) = 0.
//
// Tensors live in D x D arrays: D = 2 is the in-plane block of plane strain
// (eps_zz = 0 carries no split energy), D = 3 the full 3D tensor.  The
// eigen-decomposition is closed-form for D = 2 (half-angle formulas, no
// trigonometric calls) and cyclic Jacobi for D = 3.
#pragma once

#include "common.hpp"

namespace pff {

template <typename T> struct Consts;
template <> struct Consts<double> {
  static constexpr double rs2 = 0.70710678118654752440084436210485;
  static constexpr double s2 = 1.4142135623730950488016887242097;
  static constexpr double eps = 2.220446049250313e-16;
  static constexpr int sweeps = 10;
};
template <> struct Consts<float> {
  static constexpr float rs2 = 0.70710678118654752440f;
  static constexpr float s2 = 1.41421356237309504880f;
  static constexpr float eps = 1.1920929e-7f;
  static constexpr int sweeps = 8;
};

// Mandel vector <-> symmetric tensor.
// D = 2: [11, 22, sqrt2*12];  D = 3: [11, 22, 33, sqrt2*23, sqrt2*13, sqrt2*12].
template <typename T, int D>
__device__ __forceinline__ void mandel_to_tensor(const T* m, T (&W)[D][D]) {
  const T r = Consts<T>::rs2;
  if constexpr (D == 2) {
    W[0][0] = m[0]; W[1][1] = m[1];
    W[0][1] = W[1][0] = r * m[2];
  } else {
    W[0][0] = m[0]; W[1][1] = m[1]; W[2][2] = m[2];
    W[1][2] = W[2][1] = r * m[3];
    W[0][2] = W[2][0] = r * m[4];
    W[0][1] = W[1][0] = r * m[5];
  }
}

template <typename T, int D>
__device__ __forceinline__ void tensor_to_mandel(const T (&W)[D][D], T* m) {
  const T s = Consts<T>::s2;
  if constexpr (D == 2) {
    m[0] = W[0][0]; m[1] = W[1][1];
    m[2] = s * T(0.5) * (W[0][1] + W[1][0]);
  } else {
    m[0] = W[0][0]; m[1] = W[1][1]; m[2] = W[2][2];
    m[3] = s * T(0.5) * (W[1][2] + W[2][1]);
    m[4] = s * T(0.5) * (W[0][2] + W[2][0]);
    m[5] = s * T(0.5) * (W[0][1] + W[1][0]);
  }
}

// Eigen-decomposition E = V diag(z) V^T; column a of V is eigenvector a.
template <typename T, int D> struct Eig {
  T z[D];
  T V[D][D];
};

template <typename T>
__device__ __forceinline__ void eig_sym(const T (&E)[2][2], Eig<T, 2>& e) {
  const T m = T(0.5) * (E[0][0] + E[1][1]);
  const T h = T(0.5) * (E[0][0] - E[1][1]);
  const T b = E[0][1];
  const T R = sqrt(h * h + b * b);
  T c = T(1), s = T(0);
  if (R > T(0)) {
    const T c2 = h / R, s2 = b / R;          // cos 2t, sin 2t
    if (c2 >= T(0)) {
      c = sqrt(T(0.5) * (T(1) + c2));
      s = s2 / (T(2) * c);
    } else {
      s = sqrt(T(0.5) * (T(1) - c2));
      if (s2 < T(0)) s = -s;
      c = s2 / (T(2) * s);
    }
  }
  e.z[0] = m + R;
  e.z[1] = m - R;
  e.V[0][0] = c;  e.V[1][0] = s;    // eigenvector of m + R
  e.V[0][1] = -s; e.V[1][1] = c;    // eigenvector of m - R
}

template <typename T>
__device__ __forceinline__ void eig_sym(const T (&E)[3][3], Eig<T, 3>& e) {
  T A[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      A[i][j] = E[i][j];
      e.V[i][j] = (i == j) ? T(1) : T(0);
    }
  const T tiny = Consts<T>::eps * Consts<T>::eps;
  for (int sweep = 0; sweep < Consts<T>::sweeps; ++sweep) {
    const T off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    const T dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    if (off <= tiny * (dia + off) || off == T(0)) break;
#pragma unroll
    for (int pq = 0; pq < 3; ++pq) {
      const int p = (pq == 2) ? 1 : 0;
      const int q = (pq == 0) ? 1 : 2;
      const int o = 3 - p - q;
      const T apq = A[p][q];
      if (apq == T(0)) continue;
      // rotation annihilating A[p][q]: t = tan of the Jacobi angle
      const T theta = (A[q][q] - A[p][p]) / (T(2) * apq);
      const T at = fabs(theta);
      T t;
      if (at > T(1) / Consts<T>::eps) t = T(0.5) / theta;
      else t = (theta >= T(0) ? T(1) : T(-1)) / (at + sqrt(theta * theta + T(1)));
      const T c = T(1) / sqrt(t * t + T(1));
      const T s = t * c;
      const T app = A[p][p], aqq = A[q][q];
      A[p][p] = app - t * apq;
      A[q][q] = aqq + t * apq;
      A[p][q] = A[q][p] = T(0);
      const T aop = A[o][p], aoq = A[o][q];
      A[o][p] = A[p][o] = c * aop - s * aoq;
      A[o][q] = A[q][o] = s * aop + c * aoq;
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const T vp = e.V[r][p], vq = e.V[r][q];
        e.V[r][p] = c * vp - s * vq;
        e.V[r][q] = s * vp + c * vq;
      }
    }
  }
  e.z[0] = A[0][0];
  e.z[1] = A[1][1];
  e.z[2] = A[2][2];
}

// Evaluated split state of one voxel.
// The degraded part of the strain energy.  Spectral split: the positive
// parts <tr>+ and <zeta_a>+; isotropic model (iso): the whole strain, i.e.
// every part taken as "positive", so sigma0(+) = sigma0, P(+) = I, C = g C0
// and psi0(+) = psi0, with empty negative parts.
template <typename T, int D> struct Split {
  Eig<T, D> e;
  T tr;            // trace of eps (eps_zz = 0 in plane strain)
  T trp;           // degraded part of the trace: <tr>+ (tr when iso)
  T htr;           // Theta(tr) in the tangent's volumetric term (1 when iso)
  T zp[D];         // degraded parts of the eigenvalues: <zeta>+ (zeta when iso)
  T theta[D][D];   // multipliers of P(+) in the eigenbasis (1 when iso)
  T psi_p;         // psi0(+) (psi0 when iso): the history driver
};

// Completes the split state once sp.e holds the eigen-decomposition.
template <typename T, int D>
__device__ __forceinline__ void split_from_eig(T lam, T mu, T tr, Split<T, D>& sp, bool iso = false) {
  sp.tr = tr;
  const T trp = (iso || tr > T(0)) ? tr : T(0);
  sp.trp = trp;
  sp.htr = (iso || tr > T(0)) ? T(1) : T(0);
  T sq = T(0);
#pragma unroll
  for (int a = 0; a < D; ++a) {
    sp.zp[a] = (iso || sp.e.z[a] > T(0)) ? sp.e.z[a] : T(0);
    sq += sp.zp[a] * sp.zp[a];
  }
  sp.psi_p = T(0.5) * lam * trp * trp + mu * sq;
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      const bool ta = sp.e.z[a] > T(0), tb = sp.e.z[b] > T(0);
      const T th = (ta != tb) ? (sp.zp[a] - sp.zp[b]) / (sp.e.z[a] - sp.e.z[b]) : (ta ? T(1) : T(0));
      sp.theta[a][b] = iso ? T(1) : th;
    }
}

template <typename T, int D>
__device__ __forceinline__ void split_eval(const T* eps_m, T lam, T mu, Split<T, D>& sp, bool iso = false) {
  T E[D][D];
  mandel_to_tensor<T, D>(eps_m, E);
  eig_sym(E, sp.e);
  T tr = T(0);
#pragma unroll
  for (int i = 0; i < D; ++i) tr += E[i][i];
  split_from_eig<T, D>(lam, mu, tr, sp, iso);
}

// Unit quaternion (w, x, y, z) of a proper rotation matrix (Shepperd's
// method: branch on the largest of the trace and the diagonal entries).
template <typename T>
__device__ __forceinline__ void rot_to_quat(const T (&V)[3][3], T* q) {
  const T tr = V[0][0] + V[1][1] + V[2][2];
  if (tr > T(0)) {
    const T s = sqrt(tr + T(1)) * T(2);
    q[0] = T(0.25) * s;
    q[1] = (V[2][1] - V[1][2]) / s;
    q[2] = (V[0][2] - V[2][0]) / s;
    q[3] = (V[1][0] - V[0][1]) / s;
  } else if (V[0][0] > V[1][1] && V[0][0] > V[2][2]) {
    const T s = sqrt(T(1) + V[0][0] - V[1][1] - V[2][2]) * T(2);
    q[0] = (V[2][1] - V[1][2]) / s;
    q[1] = T(0.25) * s;
    q[2] = (V[0][1] + V[1][0]) / s;
    q[3] = (V[0][2] + V[2][0]) / s;
  } else if (V[1][1] > V[2][2]) {
    const T s = sqrt(T(1) + V[1][1] - V[0][0] - V[2][2]) * T(2);
    q[0] = (V[0][2] - V[2][0]) / s;
    q[1] = (V[0][1] + V[1][0]) / s;
    q[2] = T(0.25) * s;
    q[3] = (V[1][2] + V[2][1]) / s;
  } else {
    const T s = sqrt(T(1) + V[2][2] - V[0][0] - V[1][1]) * T(2);
    q[0] = (V[1][0] - V[0][1]) / s;
    q[1] = (V[0][2] + V[2][0]) / s;
    q[2] = (V[1][2] + V[2][1]) / s;
    q[3] = T(0.25) * s;
  }
}

// Rotation matrix of a quaternion, renormalised against storage round-off.
template <typename T>
__device__ __forceinline__ void quat_to_rot(const T* qin, T (&V)[3][3]) {
  const T n = T(1) / sqrt(qin[0] * qin[0] + qin[1] * qin[1] + qin[2] * qin[2] + qin[3] * qin[3]);
  const T w = qin[0] * n, x = qin[1] * n, y = qin[2] * n, z = qin[3] * n;
  V[0][0] = T(1) - T(2) * (y * y + z * z);
  V[0][1] = T(2) * (x * y - z * w);
  V[0][2] = T(2) * (x * z + y * w);
  V[1][0] = T(2) * (x * y + z * w);
  V[1][1] = T(1) - T(2) * (x * x + z * z);
  V[1][2] = T(2) * (y * z - x * w);
  V[2][0] = T(2) * (x * z - y * w);
  V[2][1] = T(2) * (y * z + x * w);
  V[2][2] = T(1) - T(2) * (x * x + y * y);
}

// sigma0(+) or sigma0(-) as a D x D tensor (the zz entry of plane strain is
// returned separately by the caller as lambda <tr>(+/-)).
template <typename T, int D, bool POS>
__device__ __forceinline__ void sigma0(const Split<T, D>& sp, T lam, T mu, T (&S)[D][D]) {
  const T trx = POS ? sp.trp : sp.tr - sp.trp;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      T acc = T(0);
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const T za = POS ? sp.zp[a] : sp.e.z[a] - sp.zp[a];
        acc += za * sp.e.V[i][a] * sp.e.V[j][a];
      }
      S[i][j] = T(2) * mu * acc + (i == j ? lam * trx : T(0));
    }
}

// C:w for a Mandel strain w (output Mandel), C at the split state sp.
// The eigenbasis components W' = V^T W V are formed as V^T (W V) and the
// result V (theta o W') V^T as (V Wp) V^T, upper triangles only (both are
// symmetric): about 90 multiply-adds in 3D.
template <typename T, int D>
__device__ __forceinline__ void tangent_apply(const Split<T, D>& sp, T lam, T mu, T g,
                                             const T* w_m, T* out_m) {
  T W[D][D];
  mandel_to_tensor<T, D>(w_m, W);
  const auto& V = sp.e.V;
  T WV[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      T acc = T(0);
#pragma unroll
      for (int j = 0; j < D; ++j) acc += W[i][j] * V[j][b];
      WV[i][b] = acc;
    }
  T Wp[D][D];   // theta o (V^T W V), symmetric
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = a; b < D; ++b) {
      T acc = T(0);
#pragma unroll
      for (int i = 0; i < D; ++i) acc += V[i][a] * WV[i][b];
      Wp[a][b] = sp.theta[a][b] * acc;
      Wp[b][a] = Wp[a][b];
    }
  T VW[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      T acc = T(0);
#pragma unroll
      for (int a = 0; a < D; ++a) acc += V[i][a] * Wp[a][b];
      VW[i][b] = acc;
    }
  T trw = T(0);
#pragma unroll
  for (int i = 0; i < D; ++i) trw += W[i][i];
  const T lam_eff = lam * ((g - T(1)) * sp.htr + T(1));
  T O[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = i; j < D; ++j) {
      T acc = T(0);
#pragma unroll
      for (int b = 0; b < D; ++b) acc += VW[i][b] * V[j][b];
      O[i][j] = T(2) * mu * (W[i][j] + (g - T(1)) * acc) + (i == j ? lam_eff * trw : T(0));
      O[j][i] = O[i][j];
    }
  tensor_to_mandel<T, D>(O, out_m);
}

}  // namespace pff
