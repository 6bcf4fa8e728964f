// Pipes: the point-wise stages plugged into the FFT passes.
//
//   TangentPipe   the tangent action dF(q; dq) of the crack-length system
//                 (paper Sec. 3.2, eq. CrackLength_linearization, with the
//                 history derivative of eq. Delta_history);
//   ResidualPipe  the constitutive update and the residual F(q) (eqs.
//                 System_CrackLength, newGammaFourier, history) in FP64;
//   HelmPipe      (1-m)(1/l - l Lap)(.) for the damage bootstrap;
//   ProjectPipe   plain projection of C fields and Laplacian of one field.
//
// Layouts (N voxels, x fastest; C = 3 in plane strain, 6 in 3D; Mandel
// components): a Krylov vector is [d eps (C*N) | d phi (N) | dE (1)].  The
// tangent state ts holds the strain split frame, then phi, Hs and r:
//   2D: [eps (3*N) | phi | Hs | r]                        (TS = 6 fields)
//   3D: [quaternion of the eigenbasis (4*N) | eigenvalues (3*N) | phi | Hs | r]
//       (TS = 10 fields: the 3x3 eigen-decomposition is done once per
//       Newton iteration in the FP64 residual pass, not in every apply)
// where Hs = -H when the history is loading (psi0(+) >= Hn) and +H
// otherwise, and r = phi/l - l Lap(phi) is the crack-length gradient.
#pragma once

#include "krylov.hpp"
#include "passes.hpp"
#include "pointlaw.hpp"

namespace pff {

template <int DIM> struct TsLayout {
  static constexpr int FRAME = DIM == 2 ? 3 : 7;   // fields before phi
  static constexpr int PHI = FRAME, HS = FRAME + 1, R = FRAME + 2, COUNT = FRAME + 3;
};

template <typename T, int DIM>
struct TangentPipe {
  using real = T;
  using L = TsLayout<DIM>;
  static constexpr int C = DIM == 2 ? 3 : 6;
  static constexpr int D = DIM == 2 ? 2 : 3;
  static constexpr int NF = C + 1;
  static constexpr int NRED_PRO = 1;
  static constexpr int NRED_EPI = 2;
  // Fused BiCGSTAB steps (mode 0: plain J v).  The epilogue accumulates
  // (dv, J u) (mode 1) or (J u, dv) and (J u, J u) (mode 2) over the voxel
  // entries.  With pro != 0 the prologue also forms the input u:
  //   mode 1: u = r + beta (v - omega w)   (direction update, written to vout = v)
  //   mode 2: u = r - alpha w              (intermediate residual, written to vout)
  // with the scalars of ks; the trailing (load factor) entry of u is computed
  // by every thread from the old values and stored once in ks[KS_ULAST]
  // (the finisher writes it to vout after the pass, when no block reads the
  // old value any more).  Without pro, u = v.
  struct Args {
    GridDesc g;
    Material mat;
    T l, k;
    T f[6];
    const T* ts;
    const uint8_t* pid;
    const uint8_t* mask;
    const T* v;
    T* Jv;
    T* aux;
    SpecTables<T> tab;
    int mode;
    int pro;
    int mech;        // 1: the damage rows of J are zero (mechanical operator G[C:d eps~])
    const T* lgc;    // variational toughness term l div(Gc grad d phi') of this input, or null
    const T* r;
    const T* w;
    T* vout;
    const T* dv;
    double* ks;
  };

  __device__ static T input(const Args& A, long long j) {
    if (A.pro == 0) return A.v[j];
    if (A.mode == 1) {
      const T beta = T(A.ks[KS_BETA]), omega = T(A.ks[KS_OMEGA]);
      return A.r[j] + beta * (A.v[j] - omega * A.w[j]);
    }
    const T alpha = T(A.ks[KS_ALPHA]);
    return A.r[j] - alpha * A.w[j];
  }

  __device__ static void prologue(const Args& A, long long i, T* out, double* red) {
    const long long N = A.g.N;
    const int p = A.pid[i];
    const bool m = A.mask[i] != 0;
    const T lam = T(A.mat.lam[p]), mu = T(A.mat.mu[p]), Gc = T(A.mat.Gc[p]);
    const long long last = (long long)(C + 1) * N;
    const T dE = input(A, last);
    if (A.pro != 0 && i == 0) A.ks[KS_ULAST] = double(dE);
    T w[C];
#pragma unroll
    for (int k = 0; k < C; ++k) {
      const T uk = input(A, k * N + i);
      if (A.pro != 0) A.vout[k * N + i] = uk;
      w[k] = uk + A.f[k] * dE;
    }
    const T phi = A.ts[L::PHI * N + i];
    const T Hs = A.ts[L::HS * N + i];
    const T r = A.ts[L::R * N + i];
    const T dphi = input(A, C * N + i);
    if (A.pro != 0) A.vout[C * N + i] = dphi;
    const T dphf = m ? T(0) : dphi;
    Split<T, D> sp;
    if constexpr (DIM == 2) {
      T eps[C];
#pragma unroll
      for (int k = 0; k < C; ++k) eps[k] = A.ts[k * N + i];
      split_eval<T, D>(eps, lam, mu, sp, A.mat.iso != 0);
    } else {
      T q[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) q[k] = A.ts[k * N + i];
#pragma unroll
      for (int a = 0; a < 3; ++a) sp.e.z[a] = A.ts[(4 + a) * N + i];
      quat_to_rot<T>(q, sp.e.V);
      split_from_eig<T, D>(lam, mu, sp.e.z[0] + sp.e.z[1] + sp.e.z[2], sp, A.mat.iso != 0);
    }
    const T g = (T(1) - phi) * (T(1) - phi) + A.k;
    T Cw[C];
    tangent_apply<T, D>(sp, lam, mu, g, w, Cw);
    T S[D][D];
    sigma0<T, D, true>(sp, lam, mu, S);
    T b[C];
    tensor_to_mandel<T, D>(S, b);
    const T gp = T(-2) * (T(1) - phi);            // g'(phi)
    T bw = T(0);
#pragma unroll
    for (int k = 0; k < C; ++k) {
      b[k] *= gp;
      out[k] = Cw[k] + b[k] * dphf;
      bw += b[k] * w[k];
    }
    out[C] = dphf;
    const bool chi = signbit(Hs);
    const T H = fabs(Hs);
    const T s = m ? dphi : (chi ? bw : T(0)) + (Gc / A.l + T(2) * H) * dphf;
    A.aux[i] = s;
    red[0] += double(r) * double(dphf);
  }

  __device__ static void spectral(const Args& A, int kx, int ky, int kz, cpx<T>* v) {
    spectral_proj_lap<T, DIM, C, true>(A.tab, kx, ky, kz, v);
  }

  __device__ static void epilogue(const Args& A, long long i, const T* in, double* red) {
    const long long N = A.g.N;
#pragma unroll
    for (int k = 0; k < C; ++k) A.Jv[k * N + i] = in[k];
    const bool m = A.mask[i] != 0;
    const T Gc = T(A.mat.Gc[A.pid[i]]);
    const T gterm = A.lgc ? A.lgc[i] : Gc * A.l * in[C];
    const T j2 = A.mech ? T(0) : A.aux[i] - (m ? T(0) : gterm);
    A.Jv[C * N + i] = j2;
    if (A.mode == 1) {
#pragma unroll
      for (int k = 0; k < C; ++k) red[0] += double(A.dv[k * N + i]) * double(in[k]);
      red[0] += double(A.dv[C * N + i]) * double(j2);
    } else if (A.mode == 2) {
#pragma unroll
      for (int k = 0; k < C; ++k) {
        red[0] += double(in[k]) * double(A.dv[k * N + i]);
        red[1] += double(in[k]) * double(in[k]);
      }
      red[0] += double(j2) * double(A.dv[C * N + i]);
      red[1] += double(j2) * double(j2);
    }
  }
};

// the FP32 tangent takes batched launches (the request server's inner solves)
template <int DIM> struct Batchable<TangentPipe<float, DIM>> : std::true_type {};

template <int DIM>
struct ResidualPipe {
  using real = double;
  using L = TsLayout<DIM>;
  static constexpr int C = DIM == 2 ? 3 : 6;
  static constexpr int D = DIM == 2 ? 2 : 3;
  static constexpr int NF = C + 1;
  // sums of sigma (11, 22, 33, 23, 13, 12), ||sigma||^2 over the Mandel
  // components of the strain unknowns, ||2H||^2 (scales of the residual stop)
  static constexpr int NRED_PRO = 8;
  static constexpr int NRED_EPI = 4;   // Gamma, ||F1||^2, ||F2||^2, dissipation
  struct Args {
    GridDesc g;
    Material mat;
    double l, k;
    double f[6];
    const double* eps_t;
    const double* phi;
    const double* Hn;
    double* Hcur;
    const double* E;
    double* ts;      // FP64 tangent state
    float* ts32;     // FP32 copy for the mixed-precision apply, or null
    double* rhs;     // -F, FP64 Krylov right-hand side
    float* rhs32;    // FP32 copy, or null
    double* F;
    const uint8_t* pid;
    const uint8_t* mask;
    SpecTables<double> tab;
    // Laplacian of phi computed by a separate pass, or null (then phi is the
    // (C+1)-th field of this pass).  In 2D the fields are packed in pairs
    // (11, 22), (12, phi); the round-off of a complex FFT mixes a pair, so
    // near a root, where G[sigma] is tiny, the 12 component would carry
    // errors of eps * |Lap phi| outside the range of the projection.
    const double* lap_ext;
    // dissipation control: Lap(Gc phi), for the border row dD/dphi =
    // Gc phi/l - (l/2) (Gc Lap phi + Lap(Gc phi)); null for crack-length control
    const double* lapg;
    const double* lgc;        // variational toughness term l div(Gc grad phi), or null
  };

  __device__ static void prologue(const Args& A, long long i, double* out, double* red) {
    const long long N = A.g.N;
    const int p = A.pid[i];
    const double lam = A.mat.lam[p], mu = A.mat.mu[p];
    const double E = *A.E;
    double eps[C];
#pragma unroll
    for (int k = 0; k < C; ++k) eps[k] = A.eps_t[k * N + i] + A.f[k] * E;
    const double phi = A.phi[i];
    const double Hn = A.Hn[i];
    Split<double, D> sp;
    split_eval<double, D>(eps, lam, mu, sp, A.mat.iso != 0);
    const double g = (1.0 - phi) * (1.0 - phi) + A.k;
    double Sp[D][D], Sm[D][D], Sg[D][D];
    sigma0<double, D, true>(sp, lam, mu, Sp);
    sigma0<double, D, false>(sp, lam, mu, Sm);
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b) Sg[a][b] = g * Sp[a][b] + Sm[a][b];
    double sm[C];
    tensor_to_mandel<double, D>(Sg, sm);
    const double psi = sp.psi_p;              // history driver (the whole psi0 when iso)
    const double H = psi > Hn ? psi : Hn;
    const bool chi = psi >= Hn;
    const double Hs = chi ? -H : H;
    A.Hcur[i] = Hs;
#pragma unroll
    for (int k = 0; k < C; ++k) out[k] = sm[k];
    double frame[L::FRAME];
    if constexpr (DIM == 2) {
#pragma unroll
      for (int k = 0; k < C; ++k) frame[k] = eps[k];
    } else {
      rot_to_quat<double>(sp.e.V, frame);
#pragma unroll
      for (int a = 0; a < 3; ++a) frame[4 + a] = sp.e.z[a];
    }
#pragma unroll
    for (int k = 0; k < L::FRAME; ++k) A.ts[k * N + i] = frame[k];
    A.ts[L::PHI * N + i] = phi;
    A.ts[L::HS * N + i] = Hs;
    if (A.ts32) {
#pragma unroll
      for (int k = 0; k < L::FRAME; ++k) A.ts32[k * N + i] = float(frame[k]);
      A.ts32[L::PHI * N + i] = float(phi);
      A.ts32[L::HS * N + i] = float(Hs);
    }
    out[C] = A.lap_ext ? 0.0 : phi;
    double s2 = 0.0;
#pragma unroll
    for (int k = 0; k < C; ++k) s2 += sm[k] * sm[k];
    red[6] += s2;
    red[7] += 4.0 * H * H;
    if constexpr (DIM == 2) {
      const double trp = sp.trp, trm = sp.tr - sp.trp;
      red[0] += Sg[0][0];
      red[1] += Sg[1][1];
      red[2] += g * lam * trp + lam * trm;     // sigma_zz of plane strain
      red[5] += Sg[0][1];
    } else {
      red[0] += Sg[0][0];
      red[1] += Sg[1][1];
      red[2] += Sg[2][2];
      red[3] += Sg[1][2];
      red[4] += Sg[0][2];
      red[5] += Sg[0][1];
    }
  }

  __device__ static void spectral(const Args& A, int kx, int ky, int kz, cpx<double>* v) {
    spectral_proj_lap<double, DIM, C, true>(A.tab, kx, ky, kz, v);
  }

  __device__ static void epilogue(const Args& A, long long i, const double* in, double* red) {
    const long long N = A.g.N;
    const bool m = A.mask[i] != 0;
    const double Gc = A.mat.Gc[A.pid[i]];
    const double phi = A.phi[i];
    const double H = fabs(A.Hcur[i]);
    const double lap = A.lap_ext ? A.lap_ext[i] : in[C];
    const double l = A.l;
    const double gterm = A.lgc ? A.lgc[i] : Gc * l * lap;
    const double F2 = m ? 0.0 : (Gc / l + 2.0 * H) * phi - gterm - 2.0 * H;
    const double r = A.lapg ? Gc * phi / l - 0.5 * l * (Gc * lap + A.lapg[i]) : phi / l - l * lap;
    A.ts[L::R * N + i] = r;
    if (A.ts32) A.ts32[L::R * N + i] = float(r);
    double f1 = 0.0;
#pragma unroll
    for (int k = 0; k < C; ++k) {
      A.rhs[k * N + i] = -in[k];
      if (A.rhs32) A.rhs32[k * N + i] = float(-in[k]);
      if (A.F) A.F[k * N + i] = in[k];
      f1 += in[k] * in[k];
    }
    A.rhs[C * N + i] = -F2;
    if (A.rhs32) A.rhs32[C * N + i] = float(-F2);
    if (A.F) A.F[C * N + i] = F2;
    const double gam = phi * phi / (2.0 * l) - 0.5 * l * phi * lap;
    red[0] += gam;
    red[1] += f1;
    red[2] += F2 * F2;
    red[3] += Gc * gam;                      // Gc-weighted crack functional

  }
};

// (1-m) B u with B u = (1/l + 2H/Gc) u - l Lap u: the damage equation
// divided by Gc (symmetric positive definite); H = 0 (null H) for the
// damage-free bootstrap.  H holds the signed history of the residual pass.
struct HelmPipe {
  using real = double;
  static constexpr int NF = 1;
  static constexpr int NRED_PRO = 0;
  static constexpr int NRED_EPI = 0;
  struct Args {
    GridDesc g;
    double l;
    const double* u;
    double* out;
    int mask_input;          // 1: operator (1-m) B (1-m); 0: (1-m) B
    const uint8_t* mask;
    SpecTables<double> tab;
    const double* H;         // history (|H| used), or null
    const uint8_t* pid;
    Material mat;
  };
  __device__ static void prologue(const Args& A, long long i, double* out, double*) {
    const bool m = A.mask[i] != 0;
    out[0] = (A.mask_input && m) ? 0.0 : A.u[i];
  }
  __device__ static void spectral(const Args& A, int kx, int ky, int kz, cpx<double>* v) {
    if (A.g.nz == 1) spectral_proj_lap<double, 2, 0, true>(A.tab, kx, ky, kz, v);
    else spectral_proj_lap<double, 3, 0, true>(A.tab, kx, ky, kz, v);
  }
  __device__ static void epilogue(const Args& A, long long i, const double* in, double*) {
    const bool m = A.mask[i] != 0;
    const double u = (A.mask_input && m) ? 0.0 : A.u[i];
    const double a = 1.0 / A.l + (A.H ? 2.0 * fabs(A.H[i]) / A.mat.Gc[A.pid[i]] : 0.0);
    A.out[i] = m ? 0.0 : a * u - A.l * in[0];
  }
};

// Spectral Laplacian of one FP64 field (standard frequencies, Nyquist kept).
struct LapPipe {
  using real = double;
  static constexpr int NF = 1;
  static constexpr int NRED_PRO = 0;
  static constexpr int NRED_EPI = 0;
  struct Args {
    GridDesc g;
    const double* u;
    double* out;
    SpecTables<double> tab;
    const uint8_t* pid;      // non-null: the input is Gc u (per-phase toughness of mat)
    Material mat;
  };
  __device__ static void prologue(const Args& A, long long i, double* out, double*) {
    out[0] = A.pid ? A.mat.Gc[A.pid[i]] * A.u[i] : A.u[i];
  }
  __device__ static void spectral(const Args& A, int kx, int ky, int kz, cpx<double>* v) {
    if (A.g.nz == 1) spectral_proj_lap<double, 2, 0, true>(A.tab, kx, ky, kz, v);
    else spectral_proj_lap<double, 3, 0, true>(A.tab, kx, ky, kz, v);
  }
  __device__ static void epilogue(const Args& A, long long i, const double* in, double*) { A.out[i] = in[0]; }
};

// FP64 projection of the strain block of a Krylov vector onto compatible
// fields (in place: each pass reads its rows before the last pass writes).
template <int DIM>
struct CompatPipe {
  using real = double;
  static constexpr int C = DIM == 2 ? 3 : 6;
  static constexpr int NF = C;
  static constexpr int NRED_PRO = 0;
  static constexpr int NRED_EPI = 0;
  struct Args {
    GridDesc g;
    double* x;
    SpecTables<double> tab;
  };
  __device__ static void prologue(const Args& A, long long i, double* out, double*) {
#pragma unroll
    for (int k = 0; k < C; ++k) out[k] = A.x[k * A.g.N + i];
  }
  __device__ static void spectral(const Args& A, int kx, int ky, int kz, cpx<double>* v) {
    spectral_proj_lap<double, DIM, C, false>(A.tab, kx, ky, kz, v);
  }
  __device__ static void epilogue(const Args& A, long long i, const double* in, double*) {
#pragma unroll
    for (int k = 0; k < C; ++k) A.x[k * A.g.N + i] = in[k];
  }
};

template <typename T, int DIM>
struct ProjectPipe {
  using real = T;
  static constexpr int C = DIM == 2 ? 3 : 6;
  static constexpr int NF = C + 1;
  static constexpr int NRED_PRO = 0;
  static constexpr int NRED_EPI = 0;
  struct Args {
    GridDesc g;
    const T* in;
    T* out;
    SpecTables<T> tab;
  };
  __device__ static void prologue(const Args& A, long long i, T* out, double*) {
#pragma unroll
    for (int k = 0; k < NF; ++k) out[k] = A.in[k * A.g.N + i];
  }
  __device__ static void spectral(const Args& A, int kx, int ky, int kz, cpx<T>* v) {
    spectral_proj_lap<T, DIM, C, true>(A.tab, kx, ky, kz, v);
  }
  __device__ static void epilogue(const Args& A, long long i, const T* in, double*) {
#pragma unroll
    for (int k = 0; k < NF; ++k) A.out[k * A.g.N + i] = in[k];
  }
};

}  // namespace pff
