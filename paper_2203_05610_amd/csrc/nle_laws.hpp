// Hyperelastic laws on the device: stress and tangent coefficients of the
// compressible laws in one common form, shared by the linear (P1) element
// kernels and the quadratic-displacement kernels.
//
// Paper, Sec. 2 (P = dPsi/dF) and Sec. 4 (the Cook, heartbeat and twist
// laws); M1 the compressible neo-Hookean law of the Cook workloads, M2 the
// paper's Cook law, M4 the cardiac-like law, M6 Guccione's law of the
// heartbeat test.
#pragma once

#include <hip/hip_runtime.h>

#include "nle_internal.hpp"
#include "nle_kin.hpp"

namespace nle {

// laws with a per-element fibre
template <int MAT>
__host__ __device__ constexpr bool has_fibre() {
  return MAT == NLE_MAT_M4 || MAT == NLE_MAT_M6;
}

// Coefficients of the tangent in the form
//   dP = a dF + (cF L + cFF (F:dF)) F + (cT L + cM (F:dF)) F^-T + cX F^-T dF^T F^-T
//        + h1 (dF f) (x) f + h2 ((F f).(dF f)) (F f) (x) f,
// L = F^-T : dF = tr(F^-1 dF); the fibre terms belong to law M4 only.  The
// stress is P = a F + pT F^-T + h1 (F f) (x) f.
struct Coef {
  double a, cF, cT, cM, cX, pT, cFF, h1, h2;
};

// Fibre kinematics of law M4: F f and I4 - 1 = 2 f.(H f) + |H f|^2 (unit f).
struct FibreKin {
  double Ff[3];
  double e4;
};

template <typename T>
__device__ __forceinline__ FibreKin fibre_kinematics(const T H[3][3], const T f[3]) {
  FibreKin q;
  double Hf[3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
    Hf[i] = double(H[i][0]) * double(f[0]) + double(H[i][1]) * double(f[1]) +
            double(H[i][2]) * double(f[2]);
  q.e4 = 2.0 * (double(f[0]) * Hf[0] + double(f[1]) * Hf[1] + double(f[2]) * Hf[2]) +
         Hf[0] * Hf[0] + Hf[1] * Hf[1] + Hf[2] * Hf[2];
#pragma unroll
  for (int i = 0; i < 3; ++i) q.Ff[i] = double(f[i]) + Hf[i];
  return q;
}

// Law M6 (Guccione): with R = [f s n] (n = f x s), Eb = R^T E R,
// E = (H + H^T + H^T H) / 2, the symmetric coefficients bm, bE = bm o Eb
// (entrywise) and Q = bE : Eb, the passive second Piola stress is
// S = R (C e^Q bE) R^T and its derivative dS = R dSb R^T with
// dSb = C e^Q (bm o dEb + 2 bE (bE : dEb)).
template <typename T>
struct Guc {
  T R[3][3];   // columns f, s, n
  T bE[3][3];  // bm o Eb
  T S[3][3];   // passive second Piola stress
  T Ce;        // C e^Q
  double Q;
};

template <typename T>
__device__ __forceinline__ void guccione(const T H[3][3], const T f[3], const T sh[3],
                                         const MatParams &mp, Guc<T> &g) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    g.R[i][0] = f[i];
    g.R[i][1] = sh[i];
  }
  g.R[0][2] = f[1] * sh[2] - f[2] * sh[1];
  g.R[1][2] = f[2] * sh[0] - f[0] * sh[2];
  g.R[2][2] = f[0] * sh[1] - f[1] * sh[0];
  T E[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      E[i][j] = T(0.5) * (H[i][j] + H[j][i] + H[0][i] * H[0][j] + H[1][i] * H[1][j] +
                          H[2][i] * H[2][j]);
  T W[3][3];  // E R
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int b = 0; b < 3; ++b) W[i][b] = E[i][0] * g.R[0][b] + E[i][1] * g.R[1][b] + E[i][2] * g.R[2][b];
  const double bm[3][3] = {{mp.g6[1], mp.g6[4], mp.g6[5]},
                           {mp.g6[4], mp.g6[2], mp.g6[6]},
                           {mp.g6[5], mp.g6[6], mp.g6[3]}};
  double Q = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const T eb = g.R[0][a] * W[0][b] + g.R[1][a] * W[1][b] + g.R[2][a] * W[2][b];
      g.bE[a][b] = T(bm[a][b]) * eb;
      Q += double(g.bE[a][b]) * double(eb);
    }
  g.Q = Q;
  g.Ce = T(mp.g6[0] * exp(Q));
  T Sb[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) Sb[a][b] = g.Ce * g.bE[a][b];
  T V[3][3];  // R Sb
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int b = 0; b < 3; ++b) V[i][b] = g.R[i][0] * Sb[0][b] + g.R[i][1] * Sb[1][b] + g.R[i][2] * Sb[2][b];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) g.S[i][j] = V[i][0] * g.R[j][0] + V[i][1] * g.R[j][1] + V[i][2] * g.R[j][2];
}

// dS for a symmetric strain increment dE (law M6), in the frame of g.
template <typename T>
__device__ __forceinline__ void guccione_dS(const Guc<T> &g, const T dE[3][3],
                                            const MatParams &mp, T dS[3][3]) {
  T W[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int b = 0; b < 3; ++b) W[i][b] = dE[i][0] * g.R[0][b] + dE[i][1] * g.R[1][b] + dE[i][2] * g.R[2][b];
  const T bm[3][3] = {{T(mp.g6[1]), T(mp.g6[4]), T(mp.g6[5])},
                      {T(mp.g6[4]), T(mp.g6[2]), T(mp.g6[6])},
                      {T(mp.g6[5]), T(mp.g6[6]), T(mp.g6[3])}};
  T deb[3][3], c = T(0);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      deb[a][b] = g.R[0][a] * W[0][b] + g.R[1][a] * W[1][b] + g.R[2][a] * W[2][b];
      c += g.bE[a][b] * deb[a][b];
    }
  T dSb[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) dSb[a][b] = g.Ce * (bm[a][b] * deb[a][b] + T(2) * g.bE[a][b] * c);
  T V[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int b = 0; b < 3; ++b) V[i][b] = g.R[i][0] * dSb[0][b] + g.R[i][1] * dSb[1][b] + g.R[i][2] * dSb[2][b];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) dS[i][j] = V[i][0] * g.R[j][0] + V[i][1] * g.R[j][1] + V[i][2] * g.R[j][2];
}

template <int MAT, typename T>
__device__ __forceinline__ Coef coefficients(const Kin<T> &k, const T H[3][3], const FibreKin &fk,
                                             const MatParams &mp) {
  Coef c;
  c.cFF = 0.0;
  c.h1 = 0.0;
  c.h2 = 0.0;
  if (MAT == NLE_MAT_M6) {
    // B/2 (J - 1) ln J: P_vol = pT F^-T with pT = B/2 (J ln J + J - 1), whose
    // derivative gives cT = B/2 J (ln J + 2) and cX = -pT; the passive
    // Guccione part is added from S (guccione) and the active term gamma |F f|
    // gives h1, h2 as in law M4
    const double B = mp.g6[7];
    c.a = 0.0;
    c.cF = 0.0;
    c.cM = 0.0;
    c.pT = 0.5 * B * (k.J * k.lnJ + k.jm1);
    c.cT = 0.5 * B * k.J * (k.lnJ + 2.0);
    c.cX = -c.pT;
    const double I4 = 1.0 + fk.e4;
    const double rs = rsqrt(I4);
    c.h1 = mp.gamma * rs;
    c.h2 = -mp.gamma * rs / I4;
    return c;
  }
  if (MAT == NLE_MAT_M4) {
    // Psi = a/2b (exp(b (Ib1 - 3)) - 1) + af/2bf (exp(bf e4^2) - 1) [e4 > 0]
    //       + kappa/2 (J - 1)^2 + gamma sqrt(I4),  Ib1 = J^-2/3 I1, e4 = I4 - 1
    double I1 = 0.0, trH = 0.0, hh = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      trH += double(H[i][i]);
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        I1 += double(k.F[i][j]) * double(k.F[i][j]);
        hh += double(H[i][j]) * double(H[i][j]);
      }
    }
    const double j23m1 = expm1(-2.0 / 3.0 * k.lnJ);
    const double j23 = 1.0 + j23m1;
    const double ib3 = 2.0 * trH + hh + j23m1 * I1;  // J^-2/3 I1 - 3 without cancellation
    const double A = mp.a_iso * exp(mp.b_iso * ib3) * j23;
    const double be = A * mp.b_iso * j23;
    const double vk = mp.kappa * k.J;
    c.a = A;
    c.pT = vk * k.jm1 - A * I1 / 3.0;
    c.cF = -2.0 / 3.0 * (A + be * I1);
    c.cM = c.cF;
    c.cFF = 2.0 * be;
    c.cT = 2.0 / 9.0 * (A * I1 + be * I1 * I1) + vk * (2.0 * k.J - 1.0);
    c.cX = A * I1 / 3.0 - vk * k.jm1;
    const double e4 = fk.e4, I4 = 1.0 + e4;
    double G = 0.0, Gp = 0.0;
    if (e4 > 0.0) {
      const double ex = exp(mp.b_f * e4 * e4);
      G = 2.0 * mp.a_f * e4 * ex;
      Gp = 2.0 * mp.a_f * ex * (1.0 + 2.0 * mp.b_f * e4 * e4);
    }
    const double rs = rsqrt(I4);
    c.h1 = G + mp.gamma * rs;
    c.h2 = 2.0 * Gp - mp.gamma * rs / I4;
  } else if (MAT == NLE_MAT_M2) {
    // Psi = mu/2 (J^-2/3 I1 - 3) + cvol kappa (J^2 - 1 - 2 ln J)
    double I1 = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) I1 += double(k.F[i][j]) * double(k.F[i][j]);
    const double a = mp.mu * exp(-2.0 / 3.0 * k.lnJ);
    const double j2m1 = k.jm1 * (k.jm1 + 2.0);  // J^2 - 1
    const double b = 2.0 * mp.cvol * mp.kappa * j2m1;
    c.a = a;
    c.pT = b - a * I1 / 3.0;
    c.cF = -2.0 / 3.0 * a;
    c.cM = -2.0 / 3.0 * a;
    c.cT = 2.0 / 9.0 * a * I1 + 4.0 * mp.cvol * mp.kappa * k.J * k.J;
    c.cX = a * I1 / 3.0 - b;
  } else {
    // Psi = mu/2 (I1 - 3) - mu ln J + lam/2 (ln J)^2
    c.a = mp.mu;
    c.pT = mp.lam * k.lnJ - mp.mu;
    c.cF = 0.0;
    c.cM = 0.0;
    c.cT = mp.lam;
    c.cX = mp.mu - mp.lam * k.lnJ;
  }
  return c;
}

template <int MAT, typename T>
__device__ __forceinline__ double energy_density(const Kin<T> &k, const T H[3][3],
                                                 const FibreKin &fk, const MatParams &mp) {
  // I1 - 3 = 2 tr H + H:H (no cancellation)
  double trH = 0.0, hh = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    trH += double(H[i][i]);
#pragma unroll
    for (int j = 0; j < 3; ++j) hh += double(H[i][j]) * double(H[i][j]);
  }
  const double i1m3 = 2.0 * trH + hh;
  if (MAT == NLE_MAT_M6)  // volumetric and active parts; the passive part needs the frame
    return 0.5 * mp.g6[7] * k.jm1 * k.lnJ + mp.gamma * sqrt(1.0 + fk.e4);
  if (MAT == NLE_MAT_M4) {
    double I1 = i1m3 + 3.0;
    const double j23m1 = expm1(-2.0 / 3.0 * k.lnJ);
    const double ib3 = i1m3 + j23m1 * I1;
    const double e4 = fk.e4;
    double psi = mp.a_iso / (2.0 * mp.b_iso) * expm1(mp.b_iso * ib3) +
                 0.5 * mp.kappa * k.jm1 * k.jm1 + mp.gamma * sqrt(1.0 + e4);
    if (e4 > 0.0) psi += mp.a_f / (2.0 * mp.b_f) * expm1(mp.b_f * e4 * e4);
    return psi;
  }
  if (MAT == NLE_MAT_M2) {
    const double j23 = exp(-2.0 / 3.0 * k.lnJ);
    const double j2m1 = k.jm1 * (k.jm1 + 2.0);
    return 0.5 * mp.mu * (j23 * (i1m3 + 3.0) - 3.0) + mp.cvol * mp.kappa * (j2m1 - 2.0 * k.lnJ);
  }
  return 0.5 * mp.mu * i1m3 - mp.mu * k.lnJ + 0.5 * mp.lam * k.lnJ * k.lnJ;
}


}  // namespace nle
