// Mixed quadratic-displacement / linear-pressure tetrahedra (Sec. 4, "Twist
// test"; incompressible neo-Hookean law M3):
//   L(u, p) = int mu/2 (I1 - 3) - mu ln J - p (J - 1),
//   R_u[a] = int P grad N_a,  P = mu (F - F^-T) - p J F^-T,
//   R_p[b] = -int (J - 1) lambda_b,
// with the ten quadratic shape functions (vertex a: lambda_a (2 lambda_a - 1),
// edge (a, b): 4 lambda_a lambda_b; edges (0,1), (1,2), (0,2), (0,3), (1,3),
// (2,3)) on straight-sided tetrahedra and the symmetric 4-point rule of degree
// 2 (barycentric (alpha, beta, beta, beta) and permutations, weight V/4).
//
// Unknown vector: [u (3 per displacement node) | p (one per pressure node)].
// Two passes, both deterministic: one thread per element computes the 30
// displacement and 4 pressure contributions at all quadrature points and
// stores them per (element, local node); one thread per node then sums its
// entries in increasing element order and applies the Dirichlet rows.
// Tangent (symmetric, indefinite):
//   dP = mu dF + (mu + p J) F^-T dF^T F^-T - p J L F^-T - dp J F^-T,
//   dR_p = -int J L lambda_b,   L = F^-T : dF.
// The diagonal used by the preconditioner is that of the displacement block
// and, on pressure rows, the lumped pressure mass over mu (the usual
// spectrally equivalent stand-in for the Schur complement).
//
// The paper's own twist statement (Sec. 4) is the pair quadratic displacement
// / constant pressure per element (P2-P0: the pressure test function is 1 on
// its element, R_p[e] = -int_e (J - 1)) with the polyconvex law M5
//   Psi = ap (I1 - 3) + bp (I2 - 3) - cs ln J - p (J - 1),  cs = 4 bs + 2 as,
//   P = 2 ap F + 2 bp (I1 F - F C) - (cs + p J) F^-T,
//   dP = 2 ap dF + 2 bp (2 (F:dF) F + I1 dF - dF C - F dF^T F - F F^T dF)
//        + (cs + p J) F^-T dF^T F^-T - p J L F^-T - dp J F^-T,
// I2 = |cof F|^2 = (I1^2 - C:C) / 2, C = F^T F; either law takes either pair.
// Displacement-block diagonal of M5 for dof (a, i), g = grad N_a, z = F g,
// w = F^-T g: 2 ap |g|^2 + 2 bp (z_i^2 + (I1 - (F F^T)_ii) |g|^2 - |z|^2)
// + cs w_i^2 (the pressure terms cancel, as for M3).
//
// The same elements without a pressure field (second-order displacement
// elements, Sec. 6 tables) carry the compressible law M1:
//   P = mu F + (lam ln J - mu) F^-T,
//   dP = mu dF + (mu - lam ln J) F^-T dF^T F^-T + lam L F^-T.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "nle_internal.hpp"
#include "nle_kin.hpp"
#include "nle_laws.hpp"

namespace nle {

namespace {

constexpr double QA = 0.58541019662496845446;  // (5 + 3 sqrt 5) / 20
constexpr double QB = 0.13819660112501051518;  // (5 - sqrt 5) / 20
__constant__ int EDGE_A[6] = {0, 1, 0, 0, 1, 2};
__constant__ int EDGE_B[6] = {1, 2, 2, 3, 3, 3};

template <typename T>
struct MixArgs {
  int64_t ne, nu, np;
  const int32_t *conn, *pconn;
  const T *G, *V;
  const uint8_t *umask;
  const T *x, *v;
  T *cu, *cp;
  double mu, lam;
  double ap, bp, cs;  // law M5: alpha_p, beta_p, 4 beta_s + 2 alpha_s
  MatParams mp;       // laws M2, M4, M6 (no pressure field)
  const T *fib, *sheet;  // [3][n_e] per-element fibre and sheet (M4, M6)
  double *red;
  int32_t *flag;
  const int32_t *skip;
  int32_t nomask;
};

// One quadrature point of a compressible law without a pressure field in the
// common form of nle_laws.hpp:
//   P  = a F + pT F^-T + h1 (F f) (x) f  [+ F S, law M6]
//   dP = a dF + (cF L + cFF F:dF) F + (cT L + cM F:dF) F^-T + cX F^-T dF^T F^-T
//        + h1 (dF f) (x) f + h2 ((F f).(dF f)) (F f) (x) f
//        [+ dF S + F dS(sym(F^T dF)), law M6],
// contributions w P grad N_a (residual), w dP grad N_a (action) or the
// diagonal of the point's tangent for dF = e_i (x) grad N_a.
template <typename T, int OP, int LAW>
__device__ __forceinline__ void gen_point(const MixArgs<T> &A, const T H[3][3], const Kin<T> &k,
                                          const T f[3], const T sh[3], const T gN[10][3],
                                          const T W[10][3], double w, T cu[10][3],
                                          double &eacc) {
  const MatParams &mp = A.mp;
  FibreKin fk;
  fk.e4 = 0.0;
  fk.Ff[0] = fk.Ff[1] = fk.Ff[2] = 0.0;
  if (has_fibre<LAW>()) fk = fibre_kinematics(H, f);
  Guc<T> gu;
  if (LAW == NLE_MAT_M6) guccione(H, f, sh, mp, gu);
  if (OP == OP_ENERGY) {
    double psi = energy_density<LAW>(k, H, fk, mp);
    if (LAW == NLE_MAT_M6) psi += 0.5 * mp.g6[0] * expm1(gu.Q);
    eacc += w * psi;
    return;
  }
  const Coef cf = coefficients<LAW>(k, H, fk, mp);
  T Ff[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) Ff[i] = T(fk.Ff[i]);
  const T tw = T(w);
  if (OP == OP_RES) {
    const T ca = T(cf.a), cp = T(cf.pT), ch = T(cf.h1);
    T P[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        T t = ca * k.F[i][j] + cp * k.FiT[i][j];
        if (has_fibre<LAW>()) t += ch * Ff[i] * f[j];
        if (LAW == NLE_MAT_M6)
          t += k.F[i][0] * gu.S[0][j] + k.F[i][1] * gu.S[1][j] + k.F[i][2] * gu.S[2][j];
        P[i][j] = tw * t;
      }
#pragma unroll
    for (int a = 0; a < 10; ++a)
#pragma unroll
      for (int i = 0; i < 3; ++i)
        cu[a][i] += P[i][0] * gN[a][0] + P[i][1] * gN[a][1] + P[i][2] * gN[a][2];
  } else if (OP == OP_JV) {
    T dF[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        T s = T(0);
#pragma unroll
        for (int a = 0; a < 10; ++a) s += W[a][i] * gN[a][j];
        dF[i][j] = s;
      }
    T L = T(0), FdF = T(0);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        L += k.FiT[i][j] * dF[i][j];
        FdF += k.F[i][j] * dF[i][j];
      }
    T M[3][3];  // dF^T F^-T
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        M[r][j] = dF[0][r] * k.FiT[0][j] + dF[1][r] * k.FiT[1][j] + dF[2][r] * k.FiT[2][j];
    const T sF = T(cf.cF) * L + T(cf.cFF) * FdF, sT = T(cf.cT) * L + T(cf.cM) * FdF;
    T dFf[3] = {T(0), T(0), T(0)}, s2 = T(0);
    if (has_fibre<LAW>()) {
#pragma unroll
      for (int i = 0; i < 3; ++i) dFf[i] = dF[i][0] * f[0] + dF[i][1] * f[1] + dF[i][2] * f[2];
      s2 = T(cf.h2) * (Ff[0] * dFf[0] + Ff[1] * dFf[1] + Ff[2] * dFf[2]);
    }
    T dS[3][3];
    if (LAW == NLE_MAT_M6) {
      T dE[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
          dE[i][j] = T(0.5) * (k.F[0][i] * dF[0][j] + k.F[1][i] * dF[1][j] + k.F[2][i] * dF[2][j] +
                               dF[0][i] * k.F[0][j] + dF[1][i] * k.F[1][j] + dF[2][i] * k.F[2][j]);
      guccione_dS(gu, dE, mp, dS);
    }
    T dP[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const T X = k.FiT[i][0] * M[0][j] + k.FiT[i][1] * M[1][j] + k.FiT[i][2] * M[2][j];
        T t = T(cf.a) * dF[i][j] + sF * k.F[i][j] + sT * k.FiT[i][j] + T(cf.cX) * X;
        if (has_fibre<LAW>()) t += (T(cf.h1) * dFf[i] + s2 * Ff[i]) * f[j];
        if (LAW == NLE_MAT_M6)
          t += dF[i][0] * gu.S[0][j] + dF[i][1] * gu.S[1][j] + dF[i][2] * gu.S[2][j] +
               k.F[i][0] * dS[0][j] + k.F[i][1] * dS[1][j] + k.F[i][2] * dS[2][j];
        dP[i][j] = tw * t;
      }
#pragma unroll
    for (int a = 0; a < 10; ++a)
#pragma unroll
      for (int i = 0; i < 3; ++i)
        cu[a][i] += dP[i][0] * gN[a][0] + dP[i][1] * gN[a][1] + dP[i][2] * gN[a][2];
  } else if (OP == OP_DIAG) {
    // dF = e_i (x) g: w = F^-T g, z = F g give
    // a |g|^2 + (cF + cM) w_i z_i + cFF z_i^2 + (cT + cX) w_i^2 + (h1 + h2 (Ff)_i^2) (g.f)^2
    // and, for law M6, g.S g + C e^Q (bm : dEb^2 + 2 (bE : dEb)^2) with
    // dEb = sym(rb (x) gb), rb = R^T F^T e_i, gb = R^T g
    const T c1 = T(cf.cF + cf.cM), c2 = T(cf.cT + cf.cX);
    T rb[3][3];
    if (LAW == NLE_MAT_M6) {
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int b = 0; b < 3; ++b)
          rb[i][b] = gu.R[0][b] * k.F[i][0] + gu.R[1][b] * k.F[i][1] + gu.R[2][b] * k.F[i][2];
    }
#pragma unroll
    for (int a = 0; a < 10; ++a) {
      const T gg = gN[a][0] * gN[a][0] + gN[a][1] * gN[a][1] + gN[a][2] * gN[a][2];
      const T gf = gN[a][0] * f[0] + gN[a][1] * f[1] + gN[a][2] * f[2];
      T gSg = T(0), gb[3] = {T(0), T(0), T(0)};
      if (LAW == NLE_MAT_M6) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) gSg += gN[a][i] * gu.S[i][j] * gN[a][j];
#pragma unroll
        for (int b = 0; b < 3; ++b)
          gb[b] = gu.R[0][b] * gN[a][0] + gu.R[1][b] * gN[a][1] + gu.R[2][b] * gN[a][2];
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const T wi = k.FiT[i][0] * gN[a][0] + k.FiT[i][1] * gN[a][1] + k.FiT[i][2] * gN[a][2];
        const T zi = k.F[i][0] * gN[a][0] + k.F[i][1] * gN[a][1] + k.F[i][2] * gN[a][2];
        T dg = T(cf.a) * gg + c1 * wi * zi + c2 * wi * wi + T(cf.cFF) * zi * zi;
        if (has_fibre<LAW>()) dg += (T(cf.h1) + T(cf.h2) * Ff[i] * Ff[i]) * gf * gf;
        if (LAW == NLE_MAT_M6) {
          const T bm[3][3] = {{T(mp.g6[1]), T(mp.g6[4]), T(mp.g6[5])},
                              {T(mp.g6[4]), T(mp.g6[2]), T(mp.g6[6])},
                              {T(mp.g6[5]), T(mp.g6[6]), T(mp.g6[3])}};
          T q2 = T(0), be = T(0);
#pragma unroll
          for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int q = 0; q < 3; ++q) {
              const T de = T(0.5) * (rb[i][p] * gb[q] + rb[i][q] * gb[p]);
              q2 += bm[p][q] * de * de;
              be += gu.bE[p][q] * de;
            }
          dg += gSg + gu.Ce * (q2 + T(2) * be * be);
        }
        cu[a][i] += tw * dg;
      }
    }
  }
}

// LAW: NLE_MAT_M3 or NLE_MAT_M5 (with a pressure field); NLE_MAT_M1, M2, M4
// or M6 (none).  NPE: pressure values per element, 4 (linear) or 1 (constant).
// Laws M2, M4 and M6 take the common tangent form of nle_laws.hpp at each
// point (GEN), evaluated from the state (no per-element cache).
template <typename T, int OP, int LAW, int NPE>
__global__ __launch_bounds__(NT) void k_mixed_elem(MixArgs<T> A) {
  constexpr bool PRES = LAW == NLE_MAT_M3 || LAW == NLE_MAT_M5;
  constexpr bool GEN = !PRES && LAW != NLE_MAT_M1;
  __shared__ double sh[NT / 64];
  if (A.skip && A.skip[0] != 0) return;
  const int64_t e = int64_t(blockIdx.x) * NT + threadIdx.x;
  double eacc = 0.0;
  bool bad = false;
  if (e < A.ne) {
    const uint32_t ne = uint32_t(A.ne);
    int32_t cn[10], pn[4] = {0, 0, 0, 0};
#pragma unroll
    for (int a = 0; a < 10; ++a) cn[a] = A.conn[size_t(a) * ne + e];
    if (PRES) {
#pragma unroll
      for (int b = 0; b < NPE; ++b) pn[b] = A.pconn[size_t(b) * ne + e];
    }
    T g[4][3];
#pragma unroll
    for (int a = 1; a < 4; ++a)
#pragma unroll
      for (int j = 0; j < 3; ++j) g[a][j] = A.G[size_t(3 * (a - 1) + j) * ne + e];
#pragma unroll
    for (int j = 0; j < 3; ++j) g[0][j] = -(g[1][j] + g[2][j] + g[3][j]);
    const double w = double(A.V[e]) * 0.25;
    T fe[3] = {T(0), T(0), T(0)}, se[3] = {T(0), T(0), T(0)};
    if (has_fibre<LAW>()) {
#pragma unroll
      for (int j = 0; j < 3; ++j) fe[j] = A.fib[size_t(j) * ne + e];
    }
    if (LAW == NLE_MAT_M6) {
#pragma unroll
      for (int j = 0; j < 3; ++j) se[j] = A.sheet[size_t(j) * ne + e];
    }
    T U[10][3], W[10][3], P4[4] = {T(0), T(0), T(0), T(0)}, WP[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int a = 0; a < 10; ++a) {
      const uint32_t mk = (OP == OP_JV && !A.nomask) ? A.umask[cn[a]] : 0u;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        U[a][i] = A.x[3 * int64_t(cn[a]) + i];
        if (OP == OP_JV) W[a][i] = ((mk >> i) & 1u) ? T(0) : A.v[3 * int64_t(cn[a]) + i];
      }
    }
    if (PRES) {
#pragma unroll
      for (int b = 0; b < NPE; ++b) {
        P4[b] = A.x[3 * A.nu + pn[b]];
        if (OP == OP_JV) WP[b] = A.v[3 * A.nu + pn[b]];
      }
    }
    T cu[10][3], cpv[4];
#pragma unroll
    for (int a = 0; a < 10; ++a)
#pragma unroll
      for (int i = 0; i < 3; ++i) cu[a][i] = T(0);
#pragma unroll
    for (int b = 0; b < 4; ++b) cpv[b] = T(0);
    const T mu = T(A.mu);
    const double lamd = A.lam;
    for (int q = 0; q < 4; ++q) {
      T lam[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) lam[a] = T(a == q ? QA : QB);
      // pressure shape functions at the point: barycentric (linear) or 1
      T pb[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) pb[b] = NPE == 1 ? T(b == 0 ? 1 : 0) : lam[b];
      T gN[10][3];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int j = 0; j < 3; ++j) gN[a][j] = (T(4) * lam[a] - T(1)) * g[a][j];
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const int a = EDGE_A[k], b = EDGE_B[k];
#pragma unroll
        for (int j = 0; j < 3; ++j) gN[4 + k][j] = T(4) * (lam[b] * g[a][j] + lam[a] * g[b][j]);
      }
      T H[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          T s = T(0);
#pragma unroll
          for (int a = 0; a < 10; ++a) s += U[a][i] * gN[a][j];
          H[i][j] = s;
        }
      Kin<T> k;
      kinematics(H, k);
      bad |= k.bad;
      if constexpr (GEN) {
        gen_point<T, OP, LAW>(A, H, k, fe, se, gN, W, w, cu, eacc);
        continue;
      }
      T pq = T(0);
#pragma unroll
      for (int b = 0; b < NPE; ++b) pq += pb[b] * P4[b];
      const T J = T(k.J);
      // law M5: I1 = F:F, FC = F C = F F^T F, and the stress's F coefficient
      T I1 = T(0), FC[3][3];
      if (LAW == NLE_MAT_M5 && OP != OP_ENERGY) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) I1 += k.F[i][j] * k.F[i][j];
        T B[3][3];  // F F^T
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j)
            B[i][j] = k.F[i][0] * k.F[j][0] + k.F[i][1] * k.F[j][1] + k.F[i][2] * k.F[j][2];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j)
            FC[i][j] = B[i][0] * k.F[0][j] + B[i][1] * k.F[1][j] + B[i][2] * k.F[2][j];
      }
      if (OP == OP_ENERGY) {
        double trH = 0.0, hh = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          trH += double(H[i][i]);
#pragma unroll
          for (int j = 0; j < 3; ++j) hh += double(H[i][j]) * double(H[i][j]);
        }
        if (LAW == NLE_MAT_M5) {
          // I1 - 3 = 2 tr H + H:H; with E2 = C - I = H + H^T + H^T H,
          // I2 - 3 = 2 tr E2 + ((tr E2)^2 - E2:E2) / 2 (no cancellation)
          double E2[3][3];
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
              double t = double(H[i][j]) + double(H[j][i]);
#pragma unroll
              for (int m = 0; m < 3; ++m) t += double(H[m][i]) * double(H[m][j]);
              E2[i][j] = t;
            }
          const double tE = E2[0][0] + E2[1][1] + E2[2][2];
          double ee = 0.0;
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) ee += E2[i][j] * E2[i][j];
          const double i2m3 = 2.0 * tE + 0.5 * (tE * tE - ee);
          eacc += w * (A.ap * (2.0 * trH + hh) + A.bp * i2m3 - A.cs * k.lnJ -
                       double(pq) * k.jm1);
        } else if (PRES) {
          eacc += w * (0.5 * A.mu * (2.0 * trH + hh) - A.mu * k.lnJ - double(pq) * k.jm1);
        } else {
          eacc += w * (0.5 * A.mu * (2.0 * trH + hh) - A.mu * k.lnJ + 0.5 * lamd * k.lnJ * k.lnJ);
        }
        continue;
      }
      if (OP == OP_RES) {
        T P[3][3];
        if (LAW == NLE_MAT_M5) {
          const T a2 = T(2.0 * A.ap) + T(2.0 * A.bp) * I1, b2 = T(2.0 * A.bp);
          const T cT = -(T(A.cs) + pq * J);
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
              P[i][j] = T(w) * (a2 * k.F[i][j] - b2 * FC[i][j] + cT * k.FiT[i][j]);
        } else {
          const T cT = PRES ? -(mu + pq * J) : T(lamd * k.lnJ - A.mu);
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) P[i][j] = T(w) * (mu * k.F[i][j] + cT * k.FiT[i][j]);
        }
#pragma unroll
        for (int a = 0; a < 10; ++a)
#pragma unroll
          for (int i = 0; i < 3; ++i)
            cu[a][i] += P[i][0] * gN[a][0] + P[i][1] * gN[a][1] + P[i][2] * gN[a][2];
        if (PRES) {
          const T rp = -T(w * k.jm1);
#pragma unroll
          for (int b = 0; b < NPE; ++b) cpv[b] += rp * pb[b];
        }
      } else if (OP == OP_JV) {
        T dF[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            T s = T(0);
#pragma unroll
            for (int a = 0; a < 10; ++a) s += W[a][i] * gN[a][j];
            dF[i][j] = s;
          }
        T dp = T(0);
#pragma unroll
        for (int b = 0; b < NPE; ++b) dp += pb[b] * WP[b];
        T L = T(0);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) L += k.FiT[i][j] * dF[i][j];
        T M[3][3];  // dF^T F^-T
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int j = 0; j < 3; ++j)
            M[r][j] = dF[0][r] * k.FiT[0][j] + dF[1][r] * k.FiT[1][j] + dF[2][r] * k.FiT[2][j];
        const T pJ = pq * J;
        const T cX = LAW == NLE_MAT_M5 ? T(A.cs) + pJ : (PRES ? mu + pJ : T(A.mu - lamd * k.lnJ));
        const T cT = PRES ? -(pJ * L + dp * J) : T(lamd) * L;
        T dP[3][3];
        if (LAW == NLE_MAT_M5) {
          // 2 bp (2 (F:dF) F + I1 dF - dF C - F dF^T F - F F^T dF)
          T FdF = T(0);
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) FdF += k.F[i][j] * dF[i][j];
          T Ct[3][3], G[3][3], Bt[3][3];  // C = F^T F, dF^T F, F F^T
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
              Ct[i][j] = k.F[0][i] * k.F[0][j] + k.F[1][i] * k.F[1][j] + k.F[2][i] * k.F[2][j];
              G[i][j] = dF[0][i] * k.F[0][j] + dF[1][i] * k.F[1][j] + dF[2][i] * k.F[2][j];
              Bt[i][j] = k.F[i][0] * k.F[j][0] + k.F[i][1] * k.F[j][1] + k.F[i][2] * k.F[j][2];
            }
          const T a2 = T(2.0 * A.ap) + T(2.0 * A.bp) * I1, b2 = T(2.0 * A.bp);
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
              const T X = k.FiT[i][0] * M[0][j] + k.FiT[i][1] * M[1][j] + k.FiT[i][2] * M[2][j];
              T t = a2 * dF[i][j] + T(2) * b2 * FdF * k.F[i][j];
#pragma unroll
              for (int m = 0; m < 3; ++m)
                t -= b2 * (dF[i][m] * Ct[m][j] + k.F[i][m] * G[m][j] + Bt[i][m] * dF[m][j]);
              dP[i][j] = T(w) * (t + cX * X + cT * k.FiT[i][j]);
            }
        } else {
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
              const T X = k.FiT[i][0] * M[0][j] + k.FiT[i][1] * M[1][j] + k.FiT[i][2] * M[2][j];
              dP[i][j] = T(w) * (mu * dF[i][j] + cX * X + cT * k.FiT[i][j]);
            }
        }
#pragma unroll
        for (int a = 0; a < 10; ++a)
#pragma unroll
          for (int i = 0; i < 3; ++i)
            cu[a][i] += dP[i][0] * gN[a][0] + dP[i][1] * gN[a][1] + dP[i][2] * gN[a][2];
        if (PRES) {
          const T rp = -T(w) * J * L;
#pragma unroll
          for (int b = 0; b < NPE; ++b) cpv[b] += rp * pb[b];
        }
      } else if (LAW == NLE_MAT_M5) {  // OP_DIAG of law M5 (see the header)
        T Bt[3][3];  // F F^T
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j)
            Bt[i][j] = k.F[i][0] * k.F[j][0] + k.F[i][1] * k.F[j][1] + k.F[i][2] * k.F[j][2];
        const T a2 = T(2.0 * A.ap), b2 = T(2.0 * A.bp), cs = T(A.cs);
#pragma unroll
        for (int a = 0; a < 10; ++a) {
          const T gg = gN[a][0] * gN[a][0] + gN[a][1] * gN[a][1] + gN[a][2] * gN[a][2];
          T z[3], wv[3];
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            z[i] = k.F[i][0] * gN[a][0] + k.F[i][1] * gN[a][1] + k.F[i][2] * gN[a][2];
            wv[i] = k.FiT[i][0] * gN[a][0] + k.FiT[i][1] * gN[a][1] + k.FiT[i][2] * gN[a][2];
          }
          const T zz = z[0] * z[0] + z[1] * z[1] + z[2] * z[2];
#pragma unroll
          for (int i = 0; i < 3; ++i)
            cu[a][i] += T(w) * (a2 * gg + b2 * (z[i] * z[i] + (I1 - Bt[i][i]) * gg - zz) +
                                cs * wv[i] * wv[i]);
        }
      } else {  // OP_DIAG: mu |g|^2 + mu ((F^-T g)_i)^2 (pressure terms cancel);
                // law M1: mu |g|^2 + (mu - lam ln J + lam) ((F^-T g)_i)^2
        const T ct = PRES ? mu : T(A.mu - lamd * k.lnJ + lamd);
#pragma unroll
        for (int a = 0; a < 10; ++a) {
          const T gg = gN[a][0] * gN[a][0] + gN[a][1] * gN[a][1] + gN[a][2] * gN[a][2];
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            const T t = k.FiT[i][0] * gN[a][0] + k.FiT[i][1] * gN[a][1] + k.FiT[i][2] * gN[a][2];
            cu[a][i] += T(w) * (mu * gg + ct * t * t);
          }
        }
      }
    }
    if (OP != OP_ENERGY) {
#pragma unroll
      for (int a = 0; a < 10; ++a)
#pragma unroll
        for (int i = 0; i < 3; ++i) A.cu[4 * (10 * e + a) + i] = cu[a][i];
      if (PRES && OP != OP_DIAG) {
#pragma unroll
        for (int b = 0; b < NPE; ++b) A.cp[NPE * e + b] = cpv[b];
      }
    }
  }
  if (bad && A.flag) A.flag[0] = 1;
  if (OP == OP_ENERGY) {
    double s = eacc;
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      double r = 0.0;
      for (int k = 0; k < NT / 64; ++k) r += sh[k];
      A.red[blockIdx.x] = r;
    }
  }
}

template <typename T>
struct GatherArgs {
  int64_t nu, np;
  const int32_t *u_ptr, *u_ent, *p_ptr, *p_ent;
  const uint8_t *umask;
  const double *mlump;
  const T *cu, *cp;
  const T *v;
  T *out;
  const double *fext;
  const T *fs;  // surface-load contributions (null: none)
  double s, mu;
  double *red;
  const T *ep_w;
  const double *ep_coef;
  const int32_t *skip;
  int32_t nomask;
};

template <typename T, int OP>
__global__ __launch_bounds__(NT) void k_mixed_gather(GatherArgs<T> A) {
  __shared__ double sh[NT / 64];
  if (A.skip && A.skip[0] != 0) return;
  const int64_t t = int64_t(blockIdx.x) * NT + threadIdx.x;
  const T epc = A.ep_coef ? T(A.ep_coef[0]) : T(0);
  double nrm = 0.0;
  if (t < A.nu) {
    T acc[3] = {T(0), T(0), T(0)};
    for (int q = A.u_ptr[t]; q < A.u_ptr[t + 1]; ++q) {
      const T *c = A.cu + 4 * int64_t(A.u_ent[q]);
      acc[0] += c[0];
      acc[1] += c[1];
      acc[2] += c[2];
    }
    const uint32_t mk = A.umask[t];
    if (A.fs) {
#pragma unroll
      for (int i = 0; i < 3; ++i) acc[i] += A.fs[3 * t + i];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int64_t d = 3 * t + i;
      const bool fixed = (mk >> i) & 1u;
      if (OP == OP_RES) {
        const double r = fixed ? 0.0 : double(acc[i]) - A.s * A.fext[d];
        A.out[d] = T(r);
        nrm += r * r;
      } else if (OP == OP_JV) {
        const T vd = A.v[d];
        T y = fixed ? (A.nomask ? T(0) : vd) : acc[i];
        if (A.ep_w) y -= epc * A.ep_w[d];
        A.out[d] = y;
        nrm += double(vd * y);
      } else {
        A.out[d] = fixed ? T(1) : acc[i];
      }
    }
  } else if (t < A.nu + A.np) {
    const int64_t b = t - A.nu, d = 3 * A.nu + b;
    T acc = T(0);
    if (OP != OP_DIAG)
      for (int q = A.p_ptr[b]; q < A.p_ptr[b + 1]; ++q) acc += A.cp[A.p_ent[q]];
    if (OP == OP_RES) {
      A.out[d] = acc;
      nrm += double(acc) * double(acc);
    } else if (OP == OP_JV) {
      T y = acc;
      if (A.ep_w) y -= epc * A.ep_w[d];
      A.out[d] = y;
      nrm += double(A.v[d] * y);
    } else {
      A.out[d] = T(A.mlump[b] / A.mu);
    }
  }
  if (A.red) {
    double s = nrm;
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      double r = 0.0;
      for (int k = 0; k < NT / 64; ++k) r += sh[k];
      A.red[blockIdx.x] = r;
    }
  }
}

template <typename T>
int launch_mixed(Ctx *c, int op, const T *G, const T *V, const T *x, const T *v, T *out,
                 double *red, hipError_t *err) {
  const MixedMesh &M = c->mx;
  MixArgs<T> A;
  A.ne = M.n_e;
  A.nu = M.n_u;
  A.np = M.n_p;
  A.conn = M.conn;
  A.pconn = M.pconn;
  A.G = G;
  A.V = V;
  A.umask = M.umask;
  A.x = x;
  A.v = v;
  A.cu = static_cast<T *>(M.cu);
  A.cp = static_cast<T *>(M.cp);
  A.mu = c->mat.mu;
  A.lam = c->mat.lam;
  A.ap = c->mat.a_iso;   // law M5 keeps alpha_p, beta_p and 4 beta_s + 2 alpha_s here
  A.bp = c->mat.b_iso;
  A.cs = c->mat.a_f;
  A.mp = c->mat;
  A.fib = sizeof(T) == 8 ? reinterpret_cast<const T *>(c->fib64) : reinterpret_cast<const T *>(c->fib32);
  A.sheet = sizeof(T) == 8 ? reinterpret_cast<const T *>(c->sh64) : reinterpret_cast<const T *>(c->sh32);
  A.red = red;
  A.flag = c->dflag;
  A.skip = c->elem_skip;
  A.nomask = (op == OP_JV && c->jv_nomask) ? 1 : 0;
  const int g1 = int((M.n_e + NT - 1) / NT);
  if (op == OP_ODIAG) {  // nodal blocks are defined for the P1 form only
    *err = hipErrorInvalidValue;
    return 0;
  }
  const bool pres = M.n_p > 0;
  const bool m5 = c->mat.kind == NLE_MAT_M5;
  const int kind = c->mat.kind;
#define NLE_MIXED_ELEM(OPV)                                                                    \
  if (!pres && kind == NLE_MAT_M2)                                                             \
    hipLaunchKernelGGL((k_mixed_elem<T, OPV, NLE_MAT_M2, 0>), dim3(g1), dim3(NT), 0, c->stream, A); \
  else if (!pres && kind == NLE_MAT_M4)                                                        \
    hipLaunchKernelGGL((k_mixed_elem<T, OPV, NLE_MAT_M4, 0>), dim3(g1), dim3(NT), 0, c->stream, A); \
  else if (!pres && kind == NLE_MAT_M6)                                                        \
    hipLaunchKernelGGL((k_mixed_elem<T, OPV, NLE_MAT_M6, 0>), dim3(g1), dim3(NT), 0, c->stream, A); \
  else if (!pres)                                                                              \
    hipLaunchKernelGGL((k_mixed_elem<T, OPV, NLE_MAT_M1, 0>), dim3(g1), dim3(NT), 0, c->stream, A); \
  else if (M.npe == 1 && m5)                                                                   \
    hipLaunchKernelGGL((k_mixed_elem<T, OPV, NLE_MAT_M5, 1>), dim3(g1), dim3(NT), 0, c->stream, A); \
  else if (M.npe == 1)                                                                         \
    hipLaunchKernelGGL((k_mixed_elem<T, OPV, NLE_MAT_M3, 1>), dim3(g1), dim3(NT), 0, c->stream, A); \
  else if (m5)                                                                                 \
    hipLaunchKernelGGL((k_mixed_elem<T, OPV, NLE_MAT_M5, 4>), dim3(g1), dim3(NT), 0, c->stream, A); \
  else                                                                                         \
    hipLaunchKernelGGL((k_mixed_elem<T, OPV, NLE_MAT_M3, 4>), dim3(g1), dim3(NT), 0, c->stream, A)
  switch (op) {
    case OP_RES:
      NLE_MIXED_ELEM(OP_RES);
      break;
    case OP_JV:
      NLE_MIXED_ELEM(OP_JV);
      break;
    case OP_DIAG:
      NLE_MIXED_ELEM(OP_DIAG);
      break;
    default:
      NLE_MIXED_ELEM(OP_ENERGY);
      *err = hipGetLastError();
      return g1;
  }
#undef NLE_MIXED_ELEM
  *err = hipGetLastError();
  if (*err != hipSuccess) return 0;
  // surface loads (quadratic heartbeat faces) into the node sums
  const T *fs = nullptr;
  if (op == OP_RES || op == OP_JV || op == OP_DIAG) {
    fs = static_cast<const T *>(
        surf_apply(c, op, sizeof(T) == 8 ? NLE_FP64 : NLE_FP32, x, v, nullptr, err));
    if (*err != hipSuccess) return 0;
  }
  GatherArgs<T> B;
  B.fs = fs;
  B.nu = M.n_u;
  B.np = M.n_p;
  B.u_ptr = M.u_ptr;
  B.u_ent = M.u_ent;
  B.p_ptr = M.p_ptr;
  B.p_ent = M.p_ent;
  B.umask = M.umask;
  B.mlump = M.mlump;
  B.cu = static_cast<const T *>(M.cu);
  B.cp = static_cast<const T *>(M.cp);
  B.v = v;
  B.out = out;
  B.fext = c->fext;
  B.s = c->load_scale;
  B.mu = mixed_mu_eff(c);
  B.skip = c->elem_skip;
  B.nomask = A.nomask;
  const bool jv_ep = op == OP_JV && c->ep.red;
  B.red = op == OP_RES ? red : (jv_ep ? c->ep.red : nullptr);
  B.ep_w = op == OP_JV ? static_cast<const T *>(c->ep.w) : nullptr;
  B.ep_coef = op == OP_JV ? c->ep.coef : nullptr;
  const int g2 = int((M.n_u + M.n_p + NT - 1) / NT);
  switch (op) {
    case OP_RES:
      hipLaunchKernelGGL((k_mixed_gather<T, OP_RES>), dim3(g2), dim3(NT), 0, c->stream, B);
      break;
    case OP_JV:
      hipLaunchKernelGGL((k_mixed_gather<T, OP_JV>), dim3(g2), dim3(NT), 0, c->stream, B);
      break;
    default:
      hipLaunchKernelGGL((k_mixed_gather<T, OP_DIAG>), dim3(g2), dim3(NT), 0, c->stream, B);
      break;
  }
  *err = hipGetLastError();
  return (op == OP_RES || jv_ep) ? g2 : 0;
}

template <typename T>
T *mupload(Ctx *c, const std::vector<T> &h, hipError_t *e) {
  T *d = static_cast<T *>(dalloc(c, std::max<size_t>(h.size(), 1) * sizeof(T)));
  if (!d) {
    *e = hipErrorOutOfMemory;
    return nullptr;
  }
  c->mesh_allocs.push_back(d);
  if (!h.empty()) {
    const hipError_t r =
        hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, c->stream);
    if (r != hipSuccess) *e = r;
  }
  return d;
}

// SIMPLE diagonal of the constant-pressure pair: with one pressure per
// element, row e of the pressure-displacement block lives on element e,
// B_e,(a,i) = -sum_q w_q J_q (F_q^-T grad N_a)_i, and
//   s_e = sum over the element's free dofs of B_e,(a,i)^2 / A_(a,i)(a,i),
// A's diagonal from the linearization (d = diag64, identity on Dirichlet
// dofs).  Written as s (double) and 1/s in both precisions.
__global__ __launch_bounds__(NT) void k_mixed_simple(int64_t ne, int64_t nu, const int32_t *conn,
                                                     const double *G, const double *V,
                                                     const uint8_t *umask, const double *x,
                                                     const double *d, double *sinv64,
                                                     float *sinv32, double *s_out) {
  const int64_t e = int64_t(blockIdx.x) * NT + threadIdx.x;
  if (e >= ne) return;
  const uint32_t n = uint32_t(ne);
  int32_t cn[10];
#pragma unroll
  for (int a = 0; a < 10; ++a) cn[a] = conn[size_t(a) * n + e];
  double g[4][3];
#pragma unroll
  for (int a = 1; a < 4; ++a)
#pragma unroll
    for (int j = 0; j < 3; ++j) g[a][j] = G[size_t(3 * (a - 1) + j) * n + e];
#pragma unroll
  for (int j = 0; j < 3; ++j) g[0][j] = -(g[1][j] + g[2][j] + g[3][j]);
  double U[10][3];
#pragma unroll
  for (int a = 0; a < 10; ++a)
#pragma unroll
    for (int i = 0; i < 3; ++i) U[a][i] = x[3 * int64_t(cn[a]) + i];
  const double w = V[e] * 0.25;
  double b[10][3];
#pragma unroll
  for (int a = 0; a < 10; ++a)
#pragma unroll
    for (int i = 0; i < 3; ++i) b[a][i] = 0.0;
  for (int q = 0; q < 4; ++q) {
    double lam[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) lam[a] = a == q ? QA : QB;
    double gN[10][3];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int j = 0; j < 3; ++j) gN[a][j] = (4.0 * lam[a] - 1.0) * g[a][j];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int a = EDGE_A[k], bb = EDGE_B[k];
#pragma unroll
      for (int j = 0; j < 3; ++j) gN[4 + k][j] = 4.0 * (lam[bb] * g[a][j] + lam[a] * g[bb][j]);
    }
    double H[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        double t = 0.0;
#pragma unroll
        for (int a = 0; a < 10; ++a) t += U[a][i] * gN[a][j];
        H[i][j] = t;
      }
    Kin<double> k;
    kinematics(H, k);
    const double wJ = w * k.J;
#pragma unroll
    for (int a = 0; a < 10; ++a)
#pragma unroll
      for (int i = 0; i < 3; ++i)
        b[a][i] -= wJ * (k.FiT[i][0] * gN[a][0] + k.FiT[i][1] * gN[a][1] + k.FiT[i][2] * gN[a][2]);
  }
  double sacc = 0.0;
#pragma unroll
  for (int a = 0; a < 10; ++a) {
    const uint32_t mk = umask[cn[a]];
#pragma unroll
    for (int i = 0; i < 3; ++i)
      if (!((mk >> i) & 1u)) sacc += b[a][i] * b[a][i] / d[3 * int64_t(cn[a]) + i];
  }
  s_out[e] = sacc;
  const double inv = sacc > 0.0 ? 1.0 / sacc : 0.0;
  sinv64[e] = inv;
  sinv32[e] = float(inv);
}

}  // namespace

double mixed_mu_eff(const Ctx *c) {
  // the shear modulus of the law's small-strain limit, which scales the
  // pressure mass in the Schur block: mu (M3), 2 (alpha_p + beta_p) (M5)
  return c->mat.kind == NLE_MAT_M5 ? 2.0 * (c->mat.a_iso + c->mat.b_iso) : c->mat.mu;
}

hipError_t mixed_simple_diag(Ctx *c, double *s_out) {
  const MixedMesh &M = c->mx;
  if (M.npe != 1 || !M.sinv64) return hipErrorInvalidValue;
  const int g = int((M.n_e + NT - 1) / NT);
  hipLaunchKernelGGL(k_mixed_simple, dim3(g), dim3(NT), 0, c->stream, M.n_e, M.n_u, M.conn,
                     M.G64, M.V64, M.umask, c->ulin64, c->diag64, M.sinv64, M.sinv32,
                     s_out ? s_out : M.s64);
  return hipGetLastError();
}

hipError_t schur_lower_apply(Ctx *c, int prec, bool amg, int schur, const void *b, void *x,
                             void *t1, void *t2) {
  const MixedMesh &M = c->mx;
  const int64_t nu3 = 3 * M.n_u, np = M.n_p, n = nu3 + np;
  const size_t es = prec == NLE_FP32 ? 4 : 8;
  hipError_t e;
  // x_u (the pressure part of x is overwritten below)
  if (amg)
    e = amg_apply(c, prec, b, x);
  else
    e = pc_apply(c, prec, 1, prec == NLE_FP32 ? static_cast<const void *>(c->dinv32)
                                              : static_cast<const void *>(c->dinv64),
                 b, x, n);
  if (e != hipSuccess) return e;
  // t2 = J [x_u; 0]: its pressure rows are B x_u
  e = hipMemcpyAsync(t1, x, size_t(nu3) * es, hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) return e;
  e = vec_fill(c, prec, static_cast<char *>(t1) + size_t(nu3) * es, 0.0, np);
  if (e != hipSuccess) return e;
  // the plain tangent (no Krylov epilogue)
  auto ep = c->ep;
  c->ep.w = nullptr;
  c->ep.coef = nullptr;
  c->ep.red = nullptr;
  mixed_apply(c, OP_JV, prec, prec == NLE_FP32 ? static_cast<const void *>(c->ulin32)
                                               : static_cast<const void *>(c->ulin64),
              t1, t2, nullptr, &e);
  c->ep = ep;
  if (e != hipSuccess) return e;
  const void *sinv;
  if (schur == 2)
    sinv = prec == NLE_FP32 ? static_cast<const void *>(M.sinv32)
                            : static_cast<const void *>(M.sinv64);
  else  // the pressure rows of the Jacobi data hold mu_eff / (lumped pressure mass)
    sinv = prec == NLE_FP32 ? static_cast<const void *>(c->dinv32 + nu3)
                            : static_cast<const void *>(c->dinv64 + nu3);
  return schur_p(c, prec, static_cast<const char *>(b) + size_t(nu3) * es,
                 static_cast<const char *>(t2) + size_t(nu3) * es, sinv,
                 static_cast<char *>(x) + size_t(nu3) * es, np);
}

int mixed_red_capacity(const Ctx *c) {
  return int((c->mx.n_e + NT - 1) / NT) + int((c->mx.n_u + c->mx.n_p + NT - 1) / NT) + 8;
}

int mixed_apply(Ctx *c, int op, int prec, const void *x, const void *v, void *out, double *red,
                hipError_t *err) {
  const MixedMesh &M = c->mx;
  if (prec == NLE_FP32)
    return launch_mixed<float>(c, op, M.G32, M.V32, static_cast<const float *>(x),
                               static_cast<const float *>(v), static_cast<float *>(out), red, err);
  return launch_mixed<double>(c, op, M.G64, M.V64, static_cast<const double *>(x),
                              static_cast<const double *>(v), static_cast<double *>(out), red, err);
}

nle_status upload_mixed_masks(Ctx *c) {
  NLE_HIP(c, hipMemcpyAsync(c->mx.umask, c->h_mask.data(), c->h_mask.size(), hipMemcpyHostToDevice,
                            c->stream));
  NLE_HIP(c, hipStreamSynchronize(c->stream));
  return NLE_OK;
}

nle_status build_mixed_mesh(Ctx *c, int64_t nu, const double *X, int64_t ne, const int32_t *conn,
                            int64_t np, const int32_t *pconn, int npe) {
  // np == 0: second-order displacement elements without a pressure field;
  // npe: pressure values per element (4 linear, 1 constant)
  if (nu <= 0 || ne <= 0 || np < 0) return fail(c, NLE_E_INVAL, "empty mixed mesh");
  if (npe != 4 && npe != 1) return fail(c, NLE_E_INVAL, "pressure values per element: 4 or 1");
  if (!X || !conn || (np > 0 && !pconn)) return fail(c, NLE_E_INVAL, "null mesh array");
  if (nu >= (int64_t(1) << 28) || np >= (int64_t(1) << 28) || 10 * ne >= (int64_t(1) << 31))
    return fail(c, NLE_E_UNSUPPORTED, "mixed mesh too large");
  for (int64_t k = 0; k < 10 * ne; ++k)
    if (conn[k] < 0 || conn[k] >= nu) return fail(c, NLE_E_BADMESH, "node index out of range");
  if (np > 0)
    for (int64_t k = 0; k < npe * ne; ++k)
      if (pconn[k] < 0 || pconn[k] >= np)
        return fail(c, NLE_E_BADMESH, "pressure node index out of range");
  for (int64_t i = 0; i < 3 * nu; ++i)
    if (!std::isfinite(X[i])) return fail(c, NLE_E_BADMESH, "non-finite coordinate");
  // vertex geometry: rows of D^-1, D = [X1-X0, X2-X0, X3-X0]
  std::vector<double> G(9 * ne), V(ne);
  std::vector<float> G32(9 * ne), V32(ne);
  for (int64_t e = 0; e < ne; ++e) {
    const int32_t *v = conn + 10 * e;
    double D[3][3];
    for (int i = 0; i < 3; ++i)
      for (int a = 0; a < 3; ++a) D[i][a] = X[3 * int64_t(v[a + 1]) + i] - X[3 * int64_t(v[0]) + i];
    const double det = D[0][0] * (D[1][1] * D[2][2] - D[1][2] * D[2][1]) -
                       D[0][1] * (D[1][0] * D[2][2] - D[1][2] * D[2][0]) +
                       D[0][2] * (D[1][0] * D[2][1] - D[1][1] * D[2][0]);
    if (!(det > 0.0)) {
      return fail(c, NLE_E_BADMESH,
                  "element " + std::to_string(e) + " has non-positive volume");
    }
    // inverse = cof(D)^T / det; row a of D^-1 = grad lambda_{a+1}
    double C[3][3];
    C[0][0] = D[1][1] * D[2][2] - D[1][2] * D[2][1];
    C[0][1] = D[1][2] * D[2][0] - D[1][0] * D[2][2];
    C[0][2] = D[1][0] * D[2][1] - D[1][1] * D[2][0];
    C[1][0] = D[0][2] * D[2][1] - D[0][1] * D[2][2];
    C[1][1] = D[0][0] * D[2][2] - D[0][2] * D[2][0];
    C[1][2] = D[0][1] * D[2][0] - D[0][0] * D[2][1];
    C[2][0] = D[0][1] * D[1][2] - D[0][2] * D[1][1];
    C[2][1] = D[0][2] * D[1][0] - D[0][0] * D[1][2];
    C[2][2] = D[0][0] * D[1][1] - D[0][1] * D[1][0];
    for (int a = 0; a < 3; ++a)
      for (int j = 0; j < 3; ++j) {
        const double gv = C[j][a] / det;  // (D^-1)[a][j] = cof(D)[j][a] / det
        G[size_t(3 * a + j) * ne + e] = gv;
        G32[size_t(3 * a + j) * ne + e] = float(gv);
      }
    V[e] = det / 6.0;
    V32[e] = float(V[e]);
  }
  std::vector<int32_t> cs(10 * ne), ps(np > 0 ? npe * ne : 0);
  for (int64_t e = 0; e < ne; ++e) {
    for (int a = 0; a < 10; ++a) cs[size_t(a) * ne + e] = conn[10 * e + a];
    if (np > 0)
      for (int b = 0; b < npe; ++b) ps[size_t(b) * ne + e] = pconn[npe * e + b];
  }
  // node-centred entry lists (entries in increasing element order)
  auto csr = [](int64_t n, const int32_t *cn, int per, int64_t ne_, std::vector<int32_t> *ptr,
                std::vector<int32_t> *ent) {
    ptr->assign(n + 1, 0);
    for (int64_t k = 0; k < per * ne_; ++k) (*ptr)[cn[k] + 1] += 1;
    for (int64_t g = 0; g < n; ++g) (*ptr)[g + 1] += (*ptr)[g];
    ent->assign(per * ne_, 0);
    std::vector<int32_t> pos(ptr->begin(), ptr->end() - 1);
    for (int64_t k = 0; k < per * ne_; ++k) (*ent)[pos[cn[k]]++] = int32_t(k);
  };
  std::vector<int32_t> uptr, uent, pptr, pent;
  csr(nu, conn, 10, ne, &uptr, &uent);
  std::vector<double> ml(np, 0.0);
  if (np > 0) {
    csr(np, pconn, npe, ne, &pptr, &pent);
    for (int64_t e = 0; e < ne; ++e)
      for (int b = 0; b < npe; ++b) ml[pconn[npe * e + b]] += V[e] / npe;
  } else {
    pptr.assign(1, 0);
  }

  for (void *p : c->mesh_allocs) dfree(c, p);
  c->mesh_allocs.clear();
  c->odiag64 = c->binv64 = nullptr;
  c->binv32 = nullptr;
  c->blk_valid = false;
  c->inr = decltype(c->inr)();
  amg_release(c);
  c->m = Mesh();
  c->mx = MixedMesh();
  MixedMesh &M = c->mx;
  M.n_u = nu;
  M.n_p = np;
  M.n_e = ne;
  M.npe = np > 0 ? npe : 0;
  M.h_conn.assign(conn, conn + 10 * ne);
  hipError_t herr = hipSuccess;
  M.conn = mupload(c, cs, &herr);
  M.pconn = mupload(c, ps, &herr);
  M.G64 = mupload(c, G, &herr);
  M.G32 = mupload(c, G32, &herr);
  M.V64 = mupload(c, V, &herr);
  M.V32 = mupload(c, V32, &herr);
  M.u_ptr = mupload(c, uptr, &herr);
  M.u_ent = mupload(c, uent, &herr);
  M.p_ptr = mupload(c, pptr, &herr);
  M.p_ent = mupload(c, pent, &herr);
  M.mlump = mupload(c, ml, &herr);
  const int64_t n = 3 * nu + np;
  M.umask = static_cast<uint8_t *>(dalloc(c, size_t(nu)));
  M.cu = dalloc(c, size_t(ne) * 10 * 4 * 8);
  M.cp = dalloc(c, size_t(ne) * 4 * 8);
  if (np > 0 && npe == 1) {  // SIMPLE diagonal of the constant-pressure pair
    M.s64 = static_cast<double *>(dalloc(c, size_t(ne) * 8));
    M.sinv64 = static_cast<double *>(dalloc(c, size_t(ne) * 8));
    M.sinv32 = static_cast<float *>(dalloc(c, size_t(ne) * 4));
    for (void *p : {(void *)M.s64, (void *)M.sinv64, (void *)M.sinv32}) {
      if (!p) herr = hipErrorOutOfMemory;
      c->mesh_allocs.push_back(p);
    }
  }
  double *fext = static_cast<double *>(dalloc(c, size_t(3 * nu) * 8));
  c->fext = fext;
  c->ulin64 = static_cast<double *>(dalloc(c, size_t(n) * 8));
  c->ulin32 = static_cast<float *>(dalloc(c, size_t(n) * 4));
  c->diag64 = static_cast<double *>(dalloc(c, size_t(n) * 8));
  c->dinv64 = static_cast<double *>(dalloc(c, size_t(n) * 8));
  c->dinv32 = static_cast<float *>(dalloc(c, size_t(n) * 4));
  c->partial = nullptr;
  for (void *p : {(void *)M.umask, M.cu, M.cp, (void *)fext, (void *)c->ulin64, (void *)c->ulin32,
                  (void *)c->diag64, (void *)c->dinv64, (void *)c->dinv32}) {
    if (!p) herr = hipErrorOutOfMemory;
    c->mesh_allocs.push_back(p);
  }
  c->mixed = true;
  const int64_t need = int64_t(mixed_red_capacity(c)) + 64 * int64_t(VGRID_MAX) + 64;
  if (need > c->red_cap) {
    if (c->red) dfree(c, c->red);
    c->red = static_cast<double *>(dalloc(c, size_t(need) * 8));
    if (!c->red) herr = hipErrorOutOfMemory;
    c->red_cap = need;
  }
  if (herr == hipErrorOutOfMemory) return fail(c, NLE_E_OOM, "device allocation failed");
  if (herr != hipSuccess)
    return fail(c, NLE_E_HIP, std::string("upload: ") + hipGetErrorString(herr));
  NLE_HIP(c, hipMemsetAsync(fext, 0, size_t(3 * nu) * 8, c->stream));
  NLE_HIP(c, hipMemsetAsync(M.umask, 0, size_t(nu), c->stream));
  // host mirrors used by the load and Dirichlet setters
  Mesh &m = c->m;
  m.n_nodes = nu;
  m.n_elems = ne;
  m.h_X.assign(X, X + 3 * nu);
  m.h_V = V;
  c->h_mask.assign(nu, 0);
  c->h_ftrac.assign(3 * nu, 0.0);
  c->h_fbody.assign(3 * nu, 0.0);
  c->n_dir = 0;
  c->lin64 = c->lin32 = c->lc_valid = false;
  c->load_scale = 1.0;
  NLE_HIP(c, hipStreamSynchronize(c->stream));
  c->has_mesh = true;
  return NLE_OK;
}

}  // namespace nle
