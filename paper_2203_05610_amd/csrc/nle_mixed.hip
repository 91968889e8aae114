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
// The same elements without a pressure field (second-order displacement
// elements, Sec. 6 tables) carry the compressible law M1:
//   P = mu F + (lam ln J - mu) F^-T,
//   dP = mu dF + (mu - lam ln J) F^-T dF^T F^-T + lam L F^-T.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "nle_internal.hpp"
#include "nle_kin.hpp"

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
  double *red;
  int32_t *flag;
  const int32_t *skip;
  int32_t nomask;
};

// LAW: NLE_MAT_M3 (with the linear pressure field) or NLE_MAT_M1 (none).
template <typename T, int OP, int LAW>
__global__ __launch_bounds__(NT) void k_mixed_elem(MixArgs<T> A) {
  constexpr bool PRES = LAW == NLE_MAT_M3;
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
      for (int b = 0; b < 4; ++b) pn[b] = A.pconn[size_t(b) * ne + e];
    }
    T g[4][3];
#pragma unroll
    for (int a = 1; a < 4; ++a)
#pragma unroll
      for (int j = 0; j < 3; ++j) g[a][j] = A.G[size_t(3 * (a - 1) + j) * ne + e];
#pragma unroll
    for (int j = 0; j < 3; ++j) g[0][j] = -(g[1][j] + g[2][j] + g[3][j]);
    const double w = double(A.V[e]) * 0.25;
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
      for (int b = 0; b < 4; ++b) {
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
      T pq = T(0);
#pragma unroll
      for (int b = 0; b < 4; ++b) pq += lam[b] * P4[b];
      const T J = T(k.J);
      if (OP == OP_ENERGY) {
        double trH = 0.0, hh = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          trH += double(H[i][i]);
#pragma unroll
          for (int j = 0; j < 3; ++j) hh += double(H[i][j]) * double(H[i][j]);
        }
        if (PRES)
          eacc += w * (0.5 * A.mu * (2.0 * trH + hh) - A.mu * k.lnJ - double(pq) * k.jm1);
        else
          eacc += w * (0.5 * A.mu * (2.0 * trH + hh) - A.mu * k.lnJ + 0.5 * lamd * k.lnJ * k.lnJ);
        continue;
      }
      if (OP == OP_RES) {
        const T cT = PRES ? -(mu + pq * J) : T(lamd * k.lnJ - A.mu);
        T P[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) P[i][j] = T(w) * (mu * k.F[i][j] + cT * k.FiT[i][j]);
#pragma unroll
        for (int a = 0; a < 10; ++a)
#pragma unroll
          for (int i = 0; i < 3; ++i)
            cu[a][i] += P[i][0] * gN[a][0] + P[i][1] * gN[a][1] + P[i][2] * gN[a][2];
        if (PRES) {
          const T rp = -T(w * k.jm1);
#pragma unroll
          for (int b = 0; b < 4; ++b) cpv[b] += rp * lam[b];
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
        for (int b = 0; b < 4; ++b) dp += lam[b] * WP[b];
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
        const T cX = PRES ? mu + pJ : T(A.mu - lamd * k.lnJ);
        const T cT = PRES ? -(pJ * L + dp * J) : T(lamd) * L;
        T dP[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            const T X = k.FiT[i][0] * M[0][j] + k.FiT[i][1] * M[1][j] + k.FiT[i][2] * M[2][j];
            dP[i][j] = T(w) * (mu * dF[i][j] + cX * X + cT * k.FiT[i][j]);
          }
#pragma unroll
        for (int a = 0; a < 10; ++a)
#pragma unroll
          for (int i = 0; i < 3; ++i)
            cu[a][i] += dP[i][0] * gN[a][0] + dP[i][1] * gN[a][1] + dP[i][2] * gN[a][2];
        if (PRES) {
          const T rp = -T(w) * J * L;
#pragma unroll
          for (int b = 0; b < 4; ++b) cpv[b] += rp * lam[b];
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
        for (int b = 0; b < 4; ++b) A.cp[4 * e + b] = cpv[b];
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
#define NLE_MIXED_ELEM(OPV)                                                             \
  if (pres)                                                                             \
    hipLaunchKernelGGL((k_mixed_elem<T, OPV, NLE_MAT_M3>), dim3(g1), dim3(NT), 0, c->stream, A); \
  else                                                                                  \
    hipLaunchKernelGGL((k_mixed_elem<T, OPV, NLE_MAT_M1>), dim3(g1), dim3(NT), 0, c->stream, A)
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
  GatherArgs<T> B;
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
  B.mu = c->mat.mu;
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

}  // namespace

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
                            int64_t np, const int32_t *pconn) {
  // np == 0: second-order displacement elements without a pressure field
  if (nu <= 0 || ne <= 0 || np < 0) return fail(c, NLE_E_INVAL, "empty mixed mesh");
  if (!X || !conn || (np > 0 && !pconn)) return fail(c, NLE_E_INVAL, "null mesh array");
  if (nu >= (int64_t(1) << 28) || np >= (int64_t(1) << 28) || 10 * ne >= (int64_t(1) << 31))
    return fail(c, NLE_E_UNSUPPORTED, "mixed mesh too large");
  for (int64_t k = 0; k < 10 * ne; ++k)
    if (conn[k] < 0 || conn[k] >= nu) return fail(c, NLE_E_BADMESH, "node index out of range");
  if (np > 0)
    for (int64_t k = 0; k < 4 * ne; ++k)
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
  std::vector<int32_t> cs(10 * ne), ps(np > 0 ? 4 * ne : 0);
  for (int64_t e = 0; e < ne; ++e) {
    for (int a = 0; a < 10; ++a) cs[size_t(a) * ne + e] = conn[10 * e + a];
    if (np > 0)
      for (int b = 0; b < 4; ++b) ps[size_t(b) * ne + e] = pconn[4 * e + b];
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
    csr(np, pconn, 4, ne, &pptr, &pent);
    for (int64_t e = 0; e < ne; ++e)
      for (int b = 0; b < 4; ++b) ml[pconn[4 * e + b]] += V[e] / 4.0;
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
