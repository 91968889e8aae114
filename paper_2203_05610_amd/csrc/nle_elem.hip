// Matrix-free P1 element kernels: residual, Jacobian action, tangent diagonal
// and potential, with a deterministic two-level scatter.
//
// Work unit: one workgroup per element block (a contiguous range of
// renumbered elements, spatially compact).  Phase 1 gathers the block's nodal
// state into LDS.  Phase 2 computes, one element per thread, the element
// force vector (12 values) in registers and stores it to LDS.  Phase 3 sums,
// one node slot per thread, the contributions listed in the block-local CSR
// in increasing (element, vertex) order.  A node touched by this block only
// is final and written directly; a node shared with other blocks is written
// to its slot of `partial`, and the merge kernel sums the slots of each shared
// node in block order.  No floating-point atomics: the result is bitwise
// reproducible.
#include <hip/hip_runtime.h>

#include "nle_internal.hpp"

namespace nle {

namespace {

template <typename T>
struct ElemArgs {
  const T *G;
  const T *V;
  const uint16_t *lconn;
  const uint16_t *csr_idx;
  const uint16_t *csr_end;
  const uint32_t *nodes;
  const int32_t *blk_elem;
  const int32_t *blk_node;
  int64_t n_e;
  int32_t nblk, per_xcd, nl_max, be_max;
  const T *u;         // nodal state (linearization point for Jv)
  const T *v;         // direction (Jv)
  T *out;             // r, J v or diag
  T *partial;         // shared-slot partial sums
  const double *fext; // reference external force
  double s;           // load scale
  double *red;        // per-workgroup partial sums (residual norm^2 / energy)
  int32_t *flag;      // set to 1 when some det F <= 0
  const int32_t *skip;// if non-null and *skip != 0 the launch does nothing
  MatParams mp;
};

template <typename T>
struct MergeArgs {
  const uint32_t *fx_node;
  const int32_t *fx_ptr;
  const int32_t *fx_slot;
  int64_t n_sh;
  const T *partial;
  const T *v;
  T *out;
  const double *fext;
  double s;
  double *red;
  const int32_t *skip;
};

__device__ __forceinline__ int block_id(int nblk, int per_xcd) {
  // Workgroups are dispatched round-robin over the 8 XCDs; map consecutive
  // (spatially adjacent, node-sharing) blocks onto the same XCD's L2.
  const int w = blockIdx.x;
  return per_xcd > 0 ? (w & 7) * per_xcd + (w >> 3) : w;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Fixed-order workgroup sum; the result is valid in thread 0.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T *sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  T r = 0;
  if (threadIdx.x == 0)
    for (int k = 0; k < NT / 64; ++k) r += sh[k];
  return r;
}

// Element kinematics: F = I + H, J - 1 without cancellation, ln J, F^-T.
template <typename T>
struct Kin {
  T F[3][3];
  T FiT[3][3];
  double jm1, J, lnJ;
  bool bad;
};

template <typename T>
__device__ __forceinline__ void kinematics(const T H[3][3], Kin<T> &k) {
  // det(I + H) - 1 = tr H + ((tr H)^2 - tr(H^2)) / 2 + det H, in double so the
  // volumetric terms keep their accuracy when J is close to one.
  double h[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) h[i][j] = double(H[i][j]);
  const double tr = h[0][0] + h[1][1] + h[2][2];
  double tr2 = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) tr2 += h[i][j] * h[j][i];
  const double deth = h[0][0] * (h[1][1] * h[2][2] - h[1][2] * h[2][1]) -
                      h[0][1] * (h[1][0] * h[2][2] - h[1][2] * h[2][0]) +
                      h[0][2] * (h[1][0] * h[2][1] - h[1][1] * h[2][0]);
  double jm1 = tr + 0.5 * (tr * tr - tr2) + deth;
  k.bad = !(jm1 > -1.0);
  if (k.bad) jm1 = 0.0;
  k.jm1 = jm1;
  k.J = 1.0 + jm1;
  k.lnJ = log1p(jm1);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) k.F[i][j] = H[i][j] + (i == j ? T(1) : T(0));
  const T(&F)[3][3] = k.F;
  const T ij = T(1.0 / k.J);
  // cof F / J
  k.FiT[0][0] = (F[1][1] * F[2][2] - F[1][2] * F[2][1]) * ij;
  k.FiT[0][1] = (F[1][2] * F[2][0] - F[1][0] * F[2][2]) * ij;
  k.FiT[0][2] = (F[1][0] * F[2][1] - F[1][1] * F[2][0]) * ij;
  k.FiT[1][0] = (F[0][2] * F[2][1] - F[0][1] * F[2][2]) * ij;
  k.FiT[1][1] = (F[0][0] * F[2][2] - F[0][2] * F[2][0]) * ij;
  k.FiT[1][2] = (F[0][1] * F[2][0] - F[0][0] * F[2][1]) * ij;
  k.FiT[2][0] = (F[0][1] * F[1][2] - F[0][2] * F[1][1]) * ij;
  k.FiT[2][1] = (F[0][2] * F[1][0] - F[0][0] * F[1][2]) * ij;
  k.FiT[2][2] = (F[0][0] * F[1][1] - F[0][1] * F[1][0]) * ij;
}

// Coefficients of the tangent in the form
//   dP = a dF + cF L F + (cT L + cM (F:dF)) F^-T + cX F^-T dF^T F^-T,
// L = F^-T : dF = tr(F^-1 dF).  Also the stress P = a F + pT F^-T.
struct Coef {
  double a, cF, cT, cM, cX, pT;
};

template <typename T>
__device__ __forceinline__ Coef coefficients(const Kin<T> &k, const MatParams &mp) {
  Coef c;
  if (mp.kind == NLE_MAT_M2) {
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

template <typename T>
__device__ __forceinline__ double energy_density(const Kin<T> &k, const T H[3][3],
                                                 const MatParams &mp) {
  // I1 - 3 = 2 tr H + H:H (no cancellation)
  double trH = 0.0, hh = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    trH += double(H[i][i]);
#pragma unroll
    for (int j = 0; j < 3; ++j) hh += double(H[i][j]) * double(H[i][j]);
  }
  const double i1m3 = 2.0 * trH + hh;
  if (mp.kind == NLE_MAT_M2) {
    const double j23 = exp(-2.0 / 3.0 * k.lnJ);
    const double j2m1 = k.jm1 * (k.jm1 + 2.0);
    return 0.5 * mp.mu * (j23 * (i1m3 + 3.0) - 3.0) + mp.cvol * mp.kappa * (j2m1 - 2.0 * k.lnJ);
  }
  return 0.5 * mp.mu * i1m3 - mp.mu * k.lnJ + 0.5 * mp.lam * k.lnJ * k.lnJ;
}

// Final value of one node (all three components) from its summed element
// contributions.  mk = Dirichlet bits of the node.
template <typename T, int OP>
__device__ __forceinline__ void finalize_node(uint32_t g, uint32_t mk, const T acc[3], const T *v,
                                              T *out, const double *fext, double s,
                                              double &nrm) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int64_t d = 3 * int64_t(g) + i;
    const bool fixed = (mk >> i) & 1u;
    if (OP == OP_RES) {
      const double r = fixed ? 0.0 : double(acc[i]) - s * fext[d];
      out[d] = T(r);
      nrm += r * r;
    } else if (OP == OP_JV) {
      out[d] = fixed ? v[d] : acc[i];
    } else if (OP == OP_DIAG) {
      out[d] = fixed ? T(1) : acc[i];
    }
  }
}

template <typename T, int OP>
__global__ __launch_bounds__(NT) void k_elem_block(ElemArgs<T> A) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T *lds = reinterpret_cast<T *>(lds_raw);
  const int b = block_id(A.nblk, A.per_xcd);
  if (b >= A.nblk) {  // padding workgroup of the XCD remap: contributes nothing
    if ((OP == OP_RES || OP == OP_ENERGY) && threadIdx.x == 0) A.red[blockIdx.x] = 0.0;
    return;
  }
  if (A.skip && A.skip[0] != 0) return;
  const int tid = threadIdx.x;
  const int e0 = A.blk_elem[b], ne = A.blk_elem[b + 1] - e0;
  const int p0 = A.blk_node[b], nl = A.blk_node[b + 1] - p0;
  const int NL = A.nl_max, BE = A.be_max;
  T *uS = lds;                 // [3][NL]
  T *vS = lds + 3 * NL;        // [3][NL]      (Jv only)
  T *cS = lds + 6 * NL;        // [12][BE]
  double *rs = reinterpret_cast<double *>(lds);  // reduction scratch (reused)

  // Phase 1: gather nodal state (and direction) of the block.
  for (int l = tid; l < nl; l += NT) {
    const uint32_t w = A.nodes[p0 + l];
    const int64_t g3 = 3 * int64_t(w & NODE_MASK);
    const uint32_t mk = (w >> 28) & 7u;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      uS[i * NL + l] = A.u[g3 + i];
      if (OP == OP_JV) vS[i * NL + l] = ((mk >> i) & 1u) ? T(0) : A.v[g3 + i];
    }
  }
  __syncthreads();

  // Phase 2: one element per thread.
  bool bad = false;
  double eacc = 0.0;
  for (int e = tid; e < ne; e += NT) {
    const int64_t ge = e0 + e;
    int la[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) la[a] = A.lconn[a * A.n_e + ge];
    T g[4][3];
#pragma unroll
    for (int a = 1; a < 4; ++a)
#pragma unroll
      for (int j = 0; j < 3; ++j) g[a][j] = A.G[(3 * (a - 1) + j) * A.n_e + ge];
#pragma unroll
    for (int j = 0; j < 3; ++j) g[0][j] = -(g[1][j] + g[2][j] + g[3][j]);
    const T vol = A.V[ge];
    T H[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) H[i][j] = T(0);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const T ua = uS[i * NL + la[a]];
#pragma unroll
        for (int j = 0; j < 3; ++j) H[i][j] += ua * g[a][j];
      }
    Kin<T> k;
    kinematics(H, k);
    bad |= k.bad;
    if (OP == OP_ENERGY) {
      eacc += double(vol) * energy_density(k, H, A.mp);
      continue;
    }
    const Coef cf = coefficients(k, A.mp);
    T out[4][3];
    if (OP == OP_RES) {
      const T ca = T(cf.a), cp = T(cf.pT);
      T P[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) P[i][j] = ca * k.F[i][j] + cp * k.FiT[i][j];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int i = 0; i < 3; ++i)
          out[a][i] = vol * (P[i][0] * g[a][0] + P[i][1] * g[a][1] + P[i][2] * g[a][2]);
    } else if (OP == OP_JV) {
      T dF[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) dF[i][j] = T(0);
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const T va = vS[i * NL + la[a]];
#pragma unroll
          for (int j = 0; j < 3; ++j) dF[i][j] += va * g[a][j];
        }
      T L = T(0), FdF = T(0);
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          L += k.FiT[i][j] * dF[i][j];
          FdF += k.F[i][j] * dF[i][j];
        }
      // X = F^-T dF^T F^-T = F^-T M with M = dF^T F^-T
      T M[3][3];
#pragma unroll
      for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int j = 0; j < 3; ++j)
          M[p][j] = dF[0][p] * k.FiT[0][j] + dF[1][p] * k.FiT[1][j] + dF[2][p] * k.FiT[2][j];
      const T ca = T(cf.a), cX = T(cf.cX);
      const T sF = T(cf.cF) * L, sT = T(cf.cT) * L + T(cf.cM) * FdF;
      T dP[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const T X = k.FiT[i][0] * M[0][j] + k.FiT[i][1] * M[1][j] + k.FiT[i][2] * M[2][j];
          dP[i][j] = ca * dF[i][j] + sF * k.F[i][j] + sT * k.FiT[i][j] + cX * X;
        }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int i = 0; i < 3; ++i)
          out[a][i] = vol * (dP[i][0] * g[a][0] + dP[i][1] * g[a][1] + dP[i][2] * g[a][2]);
    } else {  // OP_DIAG: dF = e_i (x) g_a, one column at a time
      const double ca = cf.a, c1 = cf.cF + cf.cM, c2 = cf.cT + cf.cX;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const T gg = g[a][0] * g[a][0] + g[a][1] * g[a][1] + g[a][2] * g[a][2];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const T w = k.FiT[i][0] * g[a][0] + k.FiT[i][1] * g[a][1] + k.FiT[i][2] * g[a][2];
          const T z = k.F[i][0] * g[a][0] + k.F[i][1] * g[a][1] + k.F[i][2] * g[a][2];
          out[a][i] = vol * (T(ca) * gg + T(c1) * w * z + T(c2) * w * w);
        }
      }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int i = 0; i < 3; ++i) cS[(3 * a + i) * BE + e] = out[a][i];
  }
  if (bad && A.flag) A.flag[0] = 1;

  if (OP == OP_ENERGY) {
    const double s = block_sum(eacc, rs);
    if (tid == 0) A.red[blockIdx.x] = s;
    return;
  }
  __syncthreads();

  // Phase 3: fixed-order node sums.
  double nrm = 0.0;
  const uint16_t *ci = A.csr_idx + 4 * int64_t(e0);
  for (int l = tid; l < nl; l += NT) {
    const int beg = l == 0 ? 0 : int(A.csr_end[p0 + l - 1]);
    const int end = A.csr_end[p0 + l];
    T acc[3] = {T(0), T(0), T(0)};
    for (int q = beg; q < end; ++q) {
      const int id = ci[q];
      const int el = id >> 2, a = id & 3;
#pragma unroll
      for (int i = 0; i < 3; ++i) acc[i] += cS[(3 * a + i) * BE + el];
    }
    const uint32_t w = A.nodes[p0 + l];
    if (w & 0x80000000u) {
      T *pp = A.partial + 3 * int64_t(p0 + l);
      pp[0] = acc[0];
      pp[1] = acc[1];
      pp[2] = acc[2];
    } else {
      finalize_node<T, OP>(w & NODE_MASK, (w >> 28) & 7u, acc, A.v, A.out, A.fext, A.s, nrm);
    }
  }
  if (OP == OP_RES) {
    const double s = block_sum(nrm, rs);
    if (tid == 0) A.red[blockIdx.x] = s;
  }
}

template <typename T, int OP>
__global__ __launch_bounds__(NT) void k_elem_merge(MergeArgs<T> A) {
  __shared__ double rs[NT / 64];
  if (A.skip && A.skip[0] != 0) return;
  const int64_t k = int64_t(blockIdx.x) * NT + threadIdx.x;
  double nrm = 0.0;
  if (k < A.n_sh) {
    T acc[3] = {T(0), T(0), T(0)};
    const int q1 = A.fx_ptr[k + 1];
    for (int q = A.fx_ptr[k]; q < q1; ++q) {
      const T *pp = A.partial + 3 * int64_t(A.fx_slot[q]);
      acc[0] += pp[0];
      acc[1] += pp[1];
      acc[2] += pp[2];
    }
    const uint32_t w = A.fx_node[k];
    finalize_node<T, OP>(w & NODE_MASK, (w >> 28) & 7u, acc, A.v, A.out, A.fext, A.s, nrm);
  }
  if (OP == OP_RES) {
    const double s = block_sum(nrm, rs);
    if (threadIdx.x == 0) A.red[blockIdx.x] = s;
  }
}

template <typename T>
int launch(Ctx *c, int op, const T *G, const T *V, const T *u, const T *v, T *out, double *red,
           hipError_t *err) {
  const Mesh &M = c->m;
  ElemArgs<T> A;
  A.G = G;
  A.V = V;
  A.lconn = M.lconn;
  A.csr_idx = M.csr_idx;
  A.csr_end = M.csr_end;
  A.nodes = M.nodes;
  A.blk_elem = M.blk_elem;
  A.blk_node = M.blk_node;
  A.n_e = M.n_elems;
  A.nblk = M.nblk;
  A.per_xcd = c->xcd_remap ? (M.nblk + 7) / 8 : 0;
  A.nl_max = M.nl_max;
  A.be_max = M.be_max;
  A.u = u;
  A.v = v;
  A.out = out;
  A.partial = static_cast<T *>(c->partial);
  A.fext = c->fext;
  A.s = c->load_scale;
  A.red = red;
  A.flag = c->dflag;
  A.skip = c->elem_skip;
  A.mp = c->mat;
  const int grid = A.per_xcd > 0 ? 8 * A.per_xcd : M.nblk;
  size_t lds = size_t(6 * M.nl_max + 12 * M.be_max) * sizeof(T);
  lds = std::max(lds, size_t(NT / 64) * sizeof(double));
  switch (op) {
    case OP_RES:
      hipLaunchKernelGGL((k_elem_block<T, OP_RES>), dim3(grid), dim3(NT), lds, c->stream, A);
      break;
    case OP_JV:
      hipLaunchKernelGGL((k_elem_block<T, OP_JV>), dim3(grid), dim3(NT), lds, c->stream, A);
      break;
    case OP_DIAG:
      hipLaunchKernelGGL((k_elem_block<T, OP_DIAG>), dim3(grid), dim3(NT), lds, c->stream, A);
      break;
    default:
      hipLaunchKernelGGL((k_elem_block<T, OP_ENERGY>), dim3(grid), dim3(NT), lds, c->stream, A);
      break;
  }
  *err = hipGetLastError();
  if (*err != hipSuccess) return 0;
  if (op == OP_ENERGY) return grid;
  int nred = (op == OP_RES) ? grid : 0;
  if (M.n_shared > 0) {
    MergeArgs<T> B;
    B.fx_node = M.fx_node;
    B.fx_ptr = M.fx_ptr;
    B.fx_slot = M.fx_slot;
    B.n_sh = M.n_shared;
    B.partial = static_cast<const T *>(c->partial);
    B.v = v;
    B.out = out;
    B.fext = c->fext;
    B.s = c->load_scale;
    B.red = red ? red + grid : nullptr;
    B.skip = c->elem_skip;
    const int g2 = int((M.n_shared + NT - 1) / NT);
    switch (op) {
      case OP_RES:
        hipLaunchKernelGGL((k_elem_merge<T, OP_RES>), dim3(g2), dim3(NT), 0, c->stream, B);
        nred += g2;
        break;
      case OP_JV:
        hipLaunchKernelGGL((k_elem_merge<T, OP_JV>), dim3(g2), dim3(NT), 0, c->stream, B);
        break;
      default:
        hipLaunchKernelGGL((k_elem_merge<T, OP_DIAG>), dim3(g2), dim3(NT), 0, c->stream, B);
        break;
    }
    *err = hipGetLastError();
  }
  return nred;
}

}  // namespace

int elem_red_capacity(const Ctx *c) {
  const Mesh &M = c->m;
  const int grid = c->xcd_remap ? 8 * ((M.nblk + 7) / 8) : M.nblk;
  return grid + int((M.n_shared + NT - 1) / NT) + 8;
}

int elem_apply(Ctx *c, int op, int prec, const void *u, const void *v, void *out, double *red,
               hipError_t *err) {
  const Mesh &M = c->m;
  if (prec == NLE_FP32)
    return launch<float>(c, op, M.G32, M.V32, static_cast<const float *>(u),
                         static_cast<const float *>(v), static_cast<float *>(out), red, err);
  return launch<double>(c, op, M.G64, M.V64, static_cast<const double *>(u),
                        static_cast<const double *>(v), static_cast<double *>(out), red, err);
}

}  // namespace nle
