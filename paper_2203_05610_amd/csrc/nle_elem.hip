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

#include <mutex>

#include "nle_internal.hpp"
#include "nle_kin.hpp"
#include "nle_laws.hpp"

namespace nle {

// Fixed device workspace of the allocation-free Jacobian action
// (nle_jv_noalloc): the shared-slot partial sums live here instead of in the
// buffer the library allocates at mesh upload.  One copy per device, held
// until the process ends; in host code the array's name is only a stand-in,
// so its address is always taken with hipGetSymbolAddress (per device, with
// that device current) and that pointer is what kernels receive.
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

hipError_t noalloc_scratch_init(int device, void **out) {
  static std::mutex mu;
  static void *ptrs[NOALLOC_MAX_DEVICES] = {};
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!ptrs[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    ptrs[device] = p;
  }
  *out = ptrs[device];
  return hipSuccess;
}

namespace {

template <typename T>
struct ElemArgs {
  const T *xr;        // [n_slots][3] slot coordinates relative to the block's first slot
  const uint4 *lcp;   // per element: 4 slot-local vertex ids, 4 contribution positions (u16)
  const uint16_t *csr_end;
  const uint32_t *nodes;
  const int32_t *mpos;
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
  int32_t nomask;     // Jv: keep v on Dirichlet dofs, zero Dirichlet rows
  // Jv epilogue (optional): out = J v - c w with c = *ep_coef, and partial sums
  // of v.out written to ep_red (one per workgroup of each kernel)
  const T *ep_w;
  const double *ep_coef;
  double *ep_red;
  MatParams mp;
  const T *fib;       // laws M4, M6: unit fibre per element, [3][n_e]
  const T *sheet;     // law M6: unit sheet direction per element, [3][n_e]
  // linearization cache: per-element tangent coefficients at u_lin, [k][n_e]
  // (written by the diagonal pass, read by the Jacobian action)
  const T *lcoef;
  double *lc64;
  float *lc32;
  const T *fs;        // surface-load contributions per dof (null without surface loads)
  // batched mode (all null for a single problem): instance of each block,
  // per-instance load scale, material (mu, lam, cvol, kappa) and done mask
  const int32_t *blk_inst;
  const double *inst_s;
  const double *inst_mat;
  const int32_t *inst_done;
  const int32_t *blk_list;  // when set, workgroup w runs block blk_list[w] (n_list of them)
  int32_t n_list;
  const T *icm;             // inertia: c * m per dof (null: none), and u_tilde
  const double *iut;
  // CG direction formed here (Jv only, see Ctx::cg): v = vz + beta * v
  const T *vz;
  const double *cg_red;
  int32_t cg_np;
  double *cg_scal;
  int32_t *cg_flag;
};

template <typename T>
struct MergeArgs {
  const uint32_t *fx_node;
  const int32_t *fx_ptr;
  int64_t n_sh;
  const T *partial;
  const T *v;
  T *out;
  const double *fext;
  double s;
  double *red;
  const int32_t *skip;
  const T *ep_w;
  const double *ep_coef;
  double *ep_red;
  const T *fs;
  int32_t nomask;
  const int32_t *mwg_inst;  // batched mode: instance of each merge workgroup
  const double *inst_s;
  const int32_t *inst_done;
  const int32_t *mwg_list;  // when set, workgroup w runs merge workgroup mwg_list[w]
  const T *vz;              // CG direction v = vz + beta * v, beta = cg_scal[BETA]
  const double *cg_scal;
  const T *u;               // state (residual with inertia)
  const T *icm;             // inertia: c * m per dof (null: none), and u_tilde
  const double *iut;
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

// Threads per workgroup of the element-block kernel: one element per thread
// at the default block size, so the LDS a block needs carries eight waves.
constexpr int NTB = 512;

// Sum of red[0..np) in the order of the vector kernels' fixed-order sum
// (256 threads, strided, then the four wave sums in order), so the value is
// bitwise the one those kernels form; broadcast to all threads.  sh: 8 doubles.
__device__ __forceinline__ double sum_partials_256(const double *red, int np, double *sh) {
  double v = 0.0;
  if (threadIdx.x < 256)
    for (int k = threadIdx.x; k < np; k += 256) v += red[k];
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = sh[0];
  for (int k = 1; k < 4; ++k) r += sh[k];
  return r;
}

// Fixed-order workgroup sum over NTH threads; the result is valid in thread 0.
template <int NTH, typename T>
__device__ __forceinline__ T block_sum(T v, T *sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  T r = 0;
  if (threadIdx.x == 0)
    for (int k = 0; k < NTH / 64; ++k) r += sh[k];
  return r;
}

// Final value of one node (all three components) from its summed element
// contributions.  mk = Dirichlet bits of the node.
// fs (nullable) holds the surface-load contributions of the same operation;
// icm (nullable) the inertia coefficients c m per dof, with u and u_tilde
// (iut) for the residual's c m (u - u_tilde).
template <typename T, int OP>
__device__ __forceinline__ void finalize_node(uint32_t g, uint32_t mk, const T acc[3], const T *v,
                                              const T *vz, T bt,
                                              T *out, const double *fext, double s,
                                              double &nrm, bool dot, const T *epw, T epc,
                                              const T *fs, int nomask, const T *icm,
                                              const double *iut, const T *u) {
  // Every load of the node's three components is issued before the
  // arithmetic and the stores come last: out may alias the inputs as far as
  // the compiler knows, so a load after a store would wait for it.
  const int64_t d0 = 3 * int64_t(g);
  T a[3], fv[3] = {T(0), T(0), T(0)};
  if (fs) {
#pragma unroll
    for (int i = 0; i < 3; ++i) fv[i] = fs[d0 + i];
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) a[i] = fs ? acc[i] + fv[i] : acc[i];
  if (OP == OP_RES) {
    double fe[3], ci[3] = {0.0, 0.0, 0.0}, uu[3] = {0.0, 0.0, 0.0}, ut[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < 3; ++i) fe[i] = fext[d0 + i];
    if (icm) {
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        ci[i] = double(icm[d0 + i]);
        uu[i] = double(u[d0 + i]);
        ut[i] = iut[d0 + i];
      }
    }
    double r[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double ra = double(a[i]);
      if (icm) ra += ci[i] * (uu[i] - ut[i]);
      r[i] = ((mk >> i) & 1u) ? 0.0 : ra - s * fe[i];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      out[d0 + i] = T(r[i]);
      nrm += r[i] * r[i];
    }
  } else if (OP == OP_JV) {
    // the direction is read only at nodes that use it: kept Dirichlet rows
    // (nomask = 0), inertia and the v.y sum (dot)
    T vd[3] = {T(0), T(0), T(0)}, cm[3] = {T(0), T(0), T(0)}, ew[3] = {T(0), T(0), T(0)};
    if (dot || icm || (mk != 0u && !nomask)) {
      if (vz) {
#pragma unroll
        for (int i = 0; i < 3; ++i) vd[i] = vz[d0 + i] + bt * v[d0 + i];
      } else {
#pragma unroll
        for (int i = 0; i < 3; ++i) vd[i] = v[d0 + i];
      }
    }
    if (icm) {
#pragma unroll
      for (int i = 0; i < 3; ++i) cm[i] = icm[d0 + i];
    }
    if (epw) {
#pragma unroll
      for (int i = 0; i < 3; ++i) ew[i] = epw[d0 + i];
    }
    T y[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      T t = ((mk >> i) & 1u) ? (nomask ? T(0) : vd[i]) : (icm ? a[i] + cm[i] * vd[i] : a[i]);
      if (epw) t -= epc * ew[i];
      y[i] = t;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      out[d0 + i] = y[i];
      if (dot) nrm += double(vd[i] * y[i]);
    }
  } else if (OP == OP_DIAG) {
    T cm[3] = {T(0), T(0), T(0)};
    if (icm) {
#pragma unroll
      for (int i = 0; i < 3; ++i) cm[i] = icm[d0 + i];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) out[d0 + i] = ((mk >> i) & 1u) ? T(1) : (icm ? a[i] + cm[i] : a[i]);
  } else if (OP == OP_ODIAG) {
    // entry i pairs components (i, i+1 mod 3): xy, yz, zx
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const bool fx = ((mk >> i) & 1u) || ((mk >> ((i + 1) % 3)) & 1u);
      out[d0 + i] = fx ? T(0) : a[i];
    }
  }
}

// Per-element input read from the element-contiguous arrays.
template <typename T>
struct ElemIn {
  uint4 lcp;   // 8 x u16: slot-local vertex ids, then contribution positions
  T f[3];      // fibre direction (laws M4, M6)
  T sh[3];     // sheet direction (law M6)
  T cx;        // law M1, Jacobian action: the cached tangent coefficient cX
  uint32_t ge; // renumbered element index
};

__device__ __forceinline__ int lo16(uint32_t w) { return int(w & 0xFFFFu); }
__device__ __forceinline__ int hi16(uint32_t w) { return int(w >> 16); }

// Per-element arrays are component-major ([k][n_e]): with a 32-bit element
// index and uniform per-component base pointers every load is a scalar base
// plus one shared 32-bit lane offset.
template <int MAT, int OP, typename T>
__device__ __forceinline__ void load_elem(const ElemArgs<T> &A, uint32_t ge, ElemIn<T> &d) {
  d.lcp = A.lcp[ge];
  const uint32_t ne = uint32_t(A.n_e);
  d.ge = ge;
  if (OP == OP_JV && MAT == NLE_MAT_M1) d.cx = A.lcoef[ge];
  if (has_fibre<MAT>()) {
#pragma unroll
    for (int j = 0; j < 3; ++j) d.f[j] = A.fib[size_t(j) * ne + ge];
  }
  if (MAT == NLE_MAT_M6) {
#pragma unroll
    for (int j = 0; j < 3; ++j) d.sh[j] = A.sheet[size_t(j) * ne + ge];
  }
}

// Element force vector (12 values, vertex-major) of one element.
// Number of cached tangent coefficients per element and law (the others
// follow from the material constants): M1 cX; M2 a, cT, cX (cF = cM = -2a/3);
// M4 a, cF (= cM), cFF, cT, cX, h1, h2; M6 cT, cX, h1, h2 (its passive part
// is formed from the state in the Jacobian action).
template <int MAT>
__host__ __device__ constexpr int n_lcoef() {
  return MAT == NLE_MAT_M1 ? 1 : (MAT == NLE_MAT_M2 ? 3 : (MAT == NLE_MAT_M6 ? 4 : 7));
}

template <int MAT>
__device__ __forceinline__ void pack_coef(const Coef &c, double q[7]) {
  if (MAT == NLE_MAT_M1) {
    q[0] = c.cX;
  } else if (MAT == NLE_MAT_M6) {
    q[0] = c.cT;
    q[1] = c.cX;
    q[2] = c.h1;
    q[3] = c.h2;
  } else if (MAT == NLE_MAT_M2) {
    q[0] = c.a;
    q[1] = c.cT;
    q[2] = c.cX;
  } else {
    q[0] = c.a;
    q[1] = c.cF;
    q[2] = c.cFF;
    q[3] = c.cT;
    q[4] = c.cX;
    q[5] = c.h1;
    q[6] = c.h2;
  }
}

template <int MAT, typename T>
__device__ __forceinline__ Coef unpack_coef(const T *lc, uint32_t ne, uint32_t ge,
                                            const MatParams &mp) {
  Coef c;
  c.pT = 0.0;
  c.cFF = 0.0;
  c.h1 = 0.0;
  c.h2 = 0.0;
  if (MAT == NLE_MAT_M1) {
    c.a = mp.mu;
    c.cF = 0.0;
    c.cM = 0.0;
    c.cT = mp.lam;
    c.cX = double(lc[ge]);
  } else if (MAT == NLE_MAT_M6) {
    c.a = 0.0;
    c.cF = 0.0;
    c.cM = 0.0;
    c.cT = double(lc[ge]);
    c.cX = double(lc[size_t(ne) + ge]);
    c.h1 = double(lc[2 * size_t(ne) + ge]);
    c.h2 = double(lc[3 * size_t(ne) + ge]);
  } else if (MAT == NLE_MAT_M2) {
    c.a = double(lc[ge]);
    c.cT = double(lc[size_t(ne) + ge]);
    c.cX = double(lc[2 * size_t(ne) + ge]);
    c.cF = -2.0 / 3.0 * c.a;
    c.cM = c.cF;
  } else {
    c.a = double(lc[ge]);
    c.cF = double(lc[size_t(ne) + ge]);
    c.cM = c.cF;
    c.cFF = double(lc[2 * size_t(ne) + ge]);
    c.cT = double(lc[3 * size_t(ne) + ge]);
    c.cX = double(lc[4 * size_t(ne) + ge]);
    c.h1 = double(lc[5 * size_t(ne) + ge]);
    c.h2 = double(lc[6 * size_t(ne) + ge]);
  }
  return c;
}

// cof A (cof A = det A A^-T), row-major
template <typename T>
__device__ __forceinline__ void cofactor3(const T A[3][3], T C[3][3]) {
  C[0][0] = A[1][1] * A[2][2] - A[1][2] * A[2][1];
  C[0][1] = A[1][2] * A[2][0] - A[1][0] * A[2][2];
  C[0][2] = A[1][0] * A[2][1] - A[1][1] * A[2][0];
  C[1][0] = A[0][2] * A[2][1] - A[0][1] * A[2][2];
  C[1][1] = A[0][0] * A[2][2] - A[0][2] * A[2][0];
  C[1][2] = A[0][1] * A[2][0] - A[0][0] * A[2][1];
  C[2][0] = A[0][1] * A[1][2] - A[0][2] * A[1][1];
  C[2][1] = A[0][2] * A[1][0] - A[0][0] * A[1][2];
  C[2][2] = A[0][0] * A[1][1] - A[0][1] * A[1][0];
}

// F = I + H and F^-T = cof(F) / det(F) in the kernel's precision (enough for
// the tangent; J - 1 and ln J are not needed once the coefficients are cached).
template <typename T>
__device__ __forceinline__ void kinematics_light(const T H[3][3], Kin<T> &k) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) k.F[i][j] = H[i][j] + (i == j ? T(1) : T(0));
  const T(&F)[3][3] = k.F;
  T c[3][3];
  c[0][0] = F[1][1] * F[2][2] - F[1][2] * F[2][1];
  c[0][1] = F[1][2] * F[2][0] - F[1][0] * F[2][2];
  c[0][2] = F[1][0] * F[2][1] - F[1][1] * F[2][0];
  c[1][0] = F[0][2] * F[2][1] - F[0][1] * F[2][2];
  c[1][1] = F[0][0] * F[2][2] - F[0][2] * F[2][0];
  c[1][2] = F[0][1] * F[2][0] - F[0][0] * F[2][1];
  c[2][0] = F[0][1] * F[1][2] - F[0][2] * F[1][1];
  c[2][1] = F[0][2] * F[1][0] - F[0][0] * F[1][2];
  c[2][2] = F[0][0] * F[1][1] - F[0][1] * F[1][0];
  const T J = F[0][0] * c[0][0] + F[0][1] * c[0][1] + F[0][2] * c[0][2];
  T ij;
  if (sizeof(T) == 8)
    ij = T(1) / J;
  else
    ij = T(__builtin_amdgcn_rcpf(float(J)));
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) k.FiT[i][j] = c[i][j] * ij;
  k.bad = false;
}

template <typename T, int OP, int MAT>
__device__ __forceinline__ void element_forces(const ElemIn<T> &d, const T *uS, const T *vS,
                                               const T *xS, int NL, const MatParams &mp,
                                               T out[4][3], bool &bad, double &eacc,
                                               const ElemArgs<T> &A, uint32_t ge) {
  const int la[4] = {lo16(d.lcp.x), hi16(d.lcp.x), lo16(d.lcp.y), hi16(d.lcp.y)};
  // geometry from the block's slot coordinates: D = [x1-x0 | x2-x0 | x3-x0],
  // grad N_a = row a-1 of D^-1 = column a-1 of cof(D) / det D (a = 1..3),
  // grad N_0 = -(grad N_1 + grad N_2 + grad N_3), V = det D / 6
  T g[4][3];
  T Vt;
  {
    T D[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const T x0 = xS[i * NL + la[0]];
#pragma unroll
      for (int a = 1; a < 4; ++a) D[i][a - 1] = xS[i * NL + la[a]] - x0;
    }
    T C[3][3];
    cofactor3(D, C);
    const T det = D[0][0] * C[0][0] + D[0][1] * C[0][1] + D[0][2] * C[0][2];
    // FP32: the hardware reciprocal (1 ulp) instead of a correctly rounded
    // division sequence; FP64 keeps the division
    T id;
    if (sizeof(T) == 8)
      id = T(1) / det;
    else
      id = T(__builtin_amdgcn_rcpf(float(det)));
#pragma unroll
    for (int a = 1; a < 4; ++a)
#pragma unroll
      for (int j = 0; j < 3; ++j) g[a][j] = C[j][a - 1] * id;
    Vt = det * T(1.0 / 6.0);
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) g[0][j] = -(g[1][j] + g[2][j] + g[3][j]);
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
  const double V = double(Vt);
  Coef cf;
  T Ff[3], f[3];
  Guc<T> gu;  // law M6: the passive Guccione part at this state
  if (OP == OP_JV) {
    // Jacobian action from the linearization cache (always present: the
    // diagonal pass of the linearization writes it)
    kinematics_light(H, k);
    cf = unpack_coef<MAT>(A.lcoef, uint32_t(A.n_e), ge, mp);
    if (MAT == NLE_MAT_M4) {
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        f[i] = d.f[i];
        Ff[i] = f[i] + H[i][0] * d.f[0] + H[i][1] * d.f[1] + H[i][2] * d.f[2];
      }
    }
  } else {
    kinematics(H, k);
    bad |= k.bad;
    FibreKin fk;
    if (has_fibre<MAT>()) fk = fibre_kinematics(H, d.f);
    if (MAT == NLE_MAT_M6 && OP != OP_ODIAG) guccione(H, d.f, d.sh, mp, gu);
    if (OP == OP_ENERGY) {
      double psi = energy_density<MAT>(k, H, fk, mp);
      if (MAT == NLE_MAT_M6) psi += 0.5 * mp.g6[0] * expm1(gu.Q);
      eacc += V * psi;
      return;
    }
    cf = coefficients<MAT>(k, H, fk, mp);
    if (OP == OP_DIAG && A.lc64) {  // (the off-diagonal pass leaves the cache)
      double q[7];
      pack_coef<MAT>(cf, q);
#pragma unroll
      for (int t = 0; t < n_lcoef<MAT>(); ++t) {
        A.lc64[size_t(t) * size_t(A.n_e) + ge] = q[t];
        A.lc32[size_t(t) * size_t(A.n_e) + ge] = float(q[t]);
      }
    }
    if (has_fibre<MAT>()) {
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        Ff[i] = T(fk.Ff[i]);
        f[i] = d.f[i];
      }
    }
  }
  if (OP == OP_RES) {
    const T ca = T(V * cf.a), cp = T(V * cf.pT);
    T P[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) P[i][j] = ca * k.F[i][j] + cp * k.FiT[i][j];
    if (MAT == NLE_MAT_M6) {  // passive part F S
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
          P[i][j] += T(V) * (k.F[i][0] * gu.S[0][j] + k.F[i][1] * gu.S[1][j] +
                             k.F[i][2] * gu.S[2][j]);
    }
    if (has_fibre<MAT>()) {
      const T ch = T(V * cf.h1);
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) P[i][j] += ch * Ff[i] * f[j];
    }
#pragma unroll
    for (int a = 1; a < 4; ++a)
#pragma unroll
      for (int i = 0; i < 3; ++i)
        out[a][i] = P[i][0] * g[a][0] + P[i][1] * g[a][1] + P[i][2] * g[a][2];
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
        if (MAT != NLE_MAT_M1) FdF += k.F[i][j] * dF[i][j];
      }
    // X = F^-T dF^T F^-T = F^-T M with M = dF^T F^-T
    T M[3][3];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        M[p][j] = dF[0][p] * k.FiT[0][j] + dF[1][p] * k.FiT[1][j] + dF[2][p] * k.FiT[2][j];
    // coefficient products in the action's own precision (V = Vt exactly)
    const T ca = Vt * T(cf.a), cX = Vt * T(cf.cX);
    const T sT = Vt * T(cf.cT) * L + (MAT != NLE_MAT_M1 ? Vt * T(cf.cM) * FdF : T(0));
    T sF = MAT != NLE_MAT_M1 ? Vt * T(cf.cF) * L : T(0);
    if (MAT == NLE_MAT_M4) sF += Vt * T(cf.cFF) * FdF;
    // fibre terms (M4): h1 (dF f) (x) f + h2 ((F f).(dF f)) (F f) (x) f
    T dFf[3] = {T(0), T(0), T(0)}, s2 = T(0);
    if (MAT == NLE_MAT_M4) {
#pragma unroll
      for (int i = 0; i < 3; ++i) dFf[i] = dF[i][0] * f[0] + dF[i][1] * f[1] + dF[i][2] * f[2];
      s2 = Vt * T(cf.h2) * (Ff[0] * dFf[0] + Ff[1] * dFf[1] + Ff[2] * dFf[2]);
      const T c1 = Vt * T(cf.h1);
#pragma unroll
      for (int i = 0; i < 3; ++i) dFf[i] *= c1;
    }
    T dP[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const T X = k.FiT[i][0] * M[0][j] + k.FiT[i][1] * M[1][j] + k.FiT[i][2] * M[2][j];
        T t = ca * dF[i][j] + sT * k.FiT[i][j] + cX * X;
        if (MAT != NLE_MAT_M1) t += sF * k.F[i][j];
        if (MAT == NLE_MAT_M4) t += (dFf[i] + s2 * Ff[i]) * f[j];
        dP[i][j] = t;
      }
#pragma unroll
    for (int a = 1; a < 4; ++a)
#pragma unroll
      for (int i = 0; i < 3; ++i)
        out[a][i] = dP[i][0] * g[a][0] + dP[i][1] * g[a][1] + dP[i][2] * g[a][2];
  } else if (OP == OP_ODIAG) {
    // entry (i, k) of vertex a's self block, k = i+1 mod 3: with w = F^-T g,
    // z = F g (g = grad N_a) and c1 = cF + cM (= 2 cF, major symmetry),
    //   V [c1/2 (w_i z_k + z_i w_k) + cFF z_i z_k + (cT + cX) w_i w_k
    //      + h2 (g.f)^2 (Ff)_i (Ff)_k]
    const double c1 = 0.5 * V * (cf.cF + cf.cM), c2 = V * (cf.cT + cf.cX);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      T w[3], z[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        w[i] = k.FiT[i][0] * g[a][0] + k.FiT[i][1] * g[a][1] + k.FiT[i][2] * g[a][2];
        z[i] = k.F[i][0] * g[a][0] + k.F[i][1] * g[a][1] + k.F[i][2] * g[a][2];
      }
      T gf2 = T(0);
      if (MAT == NLE_MAT_M4) {
        const T gf = g[a][0] * f[0] + g[a][1] * f[1] + g[a][2] * f[2];
        gf2 = gf * gf;
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const int q = (i + 1) % 3;
        T o = T(c1) * (w[i] * z[q] + z[i] * w[q]) + T(c2) * w[i] * w[q];
        if (MAT == NLE_MAT_M4) o += T(V * cf.cFF) * z[i] * z[q] + T(V * cf.h2) * gf2 * Ff[i] * Ff[q];
        out[a][i] = o;
      }
    }
    return;
  } else {  // OP_DIAG: dF = e_i (x) g_a, one column at a time
    const double ca = V * cf.a, c1 = V * (cf.cF + cf.cM), c2 = V * (cf.cT + cf.cX);
    // law M6, passive part: g.S g + dE : dS(dE) with dE = sym((F^T e_i) (x) g);
    // in the frame dEb = sym(rb (x) gb), rb = R^T F^T e_i, gb = R^T g
    T rb[3][3];  // rb[i][a] for component i
    if (MAT == NLE_MAT_M6) {
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int b = 0; b < 3; ++b)
          rb[i][b] = gu.R[0][b] * k.F[i][0] + gu.R[1][b] * k.F[i][1] + gu.R[2][b] * k.F[i][2];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const T gg = g[a][0] * g[a][0] + g[a][1] * g[a][1] + g[a][2] * g[a][2];
      T gSg = T(0), gb[3] = {T(0), T(0), T(0)};
      if (MAT == NLE_MAT_M6) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) gSg += g[a][i] * gu.S[i][j] * g[a][j];
#pragma unroll
        for (int b = 0; b < 3; ++b)
          gb[b] = gu.R[0][b] * g[a][0] + gu.R[1][b] * g[a][1] + gu.R[2][b] * g[a][2];
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const T w = k.FiT[i][0] * g[a][0] + k.FiT[i][1] * g[a][1] + k.FiT[i][2] * g[a][2];
        const T z = k.F[i][0] * g[a][0] + k.F[i][1] * g[a][1] + k.F[i][2] * g[a][2];
        T dg = T(ca) * gg + T(c1) * w * z + T(c2) * w * w;
        if (has_fibre<MAT>()) {
          const T gf = g[a][0] * f[0] + g[a][1] * f[1] + g[a][2] * f[2];
          dg += T(V * cf.cFF) * z * z + (T(V * cf.h1) + T(V * cf.h2) * Ff[i] * Ff[i]) * gf * gf;
        }
        if (MAT == NLE_MAT_M6) {
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
          dg += T(V) * (gSg + gu.Ce * (q2 + T(2) * be * be));
        }
        out[a][i] = dg;
      }
    }
    return;
  }
  // vertex 0: grad N_0 = -(grad N_1 + grad N_2 + grad N_3)
#pragma unroll
  for (int i = 0; i < 3; ++i) out[0][i] = -(out[1][i] + out[2][i] + out[3][i]);
}

// Jacobian action of one element, 12 values (vertex-major), in the action's
// precision from the coefficients cached at linearization.  Unnormalised
// forms keep the instruction count down: with d_a = x_a - x_0 (a = 1..3) and
// C the cofactor matrix of D = [d_1 d_2 d_3], grad N_a = c_a / det D (c_a
// column a-1 of C), so H = Hh / det D, dF = dFh / det D with
// Hh = sum_a (u_a - u_0) (x) c_a, dFh = sum_a (v_a - v_0) (x) c_a; with K =
// cof F = J F^-T, F^-T = K / J.  The tangent form of coefficients() then
// gives y_a = V dP grad N_a = Q c_a / (6 det D) with
//   Q = a dFh + (cF Lh / J + cFF Fh) F + (cT Lh / J + cM Fh) K / J
//       + cX / J^2 K dFh^T K + h1 (dFh f) (x) f + h2 ((F f).(dFh f)) (F f) (x) f,
// Lh = K : dFh, Fh = F : dFh; y_0 = -(y_1 + y_2 + y_3).
template <typename T, int MAT>
__device__ __forceinline__ void element_jv(const ElemIn<T> &d, const T *uS, const T *vS,
                                           const T *xS, int NL, const MatParams &mp,
                                           T out[4][3], const ElemArgs<T> &A, uint32_t ge) {
  const int la[4] = {lo16(d.lcp.x), hi16(d.lcp.x), lo16(d.lcp.y), hi16(d.lcp.y)};
  T D[3][3], DU[3][3], DV[3][3];
  {
    T x0[3], u0[3], v0[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      x0[i] = xS[i * NL + la[0]];
      u0[i] = uS[i * NL + la[0]];
      v0[i] = vS[i * NL + la[0]];
    }
#pragma unroll
    for (int a = 1; a < 4; ++a)
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        D[i][a - 1] = xS[i * NL + la[a]] - x0[i];
        DU[i][a - 1] = uS[i * NL + la[a]] - u0[i];
        DV[i][a - 1] = vS[i * NL + la[a]] - v0[i];
      }
  }
  T C[3][3];
  cofactor3(D, C);
  const T det = D[0][0] * C[0][0] + D[0][1] * C[0][1] + D[0][2] * C[0][2];
  // column a-1 of C is c_a: Hh[i][j] = sum_a DU[i][a-1] C[j][a-1]
  T F[3][3], dF[3][3];
  T id;
  if (sizeof(T) == 8)
    id = T(1) / det;
  else
    id = T(__builtin_amdgcn_rcpf(float(det)));
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const T h = DU[i][0] * C[j][0] + DU[i][1] * C[j][1] + DU[i][2] * C[j][2];
      F[i][j] = i == j ? h * id + T(1) : h * id;
      dF[i][j] = DV[i][0] * C[j][0] + DV[i][1] * C[j][1] + DV[i][2] * C[j][2];
    }
  T K[3][3];
  cofactor3(F, K);
  const T J = F[0][0] * K[0][0] + F[0][1] * K[0][1] + F[0][2] * K[0][2];
  T iJ;
  if (sizeof(T) == 8)
    iJ = T(1) / J;
  else
    iJ = T(__builtin_amdgcn_rcpf(float(J)));
  const Coef cf = unpack_coef<MAT>(A.lcoef, uint32_t(A.n_e), ge, mp);
  const T s = id * T(1.0 / 6.0);  // 1 / (6 det D)
  const T sJ = s * iJ, sJ2 = sJ * iJ;
  const T ca = T(cf.a) * s, cX = T(cf.cX) * sJ2;
  T Lh = T(0), Fh = T(0);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      Lh += K[i][j] * dF[i][j];
      if (MAT != NLE_MAT_M1) Fh += F[i][j] * dF[i][j];
    }
  T sK = T(cf.cT) * sJ2 * Lh, sF = T(0);
  if (MAT != NLE_MAT_M1) {
    sK += T(cf.cM) * sJ * Fh;
    sF = T(cf.cF) * sJ * Lh + T(cf.cFF) * s * Fh;
  }
  // fibre terms (M4, M6)
  T Ff[3] = {T(0), T(0), T(0)}, dFf[3] = {T(0), T(0), T(0)}, f[3] = {T(0), T(0), T(0)};
  T s2 = T(0);
  if (has_fibre<MAT>()) {
#pragma unroll
    for (int i = 0; i < 3; ++i) f[i] = d.f[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Ff[i] = F[i][0] * f[0] + F[i][1] * f[1] + F[i][2] * f[2];
      dFf[i] = dF[i][0] * f[0] + dF[i][1] * f[1] + dF[i][2] * f[2];
    }
    s2 = T(cf.h2) * s * (Ff[0] * dFf[0] + Ff[1] * dFf[1] + Ff[2] * dFf[2]);
    const T c1 = T(cf.h1) * s;
#pragma unroll
    for (int i = 0; i < 3; ++i) dFf[i] *= c1;
  }
  // M = dFh^T K, then Q = ca dFh + sK K + sF F + cX K M (+ fibre terms)
  T M[3][3];
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      M[p][j] = dF[0][p] * K[0][j] + dF[1][p] * K[1][j] + dF[2][p] * K[2][j];
  T Q[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const T X = K[i][0] * M[0][j] + K[i][1] * M[1][j] + K[i][2] * M[2][j];
      T t = ca * dF[i][j] + sK * K[i][j] + cX * X;
      if (MAT != NLE_MAT_M1) t += sF * F[i][j];
      if (has_fibre<MAT>()) t += (dFf[i] + s2 * Ff[i]) * f[j];
      Q[i][j] = t;
    }
  if (MAT == NLE_MAT_M6) {
    // passive Guccione part, formed from the state: s (dFh S + F dS(dEh)),
    // dEh = sym(F^T dFh)
    T H[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) H[i][j] = F[i][j] - (i == j ? T(1) : T(0));
    Guc<T> gu;
    guccione(H, d.f, d.sh, mp, gu);
    T dE[3][3], dS[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        dE[i][j] = T(0.5) * (F[0][i] * dF[0][j] + F[1][i] * dF[1][j] + F[2][i] * dF[2][j] +
                             dF[0][i] * F[0][j] + dF[1][i] * F[1][j] + dF[2][i] * F[2][j]);
    guccione_dS(gu, dE, mp, dS);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        Q[i][j] += s * (dF[i][0] * gu.S[0][j] + dF[i][1] * gu.S[1][j] + dF[i][2] * gu.S[2][j] +
                        F[i][0] * dS[0][j] + F[i][1] * dS[1][j] + F[i][2] * dS[2][j]);
  }
#pragma unroll
  for (int a = 1; a < 4; ++a)
#pragma unroll
    for (int i = 0; i < 3; ++i)
      out[a][i] = Q[i][0] * C[0][a - 1] + Q[i][1] * C[1][a - 1] + Q[i][2] * C[2][a - 1];
#pragma unroll
  for (int i = 0; i < 3; ++i) out[0][i] = -(out[1][i] + out[2][i] + out[3][i]);
}

// Law M1 written on the deformed edge matrix X = D + DU (F = X D^-1).  With
// C = cof D (column a-1 is det D grad N_a), CX = cof X (column a-1 is
// det X grad n_a, the spatial gradient), Lh = DV CX^T (det X times the
// spatial gradient of v) and G = C^T C, the action of the law's tangent (Sec. 2)
// dP = mu dF + lam (F^-T : dF) F^-T + cX F^-T dF^T F^-T on vertex a is
//   y_a = V dP grad N_a
//       = mu / (6 det D) DV G e_a + det D / (6 det X^2) (cX Lh^T + lam tr(Lh) I) CX e_a,
// since F^-T grad N_a = grad n_a, F^-T dF^T w = (dF F^-1)^T w and dF F^-1 = DV X^-1.
template <typename T>
__device__ __forceinline__ void element_jv_m1(const ElemIn<T> &d, const T *uS, const T *vS,
                                              const T *xS, int NL, const MatParams &mp,
                                              T out[4][3]) {
  const int la[4] = {lo16(d.lcp.x), hi16(d.lcp.x), lo16(d.lcp.y), hi16(d.lcp.y)};
  T D[3][3], X[3][3], DV[3][3];
  {
    T x0[3], u0[3], v0[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      x0[i] = xS[i * NL + la[0]];
      u0[i] = uS[i * NL + la[0]];
      v0[i] = vS[i * NL + la[0]];
    }
#pragma unroll
    for (int a = 1; a < 4; ++a)
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const T dx = xS[i * NL + la[a]] - x0[i];
        D[i][a - 1] = dx;
        X[i][a - 1] = dx + (uS[i * NL + la[a]] - u0[i]);
        DV[i][a - 1] = vS[i * NL + la[a]] - v0[i];
      }
  }
  T C[3][3], CX[3][3];
  cofactor3(D, C);
  cofactor3(X, CX);
  const T det = D[0][0] * C[0][0] + D[0][1] * C[0][1] + D[0][2] * C[0][2];
  const T detx = X[0][0] * CX[0][0] + X[0][1] * CX[0][1] + X[0][2] * CX[0][2];
  T id, idx;
  if (sizeof(T) == 8) {
    id = T(1) / det;
    idx = T(1) / detx;
  } else {
    id = T(__builtin_amdgcn_rcpf(float(det)));
    idx = T(__builtin_amdgcn_rcpf(float(detx)));
  }
  T Lh[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      Lh[i][j] = DV[i][0] * CX[j][0] + DV[i][1] * CX[j][1] + DV[i][2] * CX[j][2];
  const T s1 = T(mp.mu) * id * T(1.0 / 6.0);
  const T s2 = det * idx * idx * T(1.0 / 6.0);
  const T bX = d.cx * s2;
  const T bT = T(mp.lam) * s2 * (Lh[0][0] + Lh[1][1] + Lh[2][2]);
  // B = bX Lh^T + bT I and Gs = s1 C^T C (symmetric)
  T B[3][3], Gs[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) B[i][j] = i == j ? bX * Lh[j][i] + bT : bX * Lh[j][i];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b) {
      Gs[a][b] = s1 * (C[0][a] * C[0][b] + C[1][a] * C[1][b] + C[2][a] * C[2][b]);
      Gs[b][a] = Gs[a][b];
    }
#pragma unroll
  for (int a = 1; a < 4; ++a)
#pragma unroll
    for (int i = 0; i < 3; ++i)
      out[a][i] = DV[i][0] * Gs[0][a - 1] + DV[i][1] * Gs[1][a - 1] + DV[i][2] * Gs[2][a - 1] +
                  B[i][0] * CX[0][a - 1] + B[i][1] * CX[1][a - 1] + B[i][2] * CX[2][a - 1];
#pragma unroll
  for (int i = 0; i < 3; ++i) out[0][i] = -(out[1][i] + out[2][i] + out[3][i]);
}

// One shared node of the merge: its partials (contiguous, in block order)
// summed four loads at a time but added in slot order, then finalized.
template <typename T, int OP>
__device__ __forceinline__ void merge_node(const uint32_t *fx_node, const int32_t *fx_ptr,
                                           const T *partial, int64_t k, const T *v, const T *vz,
                                           T bt, T *out, const double *fext, double lscale,
                                           double &nrm, bool dot, const T *ep_w, T epc, const T *fs,
                                           int nomask, const T *icm, const double *iut,
                                           const T *u) {
  T acc[3] = {T(0), T(0), T(0)};
  const uint32_t w = fx_node[k];
  const int q0 = fx_ptr[k], q1 = fx_ptr[k + 1];
  // partials read at indexes clamped into the range, so the four loads issue
  // together without branches (entries past the range are not added)
  const int last = q1 - 1;
  for (int q = q0; q < q1; q += 4) {
    T pv[4][3];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t qq = 3 * int64_t(min(q + t, last));
#pragma unroll
      for (int i = 0; i < 3; ++i) pv[t][i] = partial[qq + i];
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (q + t < q1) {
        acc[0] += pv[t][0];
        acc[1] += pv[t][1];
        acc[2] += pv[t][2];
      }
  }
  // padding entries (batched mode aligns each instance to whole workgroups)
  // have an empty slot range and the id 0xFFFFFFFF
  if (w != 0xFFFFFFFFu)
    finalize_node<T, OP>(w & NODE_MASK, (w >> 28) & 7u, acc, v, vz, bt, out, fext, lscale, nrm,
                         dot, ep_w, epc, fs, nomask, icm, iut, u);
}

// NLC > 0: the block's slot count is at most NLC and its element count at
// most NTB, and these compile-time strides of the LDS arrays turn every
// gather and contribution address into one base plus immediate offsets;
// NLC = 0 takes the strides from the mesh (nl_max, be_max) at run time.
template <typename T, int OP, int MAT, int NLC>
__global__ __launch_bounds__(NTB) void k_elem_block(ElemArgs<T> A) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T *lds = reinterpret_cast<T *>(lds_raw);
  // Reduction partials are stored at the block's index b (consumers sum the
  // blocks of one problem instance, which are contiguous).
  const int nrun = A.blk_list ? A.n_list : A.nblk;
  const int bw = block_id(nrun, A.per_xcd);
  if (bw >= nrun) return;  // padding workgroup of the XCD remap
  const int b = A.blk_list ? A.blk_list[bw] : bw;
  if (A.skip && A.skip[0] != 0) return;
  const int inst = A.blk_inst ? A.blk_inst[b] : 0;
  if (A.inst_done && A.inst_done[inst]) return;
  MatParams mp = A.mp;
  double lscale = A.s;
  if (A.inst_mat) {
    mp.mu = A.inst_mat[4 * inst];
    mp.lam = A.inst_mat[4 * inst + 1];
    mp.cvol = A.inst_mat[4 * inst + 2];
    mp.kappa = A.inst_mat[4 * inst + 3];
  }
  if (A.inst_s) lscale = A.inst_s[inst];
  const int tid = threadIdx.x;
  const int e0 = A.blk_elem[b], ne = A.blk_elem[b + 1] - e0;
  const int p0 = A.blk_node[b], nl = A.blk_node[b + 1] - p0;
  const int NL = NLC > 0 ? NLC : A.nl_max;
  const int BE = NLC > 0 ? NTB : A.be_max;
  const int C4 = 4 * BE;
  T *uS = lds;                 // [3][NL]
  T *vS = lds + 3 * NL;        // [3][NL]      (Jv only)
  T *xS = lds + 6 * NL;        // [3][NL]      slot coordinates
  T *cS = lds + 9 * NL;        // [3][4 BE]    contributions in slot-sorted order
  // reduction scratch after the arrays, at the 8-byte aligned offset the
  // host sizes the allocation with
  double *rs = reinterpret_cast<double *>(
      lds_raw + ((size_t(9 * NL + 12 * BE) * sizeof(T) + 7) & ~size_t(7)));

  // The inputs of this thread's first element are requested before the node
  // gather so all of these loads are in flight together.
  ElemIn<T> ea;
  if (tid < ne) load_elem<MAT, OP>(A, uint32_t(e0 + tid), ea);

  // Phase 1: gather nodal state (and direction) of the block.  The first slot
  // of each thread is requested into registers together with its phase-3
  // data (word, range, partial position), which stay in registers.
  uint32_t w0 = 0;
  int beg0 = 0, end0 = 0, mp0 = -1;
  T u1[3] = {T(0), T(0), T(0)}, x1[3] = {T(0), T(0), T(0)};
  T v1[3] = {T(0), T(0), T(0)}, z1[3] = {T(0), T(0), T(0)};
  if (tid < nl) {
    w0 = A.nodes[p0 + tid];
    end0 = A.csr_end[p0 + tid];
    beg0 = tid == 0 ? 0 : int(A.csr_end[p0 + tid - 1]);
    if (OP != OP_ENERGY && (w0 & 0x80000000u)) mp0 = A.mpos[p0 + tid];
    const int64_t g3 = 3 * int64_t(w0 & NODE_MASK), s3 = 3 * int64_t(p0 + tid);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      u1[i] = A.u[g3 + i];
      x1[i] = A.xr[s3 + i];
      if (OP == OP_JV) {
        v1[i] = A.v[g3 + i];
        if (A.vz) z1[i] = A.vz[g3 + i];
      }
    }
  }

  // CG direction formed here (v = z + beta p): beta and the stopping test
  // from the previous update's partials, taken identically by every
  // workgroup while the slot loads above are in flight; block 0 records them
  // (the update kernel of this iteration reads r.z and beta)
  T bt = T(0);
  if (OP == OP_JV && A.vz) {
    const double rz = sum_partials_256(A.cg_red, A.cg_np, rs);
    const double rr = sum_partials_256(A.cg_red + VGRID_MAX, A.cg_np, rs);
    const double rzo = A.cg_scal[cgslot::RZOLD];
    int stop = 0;
    if (!(rr == rr))
      stop = 3;
    else if (rr <= A.cg_scal[cgslot::TOL2])
      stop = 1;
    else if (double(A.cg_flag[1]) >= A.cg_scal[cgslot::MAXIT])
      stop = 5;
    const double beta = rzo > 0.0 ? rz / rzo : 0.0;
    if (b == 0 && tid == 0) {
      A.cg_scal[cgslot::RZ] = rz;
      A.cg_scal[cgslot::RR] = rr;
      A.cg_scal[cgslot::BETA] = beta;
      if (stop) A.cg_flag[0] = stop;
    }
    if (stop) return;
    bt = T(beta);
  }

  if (tid < nl) {
    const uint32_t mk = (w0 >> 28) & 7u;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      uS[i * NL + tid] = u1[i];
      xS[i * NL + tid] = x1[i];
      if (OP == OP_JV) {
        const T vd = A.vz ? z1[i] + bt * v1[i] : v1[i];
        vS[i * NL + tid] = (!A.nomask && ((mk >> i) & 1u)) ? T(0) : vd;
      }
    }
  }
  for (int l = tid + NTB; l < nl; l += NTB) {
    const uint32_t w = A.nodes[p0 + l];
    const int64_t g3 = 3 * int64_t(w & NODE_MASK);
    const uint32_t mk = (w >> 28) & 7u;
    const int64_t s3 = 3 * int64_t(p0 + l);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      uS[i * NL + l] = A.u[g3 + i];
      xS[i * NL + l] = A.xr[s3 + i];
      if (OP == OP_JV) {
        const T vd = A.vz ? A.vz[g3 + i] + bt * A.v[g3 + i] : A.v[g3 + i];
        vS[i * NL + l] = (!A.nomask && ((mk >> i) & 1u)) ? T(0) : vd;
      }
    }
  }
  __syncthreads();

  // Phase 2: one element per thread at a time.
  bool bad = false;
  double eacc = 0.0;
  auto run = [&](const ElemIn<T> &d) {
    T out[4][3];
    if constexpr (OP == OP_JV && MAT == NLE_MAT_M1)
      element_jv_m1<T>(d, uS, vS, xS, NL, mp, out);
    else if constexpr (OP == OP_JV)
      element_jv<T, MAT>(d, uS, vS, xS, NL, mp, out, A, d.ge);
    else
      element_forces<T, OP, MAT>(d, uS, vS, xS, NL, mp, out, bad, eacc, A, d.ge);
    if (OP != OP_ENERGY) {
      const int cp[4] = {lo16(d.lcp.z), hi16(d.lcp.z), lo16(d.lcp.w), hi16(d.lcp.w)};
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int i = 0; i < 3; ++i) cS[i * C4 + cp[a]] = out[a][i];
    }
  };
  for (int e = tid; e < ne; e += NTB) {
    if (e != tid) load_elem<MAT, OP>(A, uint32_t(e0 + e), ea);
    run(ea);
  }
  if (bad && A.flag) A.flag[inst] = 1;

  if (OP == OP_ENERGY) {
    const double s = block_sum<NTB>(eacc, rs);
    if (tid == 0) A.red[b] = s;
    return;
  }
  __syncthreads();

  // Phase 3: node sums over contiguous ranges, in (element, vertex) order.
  double nrm = 0.0;
  const T epc = A.ep_coef ? T(A.ep_coef[0]) : T(0);
  for (int l = tid; l < nl; l += NTB) {
    const bool first = l == tid;
    const int beg = first ? beg0 : int(A.csr_end[p0 + l - 1]);
    const int end = first ? end0 : int(A.csr_end[p0 + l]);
    T acc[3] = {T(0), T(0), T(0)};
    for (int q = beg; q < end; ++q) {
#pragma unroll
      for (int i = 0; i < 3; ++i) acc[i] += cS[i * C4 + q];
    }
    const uint32_t w = first ? w0 : A.nodes[p0 + l];
    if (w & 0x80000000u) {
      const int mp = first ? mp0 : A.mpos[p0 + l];
      T *pp = A.partial + 3 * int64_t(mp);
      pp[0] = acc[0];
      pp[1] = acc[1];
      pp[2] = acc[2];
    } else {
      finalize_node<T, OP>(w & NODE_MASK, (w >> 28) & 7u, acc, A.v, A.vz, bt, A.out, A.fext,
                           lscale, nrm, A.ep_red != nullptr, A.ep_w, epc, A.fs, A.nomask, A.icm,
                           A.iut, A.u);
    }
  }
  if (OP == OP_RES || (OP == OP_JV && A.ep_red)) {
    const double s = block_sum<NTB>(nrm, rs);
    if (tid == 0) (OP == OP_RES ? A.red : A.ep_red)[b] = s;
  }
}

template <typename T, int OP>
__global__ __launch_bounds__(NT) void k_elem_merge(MergeArgs<T> A) {
  __shared__ double rs[NT / 64];
  if (A.skip && A.skip[0] != 0) return;
  const int wg = A.mwg_list ? A.mwg_list[blockIdx.x] : int(blockIdx.x);
  const int inst = A.mwg_inst ? A.mwg_inst[wg] : 0;
  if (A.inst_done && A.inst_done[inst]) return;
  const double lscale = A.inst_s ? A.inst_s[inst] : A.s;
  const int64_t k = int64_t(wg) * NT + threadIdx.x;
  double nrm = 0.0;
  if (k < A.n_sh)
    merge_node<T, OP>(A.fx_node, A.fx_ptr, A.partial, k, A.v, A.vz,
                      A.vz ? T(A.cg_scal[cgslot::BETA]) : T(0), A.out, A.fext, lscale, nrm,
                      A.ep_red != nullptr, A.ep_w, A.ep_coef ? T(A.ep_coef[0]) : T(0), A.fs,
                      A.nomask, A.icm, A.iut, A.u);
  if (OP == OP_RES || (OP == OP_JV && A.ep_red)) {
    const double s = block_sum<NT>(nrm, rs);
    if (threadIdx.x == 0) (OP == OP_RES ? A.red : A.ep_red)[wg] = s;
  }
}

// Compile-time LDS strides offered for the Jacobian action (slots per block).
constexpr int NLC_BUCKETS[] = {256, 320, 384, 512};

template <typename T, int OP, int MAT, int NLC>
void launch_block_nl(Ctx *c, ElemArgs<T> &A) {
  const int nrun = A.blk_list ? A.n_list : A.nblk;
  A.per_xcd = c->xcd_remap ? (nrun + 7) / 8 : 0;
  const int grid = A.per_xcd > 0 ? 8 * A.per_xcd : nrun;
  const int NL = NLC > 0 ? NLC : A.nl_max, BE = NLC > 0 ? NTB : A.be_max;
  size_t lds = size_t(9 * NL + 12 * BE) * sizeof(T);
  lds = (lds + 7) & ~size_t(7);
  lds += size_t(NTB / 64) * sizeof(double);  // reduction scratch after the arrays
  hipLaunchKernelGGL((k_elem_block<T, OP, MAT, NLC>), dim3(grid), dim3(NTB), lds, c->stream, A);
}

template <typename T, int OP, int MAT>
void launch_block(Ctx *c, ElemArgs<T> &A) {
  // a bucket is taken only if its LDS fits the device's per-workgroup limit
  auto fits = [&](int nlc) {
    return (size_t(9 * nlc + 12 * NTB) * sizeof(T) + 8 + NTB / 64 * 8) <= c->lds_limit;
  };
  if (OP == OP_JV && A.be_max <= NTB) {
    if (A.nl_max <= NLC_BUCKETS[0] && fits(NLC_BUCKETS[0]))
      return launch_block_nl<T, OP, MAT, NLC_BUCKETS[0]>(c, A);
    if (A.nl_max <= NLC_BUCKETS[1] && fits(NLC_BUCKETS[1]))
      return launch_block_nl<T, OP, MAT, NLC_BUCKETS[1]>(c, A);
    if (A.nl_max <= NLC_BUCKETS[2] && fits(NLC_BUCKETS[2]))
      return launch_block_nl<T, OP, MAT, NLC_BUCKETS[2]>(c, A);
    if (A.nl_max <= NLC_BUCKETS[3] && fits(NLC_BUCKETS[3]))
      return launch_block_nl<T, OP, MAT, NLC_BUCKETS[3]>(c, A);
  }
  launch_block_nl<T, OP, MAT, 0>(c, A);
}

template <typename T>
int launch(Ctx *c, int op, const T *xr, const T *u, const T *v, T *out, double *red,
           hipError_t *err) {
  const Mesh &M = c->m;
  // surface loads (follower pressure, springs): their nodal contributions are
  // computed first and added when each node is finalized
  void *fs = nullptr;
  if (c->surf.nsn > 0 && op != OP_ENERGY) {
    fs = surf_apply(c, op, sizeof(T) == 8 ? NLE_FP64 : NLE_FP32, u, v, nullptr, err);
    if (*err != hipSuccess) return 0;
  }
  ElemArgs<T> A;
  A.xr = xr;
  A.lcp = M.lcp;
  A.csr_end = M.csr_end;
  A.nodes = M.nodes;
  A.mpos = M.mpos;
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
  A.flag = c->inst_inv ? c->inst_inv : c->dflag;
  A.skip = c->elem_skip;
  A.nomask = (op == OP_JV && c->jv_nomask) ? 1 : 0;
  A.ep_w = static_cast<const T *>(c->ep.w);
  A.ep_coef = c->ep.coef;
  A.ep_red = op == OP_JV ? c->ep.red : nullptr;
  A.mp = c->mat;
  A.fib = static_cast<const T *>(sizeof(T) == 8 ? static_cast<const void *>(c->fib64)
                                                : static_cast<const void *>(c->fib32));
  A.sheet = static_cast<const T *>(sizeof(T) == 8 ? static_cast<const void *>(c->sh64)
                                                  : static_cast<const void *>(c->sh32));
  A.fs = op == OP_ENERGY ? nullptr : static_cast<T *>(fs);
  A.lcoef = nullptr;
  A.lc64 = nullptr;
  A.lc32 = nullptr;
  if (op == OP_JV)
    A.lcoef = static_cast<const T *>(sizeof(T) == 8 ? static_cast<const void *>(c->lc64)
                                                    : static_cast<const void *>(c->lc32));
  if (op == OP_DIAG && c->lc64) {
    A.lc64 = c->lc64;
    A.lc32 = c->lc32;
  }
  A.blk_inst = M.blk_inst;
  A.blk_list = c->blk_list;
  A.n_list = c->n_blist;
  A.icm = (c->inr.on && (op == OP_RES || op == OP_JV || op == OP_DIAG))
              ? static_cast<const T *>(sizeof(T) == 8 ? static_cast<const void *>(c->inr.cm64)
                                                      : static_cast<const void *>(c->inr.cm32))
              : nullptr;
  A.iut = c->inr.ut;
  A.inst_s = c->inst_s;
  A.inst_mat = c->inst_mat;
  A.inst_done = c->inst_done;
  A.vz = op == OP_JV ? static_cast<const T *>(c->cg.z) : nullptr;
  A.cg_red = c->cg.red;
  A.cg_np = c->cg.np;
  A.cg_scal = c->cg.scal;
  A.cg_flag = c->cg.flag;
  const int kind = c->mat.kind;
#define NLE_LAUNCH_BLOCK(OPV)                                             \
  if (kind == NLE_MAT_M2)                                                 \
    launch_block<T, OPV, NLE_MAT_M2>(c, A);                               \
  else if (kind == NLE_MAT_M4)                                            \
    launch_block<T, OPV, NLE_MAT_M4>(c, A);                               \
  else if (kind == NLE_MAT_M6)                                            \
    launch_block<T, OPV, NLE_MAT_M6>(c, A);                               \
  else                                                                    \
    launch_block<T, OPV, NLE_MAT_M1>(c, A);
  switch (op) {
    case OP_RES:
      NLE_LAUNCH_BLOCK(OP_RES);
      break;
    case OP_JV:
      NLE_LAUNCH_BLOCK(OP_JV);
      break;
    case OP_DIAG:
      NLE_LAUNCH_BLOCK(OP_DIAG);
      break;
    case OP_ODIAG:
      if constexpr (sizeof(T) == 8) {
        NLE_LAUNCH_BLOCK(OP_ODIAG);
      } else {
        *err = hipErrorInvalidValue;
        return 0;
      }
      break;
    default:
      NLE_LAUNCH_BLOCK(OP_ENERGY);
      break;
  }
#undef NLE_LAUNCH_BLOCK
  *err = hipGetLastError();
  if (*err != hipSuccess) return 0;
  if (op == OP_ENERGY) return M.nblk;
  int nred = (op == OP_RES || (op == OP_JV && c->ep.red)) ? M.nblk : 0;
  const int g2 = c->mwg_list ? c->n_mlist : int((M.n_shared + NT - 1) / NT);
  if (M.n_shared > 0 && g2 > 0) {
    MergeArgs<T> B;
    B.fx_node = M.fx_node;
    B.fx_ptr = M.fx_ptr;
    B.n_sh = M.n_shared;
    B.partial = static_cast<const T *>(c->partial);
    B.v = v;
    B.out = out;
    B.fext = c->fext;
    B.s = c->load_scale;
    B.red = red ? red + M.nblk : nullptr;
    B.mwg_inst = M.mwg_inst;
    B.mwg_list = c->mwg_list;
    B.inst_s = c->inst_s;
    B.inst_done = c->inst_done;
    B.skip = c->elem_skip;
    B.nomask = A.nomask;
    B.ep_w = static_cast<const T *>(c->ep.w);
    B.ep_coef = c->ep.coef;
    B.ep_red = (op == OP_JV && c->ep.red) ? c->ep.red + M.nblk : nullptr;
    B.fs = A.fs;
    B.vz = A.vz;
    B.cg_scal = c->cg.scal;
    B.u = u;
    B.icm = A.icm;
    B.iut = A.iut;
    switch (op) {
      case OP_RES:
        hipLaunchKernelGGL((k_elem_merge<T, OP_RES>), dim3(g2), dim3(NT), 0, c->stream, B);
        nred += g2;
        break;
      case OP_JV:
        hipLaunchKernelGGL((k_elem_merge<T, OP_JV>), dim3(g2), dim3(NT), 0, c->stream, B);
        if (c->ep.red) nred += g2;
        break;
      case OP_ODIAG:
        if constexpr (sizeof(T) == 8)
          hipLaunchKernelGGL((k_elem_merge<T, OP_ODIAG>), dim3(g2), dim3(NT), 0, c->stream, B);
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
  if (c->mixed) return mixed_red_capacity(c);
  const Mesh &M = c->m;
  const int grid = c->xcd_remap ? 8 * ((M.nblk + 7) / 8) : M.nblk;
  return grid + int((M.n_shared + NT - 1) / NT) + 8;
}

int elem_apply(Ctx *c, int op, int prec, const void *u, const void *v, void *out, double *red,
               hipError_t *err) {
  if (c->mixed) return mixed_apply(c, op, prec, u, v, out, red, err);
  const Mesh &M = c->m;
  if (prec == NLE_FP32)
    return launch<float>(c, op, M.xr32, static_cast<const float *>(u),
                         static_cast<const float *>(v), static_cast<float *>(out), red, err);
  return launch<double>(c, op, M.xr64, static_cast<const double *>(u),
                        static_cast<const double *>(v), static_cast<double *>(out), red, err);
}

}  // namespace nle
