// Streaming vector kernels for the Krylov and L-BFGS loops.
//
// Reductions are deterministic: each workgroup of a fixed-size grid (a
// function of the vector length only) sums its grid-stride share in a fixed
// order and writes one partial; the consumer (a later kernel) sums the
// partials in index order.  When several workgroups of the consumer need the
// same scalar, each of them repeats that identical sum, so every workgroup
// sees the same bits without another launch.
#include <hip/hip_runtime.h>

#include "nle_internal.hpp"

namespace nle {

namespace {

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Fixed-order workgroup sum, result broadcast to all threads.
template <typename T>
__device__ __forceinline__ T block_sum_all(T v, T *sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  T r = sh[0];
  for (int k = 1; k < NT / 64; ++k) r += sh[k];
  return r;
}

// Sum of red[0..np) in a fixed order, identical in every workgroup.
__device__ __forceinline__ double sum_partials(const double *red, int np, double *sh) {
  double v = 0.0;
  for (int k = threadIdx.x; k < np; k += NT) v += red[k];
  return block_sum_all(v, sh);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_fill(T *x, T val, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < n; i += int64_t(gridDim.x) * NT)
    x[i] = val;
}

template <typename S, typename D>
__global__ __launch_bounds__(NT) void k_cast_scale(const S *x, D *y, double s, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < n; i += int64_t(gridDim.x) * NT)
    y[i] = D(s * double(x[i]));
}

template <typename S, typename D>
__global__ __launch_bounds__(NT) void k_axpy(const S *x, D *y, double a, const double *ad,
                                             int64_t n) {
  const double alpha = ad ? a * ad[0] : a;
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < n; i += int64_t(gridDim.x) * NT)
    y[i] = D(double(y[i]) + alpha * double(x[i]));
}

// Newmark's average-acceleration family: predictor u~ = u + dt v + dt^2 (1/2 - beta) a
// and corrector a' = (u' - u~) / (beta dt^2), v' = v + dt ((1 - gamma) a + gamma a').
__global__ __launch_bounds__(NT) void k_newmark_predict(const double *u, const double *v,
                                                        const double *a, double *ut, double *vt,
                                                        double dt, double beta, double gamma,
                                                        int64_t n) {
  const double h2 = dt * dt * (0.5 - beta), h1 = dt * (1.0 - gamma);
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < n; i += int64_t(gridDim.x) * NT) {
    ut[i] = u[i] + dt * v[i] + h2 * a[i];
    if (vt) vt[i] = v[i] + h1 * a[i];
  }
}

__global__ __launch_bounds__(NT) void k_newmark_correct(const double *u, const double *ut,
                                                        double *v, double *a, double dt,
                                                        double beta, double gamma, int64_t n) {
  const double c = 1.0 / (beta * dt * dt);
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < n; i += int64_t(gridDim.x) * NT) {
    const double an = c * (u[i] - ut[i]);
    v[i] = v[i] + dt * ((1.0 - gamma) * a[i] + gamma * an);
    a[i] = an;
  }
}

// partials of sum_i w_i (x_i - y_i)^2
__global__ __launch_bounds__(NT) void k_wdiff2(const double *w, const double *x, const double *y,
                                               int64_t n, double *red) {
  __shared__ double sh[NT / 64];
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < n; i += int64_t(gridDim.x) * NT) {
    const double d = x[i] - y[i];
    acc += w[i] * d * d;
  }
  acc = block_sum_all(acc, sh);
  if (threadIdx.x == 0) red[blockIdx.x] = acc;
}

__global__ __launch_bounds__(NT) void k_recip(const double *d, double *di, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < n; i += int64_t(gridDim.x) * NT)
    di[i] = 1.0 / d[i];
}

__global__ __launch_bounds__(NT) void k_lift(double *u, const int64_t *dofs, const double *vals,
                                             int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < n; i += int64_t(gridDim.x) * NT)
    u[dofs[i]] = vals[i];
}

// w[d] = g_d - u[d] on the Dirichlet dofs (w is zero elsewhere)
__global__ __launch_bounds__(NT) void k_dir_delta(const double *u, const int64_t *dofs,
                                                  const double *vals, double *w, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < n; i += int64_t(gridDim.x) * NT)
    w[dofs[i]] = vals[i] - u[dofs[i]];
}

template <typename T>
__global__ __launch_bounds__(NT) void k_dot(const T *a, const T *b, int64_t n, double *red) {
  __shared__ T sh[NT / 64];
  T acc = T(0);
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < n; i += int64_t(gridDim.x) * NT)
    acc += a[i] * b[i];
  acc = block_sum_all(acc, sh);
  if (threadIdx.x == 0) red[blockIdx.x] = double(acc);
}

// out[c] = sum_k red[c * stride + k], k < np, one workgroup per c.
__global__ __launch_bounds__(NT) void k_reduce(const double *red, int np, int stride, double *out) {
  __shared__ double sh[NT / 64];
  const double s = sum_partials(red + int64_t(blockIdx.x) * stride, np, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// ------------------------------------------------------------------ CG
// Device scalars (scal[]) and flags (flag[]) shared by the CG and MINRES
// loops.  Every iteration is a fixed sequence of launches with no per-
// iteration host argument, so a chunk of iterations can be replayed as one
// graph.  A scalar written by one workgroup is only read by later kernels.
//   flag[0]: 0 running, 1 converged, 2 breakdown, 3 NaN, 5 iteration limit
//   flag[1]: completed iterations
enum {
  S_RZ = cgslot::RZ, S_RZOLD = cgslot::RZOLD, S_TOL2 = cgslot::TOL2, S_RR = cgslot::RR,
  S_B2 = cgslot::B2, S_MAXIT = cgslot::MAXIT, S_BETA = cgslot::BETA,
  // MINRES
  M_BETA = 8, M_OLDB = 9, M_ALFA = 10, M_CS = 11, M_SN = 12, M_DBAR = 13, M_EPS = 14,
  M_OLDEPS = 15, M_DELTA = 16, M_PHI = 17, M_PHIBAR = 18, M_DENOM = 19, M_COEF = 20,
  M_INVBETA = 21
};

// Preconditioner on one unit of BS consecutive entries (unit u of nu):
//   BS = 1: point Jacobi, z = d r (d the inverse diagonal; identity if null);
//   BS = 3: nodal block Jacobi, z = B r with B the symmetric inverse of the
//           node's diagonal 3x3 tangent block, d = [6][nu] component-major
//           (xx, yy, zz, xy, yz, xz).
template <int BS, typename T>
__device__ __forceinline__ void pc_unit(const T *d, int64_t u, int64_t nu, const T *r, T *z) {
  if constexpr (BS == 1) {
    z[0] = d ? d[u] * r[0] : r[0];
  } else {
    const T bxx = d[u], byy = d[nu + u], bzz = d[2 * nu + u];
    const T bxy = d[3 * nu + u], byz = d[4 * nu + u], bxz = d[5 * nu + u];
    z[0] = bxx * r[0] + bxy * r[1] + bxz * r[2];
    z[1] = bxy * r[0] + byy * r[1] + byz * r[2];
    z[2] = bxz * r[0] + byz * r[1] + bzz * r[2];
  }
}

#define UNIT_LOOP(u, nu)                                                            \
  for (int64_t u = int64_t(blockIdx.x) * NT + threadIdx.x; u < (nu); u += int64_t(gridDim.x) * NT)

template <typename T, int BS>
__global__ __launch_bounds__(NT) void k_pc_apply(const T *d, const T *x, T *y, int64_t n) {
  const int64_t nu = n / BS;
  UNIT_LOOP(u, nu) {
    T r[BS], z[BS];
#pragma unroll
    for (int c = 0; c < BS; ++c) r[c] = x[BS * u + c];
    pc_unit<BS>(d, u, nu, r, z);
#pragma unroll
    for (int c = 0; c < BS; ++c) y[BS * u + c] = z[c];
  }
}

// Symmetric 3x3 block inverses from the diagonal (d: xx yy zz per node,
// interleaved) and off-diagonal entries (o: xy yz zx per node), by cofactors
// in FP64; written as [6][nn] in FP64 and FP32.  A block that is not positive
// definite (a leading principal minor <= 0, as happens at nodes of a loaded
// tangent that has turned indefinite) gives that node the point-Jacobi
// entries instead, so the preconditioner stays symmetric positive definite
// wherever point Jacobi is.
__global__ __launch_bounds__(NT) void k_block_inv(const double *d, const double *o, double *b64,
                                                  float *b32, int64_t nn) {
  UNIT_LOOP(k, nn) {
    const double a00 = d[3 * k], a11 = d[3 * k + 1], a22 = d[3 * k + 2];
    const double a01 = o[3 * k], a12 = o[3 * k + 1], a02 = o[3 * k + 2];
    const double c00 = a11 * a22 - a12 * a12, c11 = a00 * a22 - a02 * a02;
    const double c22 = a00 * a11 - a01 * a01;
    const double c01 = a02 * a12 - a01 * a22, c12 = a01 * a02 - a00 * a12;
    const double c02 = a01 * a12 - a02 * a11;
    const double det = a00 * c00 + a01 * c01 + a02 * c02;
    double v[6];
    if (a00 > 0.0 && c22 > 0.0 && det > 0.0) {
      const double id = 1.0 / det;
      v[0] = c00 * id, v[1] = c11 * id, v[2] = c22 * id;
      v[3] = c01 * id, v[4] = c12 * id, v[5] = c02 * id;
    } else {
      v[0] = 1.0 / a00, v[1] = 1.0 / a11, v[2] = 1.0 / a22;
      v[3] = v[4] = v[5] = 0.0;
    }
#pragma unroll
    for (int t = 0; t < 6; ++t) {
      b64[t * nn + k] = v[t];
      b32[t * nn + k] = float(v[t]);
    }
  }
}

// Preconditioned CG (Hestenes-Stiefel).  One iteration: the Jacobian action
// Ap = J p (its epilogue gives the partials of p.Ap), cg_update, cg_direction.
// (The single-reduction arrangement, which carries s = A p by recurrence and
// saves one launch, was measured: in FP32 its recurrence drifts and the
// inexact Newton solves needed ~50% more iterations, so it is not used.)
template <typename T, int BS>
__global__ __launch_bounds__(NT) void k_cg_start(const T *b, T *x, T *r, T *z, T *p, const T *dinv,
                                                 int64_t n, double *red) {
  __shared__ T sh[NT / 64];
  T arz = T(0), arr = T(0);
  const int64_t nu = n / BS;
  UNIT_LOOP(k, nu) {
    T bi[BS], zi[BS];
#pragma unroll
    for (int c = 0; c < BS; ++c) {
      const int64_t i = BS * k + c;
      bi[c] = b[i];
      x[i] = T(0);
      r[i] = bi[c];
    }
    pc_unit<BS>(dinv, k, nu, bi, zi);
#pragma unroll
    for (int c = 0; c < BS; ++c) {
      z[BS * k + c] = zi[c];
      p[BS * k + c] = zi[c];
      arz += bi[c] * zi[c];
      arr += bi[c] * bi[c];
    }
  }
  arz = block_sum_all(arz, sh);
  arr = block_sum_all(arr, sh);
  if (threadIdx.x == 0) {
    red[blockIdx.x] = double(arz);
    red[VGRID_MAX + blockIdx.x] = double(arr);
  }
}

__global__ __launch_bounds__(NT) void k_cg_start2(const double *red, int np, double *scal,
                                                  int32_t *flag, double rtol, double atol,
                                                  int max_it) {
  __shared__ double sh[NT / 64];
  const double rz = sum_partials(red, np, sh);
  const double rr = sum_partials(red + VGRID_MAX, np, sh);
  if (threadIdx.x == 0) {
    const double tol2 = fmax(rtol * rtol * rr, atol * atol);
    scal[S_RZ] = rz;
    scal[S_RZOLD] = 0.0;  // the first direction is z itself (beta = 0)
    scal[S_BETA] = 0.0;
    scal[S_TOL2] = tol2;
    scal[S_RR] = rr;
    scal[S_B2] = rr;
    scal[S_MAXIT] = double(max_it);
    flag[1] = 0;
    flag[0] = (rr <= tol2) ? 1 : ((rr == rr) ? 0 : 3);
  }
}

// alpha = rz / p.Ap;  x += alpha p;  r -= alpha Ap;  z = M^-1 r; partials of
// r.z and r.r.  p.Ap partials come from the Jacobian-action epilogue.
// FUSED: the direction of this iteration is formed here as p = z + beta p
// (beta = scal[S_BETA], written by the Jacobian action that used the same
// direction) and the iteration count advances here (no direction kernel).
template <typename T, int BS, bool FUSED>
__global__ __launch_bounds__(NT) void k_cg_update(T *x, T *r, T *z, T *p, const T *Ap,
                                                  const T *dinv, int64_t n, const double *red_a,
                                                  int np_a, double *red_b, double *scal,
                                                  int32_t *flag, T *cd, T cth) {
  __shared__ double shd[NT / 64];
  __shared__ T sh[NT / 64];
  if (flag[0] != 0) return;
  const double pAp = sum_partials(red_a, np_a, shd);
  if (!(pAp > 0.0)) {  // not positive definite (or NaN): stop, keep x
    if (blockIdx.x == 0 && threadIdx.x == 0) flag[0] = (pAp == pAp) ? 2 : 3;
    return;
  }
  const double rz = scal[S_RZ];
  const double alpha = rz / pAp;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    scal[S_RZOLD] = rz;
    if (FUSED) flag[1] = flag[1] + 1;
  }
  const T a = T(alpha);
  const T bt = FUSED ? T(scal[S_BETA]) : T(0);
  T arz = T(0), arr = T(0);
  const int64_t nu = n / BS;
  UNIT_LOOP(k, nu) {
    T ri[BS], zi[BS];
#pragma unroll
    for (int c = 0; c < BS; ++c) {
      const int64_t i = BS * k + c;
      ri[c] = r[i] - a * Ap[i];
      if (FUSED) {
        const T pn = z[i] + bt * p[i];
        p[i] = pn;
        x[i] += a * pn;
      } else {
        x[i] += a * p[i];
      }
      r[i] = ri[c];
    }
    pc_unit<BS>(dinv, k, nu, ri, zi);
    if (cd) {  // the multigrid cycle's first Chebyshev step
#pragma unroll
      for (int c = 0; c < BS; ++c) {
        zi[c] = cth * zi[c];
        cd[BS * k + c] = zi[c];
      }
    }
#pragma unroll
    for (int c = 0; c < BS; ++c) {
      z[BS * k + c] = zi[c];
      arz += ri[c] * zi[c];
      arr += ri[c] * ri[c];
    }
  }
  arz = block_sum_all(arz, sh);
  arr = block_sum_all(arr, sh);
  if (threadIdx.x == 0) {
    red_b[blockIdx.x] = double(arz);
    red_b[VGRID_MAX + blockIdx.x] = double(arr);
  }
}

// beta = rz_new / rz_old;  p = z + beta p;  convergence test on r.r.
template <typename T>
__global__ __launch_bounds__(NT) void k_cg_direction(T *p, const T *z, int64_t n,
                                                     const double *red_b, int np, double *scal,
                                                     int32_t *flag) {
  __shared__ double sh[NT / 64];
  if (flag[0] != 0) return;
  const double rz = sum_partials(red_b, np, sh);
  const double rr = sum_partials(red_b + VGRID_MAX, np, sh);
  const double beta = rz / scal[S_RZOLD];
  const T bt = T(beta);
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < n; i += int64_t(gridDim.x) * NT)
    p[i] = z[i] + bt * p[i];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    scal[S_RZ] = rz;
    scal[S_RR] = rr;
    const int its = flag[1] + 1;
    flag[1] = its;
    if (!(rr == rr))
      flag[0] = 3;
    else if (rr <= scal[S_TOL2])
      flag[0] = 1;
    else if (double(its) >= scal[S_MAXIT])
      flag[0] = 5;
  }
}

// ------------------------------------------------------------------ MINRES
// Preconditioned MINRES (Paige & Saunders 1975; the Lanczos / Givens form).
// Besides the solution it carries z = A w and the true residual r = b - A x,
// so the stopping test is on ||b - A x||_2 like the other Krylov methods.
template <typename T, int BS>
__global__ __launch_bounds__(NT) void k_mr_start(const T *b, T *x, T *r1, T *r2, T *y, T *r,
                                                 T *wa, T *wb, T *za, T *zb, const T *dinv,
                                                 int64_t n, double *red) {
  __shared__ T sh[NT / 64];
  T aby = T(0), abb = T(0);
  const int64_t nu = n / BS;
  UNIT_LOOP(k, nu) {
    T bi[BS], yi[BS];
#pragma unroll
    for (int c = 0; c < BS; ++c) {
      const int64_t i = BS * k + c;
      bi[c] = b[i];
      x[i] = T(0);
      r1[i] = bi[c];
      r2[i] = bi[c];
      r[i] = bi[c];
      wa[i] = T(0);
      wb[i] = T(0);
      za[i] = T(0);
      zb[i] = T(0);
    }
    pc_unit<BS>(dinv, k, nu, bi, yi);
#pragma unroll
    for (int c = 0; c < BS; ++c) {
      y[BS * k + c] = yi[c];
      aby += bi[c] * yi[c];
      abb += bi[c] * bi[c];
    }
  }
  aby = block_sum_all(aby, sh);
  abb = block_sum_all(abb, sh);
  if (threadIdx.x == 0) {
    red[blockIdx.x] = double(aby);
    red[VGRID_MAX + blockIdx.x] = double(abb);
  }
}

__global__ __launch_bounds__(NT) void k_mr_start2(const double *red, int np, double *scal,
                                                  int32_t *flag, double rtol, double atol,
                                                  int max_it) {
  __shared__ double sh[NT / 64];
  const double by = sum_partials(red, np, sh);
  const double bb = sum_partials(red + VGRID_MAX, np, sh);
  if (threadIdx.x == 0) {
    const double tol2 = fmax(rtol * rtol * bb, atol * atol);
    const double beta1 = sqrt(fmax(by, 0.0));
    scal[S_TOL2] = tol2;
    scal[S_RR] = bb;
    scal[S_B2] = bb;
    scal[S_MAXIT] = double(max_it);
    scal[M_BETA] = beta1;
    scal[M_OLDB] = 0.0;
    scal[M_CS] = -1.0;
    scal[M_SN] = 0.0;
    scal[M_DBAR] = 0.0;
    scal[M_EPS] = 0.0;
    scal[M_PHIBAR] = beta1;
    scal[M_COEF] = 0.0;
    scal[M_INVBETA] = beta1 > 0.0 ? 1.0 / beta1 : 0.0;
    flag[1] = 0;
    if (!(bb == bb) || !(by == by))
      flag[0] = 3;
    else if (bb <= tol2)
      flag[0] = 1;
    else if (!(by > 0.0))
      flag[0] = 2;  // preconditioner not positive definite
    else
      flag[0] = 0;
  }
}

// v = y / beta (first iteration only; later iterations form v in k_mr_e)
template <typename T>
__global__ __launch_bounds__(NT) void k_mr_v(const T *y, T *v, int64_t n, const double *scal,
                                             const int32_t *flag) {
  if (flag[0] != 0) return;
  const T s = T(scal[M_INVBETA]);
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < n; i += int64_t(gridDim.x) * NT)
    v[i] = y[i] * s;
}

// After the Jacobian action (with epilogue) y = A v - coef r1 and partials of
// alfa = v.y:  av = A v;  t = y - (alfa / beta) r2;  r1 = r2;  r2 = t;
// y = M^-1 t;  partials of t.y.
template <typename T, int BS>
__global__ __launch_bounds__(NT) void k_mr_c(T *y, T *r1, T *r2, T *av, const T *dinv, int64_t n,
                                             const double *red_a, int np_a, double *red_b,
                                             double *scal, const int32_t *flag) {
  __shared__ double shd[NT / 64];
  __shared__ T sh[NT / 64];
  if (flag[0] != 0) return;
  const double alfa = sum_partials(red_a, np_a, shd);
  if (blockIdx.x == 0 && threadIdx.x == 0) scal[M_ALFA] = alfa;
  const T c = T(scal[M_COEF]);
  const T ab = T(alfa * scal[M_INVBETA]);
  T acc = T(0);
  const int64_t nu = n / BS;
  UNIT_LOOP(k, nu) {
    T t[BS], yn[BS];
#pragma unroll
    for (int q = 0; q < BS; ++q) {
      const int64_t i = BS * k + q;
      const T yi = y[i];
      const T r1i = r1[i], r2i = r2[i];
      av[i] = yi + c * r1i;
      t[q] = yi - ab * r2i;
      r1[i] = r2i;
      r2[i] = t[q];
    }
    pc_unit<BS>(dinv, k, nu, t, yn);
#pragma unroll
    for (int q = 0; q < BS; ++q) {
      y[BS * k + q] = yn[q];
      acc += t[q] * yn[q];
    }
  }
  acc = block_sum_all(acc, sh);
  if (threadIdx.x == 0) red_b[blockIdx.x] = double(acc);
}

// Scalar recurrence (one workgroup): new beta, Givens rotation, step phi;
// also the convergence test on the previous iteration's ||r||^2.
__global__ __launch_bounds__(NT) void k_mr_d(const double *red_b, int np, const double *red_r,
                                             int np_r, double *scal, int32_t *flag) {
  __shared__ double sh[NT / 64];
  if (flag[0] != 0) return;
  const double bb = sum_partials(red_b, np, sh);
  const double rr = flag[1] > 0 ? sum_partials(red_r, np_r, sh) : scal[S_RR];
  if (threadIdx.x != 0) return;
  scal[S_RR] = rr;
  if (!(rr == rr) || !(bb == bb)) {
    flag[0] = 3;
    return;
  }
  if (flag[1] > 0 && rr <= scal[S_TOL2]) {
    flag[0] = 1;
    return;
  }
  if (double(flag[1]) >= scal[S_MAXIT]) {
    flag[0] = 5;
    return;
  }
  const double alfa = scal[M_ALFA];
  const double beta_old = scal[M_BETA];
  const double beta = sqrt(fmax(bb, 0.0));
  const double cs = scal[M_CS], sn = scal[M_SN], dbar = scal[M_DBAR];
  const double oldeps = scal[M_EPS];
  const double delta = cs * dbar + sn * alfa;
  const double gbar = sn * dbar - cs * alfa;
  const double epsln = sn * beta;
  const double dbar_n = -cs * beta;
  double gamma = sqrt(gbar * gbar + beta * beta);
  gamma = fmax(gamma, 1e-300);
  const double cs_n = gbar / gamma, sn_n = beta / gamma;
  const double phibar = scal[M_PHIBAR];
  scal[M_OLDB] = beta_old;
  scal[M_BETA] = beta;
  scal[M_OLDEPS] = oldeps;
  scal[M_DELTA] = delta;
  scal[M_EPS] = epsln;
  scal[M_DBAR] = dbar_n;
  scal[M_CS] = cs_n;
  scal[M_SN] = sn_n;
  scal[M_PHI] = cs_n * phibar;
  scal[M_PHIBAR] = sn_n * phibar;
  scal[M_DENOM] = 1.0 / gamma;
  scal[M_COEF] = beta_old > 0.0 ? beta / beta_old : 0.0;
  scal[M_INVBETA] = beta > 0.0 ? 1.0 / beta : 0.0;
  flag[1] = flag[1] + 1;
}

// w = (v - oldeps w_{k-2} - delta w_{k-1}) / gamma;  x += phi w;
// z = (A v - oldeps z_{k-2} - delta z_{k-1}) / gamma;  r -= phi z;  partials
// of r.r;  next v = y / beta.
template <typename T>
__global__ __launch_bounds__(NT) void k_mr_e(T *x, T *v, const T *y, const T *av, T *wa, T *wb,
                                             T *za, T *zb, T *r, int64_t n, double *red_r,
                                             const double *scal, const int32_t *flag) {
  __shared__ T sh[NT / 64];
  if (flag[0] != 0) return;
  const T oe = T(scal[M_OLDEPS]), de = T(scal[M_DELTA]), dn = T(scal[M_DENOM]);
  const T ph = T(scal[M_PHI]), ib = T(scal[M_INVBETA]);
  T acc = T(0);
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < n; i += int64_t(gridDim.x) * NT) {
    const T w1 = wa[i], w2 = wb[i];  // w_{k-1}, w_{k-2}
    const T w = (v[i] - oe * w2 - de * w1) * dn;
    wb[i] = w1;
    wa[i] = w;
    x[i] += ph * w;
    const T z1 = za[i], z2 = zb[i];
    const T zz = (av[i] - oe * z2 - de * z1) * dn;
    zb[i] = z1;
    za[i] = zz;
    const T ri = r[i] - ph * zz;
    r[i] = ri;
    acc += ri * ri;
    v[i] = y[i] * ib;
  }
  acc = block_sum_all(acc, sh);
  if (threadIdx.x == 0) red_r[blockIdx.x] = double(acc);
}

// ------------------------------------------------------------------ GMRES
// Device data (m = cycle length): Hessenberg column j (rows 0..j+1) at
// Hp[j]; rot = cs[m], sn[m], g[m+1], y[m]; basis vector i at Vp[i]; partial
// row i at Rp[i].  scal: [0] beta (norm of r0), [1] tolerance, [2] 1 / h(j+1,
// j), [3] current residual estimate; flag: [0] done (1 converged, 3
// breakdown, 4 cycle full), [1] columns in the current cycle.
__device__ __forceinline__ double *gm_cs(double *rot, int) { return rot; }
__device__ __forceinline__ double *gm_sn(double *rot, int m) { return rot + m; }
__device__ __forceinline__ double *gm_g(double *rot, int m) { return rot + 2 * m; }
__device__ __forceinline__ double *gm_y(double *rot, int m) { return rot + 3 * m + 1; }

// table entries of one pool segment
__global__ __launch_bounds__(NT) void k_gm_tables(void **Vp, double **Hp, double **Rp, int v0,
                                                  int nv, int limit, char *vbase, size_t vb,
                                                  double *hbase, double *rbase) {
  const int t = blockIdx.x * NT + threadIdx.x;
  if (t >= nv || v0 + t >= limit) return;
  Vp[v0 + t] = vbase + size_t(t) * vb;
  // column v0 + l holds v0 + l + 2 rows
  Hp[v0 + t] = hbase + (int64_t(t) * (v0 + 2) + int64_t(t) * (t - 1) / 2);
  Rp[v0 + t] = rbase + int64_t(t) * VGRID_MAX;
}

// partials of V_i . w for i = blockIdx.y
template <typename T>
__global__ __launch_bounds__(NT) void k_gm_dots(T *const *Vp, const T *w, int64_t n,
                                                double *const *Rp, const int32_t *flag) {
  __shared__ T sh[NT / 64];
  if (flag[0] != 0) return;
  const T *vi = Vp[blockIdx.y];
  T acc = T(0);
  for (int64_t k = int64_t(blockIdx.x) * NT + threadIdx.x; k < n; k += int64_t(gridDim.x) * NT)
    acc += vi[k] * w[k];
  acc = block_sum_all(acc, sh);
  if (threadIdx.x == 0) Rp[blockIdx.y][blockIdx.x] = double(acc);
}

// hc[i] (+)= sum of partials of dot i (row Rp[i]), one workgroup per i
__global__ __launch_bounds__(NT) void k_gm_reduce(double *const *Rp, int np, double *hc, int add,
                                                  const int32_t *flag) {
  __shared__ double sh[NT / 64];
  if (flag[0] != 0) return;
  const double s = sum_partials(Rp[blockIdx.x], np, sh);
  if (threadIdx.x == 0) hc[blockIdx.x] = add ? hc[blockIdx.x] + s : s;
}

// w -= sum_{i<j1} h_i V_i, with h the second argument (pass-specific copy);
// if want_sq, partials of w.w
template <typename T>
__global__ __launch_bounds__(NT) void k_gm_sub(T *const *Vp, T *w, int64_t n, const double *h,
                                               int j1, double *red_sq, const int32_t *flag) {
  __shared__ T sh[NT / 64];
  __shared__ double hs[256];
  if (flag[0] != 0) return;
  for (int i = threadIdx.x; i < j1 && i < 256; i += NT) hs[i] = h[i];
  __syncthreads();
  T acc = T(0);
  for (int64_t k = int64_t(blockIdx.x) * NT + threadIdx.x; k < n; k += int64_t(gridDim.x) * NT) {
    double wk = double(w[k]);
    for (int i = 0; i < j1; ++i) wk -= (i < 256 ? hs[i] : h[i]) * double(Vp[i][k]);
    const T t = T(wk);
    w[k] = t;
    acc += t * t;
  }
  if (red_sq) {
    acc = block_sum_all(acc, sh);
    if (threadIdx.x == 0) red_sq[blockIdx.x] = double(acc);
  }
}

// Finish column j: h(j+1,j) = ||w||, Givens rotations, residual test.
__global__ void k_gm_col(double *const *Hp, double *rot, int m, int j, const double *red_sq,
                         int np, const double *hc1, const double *hc2, double *scal,
                         int32_t *flag, int max_cols) {
  __shared__ double sh[NT / 64];
  if (flag[0] != 0) return;
  const double ww = sum_partials(red_sq, np, sh);
  if (threadIdx.x != 0) return;
  double *col = Hp[j];
  for (int i = 0; i <= j; ++i) col[i] = hc1[i] + (hc2 ? hc2[i] : 0.0);
  const double hn = sqrt(ww);
  col[j + 1] = hn;
  double *cs = gm_cs(rot, m), *sn = gm_sn(rot, m), *g = gm_g(rot, m);
  for (int i = 0; i < j; ++i) {
    const double t = cs[i] * col[i] + sn[i] * col[i + 1];
    col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
    col[i] = t;
  }
  const double den = hypot(col[j], col[j + 1]);
  double c = 1.0, s = 0.0;
  if (den > 0.0) {
    c = col[j] / den;
    s = col[j + 1] / den;
  }
  cs[j] = c;
  sn[j] = s;
  col[j] = c * col[j] + s * col[j + 1];
  col[j + 1] = 0.0;
  g[j + 1] = -s * g[j];
  g[j] = c * g[j];
  const double res = fabs(g[j + 1]);
  scal[3] = res;
  scal[2] = hn > 0.0 ? 1.0 / hn : 0.0;
  flag[1] = j + 1;
  if (!(res == res))
    flag[0] = 3;
  else if (res <= scal[1] || hn == 0.0)
    flag[0] = 1;
  else if (j + 1 >= max_cols)
    flag[0] = 4;  // cycle full (host restarts or stops)
}

// V_{j+1} = w * scal[2]
template <typename T>
__global__ __launch_bounds__(NT) void k_gm_next(const T *w, T *vn, int64_t n, const double *scal,
                                                const int32_t *flag) {
  if (flag[0] != 0) return;
  const T s = T(scal[2]);
  for (int64_t k = int64_t(blockIdx.x) * NT + threadIdx.x; k < n; k += int64_t(gridDim.x) * NT)
    vn[k] = w[k] * s;
}

// Back substitution R(0:k,0:k) y = g(0:k), k = flag[1] (R: the rotated
// Hessenberg columns).
__global__ void k_gm_solve(double *const *Hp, double *rot, int m, const int32_t *flag) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int k = flag[1];
  double *g = gm_g(rot, m), *y = gm_y(rot, m);
  for (int i = k - 1; i >= 0; --i) {
    double s = g[i];
    for (int l = i + 1; l < k; ++l) s -= Hp[l][i] * y[l];
    const double d = Hp[i][i];
    y[i] = d != 0.0 ? s / d : 0.0;
  }
}

// x += M^-1 (sum_i y_i V_i)
template <typename T, int BS>
__global__ __launch_bounds__(NT) void k_gm_update(T *const *Vp, T *x, const T *dinv, int64_t n,
                                                  const double *rot, int m, const int32_t *flag) {
  __shared__ double ys[256];
  const int k = flag[1];
  const double *y = rot + 3 * m + 1;
  for (int i = threadIdx.x; i < k && i < 256; i += NT) ys[i] = y[i];
  __syncthreads();
  const int64_t nu = n / BS;
  UNIT_LOOP(u, nu) {
    double s[BS];
#pragma unroll
    for (int c = 0; c < BS; ++c) {
      const int64_t q = BS * u + c;
      s[c] = 0.0;
      for (int i = 0; i < k; ++i) s[c] += (i < 256 ? ys[i] : y[i]) * double(Vp[i][q]);
    }
    if constexpr (BS == 1) {
      const double d = dinv ? double(dinv[u]) : 1.0;
      x[u] = T(double(x[u]) + d * s[0]);
    } else {
      const double bxx = dinv[u], byy = dinv[nu + u], bzz = dinv[2 * nu + u];
      const double bxy = dinv[3 * nu + u], byz = dinv[4 * nu + u], bxz = dinv[5 * nu + u];
      const double z[3] = {bxx * s[0] + bxy * s[1] + bxz * s[2],
                           bxy * s[0] + byy * s[1] + byz * s[2],
                           bxz * s[0] + byz * s[1] + bzz * s[2]};
#pragma unroll
      for (int c = 0; c < 3; ++c) x[3 * u + c] = T(double(x[3 * u + c]) + z[c]);
    }
  }
}

// Start of a cycle: V_0 = r0 / ||r0|| given partials of r0.r0; initialise g.
template <typename T>
__global__ __launch_bounds__(NT) void k_gm_start(const T *r0, T *V0, int64_t n, const double *red,
                                                 int np, double *rot, int m, double *scal,
                                                 int32_t *flag, double rtol, double atol,
                                                 int first) {
  __shared__ double sh[NT / 64];
  const double rr = sum_partials(red, np, sh);
  const double beta = sqrt(rr);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (first) scal[1] = fmax(rtol * beta, atol);
    scal[0] = beta;
    scal[3] = beta;
    // g[j + 1] is written by column j before anything reads it
    gm_g(rot, m)[0] = beta;
    flag[1] = 0;
    flag[0] = !(beta == beta) ? 3 : (beta <= scal[1] ? 1 : 0);
  }
  const T s = T(beta > 0.0 ? 1.0 / beta : 0.0);
  for (int64_t k = int64_t(blockIdx.x) * NT + threadIdx.x; k < n; k += int64_t(gridDim.x) * NT)
    V0[k] = r0[k] * s;
}

// ------------------------------------------------------------------ L-BFGS
template <typename T>
__global__ __launch_bounds__(NT) void k_lb_axpy_dot(T *q, const T *y, const double *red, int np,
                                                    double rho, double *alpha_out,
                                                    const T *s_next, double *red_next, int64_t n) {
  __shared__ double shd[NT / 64];
  __shared__ T sh[NT / 64];
  const double alpha = rho * sum_partials(red, np, shd);
  if (blockIdx.x == 0 && threadIdx.x == 0) alpha_out[0] = alpha;
  const T a = T(alpha);
  T acc = T(0);
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < n; i += int64_t(gridDim.x) * NT) {
    const T qi = q[i] - a * y[i];
    q[i] = qi;
    if (s_next) acc += s_next[i] * qi;
  }
  if (red_next) {
    acc = block_sum_all(acc, sh);
    if (threadIdx.x == 0) red_next[blockIdx.x] = double(acc);
  }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_lb_axpy2_dot(T *z, const T *s, const double *red, int np,
                                                     double rho, const double *alpha,
                                                     const T *y_next, double *red_next,
                                                     int64_t n) {
  __shared__ double shd[NT / 64];
  __shared__ T sh[NT / 64];
  const double beta = rho * sum_partials(red, np, shd);
  const T cc = T(alpha[0] - beta);
  T acc = T(0);
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < n; i += int64_t(gridDim.x) * NT) {
    const T zi = z[i] + cc * s[i];
    z[i] = zi;
    if (y_next) acc += y_next[i] * zi;
  }
  if (red_next) {
    acc = block_sum_all(acc, sh);
    if (threadIdx.x == 0) red_next[blockIdx.x] = double(acc);
  }
}

}  // namespace

int vgrid(int64_t n) {
  int64_t g = (n + NT * 4 - 1) / (NT * 4);
  if (g < 1) g = 1;
  if (g > VGRID_MAX) g = VGRID_MAX;
  return int(g);
}

#define LAUNCH(kern, grid, ...) hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), 0, c->stream, __VA_ARGS__)

hipError_t vec_fill(Ctx *c, int prec, void *x, double val, int64_t n) {
  if (prec == NLE_FP32)
    LAUNCH(k_fill<float>, vgrid(n), static_cast<float *>(x), float(val), n);
  else
    LAUNCH(k_fill<double>, vgrid(n), static_cast<double *>(x), val, n);
  return hipGetLastError();
}

hipError_t vec_cast_scale(Ctx *c, int px, const void *x, int py, void *y, double s, int64_t n) {
  const int g = vgrid(n);
  if (px == NLE_FP64 && py == NLE_FP64)
    LAUNCH((k_cast_scale<double, double>), g, static_cast<const double *>(x), static_cast<double *>(y), s, n);
  else if (px == NLE_FP64)
    LAUNCH((k_cast_scale<double, float>), g, static_cast<const double *>(x), static_cast<float *>(y), s, n);
  else if (py == NLE_FP64)
    LAUNCH((k_cast_scale<float, double>), g, static_cast<const float *>(x), static_cast<double *>(y), s, n);
  else
    LAUNCH((k_cast_scale<float, float>), g, static_cast<const float *>(x), static_cast<float *>(y), s, n);
  return hipGetLastError();
}

hipError_t vec_axpy(Ctx *c, int px, const void *x, int py, void *y, double a, const double *ad,
                    int64_t n) {
  const int g = vgrid(n);
  if (px == NLE_FP64 && py == NLE_FP64)
    LAUNCH((k_axpy<double, double>), g, static_cast<const double *>(x), static_cast<double *>(y), a, ad, n);
  else if (px == NLE_FP32 && py == NLE_FP64)
    LAUNCH((k_axpy<float, double>), g, static_cast<const float *>(x), static_cast<double *>(y), a, ad, n);
  else if (px == NLE_FP64)
    LAUNCH((k_axpy<double, float>), g, static_cast<const double *>(x), static_cast<float *>(y), a, ad, n);
  else
    LAUNCH((k_axpy<float, float>), g, static_cast<const float *>(x), static_cast<float *>(y), a, ad, n);
  return hipGetLastError();
}

hipError_t pc_apply(Ctx *c, int prec, int pcb, const void *d, const void *x, void *y, int64_t n) {
  const int g = vgrid(n);
  if (prec == NLE_FP32) {
    if (pcb == 3)
      LAUNCH((k_pc_apply<float, 3>), g, static_cast<const float *>(d), static_cast<const float *>(x),
             static_cast<float *>(y), n);
    else
      LAUNCH((k_pc_apply<float, 1>), g, static_cast<const float *>(d), static_cast<const float *>(x),
             static_cast<float *>(y), n);
  } else {
    if (pcb == 3)
      LAUNCH((k_pc_apply<double, 3>), g, static_cast<const double *>(d),
             static_cast<const double *>(x), static_cast<double *>(y), n);
    else
      LAUNCH((k_pc_apply<double, 1>), g, static_cast<const double *>(d),
             static_cast<const double *>(x), static_cast<double *>(y), n);
  }
  return hipGetLastError();
}

// Schur block of the lower block-triangular preconditioner: x_p =
// -(b_p - t_p) * sinv_p (the Schur approximation -diag(1 / sinv)).
template <typename T>
__global__ __launch_bounds__(NT) void k_schur_p(const T *b, const T *t, const T *sinv, T *x,
                                                int64_t np) {
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < np; i += int64_t(gridDim.x) * NT)
    x[i] = -(b[i] - t[i]) * sinv[i];
}

hipError_t schur_p(Ctx *c, int prec, const void *b, const void *t, const void *sinv, void *x,
                   int64_t np) {
  const int g = vgrid(np);
  if (prec == NLE_FP32)
    LAUNCH(k_schur_p<float>, g, static_cast<const float *>(b), static_cast<const float *>(t),
           static_cast<const float *>(sinv), static_cast<float *>(x), np);
  else
    LAUNCH(k_schur_p<double>, g, static_cast<const double *>(b), static_cast<const double *>(t),
           static_cast<const double *>(sinv), static_cast<double *>(x), np);
  return hipGetLastError();
}

hipError_t block_inverse(Ctx *c, int64_t nn) {
  LAUNCH(k_block_inv, vgrid(nn), c->diag64, c->odiag64, c->binv64, c->binv32, nn);
  return hipGetLastError();
}

hipError_t newmark_predict(Ctx *c, const double *u, const double *v, const double *a, double *ut,
                           double *vt, double dt, double beta, double gamma, int64_t n) {
  LAUNCH(k_newmark_predict, vgrid(n), u, v, a, ut, vt, dt, beta, gamma, n);
  return hipGetLastError();
}

hipError_t newmark_correct(Ctx *c, const double *u, const double *ut, double *v, double *a,
                           double dt, double beta, double gamma, int64_t n) {
  LAUNCH(k_newmark_correct, vgrid(n), u, ut, v, a, dt, beta, gamma, n);
  return hipGetLastError();
}

int vec_wdiff2_partials(Ctx *c, const double *w, const double *x, const double *y, int64_t n,
                        double *red, hipError_t *err) {
  const int g = vgrid(n);
  LAUNCH(k_wdiff2, g, w, x, y, n, red);
  *err = hipGetLastError();
  return g;
}

hipError_t vec_recip(Ctx *c, const double *d, double *di, int64_t n) {
  LAUNCH(k_recip, vgrid(n), d, di, n);
  return hipGetLastError();
}

hipError_t vec_lift(Ctx *c, double *u) {
  if (c->n_dir == 0) return hipSuccess;
  if (!c->dir_dofs || !c->dir_vals) return hipErrorInvalidValue;  // never launch on null arrays
  LAUNCH(k_lift, vgrid(c->n_dir), u, c->dir_dofs, c->dir_vals, c->n_dir);
  return hipGetLastError();
}

hipError_t vec_dir_delta(Ctx *c, const double *u, double *w) {
  if (c->n_dir == 0) return hipSuccess;
  if (!c->dir_dofs || !c->dir_vals) return hipErrorInvalidValue;
  LAUNCH(k_dir_delta, vgrid(c->n_dir), u, c->dir_dofs, c->dir_vals, w, c->n_dir);
  return hipGetLastError();
}

int vec_dot_partials(Ctx *c, int prec, const void *a, const void *b, int64_t n, double *red,
                     hipError_t *err) {
  const int g = vgrid(n);
  if (prec == NLE_FP32)
    LAUNCH(k_dot<float>, g, static_cast<const float *>(a), static_cast<const float *>(b), n, red);
  else
    LAUNCH(k_dot<double>, g, static_cast<const double *>(a), static_cast<const double *>(b), n, red);
  *err = hipGetLastError();
  return g;
}

hipError_t reduce_scalar(Ctx *c, const double *red, int np, double *out) {
  LAUNCH(k_reduce, 1, red, np, 0, out);
  return hipGetLastError();
}

hipError_t reduce_scalars(Ctx *c, const double *red, int np, int count, double *out) {
  LAUNCH(k_reduce, count, red, np, VGRID_MAX, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ CG
hipError_t cg_start(Ctx *c, const CgArgs &a, const void *b, double rtol, double atol, int max_it,
                    bool finish) {
  const int g = vgrid(a.n);
#define CG_START(T, BS)                                                                        \
  LAUNCH((k_cg_start<T, BS>), g, static_cast<const T *>(b), static_cast<T *>(a.x),              \
         static_cast<T *>(a.r), static_cast<T *>(a.z), static_cast<T *>(a.p),                   \
         static_cast<const T *>(a.dinv), a.n, a.red_b)
  if (a.prec == NLE_FP32) {
    if (a.pcb == 3) CG_START(float, 3); else CG_START(float, 1);
  } else {
    if (a.pcb == 3) CG_START(double, 3); else CG_START(double, 1);
  }
#undef CG_START
  if (!finish) return hipGetLastError();
  return cg_start_finish(c, a, rtol, atol, max_it);
}

hipError_t cg_start_finish(Ctx *c, const CgArgs &a, double rtol, double atol, int max_it) {
  LAUNCH(k_cg_start2, 1, a.red_b, vgrid(a.n), a.scal, a.flag, rtol, atol, max_it);
  return hipGetLastError();
}

hipError_t cg_update(Ctx *c, const CgArgs &a, bool fused) {
  const int g = vgrid(a.n);
#define CG_UPD(T, BS, F)                                                                       \
  LAUNCH((k_cg_update<T, BS, F>), g, static_cast<T *>(a.x), static_cast<T *>(a.r),              \
         static_cast<T *>(a.z), static_cast<T *>(a.p), static_cast<const T *>(a.Ap),            \
         static_cast<const T *>(a.dinv), a.n, a.red_a, a.np_a, a.red_b, a.scal, a.flag,         \
         static_cast<T *>(a.cd), T(a.cth))
#define CG_UPD2(T, BS)                                                                         \
  if (fused) CG_UPD(T, BS, true); else CG_UPD(T, BS, false)
  if (a.prec == NLE_FP32) {
    if (a.pcb == 3) CG_UPD2(float, 3); else CG_UPD2(float, 1);
  } else {
    if (a.pcb == 3) CG_UPD2(double, 3); else CG_UPD2(double, 1);
  }
#undef CG_UPD2
#undef CG_UPD
  return hipGetLastError();
}

hipError_t cg_direction(Ctx *c, const CgArgs &a) {
  const int g = vgrid(a.n);
  if (a.prec == NLE_FP32)
    LAUNCH(k_cg_direction<float>, g, static_cast<float *>(a.p), static_cast<const float *>(a.z),
           a.n, a.red_b, g, a.scal, a.flag);
  else
    LAUNCH(k_cg_direction<double>, g, static_cast<double *>(a.p), static_cast<const double *>(a.z),
           a.n, a.red_b, g, a.scal, a.flag);
  return hipGetLastError();
}

// ------------------------------------------------------------------ MINRES
#define MR_PTRS(T)                                                                              \
  static_cast<T *>(a.x), static_cast<T *>(a.r1), static_cast<T *>(a.r2), static_cast<T *>(a.y), \
      static_cast<T *>(a.r), static_cast<T *>(a.wa), static_cast<T *>(a.wb),                      \
      static_cast<T *>(a.za), static_cast<T *>(a.zb), static_cast<const T *>(a.dinv)

hipError_t mr_start(Ctx *c, const MinresArgs &a, const void *b, double rtol, double atol,
                    int max_it, bool finish) {
  const int g = vgrid(a.n);
  if (a.prec == NLE_FP32) {
    if (a.pcb == 3)
      LAUNCH((k_mr_start<float, 3>), g, static_cast<const float *>(b), MR_PTRS(float), a.n, a.red_b);
    else
      LAUNCH((k_mr_start<float, 1>), g, static_cast<const float *>(b), MR_PTRS(float), a.n, a.red_b);
  } else {
    if (a.pcb == 3)
      LAUNCH((k_mr_start<double, 3>), g, static_cast<const double *>(b), MR_PTRS(double), a.n, a.red_b);
    else
      LAUNCH((k_mr_start<double, 1>), g, static_cast<const double *>(b), MR_PTRS(double), a.n, a.red_b);
  }
  if (!finish) return hipGetLastError();
  return mr_start_finish(c, a, rtol, atol, max_it);
}

hipError_t mr_start_finish(Ctx *c, const MinresArgs &a, double rtol, double atol, int max_it) {
  const int g = vgrid(a.n);
  LAUNCH(k_mr_start2, 1, a.red_b, g, a.scal, a.flag, rtol, atol, max_it);
  if (a.prec == NLE_FP32)
    LAUNCH(k_mr_v<float>, g, static_cast<const float *>(a.y), static_cast<float *>(a.v), a.n,
           a.scal, a.flag);
  else
    LAUNCH(k_mr_v<double>, g, static_cast<const double *>(a.y), static_cast<double *>(a.v), a.n,
           a.scal, a.flag);
  return hipGetLastError();
}

// the three vector / scalar steps after the Jacobian action of one iteration
hipError_t mr_iterate(Ctx *c, const MinresArgs &a,
                      hipError_t (*pc_outside)(Ctx *, const MinresArgs &)) {
  const int g = vgrid(a.n);
#define MR_C(T, BS)                                                                            \
  LAUNCH((k_mr_c<T, BS>), g, static_cast<T *>(a.y), static_cast<T *>(a.r1),                    \
         static_cast<T *>(a.r2), static_cast<T *>(a.av), static_cast<const T *>(a.dinv), a.n,   \
         a.red_a, a.np_a, a.red_b, a.scal, a.flag)
  if (a.prec == NLE_FP32) {
    if (a.pcb == 3) MR_C(float, 3); else MR_C(float, 1);
  } else {
    if (a.pcb == 3) MR_C(double, 3); else MR_C(double, 1);
  }
#undef MR_C
  if (pc_outside) {
    // the preconditioner runs outside these kernels (the multigrid cycle):
    // y = M^-1 r2 and the partials of r2.y, then the scalar and vector steps
    const hipError_t e = pc_outside(c, a);
    if (e != hipSuccess) return e;
  }
  LAUNCH(k_mr_d, 1, a.red_b, g, a.red_r, g, a.scal, a.flag);
  if (a.prec == NLE_FP32)
    LAUNCH(k_mr_e<float>, g, static_cast<float *>(a.x), static_cast<float *>(a.v),
           static_cast<const float *>(a.y), static_cast<const float *>(a.av),
           static_cast<float *>(a.wa), static_cast<float *>(a.wb), static_cast<float *>(a.za),
           static_cast<float *>(a.zb), static_cast<float *>(a.r), a.n, a.red_r, a.scal, a.flag);
  else
    LAUNCH(k_mr_e<double>, g, static_cast<double *>(a.x), static_cast<double *>(a.v),
           static_cast<const double *>(a.y), static_cast<const double *>(a.av),
           static_cast<double *>(a.wa), static_cast<double *>(a.wb), static_cast<double *>(a.za),
           static_cast<double *>(a.zb), static_cast<double *>(a.r), a.n, a.red_r, a.scal, a.flag);
  return hipGetLastError();
}

// ------------------------------------------------------------------ GMRES
hipError_t gmres_tables(Ctx *c, const GmresArgs &a, int v0, int nv, int limit, void *vbase,
                        size_t vb, double *hbase, double *rbase) {
  if (nv <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gm_tables, dim3((nv + NT - 1) / NT), dim3(NT), 0, c->stream, a.Vp, a.Hp,
                     a.Rp, v0, nv, limit, static_cast<char *>(vbase), vb, hbase, rbase);
  return hipGetLastError();
}

hipError_t gmres_start(Ctx *c, const GmresArgs &a, const void *r0, double rtol, double atol,
                       int first) {
  const int g = vgrid(a.n);
  hipError_t e;
  double *red = a.hR[0];
  vec_dot_partials(c, a.prec, r0, r0, a.n, red, &e);
  if (e != hipSuccess) return e;
  if (a.prec == NLE_FP32)
    LAUNCH(k_gm_start<float>, g, static_cast<const float *>(r0), static_cast<float *>(a.hV[0]),
           a.n, red, g, a.rot, a.m, a.scal, a.flag, rtol, atol, first);
  else
    LAUNCH(k_gm_start<double>, g, static_cast<const double *>(r0), static_cast<double *>(a.hV[0]),
           a.n, red, g, a.rot, a.m, a.scal, a.flag, rtol, atol, first);
  return hipGetLastError();
}

// partials of V_i . w, i <= j, into rows 0..j
hipError_t gmres_multidot(Ctx *c, const GmresArgs &a, int j) {
  const int g = vgrid(a.n);
  if (a.prec == NLE_FP32)
    hipLaunchKernelGGL(k_gm_dots<float>, dim3(g, j + 1), dim3(NT), 0, c->stream,
                       reinterpret_cast<float *const *>(a.Vp), static_cast<const float *>(a.w),
                       a.n, a.Rp, a.flag);
  else
    hipLaunchKernelGGL(k_gm_dots<double>, dim3(g, j + 1), dim3(NT), 0, c->stream,
                       reinterpret_cast<double *const *>(a.Vp), static_cast<const double *>(a.w),
                       a.n, a.Rp, a.flag);
  return hipGetLastError();
}

// pass p: reduce the j+1 dots into hc_p (scal area p), subtract; the last
// pass also produces partials of w.w.
hipError_t gmres_subtract(Ctx *c, const GmresArgs &a, int j, int pass, int want_sq) {
  const int g = vgrid(a.n);
  double *hc = a.scal + 8 + pass * (a.m + 1);
  hipLaunchKernelGGL(k_gm_reduce, dim3(j + 1), dim3(NT), 0, c->stream, a.Rp, g, hc, 0, a.flag);
  double *red_sq = want_sq ? a.redsq : nullptr;
  if (a.prec == NLE_FP32)
    LAUNCH(k_gm_sub<float>, g, reinterpret_cast<float *const *>(a.Vp), static_cast<float *>(a.w),
           a.n, hc, j + 1, red_sq, a.flag);
  else
    LAUNCH(k_gm_sub<double>, g, reinterpret_cast<double *const *>(a.Vp),
           static_cast<double *>(a.w), a.n, hc, j + 1, red_sq, a.flag);
  return hipGetLastError();
}

// Modified Gram-Schmidt step i: h_i = V_i . w (reduced), w -= h_i V_i.  The
// coefficient is accumulated into the pass-0 column area.
hipError_t gmres_mgs_step(Ctx *c, const GmresArgs &a, int i, int j) {
  const int g = vgrid(a.n);
  hipError_t e;
  const int64_t n = a.n;
  vec_dot_partials(c, a.prec, a.hV[i], a.w, n, a.hR[0], &e);
  if (e != hipSuccess) return e;
  double *hc = a.scal + 8;
  hipLaunchKernelGGL(k_gm_reduce, dim3(1), dim3(NT), 0, c->stream, a.Rp, g, hc + i, 0, a.flag);
  const bool last = (i == j);
  double *red_sq = last ? a.redsq : nullptr;
  if (a.prec == NLE_FP32)
    LAUNCH(k_gm_sub<float>, g, reinterpret_cast<float *const *>(a.Vp) + i,
           static_cast<float *>(a.w), n, hc + i, 1, red_sq, a.flag);
  else
    LAUNCH(k_gm_sub<double>, g, reinterpret_cast<double *const *>(a.Vp) + i,
           static_cast<double *>(a.w), n, hc + i, 1, red_sq, a.flag);
  return hipGetLastError();
}

hipError_t gmres_finish_col(Ctx *c, const GmresArgs &a, int j, int mgs) {
  const int g = vgrid(a.n);
  const double *hc1 = a.scal + 8;
  const double *hc2 = mgs ? nullptr : a.scal + 8 + (a.m + 1);
  hipLaunchKernelGGL(k_gm_col, dim3(1), dim3(NT), 0, c->stream, a.Hp, a.rot, a.m, j, a.redsq, g,
                     hc1, hc2, a.scal, a.flag, a.m);
  void *vn = a.hV[j + 1];
  if (a.prec == NLE_FP32)
    LAUNCH(k_gm_next<float>, g, static_cast<const float *>(a.w), static_cast<float *>(vn), a.n,
           a.scal, a.flag);
  else
    LAUNCH(k_gm_next<double>, g, static_cast<const double *>(a.w), static_cast<double *>(vn), a.n,
           a.scal, a.flag);
  return hipGetLastError();
}

hipError_t gmres_update_x(Ctx *c, const GmresArgs &a) {
  hipLaunchKernelGGL(k_gm_solve, dim3(1), dim3(64), 0, c->stream, a.Hp, a.rot, a.m, a.flag);
  const int g = vgrid(a.n);
#define GM_UPD(T, BS)                                                                          \
  LAUNCH((k_gm_update<T, BS>), g, reinterpret_cast<T *const *>(a.Vp), static_cast<T *>(a.x),    \
         static_cast<const T *>(a.dinv), a.n, a.rot, a.m, a.flag)
  if (a.prec == NLE_FP32) {
    if (a.pcb == 3) GM_UPD(float, 3); else GM_UPD(float, 1);
  } else {
    if (a.pcb == 3) GM_UPD(double, 3); else GM_UPD(double, 1);
  }
#undef GM_UPD
  return hipGetLastError();
}

// ------------------------------------------------------------------ L-BFGS
hipError_t lbfgs_dot(Ctx *c, int prec, const void *s, const void *q, int64_t n, double *red,
                     int *np) {
  hipError_t e;
  *np = vec_dot_partials(c, prec, s, q, n, red, &e);
  return e;
}

hipError_t lbfgs_axpy_dot(Ctx *c, int prec, void *q, const void *y, const double *red, int np,
                          double rho, double *alpha_out, const void *s_next, double *red_next,
                          int64_t n) {
  const int g = vgrid(n);
  if (prec == NLE_FP32)
    LAUNCH(k_lb_axpy_dot<float>, g, static_cast<float *>(q), static_cast<const float *>(y), red, np,
           rho, alpha_out, static_cast<const float *>(s_next), red_next, n);
  else
    LAUNCH(k_lb_axpy_dot<double>, g, static_cast<double *>(q), static_cast<const double *>(y), red,
           np, rho, alpha_out, static_cast<const double *>(s_next), red_next, n);
  return hipGetLastError();
}

hipError_t lbfgs_axpy2_dot(Ctx *c, int prec, void *z, const void *s, const double *red, int np,
                           double rho, const double *alpha, const void *y_next, double *red_next,
                           int64_t n) {
  const int g = vgrid(n);
  if (prec == NLE_FP32)
    LAUNCH(k_lb_axpy2_dot<float>, g, static_cast<float *>(z), static_cast<const float *>(s), red, np,
           rho, alpha, static_cast<const float *>(y_next), red_next, n);
  else
    LAUNCH(k_lb_axpy2_dot<double>, g, static_cast<double *>(z), static_cast<const double *>(s), red,
           np, rho, alpha, static_cast<const double *>(y_next), red_next, n);
  return hipGetLastError();
}

}  // namespace nle
