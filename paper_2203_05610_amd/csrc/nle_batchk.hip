// Vector kernels of the batched solver.  The union vector of all instances is
// cut into segments of at most SEG dofs that never span two instances; one
// workgroup per segment, one partial per segment.  Every scalar of the Krylov
// recurrences is per instance; a workgroup sums the partials of its own
// instance (segments, or element blocks and merge workgroups) in index order,
// so instances never mix and results do not depend on the batch.
#include <hip/hip_runtime.h>

#include "nle_batch.hpp"

namespace nle {

namespace {

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

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

__device__ __forceinline__ double range_sum(const double *red, int a, int b, double *sh) {
  double v = 0.0;
  for (int k = a + int(threadIdx.x); k < b; k += NT) v += red[k];
  return block_sum_all(v, sh);
}

// Sum of instance i's element-kernel partials: its blocks, then its merge
// workgroups (stored after all nblk block partials).
__device__ __forceinline__ double elem_sum(const BatchDev &B, const double *red, int i, double *sh) {
  const double a = range_sum(red, B.inst_blk[i], B.inst_blk[i + 1], sh);
  const double b = range_sum(red, B.nblk + B.inst_mwg[i], B.nblk + B.inst_mwg[i + 1], sh);
  return a + b;
}

__device__ __forceinline__ double seg_sum(const BatchDev &B, const double *red, int i, double *sh) {
  return range_sum(red, B.inst_seg[i], B.inst_seg[i + 1], sh);
}

#define SEG_LOOP(B, s, d) for (int64_t d = B.seg_beg[s] + threadIdx.x; d < B.seg_beg[s + 1]; d += NT)

// ---- per-instance reductions -------------------------------------------------
// out[i] = instance i's sum of element partials (one workgroup per instance)
__global__ __launch_bounds__(NT) void kb_reduce_elem(BatchDev B, const double *red, double *out) {
  __shared__ double sh[NT / 64];
  const int i = blockIdx.x;
  const double s = elem_sum(B, red, i, sh);
  if (threadIdx.x == 0) out[i] = s;
}

__global__ __launch_bounds__(NT) void kb_reduce_seg(BatchDev B, const double *red, double *out) {
  __shared__ double sh[NT / 64];
  const int i = blockIdx.x;
  const double s = seg_sum(B, red, i, sh);
  if (threadIdx.x == 0) out[i] = s;
}

// ---- elementwise with per-instance coefficients ---------------------------------
// y = coef[i] * x (types may differ)
template <typename S, typename D>
__global__ __launch_bounds__(NT) void kb_scale(BatchDev B, const S *x, D *y, const double *coef) {
  const int s = blockIdx.x, i = B.seg_inst[s];
  const double a = coef[i];
  SEG_LOOP(B, s, d) y[d] = D(a * double(x[d]));
}

// y += coef[i] * x, skipped where coef[i] == 0
template <typename S, typename D>
__global__ __launch_bounds__(NT) void kb_axpy(BatchDev B, const S *x, D *y, const double *coef) {
  const int s = blockIdx.x, i = B.seg_inst[s];
  const double a = coef[i];
  if (a == 0.0) return;
  SEG_LOOP(B, s, d) y[d] = D(double(y[d]) + a * double(x[d]));
}

// dst = src where mask[i] != 0
__global__ __launch_bounds__(NT) void kb_copy(BatchDev B, const double *src, double *dst,
                                              const int32_t *mask) {
  const int s = blockIdx.x, i = B.seg_inst[s];
  if (!mask[i]) return;
  SEG_LOOP(B, s, d) dst[d] = src[d];
}

// t -= b; partials of t.t per segment
template <typename T>
__global__ __launch_bounds__(NT) void kb_sub_norm(BatchDev B, T *t, const T *b, double *red) {
  __shared__ T sh[NT / 64];
  const int s = blockIdx.x;
  T acc = T(0);
  SEG_LOOP(B, s, d) {
    const T v = t[d] - b[d];
    t[d] = v;
    acc += v * v;
  }
  acc = block_sum_all(acc, sh);
  if (threadIdx.x == 0) red[s] = double(acc);
}

// ---- batched L-BFGS: pairs in per-instance ring slots ----------------------------
// The pairs (s_j, y_j) of all instances live in [m][n] arrays; instance i's
// pair of a given age sits in slot[i] (negative: the instance has none).
// partials of base[slot].x per segment
template <typename T>
__global__ __launch_bounds__(NT) void kb_dot_slot(BatchDev B, const T *base, int64_t stride,
                                                  const int32_t *slot, const T *x, double *red) {
  __shared__ T sh[NT / 64];
  const int s = blockIdx.x, i = B.seg_inst[s];
  const int k = slot[i];
  T acc = T(0);
  if (k >= 0) {
    const T *v = base + int64_t(k) * stride;
    SEG_LOOP(B, s, d) acc += v[d] * x[d];
  }
  acc = block_sum_all(acc, sh);
  if (threadIdx.x == 0) red[s] = double(acc);
}

// y += coef[i] * base[slot[i]] (nothing where slot < 0 or coef == 0)
template <typename S, typename D>
__global__ __launch_bounds__(NT) void kb_axpy_slot(BatchDev B, D *y, const S *base, int64_t stride,
                                                   const int32_t *slot, const double *coef) {
  const int s = blockIdx.x, i = B.seg_inst[s];
  const int k = slot[i];
  const double a = coef[i];
  if (k < 0 || a == 0.0) return;
  const S *v = base + int64_t(k) * stride;
  SEG_LOOP(B, s, d) y[d] = D(double(y[d]) + a * double(v[d]));
}

// base[slot[i]] = coef[i] * x (where slot >= 0)
template <typename T>
__global__ __launch_bounds__(NT) void kb_store_slot(BatchDev B, T *base, int64_t stride,
                                                    const int32_t *slot, const T *x,
                                                    const double *coef) {
  const int s = blockIdx.x, i = B.seg_inst[s];
  const int k = slot[i];
  if (k < 0) return;
  const T a = T(coef[i]);
  T *v = base + int64_t(k) * stride;
  SEG_LOOP(B, s, d) v[d] = a * x[d];
}

// The new pair of each instance with slot >= 0: y = g - g_prev into
// Ybase[slot] (rounded to T), and per-segment partials of s.y, s.s, y.y
// (s = Sbase[slot]) at red[0, nseg), red[nseg, 2 nseg), red[2 nseg, 3 nseg).
template <typename T>
__global__ __launch_bounds__(NT) void kb_lbfgs_pair(BatchDev B, const T *Sbase, T *Ybase,
                                                    int64_t stride, const int32_t *slot,
                                                    const double *g, const double *gp,
                                                    double *red) {
  __shared__ T sh[NT / 64];
  const int s = blockIdx.x, i = B.seg_inst[s];
  const int k = slot[i];
  T sy = T(0), ss = T(0), yy = T(0);
  if (k >= 0) {
    const T *sv = Sbase + int64_t(k) * stride;
    T *yv = Ybase + int64_t(k) * stride;
    SEG_LOOP(B, s, d) {
      const T y = T(g[d] - gp[d]);
      yv[d] = y;
      const T sd = sv[d];
      sy += sd * y;
      ss += sd * sd;
      yy += y * y;
    }
  }
  sy = block_sum_all(sy, sh);
  ss = block_sum_all(ss, sh);
  yy = block_sum_all(yy, sh);
  if (threadIdx.x == 0) {
    red[s] = double(sy);
    red[B.nseg + s] = double(ss);
    red[2 * B.nseg + s] = double(yy);
  }
}

// per instance: first loop alpha = rho dot, coef = -alpha; second loop
// coef = alpha - rho dot (beta)
__global__ __launch_bounds__(NT) void kb_lbfgs_coef(int n, const double *rho, const double *dot,
                                                    double *alpha, double *coef, int second) {
  const int i = int(blockIdx.x) * NT + int(threadIdx.x);
  if (i >= n) return;
  if (second)
    coef[i] = alpha[i] - rho[i] * dot[i];
  else {
    alpha[i] = rho[i] * dot[i];
    coef[i] = -alpha[i];
  }
}

// ---- batched CG ----------------------------------------------------------------
// scal[i*BS + k]: 0 rz, 1 rz_old, 2 tol^2, 3 r.r ; done[i], its[i]
template <typename T>
__global__ __launch_bounds__(NT) void kb_cg_start(BatchDev B, const T *b, T *x, T *r, T *z, T *p,
                                                  const T *dinv, double *red) {
  __shared__ T sh[NT / 64];
  const int s = blockIdx.x;
  T arz = T(0), arr = T(0);
  SEG_LOOP(B, s, d) {
    const T bi = b[d];
    const T zi = dinv[d] * bi;
    x[d] = T(0);
    r[d] = bi;
    z[d] = zi;
    p[d] = zi;
    arz += bi * zi;
    arr += bi * bi;
  }
  arz = block_sum_all(arz, sh);
  arr = block_sum_all(arr, sh);
  if (threadIdx.x == 0) {
    red[s] = double(arz);
    red[B.nseg + s] = double(arr);
  }
}

__global__ __launch_bounds__(NT) void kb_cg_start2(BatchDev B, const double *red, double *scal,
                                                   int32_t *done, int32_t *its, const double *rtol,
                                                   const double *atol, const int32_t *active,
                                                   int max_it) {
  __shared__ double sh[NT / 64];
  const int i = blockIdx.x;
  const double rz = seg_sum(B, red, i, sh);
  const double rr = seg_sum(B, red + B.nseg, i, sh);
  if (threadIdx.x == 0) {
    const double tol2 = fmax(rtol[i] * rtol[i] * rr, atol[i] * atol[i]);
    double *S = scal + BS * i;
    S[0] = rz;
    S[2] = tol2;
    S[3] = rr;
    S[4] = double(max_it);
    its[i] = 0;
    done[i] = !active[i] ? 1 : (rr <= tol2 ? 1 : (rr == rr ? 0 : 3));
  }
}

template <typename T>
__global__ __launch_bounds__(NT) void kb_cg_update(BatchDev B, T *x, T *r, T *z, const T *p,
                                                   const T *Ap, const T *dinv, const double *red_a,
                                                   double *red_b, double *scal, int32_t *done) {
  __shared__ double shd[NT / 64];
  __shared__ T sh[NT / 64];
  const int s = B.seg_list ? B.seg_list[blockIdx.x] : int(blockIdx.x), i = B.seg_inst[s];
  if (done[i] != 0) return;
  const double pAp = elem_sum(B, red_a, i, shd);
  double *S = scal + BS * i;
  const bool first = s == B.inst_seg[i];
  if (!(pAp > 0.0)) {
    if (first && threadIdx.x == 0) done[i] = (pAp == pAp) ? 2 : 3;
    return;
  }
  const double rz = S[0];
  if (first && threadIdx.x == 0) S[1] = rz;
  const T a = T(rz / pAp);
  T arz = T(0), arr = T(0);
  SEG_LOOP(B, s, d) {
    const T ri = r[d] - a * Ap[d];
    const T zi = dinv[d] * ri;
    x[d] += a * p[d];
    r[d] = ri;
    z[d] = zi;
    arz += ri * zi;
    arr += ri * ri;
  }
  arz = block_sum_all(arz, sh);
  arr = block_sum_all(arr, sh);
  if (threadIdx.x == 0) {
    red_b[s] = double(arz);
    red_b[B.nseg + s] = double(arr);
  }
}

template <typename T>
__global__ __launch_bounds__(NT) void kb_cg_direction(BatchDev B, T *p, const T *z,
                                                      const double *red_b, double *scal,
                                                      int32_t *done, int32_t *its) {
  __shared__ double sh[NT / 64];
  const int s = B.seg_list ? B.seg_list[blockIdx.x] : int(blockIdx.x), i = B.seg_inst[s];
  if (done[i] != 0) return;
  const double rz = seg_sum(B, red_b, i, sh);
  const double rr = seg_sum(B, red_b + B.nseg, i, sh);
  double *S = scal + BS * i;
  const T bt = T(rz / S[1]);
  SEG_LOOP(B, s, d) p[d] = z[d] + bt * p[d];
  if (s == B.inst_seg[i] && threadIdx.x == 0) {
    S[0] = rz;
    S[3] = rr;
    const int k = its[i] + 1;
    its[i] = k;
    if (!(rr == rr))
      done[i] = 3;
    else if (rr <= S[2])
      done[i] = 1;
    else if (double(k) >= S[4])
      done[i] = 5;
  }
}

}  // namespace

#define BLAUNCH(kern, grid, ...) hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), 0, c->stream, __VA_ARGS__)

hipError_t batch_reduce_elem(Ctx *c, const BatchDev &B, const double *red, double *out) {
  BLAUNCH(kb_reduce_elem, B.n_inst, B, red, out);
  return hipGetLastError();
}

hipError_t batch_reduce_seg(Ctx *c, const BatchDev &B, const double *red, double *out) {
  BLAUNCH(kb_reduce_seg, B.n_inst, B, red, out);
  return hipGetLastError();
}

hipError_t batch_scale(Ctx *c, const BatchDev &B, int px, const void *x, int py, void *y,
                       const double *coef) {
  if (px == NLE_FP64 && py == NLE_FP64)
    BLAUNCH((kb_scale<double, double>), B.nseg, B, static_cast<const double *>(x), static_cast<double *>(y), coef);
  else if (px == NLE_FP64)
    BLAUNCH((kb_scale<double, float>), B.nseg, B, static_cast<const double *>(x), static_cast<float *>(y), coef);
  else if (py == NLE_FP64)
    BLAUNCH((kb_scale<float, double>), B.nseg, B, static_cast<const float *>(x), static_cast<double *>(y), coef);
  else
    BLAUNCH((kb_scale<float, float>), B.nseg, B, static_cast<const float *>(x), static_cast<float *>(y), coef);
  return hipGetLastError();
}

hipError_t batch_axpy(Ctx *c, const BatchDev &B, int px, const void *x, int py, void *y,
                      const double *coef) {
  if (px == NLE_FP64 && py == NLE_FP64)
    BLAUNCH((kb_axpy<double, double>), B.nseg, B, static_cast<const double *>(x), static_cast<double *>(y), coef);
  else if (px == NLE_FP32 && py == NLE_FP64)
    BLAUNCH((kb_axpy<float, double>), B.nseg, B, static_cast<const float *>(x), static_cast<double *>(y), coef);
  else if (px == NLE_FP64)
    BLAUNCH((kb_axpy<double, float>), B.nseg, B, static_cast<const double *>(x), static_cast<float *>(y), coef);
  else
    BLAUNCH((kb_axpy<float, float>), B.nseg, B, static_cast<const float *>(x), static_cast<float *>(y), coef);
  return hipGetLastError();
}

hipError_t batch_copy(Ctx *c, const BatchDev &B, const double *src, double *dst,
                      const int32_t *mask) {
  BLAUNCH(kb_copy, B.nseg, B, src, dst, mask);
  return hipGetLastError();
}

hipError_t batch_sub_norm(Ctx *c, const BatchDev &B, int prec, void *t, const void *b, double *red) {
  if (prec == NLE_FP32)
    BLAUNCH(kb_sub_norm<float>, B.nseg, B, static_cast<float *>(t), static_cast<const float *>(b), red);
  else
    BLAUNCH(kb_sub_norm<double>, B.nseg, B, static_cast<double *>(t), static_cast<const double *>(b), red);
  return hipGetLastError();
}

hipError_t batch_dot_slot(Ctx *c, const BatchDev &B, int prec, const void *base, int64_t stride,
                          const int32_t *slot, const void *x, double *red) {
  if (prec == NLE_FP32)
    BLAUNCH(kb_dot_slot<float>, B.nseg, B, static_cast<const float *>(base), stride, slot,
            static_cast<const float *>(x), red);
  else
    BLAUNCH(kb_dot_slot<double>, B.nseg, B, static_cast<const double *>(base), stride, slot,
            static_cast<const double *>(x), red);
  return hipGetLastError();
}

hipError_t batch_axpy_slot(Ctx *c, const BatchDev &B, int px, const void *base, int64_t stride,
                           const int32_t *slot, int py, void *y, const double *coef) {
  if (px == NLE_FP32 && py == NLE_FP64)
    BLAUNCH((kb_axpy_slot<float, double>), B.nseg, B, static_cast<double *>(y),
            static_cast<const float *>(base), stride, slot, coef);
  else if (px == NLE_FP32)
    BLAUNCH((kb_axpy_slot<float, float>), B.nseg, B, static_cast<float *>(y),
            static_cast<const float *>(base), stride, slot, coef);
  else if (py == NLE_FP64)
    BLAUNCH((kb_axpy_slot<double, double>), B.nseg, B, static_cast<double *>(y),
            static_cast<const double *>(base), stride, slot, coef);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t batch_store_slot(Ctx *c, const BatchDev &B, int prec, void *base, int64_t stride,
                            const int32_t *slot, const void *x, const double *coef) {
  if (prec == NLE_FP32)
    BLAUNCH(kb_store_slot<float>, B.nseg, B, static_cast<float *>(base), stride, slot,
            static_cast<const float *>(x), coef);
  else
    BLAUNCH(kb_store_slot<double>, B.nseg, B, static_cast<double *>(base), stride, slot,
            static_cast<const double *>(x), coef);
  return hipGetLastError();
}

hipError_t batch_lbfgs_pair(Ctx *c, const BatchDev &B, int prec, const void *Sbase, void *Ybase,
                            int64_t stride, const int32_t *slot, const double *g, const double *gp,
                            double *red) {
  if (prec == NLE_FP32)
    BLAUNCH(kb_lbfgs_pair<float>, B.nseg, B, static_cast<const float *>(Sbase),
            static_cast<float *>(Ybase), stride, slot, g, gp, red);
  else
    BLAUNCH(kb_lbfgs_pair<double>, B.nseg, B, static_cast<const double *>(Sbase),
            static_cast<double *>(Ybase), stride, slot, g, gp, red);
  return hipGetLastError();
}

hipError_t batch_lbfgs_coef(Ctx *c, int n, const double *rho, const double *dot, double *alpha,
                            double *coef, int second) {
  BLAUNCH(kb_lbfgs_coef, (n + NT - 1) / NT, n, rho, dot, alpha, coef, second);
  return hipGetLastError();
}

hipError_t batch_cg_start(Ctx *c, const BatchDev &B, const BatchCg &a, const void *b,
                          const double *rtol, const double *atol, const int32_t *active, int max_it) {
  if (a.prec == NLE_FP32)
    BLAUNCH(kb_cg_start<float>, B.nseg, B, static_cast<const float *>(b), static_cast<float *>(a.x),
            static_cast<float *>(a.r), static_cast<float *>(a.z), static_cast<float *>(a.p),
            static_cast<const float *>(a.dinv), a.red_b);
  else
    BLAUNCH(kb_cg_start<double>, B.nseg, B, static_cast<const double *>(b), static_cast<double *>(a.x),
            static_cast<double *>(a.r), static_cast<double *>(a.z), static_cast<double *>(a.p),
            static_cast<const double *>(a.dinv), a.red_b);
  BLAUNCH(kb_cg_start2, B.n_inst, B, a.red_b, a.scal, a.done, a.its, rtol, atol, active, max_it);
  return hipGetLastError();
}

hipError_t batch_cg_step(Ctx *c, const BatchDev &B, const BatchCg &a) {
  const int g = B.seg_list ? B.n_slist : B.nseg;
  if (a.prec == NLE_FP32) {
    BLAUNCH(kb_cg_update<float>, g, B, static_cast<float *>(a.x), static_cast<float *>(a.r),
            static_cast<float *>(a.z), static_cast<const float *>(a.p), static_cast<const float *>(a.Ap),
            static_cast<const float *>(a.dinv), a.red_a, a.red_b, a.scal, a.done);
    BLAUNCH(kb_cg_direction<float>, g, B, static_cast<float *>(a.p), static_cast<const float *>(a.z),
            a.red_b, a.scal, a.done, a.its);
  } else {
    BLAUNCH(kb_cg_update<double>, g, B, static_cast<double *>(a.x), static_cast<double *>(a.r),
            static_cast<double *>(a.z), static_cast<const double *>(a.p),
            static_cast<const double *>(a.Ap), static_cast<const double *>(a.dinv), a.red_a, a.red_b,
            a.scal, a.done);
    BLAUNCH(kb_cg_direction<double>, g, B, static_cast<double *>(a.p), static_cast<const double *>(a.z),
            a.red_b, a.scal, a.done, a.its);
  }
  return hipGetLastError();
}

}  // namespace nle
