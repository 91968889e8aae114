// Kernels of the aggregation multigrid: probing of the level-1 Galerkin
// operator, the power iteration of the finest level, and the V-cycle's
// smoother, restriction, prolongation, sparse residual and dense coarse solve.
// Every sum runs in a fixed order (one thread, or one wave with a fixed
// butterfly, per output entry), so the
// cycle is bitwise repeatable.

#include <hip/hip_runtime.h>

#include "nle_amg.hpp"

namespace nle {
namespace {

#define LAUNCH(kern, grid, ...) \
  hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), 0, c->stream, __VA_ARGS__)

inline int grid_for(int64_t n) {
  const int64_t g = (n + NT - 1) / NT;
  return int(g < 1 ? 1 : (g > 65535 ? 65535 : g));
}

// one wave64 per item
inline int grid_waves(int64_t n) { return grid_for(64 * n); }

// z[r] = coefficient k of row r's aggregate when that aggregate has colour
// `colour` and at least k+1 coarse dofs, else 0
__global__ __launch_bounds__(NT) void k_probe(double *z, const double *pv, const int32_t *pk,
                                              const int32_t *dcol, int colour, int k, int64_t n) {
  for (int64_t r = int64_t(blockIdx.x) * NT + threadIdx.x; r < n; r += int64_t(gridDim.x) * NT)
    z[r] = (dcol[r] == colour && k < pk[r]) ? pv[6 * r + k] : 0.0;
}

__global__ __launch_bounds__(NT) void k_extract(const double *y, const double *pv,
                                                AmgTasks t, int k, double *val) {
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < t.n;
       i += int64_t(gridDim.x) * NT) {
    if (k >= t.ka[i]) continue;
    const int kp = t.kp[i];
    double s = 0.0;
    for (int32_t q = t.beg[i]; q < t.end[i]; ++q) {
      const int64_t nd = t.nodes[q];
#pragma unroll
      for (int d = 0; d < 3; ++d) s += pv[6 * (3 * nd + d) + kp] * y[3 * nd + d];
    }
    val[t.dest[i] + k] = s;
  }
}

__global__ __launch_bounds__(NT) void k_power(const double *t, const double *dinv,
                                              const double *x, double *y, int64_t n,
                                              double *red) {
  __shared__ double sh[NT / 64];
  double ay = 0.0, ax = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < n; i += int64_t(gridDim.x) * NT) {
    const double v = dinv[i] * t[i];
    y[i] = v;
    ay += v * v;
    ax += x[i] * x[i];
  }
  // fixed-order workgroup sums (wave shuffles, then the four waves in order)
  for (int o = 32; o > 0; o >>= 1) {
    ay += __shfl_xor(ay, o);
    ax += __shfl_xor(ax, o);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = ay;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = sh[0];
    for (int w = 1; w < NT / 64; ++w) s += sh[w];
    red[blockIdx.x] = s;
  }
  __syncthreads();
  if (lane == 0) sh[wid] = ax;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = sh[0];
    for (int w = 1; w < NT / 64; ++w) s += sh[w];
    red[VGRID_MAX + blockIdx.x] = s;
  }
}

__global__ __launch_bounds__(NT) void k_power_scale(const double *y, const double *s, double *x,
                                                    int64_t n) {
  const double f = 1.0 / sqrt(s[0]);
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < n; i += int64_t(gridDim.x) * NT)
    x[i] = y[i] * f;
}

// Sum over a wave64 in a fixed butterfly order (the same on every run).
template <typename T>
__device__ __forceinline__ T wave_total(T s) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  return s;
}

// Chebyshev smoother on the finest level.  First step from x = 0:
// d = D^-1 b / theta, x = d.  Any other step, with t = A x:
// d <- cd d + cr D^-1 (b - t), x += d (cd = 0 restarts the recurrence);
// with red set also the per-workgroup partials of b . x (the r.z of CG).
template <typename T>
__global__ __launch_bounds__(NT) void k_cheb_first(T *x, T *d, const T *b, const T *dinv,
                                                   T inv_theta, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < n; i += int64_t(gridDim.x) * NT) {
    const T di = inv_theta * (dinv[i] * b[i]);
    d[i] = di;
    x[i] = di;
  }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_cheb_step(T *x, T *d, const T *b, const T *t,
                                                  const T *dinv, T cd, T cr, int64_t n,
                                                  double *red) {
  __shared__ double sh[NT / 64];
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * NT + threadIdx.x; i < n; i += int64_t(gridDim.x) * NT) {
    const T r = dinv[i] * (b[i] - t[i]);
    const T di = cd == T(0) ? cr * r : cd * d[i] + cr * r;
    d[i] = di;
    const T xi = x[i] + di;
    x[i] = xi;
    acc += double(b[i]) * double(xi);
  }
  if (!red) return;
  acc = wave_total(acc);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = sh[0];
    for (int k = 1; k < NT / 64; ++k) s += sh[k];
    red[blockIdx.x] = s;
  }
}

// t = A x for a coarse level's operator (the power estimate of its Jacobi
// weight): one wave per row, fixed-order wave sum.
__global__ __launch_bounds__(NT) void k_csr_mv(double *t, const double *x, const int32_t *rp,
                                               const int32_t *ci, const double *v, int64_t n) {
  const int lane = threadIdx.x & 63;
  const int64_t w0 = (int64_t(blockIdx.x) * NT + threadIdx.x) >> 6;
  const int64_t nw = (int64_t(gridDim.x) * NT) >> 6;
  for (int64_t i = w0; i < n; i += nw) {
    double s = 0.0;
    for (int32_t q = rp[i] + lane; q < rp[i + 1]; q += 64) s += v[q] * x[ci[q]];
    s = wave_total(s);
    if (lane == 0) t[i] = s;
  }
}

// Coarse-level kernels run one wave per row (rows of the coarse operators
// hold ~100 entries and there are only a few thousand rows: a thread per row
// would leave most of the chip idle); lanes stride over the row, then a
// fixed-order wave sum.

// Pre-smoothing from zero fused with the residual: x = w D^-1 b and
// r = b - A x, the x_j formed in place from b_j (the same arithmetic as the
// separate smoothing step, so the result is identical).
template <typename T>
__global__ __launch_bounds__(NT) void k_csr_pre(T *x, T *r, const T *b, const T *dinv, T w,
                                                const int32_t *rp, const int32_t *ci, const T *v,
                                                int64_t n) {
  const int lane = threadIdx.x & 63;
  const int64_t w0 = (int64_t(blockIdx.x) * NT + threadIdx.x) >> 6;
  const int64_t nw = (int64_t(gridDim.x) * NT) >> 6;
  for (int64_t i = w0; i < n; i += nw) {
    T s = T(0);
    for (int32_t q = rp[i] + lane; q < rp[i + 1]; q += 64) {
      const int32_t j = ci[q];
      s += v[q] * (w * (dinv[j] * b[j]));
    }
    s = wave_total(s);
    if (lane == 0) {
      x[i] = w * (dinv[i] * b[i]);
      r[i] = b[i] - s;
    }
  }
}

// Post-smoothing fused with its residual: xo = x + w D^-1 (b - A x) into a
// separate vector (other rows still read x).
template <typename T>
__global__ __launch_bounds__(NT) void k_csr_post(T *xo, const T *x, const T *b, const T *dinv,
                                                 T w, const int32_t *rp, const int32_t *ci,
                                                 const T *v, int64_t n) {
  const int lane = threadIdx.x & 63;
  const int64_t w0 = (int64_t(blockIdx.x) * NT + threadIdx.x) >> 6;
  const int64_t nw = (int64_t(gridDim.x) * NT) >> 6;
  for (int64_t i = w0; i < n; i += nw) {
    T s = T(0);
    for (int32_t q = rp[i] + lane; q < rp[i + 1]; q += 64) s += v[q] * x[ci[q]];
    s = wave_total(s);
    if (lane == 0) {
      const T r = b[i] - s;
      xo[i] = x[i] + w * (dinv[i] * r);
    }
  }
}

// One wave per coarse dof: the rows of its aggregate, strided over the lanes.
template <typename T>
__global__ __launch_bounds__(NT) void k_restrict(T *bc, const T *b, const T *t, AmgXfer<T> X) {
  const int lane = threadIdx.x & 63;
  const int64_t w0 = (int64_t(blockIdx.x) * NT + threadIdx.x) >> 6;
  const int64_t nw = (int64_t(gridDim.x) * NT) >> 6;
  for (int64_t R = w0; R < X.nc; R += nw) {
    const int i = X.ri[R];
    T s = T(0);
    for (int32_t q = X.rs[R] + lane; q < X.re[R]; q += 64) {
      const int64_t r = X.arows[q];
      const T v = t ? b[r] - t[r] : b[r];
      s += X.pv[6 * r + i] * v;
    }
    s = wave_total(s);
    if (lane == 0) bc[R] = s;
  }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_prolong(T *x, const T *xc, AmgXfer<T> X) {
  for (int64_t r = int64_t(blockIdx.x) * NT + threadIdx.x; r < X.n; r += int64_t(gridDim.x) * NT) {
    const int k = X.pk[r];
    if (k == 0) continue;
    const int32_t o = X.poff[r];
    T s = T(0);
    for (int i = 0; i < k; ++i) s += X.pv[6 * r + i] * xc[o + i];
    x[r] += s;
  }
}

// coarsest solve: one wave per row of the dense inverse
template <typename T>
__global__ __launch_bounds__(NT) void k_dense_mv(T *x, const T *A, const T *b, int64_t n) {
  const int lane = threadIdx.x & 63;
  const int64_t w0 = (int64_t(blockIdx.x) * NT + threadIdx.x) >> 6;
  const int64_t nw = (int64_t(gridDim.x) * NT) >> 6;
  for (int64_t i = w0; i < n; i += nw) {
    T s = T(0);
    const T *row = A + i * n;
    for (int64_t j = lane; j < n; j += 64) s += row[j] * b[j];
    s = wave_total(s);
    if (lane == 0) x[i] = s;
  }
}

template <typename T>
AmgXfer<T> typed(const AmgXfer<void> &X) {
  return AmgXfer<T>{X.poff, X.pk, static_cast<const T *>(X.pv), X.rs, X.re, X.ri, X.arows,
                    X.n, X.nc};
}

}  // namespace

hipError_t amg_probe_vec(Ctx *c, double *z, const double *pv0, const int32_t *pk0,
                         const int32_t *dcol, int colour, int k, int64_t n) {
  LAUNCH(k_probe, grid_for(n), z, pv0, pk0, dcol, colour, k, n);
  return hipGetLastError();
}

hipError_t amg_extract(Ctx *c, const double *y, const double *pv0, const AmgTasks &t, int k,
                       double *val) {
  if (t.n == 0) return hipSuccess;
  LAUNCH(k_extract, grid_for(t.n), y, pv0, t, k, val);
  return hipGetLastError();
}

hipError_t amg_csr_mv(Ctx *c, double *t, const double *x, const int32_t *rp, const int32_t *ci,
                      const double *v, int64_t n) {
  LAUNCH(k_csr_mv, grid_waves(n), t, x, rp, ci, v, n);
  return hipGetLastError();
}

int amg_power_partials(Ctx *c, const double *t, const double *dinv, const double *x, double *y,
                       int64_t n, double *red, hipError_t *err) {
  const int g = vgrid(n);
  LAUNCH(k_power, g, t, dinv, x, y, n, red);
  *err = hipGetLastError();
  return g;
}

hipError_t amg_power_scale(Ctx *c, const double *y, const double *s, double *x, int64_t n) {
  LAUNCH(k_power_scale, vgrid(n), y, s, x, n);
  return hipGetLastError();
}

hipError_t amg_cheb_first(Ctx *c, int prec, void *x, void *d, const void *b, const void *dinv,
                          double inv_theta, int64_t n) {
  if (prec == NLE_FP32)
    LAUNCH(k_cheb_first<float>, vgrid(n), static_cast<float *>(x), static_cast<float *>(d),
           static_cast<const float *>(b), static_cast<const float *>(dinv), float(inv_theta), n);
  else
    LAUNCH(k_cheb_first<double>, vgrid(n), static_cast<double *>(x), static_cast<double *>(d),
           static_cast<const double *>(b), static_cast<const double *>(dinv), inv_theta, n);
  return hipGetLastError();
}

int amg_cheb_step(Ctx *c, int prec, void *x, void *d, const void *b, const void *t,
                  const void *dinv, double cd, double cr, int64_t n, double *red,
                  hipError_t *err) {
  const int g = vgrid(n);
  if (prec == NLE_FP32)
    LAUNCH(k_cheb_step<float>, g, static_cast<float *>(x), static_cast<float *>(d),
           static_cast<const float *>(b), static_cast<const float *>(t),
           static_cast<const float *>(dinv), float(cd), float(cr), n, red);
  else
    LAUNCH(k_cheb_step<double>, g, static_cast<double *>(x), static_cast<double *>(d),
           static_cast<const double *>(b), static_cast<const double *>(t),
           static_cast<const double *>(dinv), cd, cr, n, red);
  *err = hipGetLastError();
  return g;
}

hipError_t amg_csr_pre(Ctx *c, int prec, void *x, void *r, const void *b, const void *dinv,
                       double w, const int32_t *rp, const int32_t *ci, const void *v, int64_t n) {
  if (prec == NLE_FP32)
    LAUNCH(k_csr_pre<float>, grid_waves(n), static_cast<float *>(x), static_cast<float *>(r),
           static_cast<const float *>(b), static_cast<const float *>(dinv), float(w), rp, ci,
           static_cast<const float *>(v), n);
  else
    LAUNCH(k_csr_pre<double>, grid_waves(n), static_cast<double *>(x), static_cast<double *>(r),
           static_cast<const double *>(b), static_cast<const double *>(dinv), w, rp, ci,
           static_cast<const double *>(v), n);
  return hipGetLastError();
}

hipError_t amg_csr_post(Ctx *c, int prec, void *xo, const void *x, const void *b,
                        const void *dinv, double w, const int32_t *rp, const int32_t *ci,
                        const void *v, int64_t n) {
  if (prec == NLE_FP32)
    LAUNCH(k_csr_post<float>, grid_waves(n), static_cast<float *>(xo),
           static_cast<const float *>(x), static_cast<const float *>(b),
           static_cast<const float *>(dinv), float(w), rp, ci, static_cast<const float *>(v), n);
  else
    LAUNCH(k_csr_post<double>, grid_waves(n), static_cast<double *>(xo),
           static_cast<const double *>(x), static_cast<const double *>(b),
           static_cast<const double *>(dinv), w, rp, ci, static_cast<const double *>(v), n);
  return hipGetLastError();
}

hipError_t amg_restrict(Ctx *c, int prec, void *bc, const void *b, const void *t,
                        const AmgXfer<void> &X) {
  if (prec == NLE_FP32)
    LAUNCH(k_restrict<float>, grid_waves(X.nc), static_cast<float *>(bc),
           static_cast<const float *>(b), static_cast<const float *>(t), typed<float>(X));
  else
    LAUNCH(k_restrict<double>, grid_waves(X.nc), static_cast<double *>(bc),
           static_cast<const double *>(b), static_cast<const double *>(t), typed<double>(X));
  return hipGetLastError();
}

hipError_t amg_prolong_add(Ctx *c, int prec, void *x, const void *xc, const AmgXfer<void> &X) {
  if (prec == NLE_FP32)
    LAUNCH(k_prolong<float>, grid_for(X.n), static_cast<float *>(x),
           static_cast<const float *>(xc), typed<float>(X));
  else
    LAUNCH(k_prolong<double>, grid_for(X.n), static_cast<double *>(x),
           static_cast<const double *>(xc), typed<double>(X));
  return hipGetLastError();
}

hipError_t amg_dense_mv(Ctx *c, int prec, void *x, const void *Ainv, const void *b, int64_t n) {
  if (prec == NLE_FP32)
    LAUNCH(k_dense_mv<float>, grid_waves(n), static_cast<float *>(x),
           static_cast<const float *>(Ainv), static_cast<const float *>(b), n);
  else
    LAUNCH(k_dense_mv<double>, grid_waves(n), static_cast<double *>(x),
           static_cast<const double *>(Ainv), static_cast<const double *>(b), n);
  return hipGetLastError();
}

}  // namespace nle
