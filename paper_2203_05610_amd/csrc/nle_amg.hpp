// Aggregation multigrid: declarations shared by the host setup (nle_amg.cpp)
// and its kernels (nle_amgk.hip).
#pragma once

#include "nle_internal.hpp"

namespace nle {

// One level's transfer to the next coarser level (device arrays): every row r
// of this level belongs to one aggregate whose coarse dofs are
// poff[r] .. poff[r] + pk[r] - 1, with coefficients pv[6 r + i]; coarse dof
// R sums pv[6 r + ri[R]] over the rows arows[rs[R] .. re[R]) of its aggregate.
template <typename T>
struct AmgXfer {
  const int32_t *poff, *pk;
  const T *pv;
  const int32_t *rs, *re, *ri, *arows;
  int64_t n, nc;
};

// Probing tasks of one colour: coarse entry dest + k of the level-1 operator
// is the sum over nodes nodes[beg .. end) of pv0[3 n + d][kp] y[3 n + d].
struct AmgTasks {
  const int32_t *beg, *end, *kp, *ka;
  const int64_t *dest;
  const int32_t *nodes;
  int32_t n;
};

hipError_t amg_probe_vec(Ctx *c, double *z, const double *pv0, const int32_t *pk0,
                         const int32_t *dcol, int colour, int k, int64_t n);
hipError_t amg_extract(Ctx *c, const double *y, const double *pv0, const AmgTasks &t, int k,
                       double *val);
// t = A x for a coarse level's CSR operator (FP64)
hipError_t amg_csr_mv(Ctx *c, double *t, const double *x, const int32_t *rp, const int32_t *ci,
                      const double *v, int64_t n);
// y = dinv * t; partials of y.y at red[0..g) and x.x at red[VGRID_MAX..)
int amg_power_partials(Ctx *c, const double *t, const double *dinv, const double *x, double *y,
                       int64_t n, double *red, hipError_t *err);
// x = y / sqrt(*s)
hipError_t amg_power_scale(Ctx *c, const double *y, const double *s, double *x, int64_t n);

// V-cycle pieces (prec: NLE_FP64 or NLE_FP32, vectors and matrices in it)
// Chebyshev smoother steps on the finest level: first from x = 0 (x = d =
// D^-1 b / theta), then d <- cd d + cr D^-1 (b - t), x += d, with the
// per-workgroup partials of b . x at red[0 .. vgrid(n)) (if not null; returns the count)
hipError_t amg_cheb_first(Ctx *c, int prec, void *x, void *d, const void *b, const void *dinv,
                          double inv_theta, int64_t n);
int amg_cheb_step(Ctx *c, int prec, void *x, void *d, const void *b, const void *t,
                  const void *dinv, double cd, double cr, int64_t n, double *red,
                  hipError_t *err);
// coarse-level smoothing fused with the sparse residual:
// pre: x = w D^-1 b, r = b - A x;  post: xo = x + w D^-1 (b - A x) (xo != x)
hipError_t amg_csr_pre(Ctx *c, int prec, void *x, void *r, const void *b, const void *dinv,
                       double w, const int32_t *rp, const int32_t *ci, const void *v, int64_t n);
hipError_t amg_csr_post(Ctx *c, int prec, void *xo, const void *x, const void *b,
                        const void *dinv, double w, const int32_t *rp, const int32_t *ci,
                        const void *v, int64_t n);
// bc = P^T (b - t) (t may be null: bc = P^T b)
hipError_t amg_restrict(Ctx *c, int prec, void *bc, const void *b, const void *t,
                        const AmgXfer<void> &X);
// x += P xc
hipError_t amg_prolong_add(Ctx *c, int prec, void *x, const void *xc, const AmgXfer<void> &X);
// x = Ainv b (dense, row-major n x n)
hipError_t amg_dense_mv(Ctx *c, int prec, void *x, const void *Ainv, const void *b, int64_t n);

}  // namespace nle
