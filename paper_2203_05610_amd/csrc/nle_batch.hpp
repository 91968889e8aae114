// Batched solver: declarations shared by the host driver and its kernels.
#pragma once

#include "nle_internal.hpp"

namespace nle {

constexpr int BS = 8;            // per-instance scalar stride of the batched CG
constexpr int64_t SEG = 4096;    // dofs per vector segment (one workgroup)

// Segment and instance tables on the device (passed by value to kernels).
struct BatchDev {
  int32_t n_inst = 0, nseg = 0, nblk = 0;
  const int32_t *seg_inst = nullptr;  // [nseg] instance of each segment
  const int64_t *seg_beg = nullptr;   // [nseg+1] first dof of each segment
  const int32_t *inst_seg = nullptr;  // [n_inst+1] segment offsets
  const int32_t *inst_blk = nullptr;  // [n_inst+1] element-block offsets
  const int32_t *inst_mwg = nullptr;  // [n_inst+1] merge-workgroup offsets
  // when set, a launch covers only the listed segments (one workgroup each)
  const int32_t *seg_list = nullptr;
  int32_t n_slist = 0;
};

struct BatchCg {
  int prec;
  void *x, *r, *z, *p, *Ap;
  const void *dinv;
  double *red_a;   // element partials of p.Ap (blocks, then merge workgroups)
  double *red_b;   // segment partials of (r.z, r.r): 2 x nseg
  double *scal;    // [n_inst][BS]
  int32_t *done;   // [n_inst] 0 running, 1 converged, 2 breakdown, 3 NaN, 5 limit
  int32_t *its;    // [n_inst]
};

hipError_t batch_reduce_elem(Ctx *c, const BatchDev &B, const double *red, double *out);
hipError_t batch_reduce_seg(Ctx *c, const BatchDev &B, const double *red, double *out);
hipError_t batch_scale(Ctx *c, const BatchDev &B, int px, const void *x, int py, void *y,
                       const double *coef);
hipError_t batch_axpy(Ctx *c, const BatchDev &B, int px, const void *x, int py, void *y,
                      const double *coef);
hipError_t batch_copy(Ctx *c, const BatchDev &B, const double *src, double *dst,
                      const int32_t *mask);
hipError_t batch_sub_norm(Ctx *c, const BatchDev &B, int prec, void *t, const void *b, double *red);
hipError_t batch_cg_start(Ctx *c, const BatchDev &B, const BatchCg &a, const void *b,
                          const double *rtol, const double *atol, const int32_t *active,
                          int max_it);
hipError_t batch_cg_step(Ctx *c, const BatchDev &B, const BatchCg &a);
// batched L-BFGS (pairs in per-instance ring slots of [m][stride] arrays)
hipError_t batch_dot_slot(Ctx *c, const BatchDev &B, int prec, const void *base, int64_t stride,
                          const int32_t *slot, const void *x, double *red);
hipError_t batch_axpy_slot(Ctx *c, const BatchDev &B, int px, const void *base, int64_t stride,
                           const int32_t *slot, int py, void *y, const double *coef);
hipError_t batch_store_slot(Ctx *c, const BatchDev &B, int prec, void *base, int64_t stride,
                            const int32_t *slot, const void *x, const double *coef);
hipError_t batch_lbfgs_pair(Ctx *c, const BatchDev &B, int prec, const void *Sbase, void *Ybase,
                            int64_t stride, const int32_t *slot, const double *g, const double *gp,
                            double *red);
hipError_t batch_lbfgs_coef(Ctx *c, int n, const double *rho, const double *dot, double *alpha,
                            double *coef, int second);

}  // namespace nle
