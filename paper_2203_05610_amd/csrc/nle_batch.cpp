// Batched solver: many independent quasi-static problems (uneven meshes,
// materials and loads) solved together.  The instances form one disjoint-union
// mesh; every launch (residual, linearization, Jacobian action, CG step)
// covers all of them, while every decision (Newton convergence, Krylov
// tolerance, step length, load-step cutback) is taken per instance.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <new>

#include "nle_batch.hpp"

namespace nle {

nle_status read_scalars(Ctx *c, const void *dev, size_t bytes);
nle_status linearize(Ctx *c, const double *u, int prec);
nle_status jv(Ctx *c, const void *v, void *y, int prec);

namespace {

struct Inst {
  std::vector<double> X;
  std::vector<int32_t> conn;
  double params[3] = {0, 0, 0.25};
  std::vector<int64_t> ddofs;
  std::vector<double> dvals;
  std::vector<int32_t> tri;
  double t[3] = {0, 0, 0};
  std::vector<double> scales;
};

struct Batch {
  nle_ctx *ctx = nullptr;
  Ctx *c = nullptr;
  int32_t kind = 0;
  std::vector<Inst> inst;
  bool finalized = false;
  std::string err;
  BatchDev B;
  std::vector<int64_t> node_off;
  std::vector<int32_t> h_inst_seg;  // [n_inst+1] segment offsets
  std::vector<void *> allocs;
  // per-instance device arrays
  double *d_coef = nullptr, *d_rtol = nullptr, *d_atol = nullptr, *d_out = nullptr;
  double *d_kscal = nullptr;
  int32_t *d_mask = nullptr, *d_active = nullptr, *d_kdone = nullptr, *d_kits = nullptr;
  int32_t *d_inv = nullptr;
  // work lists of the instances taking a Newton step (blocks, merge
  // workgroups, segments), rebuilt every round
  int32_t *d_blist = nullptr, *d_mlist = nullptr, *d_slist = nullptr;
  double *h_pin = nullptr;  // pinned host staging, 16 n_inst doubles
};

nle_status bfail(Batch *b, nle_status s, const std::string &m) {
  if (b) b->err = m;
  return s;
}

#define BHIP(b, call)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess) return bfail((b), NLE_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <typename T>
T *bupload(Batch *b, const std::vector<T> &h, hipError_t *e) {
  T *d = static_cast<T *>(dalloc(b->c, std::max<size_t>(h.size(), 1) * sizeof(T)));
  if (!d) {
    *e = hipErrorOutOfMemory;
    return nullptr;
  }
  b->allocs.push_back(d);
  if (!h.empty()) {
    hipError_t r = hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, b->c->stream);
    if (r != hipSuccess) *e = r;
  }
  return d;
}

template <typename T>
T *balloc(Batch *b, size_t n, hipError_t *e) {
  T *d = static_cast<T *>(dalloc(b->c, std::max<size_t>(n, 1) * sizeof(T)));
  if (!d) *e = hipErrorOutOfMemory;
  b->allocs.push_back(d);
  return d;
}

nle_status finalize(Batch *b) {
  Ctx *c = b->c;
  const int32_t n = int32_t(b->inst.size());
  if (n < 1) return bfail(b, NLE_E_STATE, "empty batch");
  std::vector<int64_t> ie(n + 1, 0), in(n + 1, 0);
  for (int32_t i = 0; i < n; ++i) {
    ie[i + 1] = ie[i] + int64_t(b->inst[i].conn.size() / 4);
    in[i + 1] = in[i] + int64_t(b->inst[i].X.size() / 3);
  }
  const int64_t ne = ie[n], nn = in[n];
  std::vector<double> X(3 * nn);
  std::vector<int32_t> conn(4 * ne);
  for (int32_t i = 0; i < n; ++i) {
    std::copy(b->inst[i].X.begin(), b->inst[i].X.end(), X.begin() + 3 * in[i]);
    for (size_t k = 0; k < b->inst[i].conn.size(); ++k)
      conn[4 * ie[i] + k] = int32_t(b->inst[i].conn[k] + in[i]);
  }
  if (nn >= (int64_t(1) << 28) || ne >= (int64_t(1) << 31))
    return bfail(b, NLE_E_UNSUPPORTED, "batch too large");
  c->has_mesh = false;
  drop_graph(c);
  nle_status s = build_mesh(c, nn, X.data(), ne, conn.data(), &ie, &in);
  if (s != NLE_OK) return bfail(b, s, c->err);
  // Dirichlet mask and values of the union
  std::vector<int64_t> dd;
  std::vector<double> dv;
  for (int32_t i = 0; i < n; ++i)
    for (size_t k = 0; k < b->inst[i].ddofs.size(); ++k) {
      dd.push_back(b->inst[i].ddofs[k] + 3 * in[i]);
      dv.push_back(b->inst[i].dvals[k]);
    }
  c->has_mesh = true;
  s = nle_set_dirichlet(b->ctx, int64_t(dd.size()), dd.data(), dv.data());
  if (s != NLE_OK) return bfail(b, s, c->err);
  // dead tractions of every instance
  std::vector<double> f(3 * nn, 0.0);
  for (int32_t i = 0; i < n; ++i) {
    const Inst &I = b->inst[i];
    for (size_t k = 0; k + 2 < I.tri.size(); k += 3) {
      const int32_t v[3] = {I.tri[k], I.tri[k + 1], I.tri[k + 2]};
      double e1[3], e2[3];
      for (int q = 0; q < 3; ++q) {
        e1[q] = I.X[3 * v[1] + q] - I.X[3 * v[0] + q];
        e2[q] = I.X[3 * v[2] + q] - I.X[3 * v[0] + q];
      }
      const double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2],
                   cz = e1[0] * e2[1] - e1[1] * e2[0];
      const double area = 0.5 * std::sqrt(cx * cx + cy * cy + cz * cz);
      for (int a = 0; a < 3; ++a)
        for (int q = 0; q < 3; ++q) f[3 * (in[i] + v[a]) + q] += I.t[q] * area / 3.0;
    }
  }
  BHIP(b, hipMemcpyAsync(c->fext, f.data(), f.size() * 8, hipMemcpyHostToDevice, c->stream));
  c->h_ftrac = f;
  // material
  MatParams m{};
  m.kind = b->kind;
  m.mu = b->inst[0].params[0];
  m.lam = b->inst[0].params[1];
  m.cvol = b->inst[0].params[2];
  m.kappa = m.lam + 2.0 * m.mu / 3.0;
  c->mat = m;
  c->has_mat = true;
  std::vector<double> mat(4 * n);
  for (int32_t i = 0; i < n; ++i) {
    mat[4 * i] = b->inst[i].params[0];
    mat[4 * i + 1] = b->inst[i].params[1];
    mat[4 * i + 2] = b->inst[i].params[2];
    mat[4 * i + 3] = b->inst[i].params[1] + 2.0 * b->inst[i].params[0] / 3.0;
  }
  // segments (instance-aligned)
  std::vector<int32_t> seg_inst, inst_seg(n + 1, 0);
  std::vector<int64_t> seg_beg;
  for (int32_t i = 0; i < n; ++i) {
    for (int64_t d = 3 * in[i]; d < 3 * in[i + 1]; d += SEG) {
      seg_inst.push_back(i);
      seg_beg.push_back(d);
    }
    inst_seg[i + 1] = int32_t(seg_inst.size());
  }
  seg_beg.push_back(3 * nn);
  for (void *p : b->allocs) dfree(c, p);
  b->allocs.clear();
  hipError_t e = hipSuccess;
  b->B.n_inst = n;
  b->B.nseg = int32_t(seg_inst.size());
  b->B.nblk = c->m.nblk;
  b->B.seg_inst = bupload(b, seg_inst, &e);
  b->B.seg_beg = bupload(b, seg_beg, &e);
  b->B.inst_seg = bupload(b, inst_seg, &e);
  b->h_inst_seg = inst_seg;
  b->B.inst_blk = bupload(b, c->m.h_inst_blk, &e);
  b->B.inst_mwg = bupload(b, c->m.h_inst_mwg, &e);
  c->inst_mat = bupload(b, mat, &e);
  c->inst_s = balloc<double>(b, n, &e);
  c->inst_inv = balloc<int32_t>(b, n, &e);
  b->d_coef = balloc<double>(b, n, &e);
  b->d_rtol = balloc<double>(b, n, &e);
  b->d_atol = balloc<double>(b, n, &e);
  b->d_out = balloc<double>(b, 4 * n, &e);
  b->d_kscal = balloc<double>(b, size_t(BS) * n, &e);
  b->d_mask = balloc<int32_t>(b, n, &e);
  b->d_active = balloc<int32_t>(b, n, &e);
  b->d_kdone = balloc<int32_t>(b, n, &e);
  b->d_kits = balloc<int32_t>(b, n, &e);
  b->d_blist = balloc<int32_t>(b, size_t(std::max(1, c->m.nblk)), &e);
  b->d_mlist = balloc<int32_t>(b, size_t(std::max(1, c->m.n_mwg)), &e);
  b->d_slist = balloc<int32_t>(b, size_t(std::max(1, b->B.nseg)), &e);
  if (e != hipSuccess) return bfail(b, NLE_E_OOM, "batch allocation failed");
  // reduction space: element partials (blocks + merge workgroups) and segments
  const int64_t need = int64_t(elem_red_capacity(c)) + 4 * int64_t(b->B.nseg) + 64;
  if (need > c->red_cap) {
    dfree(c, c->red);
    c->red = static_cast<double *>(dalloc(c, size_t(need) * 8));
    if (!c->red) return bfail(b, NLE_E_OOM, "batch allocation failed");
    c->red_cap = need;
  }
  if (b->h_pin) (void)hipHostFree(b->h_pin);
  BHIP(b, hipHostMalloc(&b->h_pin, size_t(16) * n * 8));
  b->node_off = in;
  BHIP(b, hipStreamSynchronize(c->stream));
  b->finalized = true;
  return NLE_OK;
}

// Element-block size for the batch: re-partition the union mesh with each
// candidate and time the whole batch's Jacobian action (precision prec, at the
// lifted zero state), keeping the fastest.
nle_status autotune(Batch *b, int prec, double budget_ms, int32_t *chosen) {
  Ctx *c = b->c;
  const int32_t cand[] = {128, 256, 512, 1024};
  const int ncand = 4;
  const int64_t nd = 3 * c->m.n_nodes;
  const size_t es = prec == NLE_FP32 ? 4 : 8;
  double *u = static_cast<double *>(dalloc(c, size_t(nd) * 8));
  void *v = dalloc(c, size_t(nd) * es);
  void *y = dalloc(c, size_t(nd) * es);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  struct Free {
    Ctx *c;
    void *p[3];
    hipEvent_t *e[2];
    ~Free() {
      for (void *q : p) dfree(c, q);
      for (hipEvent_t *q : e)
        if (*q) (void)hipEventDestroy(*q);
    }
  } fr{c, {u, v, y}, {&e0, &e1}};
  if (!u || !v || !y) return bfail(b, NLE_E_OOM, "autotune allocation failed");
  BHIP(b, hipEventCreate(&e0));
  BHIP(b, hipEventCreate(&e1));
  const int32_t be0 = c->be_req;
  int32_t best = -1, current = -1;  // fastest so far, partition now in place
  double best_ms = 0.0;
  for (int k = 0; k < ncand; ++k) {
    c->be_req = cand[k];
    b->finalized = false;
    nle_status s = finalize(b);
    if (s == NLE_E_UNSUPPORTED) continue;  // the block's LDS need exceeds the device's
    if (s != NLE_OK) {
      c->be_req = be0;
      return s;
    }
    current = cand[k];
    BHIP(b, vec_fill(c, NLE_FP64, u, 0.0, nd));
    BHIP(b, vec_lift(c, u));
    s = linearize(c, u, prec);
    if (s != NLE_OK) return bfail(b, s, c->err);
    BHIP(b, vec_fill(c, prec, v, 1.0, nd));
    hipError_t e = hipSuccess;
    for (int w = 0; w < 2 && e == hipSuccess; ++w) elem_apply(c, OP_JV, prec, prec == NLE_FP32 ? (const void *)c->ulin32 : (const void *)c->ulin64, v, y, nullptr, &e);
    // one timed call sizes the repetition count to this candidate's share
    int reps = 1;
    float ms = 0.0f;
    for (int pass = 0; pass < 2 && e == hipSuccess; ++pass) {
      BHIP(b, hipEventRecord(e0, c->stream));
      for (int r = 0; r < reps && e == hipSuccess; ++r)
        elem_apply(c, OP_JV, prec, prec == NLE_FP32 ? (const void *)c->ulin32 : (const void *)c->ulin64, v, y, nullptr, &e);
      BHIP(b, hipEventRecord(e1, c->stream));
      BHIP(b, hipEventSynchronize(e1));
      BHIP(b, hipEventElapsedTime(&ms, e0, e1));
      if (pass == 0) {
        const double share = budget_ms / ncand;
        reps = int(std::min(200.0, std::max(3.0, share / std::max(double(ms), 1e-3))));
      }
    }
    if (e != hipSuccess) return bfail(b, NLE_E_HIP, std::string("autotune: ") + hipGetErrorString(e));
    const double per = double(ms) / reps;
    if (best < 0 || per < best_ms) {
      best = cand[k];
      best_ms = per;
    }
  }
  if (best < 0) {
    c->be_req = be0;
    b->finalized = false;
    nle_status s = finalize(b);
    return s != NLE_OK ? s : bfail(b, NLE_E_UNSUPPORTED, "no block size fits the device");
  }
  c->be_req = best;
  if (best != current) {
    b->finalized = false;
    nle_status s = finalize(b);
    if (s != NLE_OK) return s;
  }
  c->lin64 = c->lin32 = c->lc_valid = false;
  if (chosen) *chosen = best;
  return NLE_OK;
}

// Per-instance state of the outer loop.
struct IState {
  int step = 0;           // index of the next scheduled load scale
  double s_prev = 0.0;    // last converged load scale
  double s_cur = 0.0;     // load scale being solved
  bool need_r0 = true;
  bool finished = false;
  bool newton = false;    // takes a Newton step this round
  double r0 = 0, rn = 0, rn_prev = 0, linres = 0, eta_prev = 0, eta = 0;
  int k = 0;              // Newton iterations in the current load step
  int cuts = 0;
  int nit = 0;
  int64_t lit = 0, njv = 0, nres = 0;
  int status = NLE_OK;
};

nle_status solve(Batch *b, int method, const nle_solver_opts &o, double *u, nle_report *reports,
                 double *t_ms) {
  Ctx *c = b->c;
  const int32_t n = b->B.n_inst;
  const int prec = o.precision == NLE_PREC_MIXED ? NLE_FP32 : NLE_FP64;
  const size_t es = prec == NLE_FP32 ? 4 : 8;
  const int64_t nd = 3 * c->m.n_nodes;
  const bool inexact = method == NLE_INK;
  const int max_cuts = 8;
  // workspace: r, backup (double); b, dx, tmp, CG r z p Ap (prec)
  const size_t v64 = (size_t(nd) * 8 + 255) & ~size_t(255), vp = (size_t(nd) * es + 255) & ~size_t(255);
  if (c->ws_bytes < 2 * v64 + 7 * vp) {
    drop_graph(c);
    for (void *p : c->ws_allocs) dfree(c, p);
    c->ws_allocs.clear();
    c->ws = dalloc(c, 2 * v64 + 7 * vp);
    if (!c->ws) {
      c->ws_bytes = 0;
      return bfail(b, NLE_E_OOM, "batch workspace allocation failed");
    }
    c->ws_allocs.push_back(c->ws);
    c->ws_bytes = 2 * v64 + 7 * vp;
  }
  char *w = static_cast<char *>(c->ws);
  double *r = reinterpret_cast<double *>(w);
  double *ub = reinterpret_cast<double *>(w + v64);
  void *bv = w + 2 * v64, *dx = w + 2 * v64 + vp, *tmp = w + 2 * v64 + 2 * vp;
  BatchCg cg;
  cg.prec = prec;
  cg.x = dx;
  cg.r = w + 2 * v64 + 3 * vp;
  cg.z = w + 2 * v64 + 4 * vp;
  cg.p = w + 2 * v64 + 5 * vp;
  cg.Ap = w + 2 * v64 + 6 * vp;
  cg.dinv = prec == NLE_FP32 ? static_cast<const void *>(c->dinv32) : static_cast<const void *>(c->dinv64);
  const int cap = elem_red_capacity(c);
  cg.red_a = c->red;
  cg.red_b = c->red + cap;
  cg.scal = b->d_kscal;
  cg.done = b->d_kdone;
  cg.its = b->d_kits;
  const void *ulin = prec == NLE_FP32 ? static_cast<const void *>(c->ulin32) : static_cast<const void *>(c->ulin64);

  hipEvent_t e0, e1;
  BHIP(b, hipEventCreate(&e0));
  BHIP(b, hipEventCreate(&e1));
  BHIP(b, hipEventRecord(e0, c->stream));
  std::vector<IState> S(n);
  for (int32_t i = 0; i < n; ++i) {
    S[i].s_cur = b->inst[i].scales.empty() ? 1.0 : b->inst[i].scales[0];
    if (b->inst[i].scales.empty()) S[i].finished = true;
  }
  NLE_HIP(c, vec_lift(c, u));
  BHIP(b, hipMemcpyAsync(ub, u, size_t(nd) * 8, hipMemcpyDeviceToDevice, c->stream));
  std::vector<double> hs(n), hcoef(n), hrtol(n), hatol(n);
  std::vector<int32_t> hmask(n), hact(n);
  std::vector<int32_t> hblist, hmlist, hslist;
  const std::vector<int32_t> &hinst_seg = b->h_inst_seg;
  auto upload_d = [&](double *dst, const std::vector<double> &v) {
    return hipMemcpyAsync(dst, v.data(), size_t(n) * 8, hipMemcpyHostToDevice, c->stream);
  };
  auto upload_i = [&](int32_t *dst, const std::vector<int32_t> &v) {
    return hipMemcpyAsync(dst, v.data(), size_t(n) * 4, hipMemcpyHostToDevice, c->stream);
  };
  nle_status st = NLE_OK;
  for (int round = 0; round < 100000; ++round) {
    bool any = false;
    for (int32_t i = 0; i < n; ++i) any |= !S[i].finished;
    if (!any) break;
    // ---- residuals of all unfinished instances ---------------------------
    for (int32_t i = 0; i < n; ++i) {
      hs[i] = S[i].s_cur;
      hmask[i] = S[i].finished ? 1 : 0;
    }
    BHIP(b, upload_d(c->inst_s, hs));
    BHIP(b, upload_i(b->d_mask, hmask));
    BHIP(b, hipMemsetAsync(c->inst_inv, 0, size_t(n) * 4, c->stream));
    c->inst_done = b->d_mask;
    hipError_t e;
    elem_apply(c, OP_RES, NLE_FP64, u, nullptr, r, c->red, &e);
    if (e != hipSuccess) return bfail(b, NLE_E_HIP, "batched residual");
    BHIP(b, batch_reduce_elem(c, b->B, c->red, b->d_out));
    BHIP(b, hipMemcpyAsync(b->h_pin, b->d_out, size_t(n) * 8, hipMemcpyDeviceToHost, c->stream));
    BHIP(b, hipMemcpyAsync(b->h_pin + n, c->inst_inv, size_t(n) * 4, hipMemcpyDeviceToHost, c->stream));
    BHIP(b, hipStreamSynchronize(c->stream));
    c->inst_done = nullptr;
    const int32_t *inv = reinterpret_cast<const int32_t *>(b->h_pin + n);
    // ---- per-instance decisions --------------------------------------------
    std::vector<int32_t> restore(n, 0), save(n, 0);
    bool any_newton = false;
    for (int32_t i = 0; i < n; ++i) {
      IState &I = S[i];
      I.newton = false;
      if (I.finished) continue;
      I.nres += 1;
      const double rn = std::sqrt(b->h_pin[i]);
      bool failed = inv[i] != 0 || !std::isfinite(rn);
      if (!failed && I.need_r0) {
        I.r0 = rn;
        I.need_r0 = false;
        I.k = 0;
      }
      const double tol = std::max(o.snes_rtol * I.r0, o.snes_atol);
      if (!failed && rn <= tol) {  // load step converged
        // after a cutback the converged scale lies below the scheduled one,
        // which is then tried again
        const std::vector<double> &sc = b->inst[i].scales;
        save[i] = 1;
        I.s_prev = I.s_cur;
        I.rn = rn;
        while (I.step < int(sc.size()) && sc[I.step] <= I.s_cur) I.step += 1;
        if (I.step >= int(sc.size())) {
          I.finished = true;
          I.status = NLE_OK;
        } else {
          I.s_cur = sc[I.step];
          I.need_r0 = true;
        }
        continue;
      }
      if (!failed && I.k >= o.snes_max_it) failed = true;
      if (failed) {  // restore the last converged state and halve the increment
        restore[i] = 1;
        if (I.cuts >= max_cuts) {
          I.finished = true;
          I.status = inv[i] ? NLE_DIVERGED_INVERTED : (std::isfinite(rn) ? NLE_DIVERGED_MAXIT : NLE_DIVERGED_NAN);
          continue;
        }
        I.cuts += 1;
        I.s_cur = 0.5 * (I.s_prev + I.s_cur);
        I.need_r0 = true;
        continue;
      }
      // Newton step for this instance
      I.newton = true;
      any_newton = true;
      double eta = o.ksp_rtol, atol = o.ksp_atol;
      if (inexact) {
        if (I.k == 0) {
          eta = std::min(o.ew_rtol0, o.ew_rtolmax);
        } else if (o.ew_version == 2) {
          eta = o.ew_gamma * std::pow(rn / I.rn_prev, o.ew_alpha);
          const double stol = o.ew_gamma * std::pow(I.eta_prev, o.ew_alpha);
          if (stol > o.ew_threshold) eta = std::max(eta, stol);
        } else {
          eta = std::fabs(rn - I.linres) / I.rn_prev;
          const double stol = std::pow(I.eta_prev, o.ew_alpha2);
          if (stol > o.ew_threshold) eta = std::max(eta, stol);
        }
        eta = std::max(std::min(eta, o.ew_rtolmax), o.ew_rtolmin);
        if (prec == NLE_FP32) eta = std::max(eta, 1e-4);  // FP32 Krylov floor
        atol = o.ink_ksp_atol;
      }
      I.eta = eta;
      I.rn = rn;
      hrtol[i] = eta;
      hatol[i] = atol / rn;
    }
    // backups / restores of whole instances
    bool any_r = false, any_s = false;
    for (int32_t i = 0; i < n; ++i) {
      any_r |= restore[i] != 0;
      any_s |= save[i] != 0;
    }
    if (any_r) {
      BHIP(b, upload_i(b->d_mask, restore));
      BHIP(b, batch_copy(c, b->B, ub, u, b->d_mask));
    }
    if (any_s) {
      BHIP(b, upload_i(b->d_mask, save));
      BHIP(b, batch_copy(c, b->B, u, ub, b->d_mask));
    }
    if (!any_newton) continue;
    // ---- linearize (all instances; the cost is one pass) --------------------
    for (int32_t i = 0; i < n; ++i) hact[i] = S[i].newton ? 1 : 0;
    for (int32_t i = 0; i < n; ++i) hmask[i] = S[i].newton ? 0 : 1;
    BHIP(b, upload_i(b->d_mask, hmask));
    c->inst_done = b->d_mask;
    st = linearize(c, u, prec);
    c->inst_done = nullptr;
    if (st != NLE_OK) return bfail(b, st, c->err);
    // b = -r / ||r_i||
    for (int32_t i = 0; i < n; ++i) hcoef[i] = S[i].newton ? -1.0 / S[i].rn : 0.0;
    BHIP(b, upload_d(b->d_coef, hcoef));
    BHIP(b, batch_scale(c, b->B, NLE_FP64, r, prec, bv, b->d_coef));
    BHIP(b, upload_d(b->d_rtol, hrtol));
    BHIP(b, upload_d(b->d_atol, hatol));
    BHIP(b, upload_i(b->d_active, hact));
    // ---- batched CG ------------------------------------------------------------
    BHIP(b, batch_cg_start(c, b->B, cg, bv, b->d_rtol, b->d_atol, b->d_active, o.ksp_max_it));
    // The iterations launch only the work of the instances still iterating
    // (blocks, merge workgroups, segments from per-round lists): instances
    // take very different iteration counts, and the lists are rebuilt (and
    // the chunk graph recaptured) whenever the listed blocks could halve.
    BatchDev BL = b->B;
    BL.seg_list = b->d_slist;
    struct ClearLists {
      Ctx *c;
      ~ClearLists() {
        c->blk_list = c->mwg_list = nullptr;
        c->n_blist = c->n_mlist = 0;
      }
    } clear_lists{c};
    auto set_lists = [&](const int32_t *done) -> hipError_t {
      hblist.clear();
      hmlist.clear();
      hslist.clear();
      for (int32_t i = 0; i < n; ++i) {
        if (!S[i].newton || (done && done[i] != 0)) continue;
        for (int32_t q = c->m.h_inst_blk[i]; q < c->m.h_inst_blk[i + 1]; ++q) hblist.push_back(q);
        for (int32_t q = c->m.h_inst_mwg[i]; q < c->m.h_inst_mwg[i + 1]; ++q) hmlist.push_back(q);
        for (int32_t q = hinst_seg[i]; q < hinst_seg[i + 1]; ++q) hslist.push_back(q);
      }
      hipError_t r = hipSuccess;
      if (!hblist.empty())
        r = hipMemcpyAsync(b->d_blist, hblist.data(), hblist.size() * 4, hipMemcpyHostToDevice,
                           c->kstream);
      if (r == hipSuccess && !hmlist.empty())
        r = hipMemcpyAsync(b->d_mlist, hmlist.data(), hmlist.size() * 4, hipMemcpyHostToDevice,
                           c->kstream);
      if (r == hipSuccess && !hslist.empty())
        r = hipMemcpyAsync(b->d_slist, hslist.data(), hslist.size() * 4, hipMemcpyHostToDevice,
                           c->kstream);
      BL.n_slist = int32_t(hslist.size());
      c->blk_list = b->d_blist;
      c->n_blist = int32_t(hblist.size());
      c->mwg_list = b->d_mlist;
      c->n_mlist = int32_t(hmlist.size());
      return r;
    };
    auto iter = [&]() -> hipError_t {
      hipError_t err;
      elem_apply(c, OP_JV, prec, ulin, cg.p, cg.Ap, nullptr, &err);
      if (err != hipSuccess) return err;
      return batch_cg_step(c, BL, cg);
    };
    const int chunk = std::max(1, o.check_every);
    auto ensure_graph = [&]() -> nle_status {
      std::vector<uint64_t> key = {7, uint64_t(prec), uint64_t(nd), uint64_t(chunk),
                                   uint64_t(uintptr_t(c->ws)), uint64_t(uintptr_t(c->red)),
                                   uint64_t(uintptr_t(ulin)),
                                   uint64_t(uintptr_t(c->lc_valid ? c->lc64 : nullptr)),
                                   uint64_t(hblist.size()), uint64_t(hmlist.size()),
                                   uint64_t(hslist.size()), uint64_t(uintptr_t(b->d_blist))};
      if (c->gkey == key) return NLE_OK;
      drop_graph(c);
      c->inst_done = b->d_kdone;
      c->ep.w = nullptr;
      c->ep.coef = nullptr;
      c->ep.red = cg.red_a;
      hipError_t eb = hipStreamBeginCapture(c->kstream, hipStreamCaptureModeThreadLocal);
      if (eb != hipSuccess) {
        c->inst_done = nullptr;
        c->ep.red = nullptr;
        return bfail(b, NLE_E_HIP, "capture");
      }
      hipStream_t user = c->stream;
      c->stream = c->kstream;
      hipError_t ei = hipSuccess;
      for (int q = 0; q < chunk && ei == hipSuccess; ++q) ei = iter();
      c->stream = user;
      hipGraph_t g = nullptr;
      hipError_t ee = hipStreamEndCapture(c->kstream, &g);
      c->inst_done = nullptr;
      c->ep.red = nullptr;
      if (ei != hipSuccess || ee != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return bfail(b, NLE_E_HIP, "batched CG capture");
      }
      hipGraphExec_t ex = nullptr;
      if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return bfail(b, NLE_E_HIP, "batched CG instantiate");
      }
      c->graph = g;
      c->gexec = ex;
      c->gkey = key;
      return NLE_OK;
    };
    BHIP(b, hipEventRecord(c->ev_a, c->stream));
    BHIP(b, hipStreamWaitEvent(c->kstream, c->ev_a, 0));
    BHIP(b, set_lists(nullptr));
    {
      const nle_status sg = ensure_graph();
      if (sg != NLE_OK) return sg;
    }
    for (int done_its = 0; done_its < o.ksp_max_it; done_its += chunk) {
      BHIP(b, hipGraphLaunch(c->gexec, c->kstream));
      BHIP(b, hipMemcpyAsync(b->h_pin, b->d_kdone, size_t(n) * 4, hipMemcpyDeviceToHost, c->kstream));
      BHIP(b, hipStreamSynchronize(c->kstream));
      const int32_t *dn = reinterpret_cast<const int32_t *>(b->h_pin);
      bool all = true;
      size_t left = 0;
      for (int32_t i = 0; i < n; ++i) {
        all &= dn[i] != 0;
        if (S[i].newton && dn[i] == 0)
          left += size_t(c->m.h_inst_blk[i + 1] - c->m.h_inst_blk[i]);
      }
      if (all) break;
      if (2 * left <= hblist.size()) {
        std::vector<int32_t> dcopy(dn, dn + n);
        BHIP(b, set_lists(dcopy.data()));
        const nle_status sg = ensure_graph();
        if (sg != NLE_OK) return sg;
      }
    }
    BHIP(b, hipMemcpyAsync(b->h_pin, b->d_kits, size_t(n) * 4, hipMemcpyDeviceToHost, c->kstream));
    BHIP(b, hipMemcpyAsync(reinterpret_cast<int32_t *>(b->h_pin) + n, b->d_kdone, size_t(n) * 4,
                           hipMemcpyDeviceToHost, c->kstream));
    BHIP(b, hipStreamSynchronize(c->kstream));
    BHIP(b, hipEventRecord(c->ev_b, c->kstream));
    BHIP(b, hipStreamWaitEvent(c->stream, c->ev_b, 0));
    c->blk_list = c->mwg_list = nullptr;  // the steps below cover every stepping instance
    c->n_blist = c->n_mlist = 0;
    {
      const int32_t *its = reinterpret_cast<const int32_t *>(b->h_pin);
      for (int32_t i = 0; i < n; ++i)
        if (S[i].newton) {
          S[i].lit += its[i];
          S[i].njv += its[i];
        }
    }
    // ---- iNK: ||r + J du|| per instance ------------------------------------------
    if (inexact) {
      for (int32_t i = 0; i < n; ++i) hmask[i] = S[i].newton ? 0 : 1;
      BHIP(b, upload_i(b->d_mask, hmask));
      c->inst_done = b->d_mask;
      nle_status s2 = jv(c, dx, tmp, prec);
      c->inst_done = nullptr;
      if (s2 != NLE_OK) return bfail(b, s2, c->err);
      BHIP(b, batch_sub_norm(c, b->B, prec, tmp, bv, c->red));
      BHIP(b, batch_reduce_seg(c, b->B, c->red, b->d_out));
      BHIP(b, hipMemcpyAsync(b->h_pin, b->d_out, size_t(n) * 8, hipMemcpyDeviceToHost, c->stream));
      BHIP(b, hipStreamSynchronize(c->stream));
      for (int32_t i = 0; i < n; ++i)
        if (S[i].newton) {
          S[i].njv += 1;
          S[i].linres = S[i].rn * std::sqrt(b->h_pin[i]);
          S[i].eta_prev = S[i].eta;
        }
    }
    // ---- u += ||r_i|| dx ---------------------------------------------------------
    for (int32_t i = 0; i < n; ++i) hcoef[i] = S[i].newton ? S[i].rn : 0.0;
    BHIP(b, upload_d(b->d_coef, hcoef));
    BHIP(b, batch_axpy(c, b->B, prec, dx, NLE_FP64, u, b->d_coef));
    for (int32_t i = 0; i < n; ++i)
      if (S[i].newton) {
        S[i].rn_prev = S[i].rn;
        S[i].k += 1;
        S[i].nit += 1;
      }
  }
  BHIP(b, hipEventRecord(e1, c->stream));
  BHIP(b, hipEventSynchronize(e1));
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (t_ms) *t_ms = ms;
  nle_status worst = NLE_OK;
  for (int32_t i = 0; i < n; ++i) {
    if (S[i].status != NLE_OK) worst = S[i].status;
    if (reports) {
      nle_report &R = reports[i];
      R.status = S[i].status;
      R.nit = S[i].nit;
      R.lit_total = S[i].lit;
      R.n_jv = S[i].njv;
      R.n_residual = S[i].nres;
      R.bfgs_skipped = S[i].cuts;  // load-step cutbacks of this instance
      R.rnorm0 = S[i].r0;
      R.rnorm_final = S[i].rn;
      R.t_ms = ms;
    }
  }
  return worst;
}

}  // namespace

}  // namespace nle

using namespace nle;

struct nle_batch {
  Batch b;
};

extern "C" {

nle_status nle_batch_create(nle_batch **out, int32_t device, void *stream,
                            const nle_allocator *alloc) {
  if (!out) return NLE_E_INVAL;
  *out = nullptr;
  nle_batch *h = new (std::nothrow) nle_batch();
  if (!h) return NLE_E_OOM;
  nle_status s = nle_create(&h->b.ctx, device, stream, alloc);
  if (s != NLE_OK) {
    delete h;
    return s;
  }
  h->b.c = reinterpret_cast<Ctx *>(h->b.ctx);
  *out = h;
  return NLE_OK;
}

void nle_batch_destroy(nle_batch *h) {
  if (!h) return;
  Ctx *c = h->b.c;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  c->inst_s = nullptr;
  c->inst_mat = nullptr;
  c->inst_inv = nullptr;
  c->inst_done = nullptr;
  for (void *p : h->b.allocs) dfree(c, p);
  if (h->b.h_pin) (void)hipHostFree(h->b.h_pin);
  nle_destroy(h->b.ctx);
  delete h;
}

const char *nle_batch_last_error(const nle_batch *h) {
  if (!h) return "null batch";
  return h->b.err.c_str();
}

nle_status nle_batch_add(nle_batch *h, int64_t n_nodes, const double *X, int64_t n_elems,
                         const int32_t *conn, int32_t mat_kind, const double *params,
                         int32_t n_params, int64_t n_dir, const int64_t *dofs,
                         const double *values, int64_t n_faces, const int32_t *tri,
                         const double *traction, int32_t n_scales, const double *scales,
                         int32_t *id) {
  if (!h) return NLE_E_INVAL;
  Batch *b = &h->b;
  try {
    if (b->finalized) return bfail(b, NLE_E_STATE, "batch already finalized");
    if (n_nodes <= 0 || n_elems <= 0 || !X || !conn || !params || n_scales < 1 || !scales)
      return bfail(b, NLE_E_INVAL, "bad instance arrays");
    if (mat_kind != NLE_MAT_M1 && mat_kind != NLE_MAT_M2)
      return bfail(b, NLE_E_UNSUPPORTED, "unknown material kind");
    if (!b->inst.empty() && mat_kind != b->kind)
      return bfail(b, NLE_E_INVAL, "all instances of a batch use one material law");
    if (n_params != 2 && !(mat_kind == NLE_MAT_M2 && n_params == 3))
      return bfail(b, NLE_E_INVAL, "bad material parameter count");
    Inst I;
    I.X.assign(X, X + 3 * n_nodes);
    I.conn.assign(conn, conn + 4 * n_elems);
    for (int32_t v : I.conn)
      if (v < 0 || v >= n_nodes) return bfail(b, NLE_E_BADMESH, "node index out of range");
    I.params[0] = params[0];
    I.params[1] = params[1];
    I.params[2] = n_params == 3 ? params[2] : 0.25;
    if (!(I.params[0] > 0.0)) return bfail(b, NLE_E_INVAL, "mu must be positive");
    if (n_dir > 0) {
      if (!dofs || !values) return bfail(b, NLE_E_INVAL, "bad Dirichlet arrays");
      I.ddofs.assign(dofs, dofs + n_dir);
      I.dvals.assign(values, values + n_dir);
      for (int64_t d : I.ddofs)
        if (d < 0 || d >= 3 * n_nodes) return bfail(b, NLE_E_INVAL, "Dirichlet dof out of range");
    }
    if (n_faces > 0) {
      if (!tri || !traction) return bfail(b, NLE_E_INVAL, "bad traction arrays");
      I.tri.assign(tri, tri + 3 * n_faces);
      for (int32_t v : I.tri)
        if (v < 0 || v >= n_nodes) return bfail(b, NLE_E_INVAL, "face node out of range");
      I.t[0] = traction[0];
      I.t[1] = traction[1];
      I.t[2] = traction[2];
    }
    I.scales.assign(scales, scales + n_scales);
    for (int32_t k = 0; k < n_scales; ++k)
      if (!std::isfinite(I.scales[k]) || !(I.scales[k] > (k ? I.scales[k - 1] : 0.0)))
        return bfail(b, NLE_E_INVAL, "load scales must be positive and increasing");
    b->kind = mat_kind;
    b->inst.push_back(std::move(I));
    if (id) *id = int32_t(b->inst.size()) - 1;
    return NLE_OK;
  } catch (const std::bad_alloc &) {
    return bfail(b, NLE_E_OOM, "host allocation failed");
  }
}

nle_status nle_batch_finalize(nle_batch *h) {
  if (!h) return NLE_E_INVAL;
  Batch *b = &h->b;
  if (hipSetDevice(b->c->device) != hipSuccess) return bfail(b, NLE_E_HIP, "hipSetDevice");
  try {
    return finalize(b);
  } catch (const std::bad_alloc &) {
    return bfail(b, NLE_E_OOM, "host allocation failed");
  }
}

nle_status nle_batch_autotune(nle_batch *h, int32_t prec, double budget_ms, int32_t *block_size) {
  if (!h) return NLE_E_INVAL;
  Batch *b = &h->b;
  if (!b->finalized) return bfail(b, NLE_E_STATE, "nle_batch_finalize first");
  if (prec != NLE_FP32 && prec != NLE_FP64) return bfail(b, NLE_E_INVAL, "bad precision");
  if (!(budget_ms > 0.0)) return bfail(b, NLE_E_INVAL, "budget_ms must be positive");
  if (hipSetDevice(b->c->device) != hipSuccess) return bfail(b, NLE_E_HIP, "hipSetDevice");
  try {
    return autotune(b, prec, budget_ms, block_size);
  } catch (const std::bad_alloc &) {
    return bfail(b, NLE_E_OOM, "host allocation failed");
  }
}

nle_status nle_batch_layout(const nle_batch *h, int64_t *node_offsets) {
  if (!h || !node_offsets) return NLE_E_INVAL;
  if (!h->b.finalized) return NLE_E_STATE;
  std::copy(h->b.node_off.begin(), h->b.node_off.end(), node_offsets);
  return NLE_OK;
}

nle_status nle_batch_solve(nle_batch *h, int32_t method, const nle_solver_opts *o, double *u,
                           nle_report *reports, double *t_ms) {
  if (!h) return NLE_E_INVAL;
  Batch *b = &h->b;
  if (!b->finalized) return bfail(b, NLE_E_STATE, "nle_batch_finalize first");
  if (!o || !u) return bfail(b, NLE_E_INVAL, "null argument");
  if (method != NLE_NK && method != NLE_INK)
    return bfail(b, NLE_E_UNSUPPORTED, "batched solves support NK and iNK");
  if (o->ksp_type != NLE_KSP_CG) return bfail(b, NLE_E_UNSUPPORTED, "batched Krylov is CG");
  if (o->pc != NLE_PC_JACOBI) return bfail(b, NLE_E_UNSUPPORTED, "batched preconditioner is Jacobi");
  if (hipSetDevice(b->c->device) != hipSuccess) return bfail(b, NLE_E_HIP, "hipSetDevice");
  try {
    nle_status s = solve(b, method, *o, u, reports, t_ms);
    b->c->inst_done = nullptr;
    b->c->ep.red = nullptr;
    return s;
  } catch (const std::bad_alloc &) {
    b->c->inst_done = nullptr;
    return bfail(b, NLE_E_OOM, "host allocation failed");
  }
}

}  // extern "C"
