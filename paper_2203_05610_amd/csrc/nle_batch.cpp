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
  int64_t replays = 0;      // replays of captured Krylov chunks (graph launches)
  // the tail: when at most tail_max instances are unfinished, or (NK, iNK)
  // when an instance's batched CG solve of a round takes more than tail_its
  // iterations, it is finished alone with the single-problem solver and
  // preconditioner tail_pc
  int32_t tail_max = 0, tail_its = 0, tail_pc = NLE_PC_AMG;
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
  int skipped = 0;        // L-BFGS pairs rejected by the curvature test
  int nit = 0;
  int64_t lit = 0, njv = 0, nres = 0;
  int status = NLE_OK;
};

// Batched CG on the instances flagged in `active`, b -> cg.x from zero with
// the per-instance tolerances already in b->d_rtol / d_atol: chunks of
// `chunk` iterations are captured as a graph and replayed; the launches cover
// only the work of the instances still iterating (blocks, merge workgroups,
// segments from per-round lists), which are rebuilt (and the graph
// recaptured) whenever the listed blocks could halve.  its[i] receives the
// iterations of instance i.
nle_status batch_cg(Batch *b, const BatchCg &cg, int prec, const void *ulin, const void *bv,
                    const std::vector<char> &active, int max_it, int chunk,
                    std::vector<int32_t> *its_out) {
  Ctx *c = b->c;
  const int32_t n = b->B.n_inst;
  const int64_t nd = 3 * c->m.n_nodes;
  std::vector<int32_t> hact(n), hblist, hmlist, hslist;
  for (int32_t i = 0; i < n; ++i) hact[i] = active[i] ? 1 : 0;
  BHIP(b, hipMemcpyAsync(b->d_active, hact.data(), size_t(n) * 4, hipMemcpyHostToDevice,
                         c->stream));
  BHIP(b, batch_cg_start(c, b->B, cg, bv, b->d_rtol, b->d_atol, b->d_active, max_it));
  const std::vector<int32_t> &hinst_seg = b->h_inst_seg;
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
      if (!active[i] || (done && done[i] != 0)) continue;
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
  auto ensure_graph = [&]() -> nle_status {
    std::vector<uint64_t> key = {7, uint64_t(prec), uint64_t(nd), uint64_t(chunk),
                                 uint64_t(uintptr_t(c->ws)), uint64_t(uintptr_t(c->red)),
                                 uint64_t(uintptr_t(ulin)), uint64_t(uintptr_t(cg.x)),
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
  for (int done_its = 0; done_its < max_it; done_its += chunk) {
    BHIP(b, hipGraphLaunch(c->gexec, c->kstream));
    b->replays += 1;
    BHIP(b, hipMemcpyAsync(b->h_pin, b->d_kdone, size_t(n) * 4, hipMemcpyDeviceToHost, c->kstream));
    BHIP(b, hipStreamSynchronize(c->kstream));
    const int32_t *dn = reinterpret_cast<const int32_t *>(b->h_pin);
    bool all = true;
    size_t left = 0;
    for (int32_t i = 0; i < n; ++i) {
      all &= dn[i] != 0;
      if (active[i] && dn[i] == 0) left += size_t(c->m.h_inst_blk[i + 1] - c->m.h_inst_blk[i]);
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
  const int32_t *its = reinterpret_cast<const int32_t *>(b->h_pin);
  its_out->assign(its, its + n);
  return NLE_OK;
}

// Finish instance i alone (the tail of a batch solve): a context of its own on
// the batch's stream and allocator, the single-problem solver with the batch's
// method and options but preconditioner tail_pc, from the last converged state
// (ub) over the current scale and the rest of the schedule, a failed increment
// halved as in the batch rounds (the same budget of cutbacks).  The result, or
// the last converged state if the schedule fails, goes to u.
template <typename St>
nle_status finish_alone(Batch *b, int32_t i, int method, const nle_solver_opts &o, double *u,
                        const double *ub, St &I, int max_cuts) {
  Ctx *c = b->c;
  const Inst &in = b->inst[size_t(i)];
  const int64_t nn = int64_t(in.X.size() / 3), ne = int64_t(in.conn.size() / 4);
  const int64_t d0 = 3 * b->node_off[size_t(i)], nd = 3 * nn;
  nle_ctx *sub = nullptr;
  nle_status st = nle_create(&sub, c->device, c->stream, &c->al);
  if (st != NLE_OK) return bfail(b, st, "tail: context creation failed");
  struct Guard {
    Ctx *c;
    nle_ctx *sub;
    double *us = nullptr, *usb = nullptr;
    ~Guard() {
      if (us) dfree(c, us);
      if (usb) dfree(c, usb);
      nle_destroy(sub);
    }
  } g{c, sub};
  auto sfail = [&](nle_status s2) {
    return bfail(b, s2, std::string("tail: ") + nle_last_error(sub));
  };
  if ((st = nle_upload_mesh(sub, nn, in.X.data(), ne, 4, in.conn.data())) != NLE_OK)
    return sfail(st);
  const int32_t np = b->kind == NLE_MAT_M2 ? 3 : 2;
  if ((st = nle_set_material(sub, b->kind, in.params, np)) != NLE_OK) return sfail(st);
  if ((st = nle_set_dirichlet(sub, int64_t(in.ddofs.size()), in.ddofs.data(), in.dvals.data())) !=
      NLE_OK)
    return sfail(st);
  if (!in.tri.empty() &&
      (st = nle_set_traction(sub, int64_t(in.tri.size() / 3), in.tri.data(), in.t)) != NLE_OK)
    return sfail(st);
  g.us = static_cast<double *>(dalloc(c, size_t(nd) * 8));
  g.usb = static_cast<double *>(dalloc(c, size_t(nd) * 8));
  if (!g.us || !g.usb) return bfail(b, NLE_E_OOM, "tail: device allocation failed");
  BHIP(b, hipMemcpyAsync(g.us, ub + d0, size_t(nd) * 8, hipMemcpyDeviceToDevice, c->stream));
  BHIP(b, hipMemcpyAsync(g.usb, ub + d0, size_t(nd) * 8, hipMemcpyDeviceToDevice, c->stream));
  nle_solver_opts oo = o;
  oo.pc = b->tail_pc;
  auto solver = method == NLE_NK ? nle_solve_nk : (method == NLE_INK ? nle_solve_ink : nle_solve_bfgs);
  std::vector<double> tg{I.s_cur};
  for (size_t k = size_t(I.step); k < in.scales.size(); ++k)
    if (in.scales[k] > I.s_cur) tg.push_back(in.scales[k]);
  double s_prev = I.s_prev;
  int status = NLE_OK;
  size_t k = 0;
  while (k < tg.size()) {
    if ((st = nle_set_load_scale(sub, tg[k])) != NLE_OK) return sfail(st);
    nle_report rep{};
    st = solver(sub, g.us, &oo, &rep);
    if (st < 0) return sfail(st);
    I.nit += rep.nit;
    I.lit += rep.lit_total;
    I.njv += rep.n_jv;
    I.nres += rep.n_residual;
    I.skipped += rep.bfgs_skipped;
    I.rn = rep.rnorm_final;
    if (st == NLE_OK) {
      BHIP(b, hipMemcpyAsync(g.usb, g.us, size_t(nd) * 8, hipMemcpyDeviceToDevice, c->stream));
      s_prev = tg[k];
      ++k;
      continue;
    }
    BHIP(b, hipMemcpyAsync(g.us, g.usb, size_t(nd) * 8, hipMemcpyDeviceToDevice, c->stream));
    if (I.cuts >= max_cuts) {
      status = st;
      break;
    }
    I.cuts += 1;
    tg.insert(tg.begin() + std::ptrdiff_t(k), 0.5 * (s_prev + tg[k]));
  }
  BHIP(b, hipMemcpyAsync(u + d0, g.us, size_t(nd) * 8, hipMemcpyDeviceToDevice, c->stream));
  BHIP(b, hipStreamSynchronize(c->stream));
  I.s_prev = s_prev;
  I.finished = true;
  I.status = status;
  return NLE_OK;
}

// Finish every unfinished instance alone once at most tail_max remain
// (returns true when it did).
template <typename St>
nle_status maybe_tail(Batch *b, int method, const nle_solver_opts &o, double *u, const double *ub,
                      std::vector<St> &S, int max_cuts, bool *done) {
  *done = false;
  int left = 0;
  for (const St &I : S) left += I.finished ? 0 : 1;
  if (b->tail_max <= 0 || left == 0 || left > b->tail_max) return NLE_OK;
  for (size_t i = 0; i < S.size(); ++i)
    if (!S[i].finished) {
      const nle_status st = finish_alone(b, int32_t(i), method, o, u, ub, S[i], max_cuts);
      if (st != NLE_OK) return st;
    }
  *done = true;
  return NLE_OK;
}

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
  std::vector<int32_t> hmask(n);
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
    {
      bool tail = false;
      st = maybe_tail(b, method, o, u, ub, S, max_cuts, &tail);
      if (st != NLE_OK) return st;
      if (tail) break;
    }
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
    // ---- batched CG ------------------------------------------------------------
    {
      std::vector<char> act(n);
      for (int32_t i = 0; i < n; ++i) act[i] = S[i].newton ? 1 : 0;
      std::vector<int32_t> its;
      st = batch_cg(b, cg, prec, ulin, bv, act, o.ksp_max_it, std::max(1, o.check_every), &its);
      if (st != NLE_OK) return st;
      for (int32_t i = 0; i < n; ++i)
        if (S[i].newton) {
          S[i].lit += its[i];
          S[i].njv += its[i];
        }
      // instances whose solve took more than tail_its iterations leave the
      // rounds (the rest of this round skips them) and are finished alone
      if (b->tail_its > 0)
        for (int32_t i = 0; i < n; ++i)
          if (S[i].newton && its[i] > b->tail_its) {
            S[i].newton = false;
            st = finish_alone(b, i, method, o, u, ub, S[i], max_cuts);
            if (st != NLE_OK) return st;
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
      R.bfgs_skipped = S[i].skipped;
      R.cutbacks = S[i].cuts;
      R.rnorm0 = S[i].r0;
      R.rnorm_final = S[i].rn;
      R.t_ms = ms;
    }
  }
  return worst;
}

// Batched L-BFGS (Sec. 3; the single-problem solver's algorithm per
// instance): every round evaluates the residuals of all unfinished instances,
// takes the per-instance decisions (converged -> next load scale; diverged ->
// restore and halve the increment; otherwise one BFGS iteration), forms the
// new pairs (y = g - g_prev, curvature test), re-linearizes the instances
// whose H0 is due (first iteration of a load step, or every h0_refresh
// iterations, dropping their pairs), and runs the two-loop recursion for all
// stepping instances at once: pairs sit in per-instance ring slots of [m+1]
// union vectors, every dot product is reduced per instance, H0 is the point
// Jacobi inverse (BFGS-preonly) or a batched CG solve (inexact BFGS).
nle_status solve_bfgs(Batch *b, const nle_solver_opts &o, double *u, nle_report *reports,
                      double *t_ms) {
  Ctx *c = b->c;
  const int32_t n = b->B.n_inst;
  const int prec = o.precision == NLE_PREC_MIXED ? NLE_FP32 : NLE_FP64;
  const size_t es = prec == NLE_FP32 ? 4 : 8;
  const int64_t nd = 3 * c->m.n_nodes;
  const int max_cuts = 8;
  const int m = std::max(1, o.qn_m), ms = m + 1;  // pairs, ring slots
  const bool ksp_h0 = o.h0 == NLE_H0_KSP;
  // workspace: r, backup, g_prev (double); q, z, CG x r z p Ap (prec); S, Y
  // [ms] (prec); per-instance tables
  const size_t v64 = (size_t(nd) * 8 + 255) & ~size_t(255), vp = (size_t(nd) * es + 255) & ~size_t(255);
  const size_t tab = (size_t(n) * (4 + 8) * size_t(3 * ms + 4) + 255) & ~size_t(255);
  const size_t need = 3 * v64 + size_t(7 + 2 * ms) * vp + tab;
  if (c->ws_bytes < need) {
    drop_graph(c);
    for (void *p : c->ws_allocs) dfree(c, p);
    c->ws_allocs.clear();
    c->ws = dalloc(c, need);
    if (!c->ws) {
      c->ws_bytes = 0;
      return bfail(b, NLE_E_OOM, "batch workspace allocation failed");
    }
    c->ws_allocs.push_back(c->ws);
    c->ws_bytes = need;
  }
  char *w = static_cast<char *>(c->ws);
  double *r = reinterpret_cast<double *>(w);
  double *ub = reinterpret_cast<double *>(w + v64);
  double *gp = reinterpret_cast<double *>(w + 2 * v64);
  char *wp = w + 3 * v64;
  void *q = wp, *z = wp + vp;
  BatchCg cg;
  cg.prec = prec;
  cg.x = z;
  cg.r = wp + 2 * vp;
  cg.z = wp + 3 * vp;
  cg.p = wp + 4 * vp;
  cg.Ap = wp + 5 * vp;
  void *qs = wp + 6 * vp;  // the scaled right-hand side of the H0 solve
  void *Sb = wp + 7 * vp, *Yb = wp + size_t(7 + ms) * vp;
  const int64_t stride = int64_t(vp / es);
  char *tb = wp + size_t(7 + 2 * ms) * vp;
  int32_t *d_slot = reinterpret_cast<int32_t *>(tb);             // [ms][n] slots by age
  double *d_rho = reinterpret_cast<double *>(tb + size_t(n) * 4 * ms);  // [ms][n]
  double *d_alpha = d_rho + size_t(ms) * n;                       // [ms][n]
  double *d_dot = d_alpha + size_t(ms) * n;                       // [n]
  double *d_cf = d_dot + n;                                       // [n]
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
  struct BState {
    int step = 0;
    double s_prev = 0.0, s_cur = 0.0;
    bool need_r0 = true, finished = false, active = false;
    double r0 = 0, rn = 0;
    int k = 0, k_lin = 0, cuts = 0, skipped = 0, nit = 0;
    int64_t lit = 0, njv = 0, nres = 0;
    int status = NLE_OK;
    int pos = 0, np = 0;     // ring: pairs in slots pos-np .. pos-1, pos free
    bool have_prev = false;  // S[pos] holds the last step, gp its gradient
    bool need_lin = true;
    std::vector<double> rho;
  };
  std::vector<BState> S(n);
  for (int32_t i = 0; i < n; ++i) {
    S[i].s_cur = b->inst[i].scales.empty() ? 1.0 : b->inst[i].scales[0];
    if (b->inst[i].scales.empty()) S[i].finished = true;
    S[i].rho.assign(ms, 0.0);
  }
  NLE_HIP(c, vec_lift(c, u));
  BHIP(b, hipMemcpyAsync(ub, u, size_t(nd) * 8, hipMemcpyDeviceToDevice, c->stream));
  std::vector<double> hs(n), hcoef(n), hd(n), hrtol(n), hatol(n);
  std::vector<int32_t> hmask(n), hslot(size_t(ms) * n);
  std::vector<double> hrho(size_t(ms) * n);
  auto upload_d = [&](double *dst, const std::vector<double> &v) {
    return hipMemcpyAsync(dst, v.data(), v.size() * 8, hipMemcpyHostToDevice, c->stream);
  };
  auto upload_i = [&](int32_t *dst, const std::vector<int32_t> &v) {
    return hipMemcpyAsync(dst, v.data(), v.size() * 4, hipMemcpyHostToDevice, c->stream);
  };
  // per-instance sums of segment partials (count arrays of nseg) into host
  auto seg_sums = [&](const double *red, int count, double *host) -> nle_status {
    for (int k = 0; k < count; ++k)
      BHIP(b, batch_reduce_seg(c, b->B, red + size_t(k) * b->B.nseg, b->d_out + size_t(k) * n));
    BHIP(b, hipMemcpyAsync(host, b->d_out, size_t(count) * n * 8, hipMemcpyDeviceToHost, c->stream));
    BHIP(b, hipStreamSynchronize(c->stream));
    return NLE_OK;
  };
  nle_status st = NLE_OK;
  for (int round = 0; round < 1000000; ++round) {
    bool any = false;
    for (int32_t i = 0; i < n; ++i) any |= !S[i].finished;
    if (!any) break;
    {
      bool tail = false;
      st = maybe_tail(b, NLE_BFGS, o, u, ub, S, max_cuts, &tail);
      if (st != NLE_OK) return st;
      if (tail) break;
    }
    // ---- residuals (the gradients g) of all unfinished instances -------------
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
    c->inst_done = nullptr;
    if (e != hipSuccess) return bfail(b, NLE_E_HIP, "batched residual");
    BHIP(b, batch_reduce_elem(c, b->B, c->red, b->d_out));
    BHIP(b, hipMemcpyAsync(b->h_pin, b->d_out, size_t(n) * 8, hipMemcpyDeviceToHost, c->stream));
    BHIP(b, hipMemcpyAsync(b->h_pin + n, c->inst_inv, size_t(n) * 4, hipMemcpyDeviceToHost, c->stream));
    BHIP(b, hipStreamSynchronize(c->stream));
    std::vector<double> rn2(b->h_pin, b->h_pin + n);
    std::vector<int32_t> inv(reinterpret_cast<const int32_t *>(b->h_pin + n),
                             reinterpret_cast<const int32_t *>(b->h_pin + n) + n);
    // ---- the new pairs of instances that stepped last round ------------------
    {
      bool anyp = false;
      for (int32_t i = 0; i < n; ++i) {
        const bool p = !S[i].finished && S[i].have_prev && inv[i] == 0 && std::isfinite(rn2[i]);
        hslot[i] = p ? S[i].pos : -1;
        anyp |= p;
      }
      if (anyp) {
        std::vector<int32_t> sl(hslot.begin(), hslot.begin() + n);
        BHIP(b, upload_i(d_slot, sl));
        BHIP(b, batch_lbfgs_pair(c, b->B, prec, Sb, Yb, stride, d_slot, r, gp, c->red));
        std::vector<double> cur(3 * size_t(n));
        st = seg_sums(c->red, 3, cur.data());
        if (st != NLE_OK) return st;
        for (int32_t i = 0; i < n; ++i) {
          if (hslot[i] < 0) continue;
          BState &I = S[i];
          const double sy = cur[i], ss = cur[n + i], yy = cur[2 * n + i];
          if (sy > o.curvature_eps * std::sqrt(ss * yy) && std::isfinite(sy)) {
            I.rho[I.pos] = 1.0 / sy;
            I.pos = (I.pos + 1) % ms;
            I.np = std::min(I.np + 1, m);
          } else {
            I.skipped += 1;
          }
        }
      }
    }
    // ---- per-instance decisions --------------------------------------------
    std::vector<int32_t> restore(n, 0), save(n, 0);
    bool any_step = false;
    for (int32_t i = 0; i < n; ++i) {
      BState &I = S[i];
      I.active = false;
      if (I.finished) continue;
      I.nres += 1;
      const double rn = std::sqrt(rn2[i]);
      bool failed = inv[i] != 0 || !std::isfinite(rn);
      if (!failed && I.need_r0) {
        I.r0 = rn;
        I.need_r0 = false;
        I.k = 0;
      }
      const double tol = std::max(o.snes_rtol * I.r0, o.snes_atol);
      auto reset_qn = [&]() {
        I.np = 0;
        I.have_prev = false;
        I.need_lin = true;
      };
      if (!failed && rn <= tol) {  // load step converged
        const std::vector<double> &sc = b->inst[i].scales;
        save[i] = 1;
        I.s_prev = I.s_cur;
        I.rn = rn;
        reset_qn();
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
      if (failed) {
        restore[i] = 1;
        reset_qn();
        if (I.cuts >= max_cuts) {
          I.finished = true;
          I.status = inv[i] ? NLE_DIVERGED_INVERTED
                            : (std::isfinite(rn) ? NLE_DIVERGED_MAXIT : NLE_DIVERGED_NAN);
          continue;
        }
        I.cuts += 1;
        I.s_cur = 0.5 * (I.s_prev + I.s_cur);
        I.need_r0 = true;
        continue;
      }
      if (o.h0_refresh > 0 && I.k_lin >= o.h0_refresh) {  // periodic reassembly
        I.need_lin = true;
        I.np = 0;
      }
      I.active = true;
      I.rn = rn;
      any_step = true;
    }
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
    if (!any_step) continue;
    // ---- H0 of the instances that need it: linearize those at u -------------
    {
      bool anyl = false;
      for (int32_t i = 0; i < n; ++i) {
        const bool l = S[i].active && S[i].need_lin;
        hmask[i] = l ? 1 : 0;
        anyl |= l;
      }
      if (anyl) {
        BHIP(b, upload_i(b->d_mask, hmask));
        BHIP(b, batch_copy(c, b->B, u, c->ulin64, b->d_mask));  // only their states move
        for (int32_t i = 0; i < n; ++i) hmask[i] = hmask[i] ? 0 : 1;
        BHIP(b, upload_i(b->d_mask, hmask));
        c->inst_done = b->d_mask;
        st = linearize(c, c->ulin64, prec);
        c->inst_done = nullptr;
        if (st != NLE_OK) return bfail(b, st, c->err);
        for (int32_t i = 0; i < n; ++i)
          if (S[i].active && S[i].need_lin) {
            S[i].need_lin = false;
            S[i].k_lin = 0;
          }
      }
    }
    // ---- two-loop recursion, all stepping instances together ----------------
    int mmax = 0;
    for (int32_t i = 0; i < n; ++i)
      if (S[i].active) mmax = std::max(mmax, S[i].np);
    for (int a = 0; a < mmax; ++a)
      for (int32_t i = 0; i < n; ++i) {
        const BState &I = S[i];
        const bool has = I.active && a < I.np;
        const int sl = has ? (I.pos - 1 - a + 2 * ms) % ms : -1;
        hslot[size_t(a) * n + i] = sl;
        hrho[size_t(a) * n + i] = has ? I.rho[sl] : 0.0;
      }
    if (mmax > 0) {
      BHIP(b, hipMemcpyAsync(d_slot, hslot.data(), size_t(mmax) * n * 4, hipMemcpyHostToDevice,
                             c->stream));
      BHIP(b, hipMemcpyAsync(d_rho, hrho.data(), size_t(mmax) * n * 8, hipMemcpyHostToDevice,
                             c->stream));
    }
    // q = g / ||g_i|| on the stepping instances, zero elsewhere
    for (int32_t i = 0; i < n; ++i) hcoef[i] = S[i].active ? 1.0 / S[i].rn : 0.0;
    BHIP(b, upload_d(b->d_coef, hcoef));
    BHIP(b, batch_scale(c, b->B, NLE_FP64, r, prec, q, b->d_coef));
    for (int a = 0; a < mmax; ++a) {  // newest to oldest: alpha = rho s.q, q -= alpha y
      const int32_t *sl = d_slot + size_t(a) * n;
      BHIP(b, batch_dot_slot(c, b->B, prec, Sb, stride, sl, q, c->red));
      BHIP(b, batch_reduce_seg(c, b->B, c->red, d_dot));
      BHIP(b, batch_lbfgs_coef(c, n, d_rho + size_t(a) * n, d_dot, d_alpha + size_t(a) * n, d_cf, 0));
      BHIP(b, batch_axpy_slot(c, b->B, prec, Yb, stride, sl, prec, q, d_cf));
    }
    // z = H0 q
    if (ksp_h0) {
      for (int32_t i = 0; i < n; ++i) {
        hrtol[i] = o.h0_rtol;
        hatol[i] = S[i].active ? o.h0_atol / S[i].rn : 0.0;
      }
      BHIP(b, upload_d(b->d_rtol, hrtol));
      BHIP(b, upload_d(b->d_atol, hatol));
      BHIP(b, hipMemcpyAsync(qs, q, size_t(nd) * es, hipMemcpyDeviceToDevice, c->stream));
      std::vector<char> act(n);
      for (int32_t i = 0; i < n; ++i) act[i] = S[i].active ? 1 : 0;
      std::vector<int32_t> its;
      st = batch_cg(b, cg, prec, ulin, qs, act, o.ksp_max_it, std::max(1, o.check_every), &its);
      if (st != NLE_OK) return st;
      for (int32_t i = 0; i < n; ++i)
        if (S[i].active) {
          S[i].lit += its[i];
          S[i].njv += its[i];
        }
    } else if (o.pc == NLE_PC_JACOBI) {
      BHIP(b, pc_apply(c, prec, 1, cg.dinv, q, z, nd));
    } else {
      BHIP(b, hipMemcpyAsync(z, q, size_t(nd) * es, hipMemcpyDeviceToDevice, c->stream));
    }
    for (int a = mmax - 1; a >= 0; --a) {  // oldest to newest: z += (alpha - rho y.z) s
      const int32_t *sl = d_slot + size_t(a) * n;
      BHIP(b, batch_dot_slot(c, b->B, prec, Yb, stride, sl, z, c->red));
      BHIP(b, batch_reduce_seg(c, b->B, c->red, d_dot));
      BHIP(b, batch_lbfgs_coef(c, n, d_rho + size_t(a) * n, d_dot, d_alpha + size_t(a) * n, d_cf, 1));
      BHIP(b, batch_axpy_slot(c, b->B, prec, Sb, stride, sl, prec, z, d_cf));
    }
    // ---- step p = -||g_i|| z into the free slot; u += p; g_prev = g ------------
    {
      std::vector<int32_t> sl(n);
      for (int32_t i = 0; i < n; ++i) {
        sl[i] = S[i].active ? S[i].pos : -1;
        hcoef[i] = S[i].active ? -S[i].rn : 0.0;
        hd[i] = S[i].active ? 1.0 : 0.0;
        hmask[i] = S[i].active ? 1 : 0;
      }
      BHIP(b, upload_i(d_slot, sl));
      BHIP(b, upload_d(b->d_coef, hcoef));
      BHIP(b, batch_store_slot(c, b->B, prec, Sb, stride, d_slot, z, b->d_coef));
      BHIP(b, upload_d(d_cf, hd));
      BHIP(b, batch_axpy_slot(c, b->B, prec, Sb, stride, d_slot, NLE_FP64, u, d_cf));
      BHIP(b, upload_i(b->d_mask, hmask));
      BHIP(b, batch_copy(c, b->B, r, gp, b->d_mask));
    }
    for (int32_t i = 0; i < n; ++i)
      if (S[i].active) {
        S[i].have_prev = true;
        S[i].k += 1;
        S[i].k_lin += 1;
        S[i].nit += 1;
      }
  }
  BHIP(b, hipEventRecord(e1, c->stream));
  BHIP(b, hipEventSynchronize(e1));
  float ms_t = 0.f;
  (void)hipEventElapsedTime(&ms_t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (t_ms) *t_ms = ms_t;
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
      R.bfgs_skipped = S[i].skipped;
      R.cutbacks = S[i].cuts;
      R.rnorm0 = S[i].r0;
      R.rnorm_final = S[i].rn;
      R.t_ms = ms_t;
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

nle_status nle_batch_set_tail(nle_batch *h, int32_t max_tail, int32_t max_its, int32_t pc) {
  if (!h) return NLE_E_INVAL;
  Batch *b = &h->b;
  if (max_tail < 0 || max_its < 0) return bfail(b, NLE_E_INVAL, "max_tail and max_its must be >= 0");
  if (pc != NLE_PC_NONE && pc != NLE_PC_JACOBI && pc != NLE_PC_BJACOBI3 && pc != NLE_PC_AMG)
    return bfail(b, NLE_E_INVAL, "bad tail preconditioner");
  b->tail_max = max_tail;
  b->tail_its = max_its;
  b->tail_pc = pc;
  return NLE_OK;
}

nle_status nle_batch_solve(nle_batch *h, int32_t method, const nle_solver_opts *o, double *u,
                           nle_report *reports, double *t_ms) {
  if (!h) return NLE_E_INVAL;
  Batch *b = &h->b;
  if (!b->finalized) return bfail(b, NLE_E_STATE, "nle_batch_finalize first");
  if (!o || !u) return bfail(b, NLE_E_INVAL, "null argument");
  if (method != NLE_NK && method != NLE_INK && method != NLE_BFGS)
    return bfail(b, NLE_E_INVAL, "bad method");
  if (o->precision != NLE_PREC_FP64 && o->precision != NLE_PREC_MIXED)
    return bfail(b, NLE_E_INVAL, "bad precision");
  if (o->ksp_type != NLE_KSP_CG) return bfail(b, NLE_E_UNSUPPORTED, "batched Krylov is CG");
  if (o->pc != NLE_PC_JACOBI && !(method == NLE_BFGS && o->h0 == NLE_H0_PREONLY &&
                                  o->pc == NLE_PC_NONE))
    return bfail(b, NLE_E_UNSUPPORTED, "batched preconditioner is Jacobi");
  if (method == NLE_BFGS && (o->qn_m < 1 || o->qn_m > 64 || o->h0_refresh < 0))
    return bfail(b, NLE_E_INVAL, "bad BFGS memory or refresh");
  if (o->ksp_max_it < 1 || o->snes_max_it < 0) return bfail(b, NLE_E_INVAL, "bad iteration limits");
  if (hipSetDevice(b->c->device) != hipSuccess) return bfail(b, NLE_E_HIP, "hipSetDevice");
  try {
    nle_status s = method == NLE_BFGS ? solve_bfgs(b, *o, u, reports, t_ms)
                                      : solve(b, method, *o, u, reports, t_ms);
    b->c->inst_done = nullptr;
    b->c->ep.red = nullptr;
    return s;
  } catch (const std::bad_alloc &) {
    b->c->inst_done = nullptr;
    return bfail(b, NLE_E_OOM, "host allocation failed");
  }
}

}  // extern "C"
