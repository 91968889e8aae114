// Nonlinear and Krylov solver control (host side; every vector operation runs
// in the library's kernels, scalars stay on the device between host checks).
//
// Paper, Sec. 3 and App. A:
//  NK   : Newton with a Krylov solve of J du = -r to rtol 1e-6 / atol 1e-10,
//         full step (line search "basic").
//  iNK  : the same with the Eisenstat-Walker relative tolerance
//         (eta_0 = 0.1, eta_max = 0.1) and atol 1e-14.
//  BFGS : limited-memory inverse update (two-loop recursion); H0 from the
//         tangent at the first iterate of the step, as one preconditioner
//         application (BFGS-preonly) or a Krylov solve with rtol 1e-2
//         (inexact BFGS); no scalar scaling of H0; full step.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>

#include "nle_internal.hpp"

namespace nle {

nle_status read_scalars(Ctx *c, const void *dev, size_t bytes);
nle_status residual_norm(Ctx *c, const double *u, double *r, double *rn, bool *inv);
nle_status linearize(Ctx *c, const double *u, int prec);
nle_status jv(Ctx *c, const void *v, void *y, int prec);

// The captured Krylov chunk bakes in kernel arguments (pointers, sizes and
// material parameters); it is dropped whenever any of them may change.
void drop_graph(Ctx *c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->gexec = nullptr;
  c->graph = nullptr;
  c->gkey.clear();
}

void gmres_pool_release(Ctx *c) {
  if (c->gm_segs.empty()) return;
  (void)hipStreamSynchronize(c->stream);
  for (const Ctx::GmSeg &g : c->gm_segs) dfree(c, g.p);
  c->gm_segs.clear();
  c->gm_hv.clear();
  c->gm_hr.clear();
  c->gm_vb = 0;
}

namespace {

constexpr double GOLDEN = 1.6180339887498949;

// Workspace: one device allocation grown on demand, carved sequentially.
struct Carver {
  char *base;
  size_t off = 0;
  void *take(size_t bytes) {
    void *p = base + off;
    off += (bytes + 255) & ~size_t(255);
    return p;
  }
};

nle_status ensure_ws(Ctx *c, size_t bytes) {
  if (c->ws_bytes >= bytes) return NLE_OK;
  NLE_HIP(c, hipStreamSynchronize(c->stream));
  drop_graph(c);
  for (void *p : c->ws_allocs) dfree(c, p);
  c->ws_allocs.clear();
  c->ws = dalloc(c, bytes);
  if (!c->ws) {
    c->ws_bytes = 0;
    return fail(c, NLE_E_OOM, "solver workspace allocation failed");
  }
  c->ws_allocs.push_back(c->ws);
  c->ws_bytes = bytes;
  return NLE_OK;
}

struct KspOpts {
  int type, orth, pc, restart, max_it, check_every;
  double rtol, atol;
  int cg_launches;
  int schur = 0;  // displacement / pressure meshes: NLE_SCHUR_* (GMRES)
};

struct KspResult {
  int its = 0;
  int flag = 0;  // 1 converged, 0 max_it, 2 indefinite, 3 NaN
};

inline size_t esz(int prec) { return prec == NLE_FP32 ? 4 : 8; }

size_t ksp_bytes(const KspOpts &o, int64_t n, int prec) {
  const size_t v = (size_t(n) * esz(prec) + 255) & ~size_t(255);
  if (o.type == NLE_KSP_CG) return 4 * v + 4096;
  if (o.type == NLE_KSP_MINRES) return 11 * v + 4096;
  // GMRES: the basis itself grows in the pool (gmres_reserve); the workspace
  // holds two work vectors, the pointer tables and the O(m) scalars
  const size_t m = size_t(o.restart > 0 ? std::min(o.restart, o.max_it) : o.max_it);
  return size_t(2 + (o.schur ? 2 : 0)) * v + 3 * (m + 1) * 8 + (4 * m + 4) * 8 +
         size_t(VGRID_MAX) * 8 + (8 + 2 * (m + 1)) * 8 + 8 * 256;
}

// Basis pool growth: the next segment holds max(64, half the vectors so far)
// vectors, at most up to the cycle's m + 1.  A segment carries its vectors,
// the Hessenberg columns of the same indices (column j: j + 2 rows) and one
// partial row per vector.
size_t gm_seg_bytes(size_t vb, int v0, int nv) {
  const size_t hcols = size_t(nv) * size_t(v0 + 2) + size_t(nv) * size_t(nv - 1) / 2;
  return size_t(nv) * vb + ((hcols * 8 + 255) & ~size_t(255)) + size_t(nv) * VGRID_MAX * 8;
}

int gm_pool_vectors(const Ctx *c) {
  return c->gm_segs.empty() ? 0 : c->gm_segs.back().v0 + c->gm_segs.back().nv;
}

// Make at least `need` (<= m + 1) basis vectors available and their table
// entries valid; `filled` counts the entries already written for this solve.
nle_status gmres_reserve(Ctx *c, const GmresArgs &a, size_t vb, int need, int *filled) {
  if (c->gm_vb != vb) {
    gmres_pool_release(c);
    c->gm_vb = vb;
  }
  while (gm_pool_vectors(c) < need) {
    const int have = gm_pool_vectors(c);
    const int nv = std::min(a.m + 1 - have, std::max(64, have / 2));
    const size_t bytes = gm_seg_bytes(vb, have, nv);
    void *p = dalloc(c, bytes);
    if (!p)
      return fail(c, NLE_E_OOM, "GMRES basis growth to " + std::to_string(have + nv) +
                                    " vectors failed (" + std::to_string(bytes >> 20) + " MiB)");
    Ctx::GmSeg g;
    g.p = p;
    g.v0 = have;
    g.nv = nv;
    g.vbase = p;
    g.hbase = reinterpret_cast<double *>(static_cast<char *>(p) + size_t(nv) * vb);
    const size_t hcols = size_t(nv) * size_t(have + 2) + size_t(nv) * size_t(nv - 1) / 2;
    g.rbase = reinterpret_cast<double *>(reinterpret_cast<char *>(g.hbase) +
                                         ((hcols * 8 + 255) & ~size_t(255)));
    c->gm_segs.push_back(g);
    for (int i = 0; i < nv; ++i) {
      c->gm_hv.push_back(static_cast<char *>(p) + size_t(i) * vb);
      c->gm_hr.push_back(g.rbase + size_t(i) * VGRID_MAX);
    }
  }
  // table entries of the segments not yet written in this solve
  for (const Ctx::GmSeg &g : c->gm_segs) {
    if (g.v0 + g.nv <= *filled || g.v0 >= a.m + 1) continue;
    NLE_HIP(c, gmres_tables(c, a, g.v0, g.nv, a.m + 1, g.vbase, vb, g.hbase, g.rbase));
  }
  *filled = std::max(*filled, std::min(gm_pool_vectors(c), a.m + 1));
  return NLE_OK;
}

// Run `iteration` (which queues one Krylov iteration on c->stream) until the
// device flag leaves 0: chunks of `chunk` iterations are captured once as a
// graph and replayed; the flag is read after each replay.
template <typename F>
nle_status run_chunks(Ctx *c, const std::vector<uint64_t> &key, int chunk, int max_it,
                      int32_t *flag, F &&iteration) {
  if (c->gkey != key) {
    drop_graph(c);
    NLE_HIP(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int i = 0; i < chunk && e == hipSuccess; ++i) e = iteration();
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(c->stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(c, NLE_E_HIP, std::string("graph capture: ") +
                                    hipGetErrorString(e != hipSuccess ? e : e2));
    }
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      return fail(c, NLE_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    c->graph = g;
    c->gexec = ex;
    c->gkey = key;
  }
  // Stagnation: the squared residual norm (scalar slot 3 of both CG and
  // MINRES) has not dropped 2% below its best value for max(4000, its/4)
  // iterations.  This happens when the solve precision's rounding floor lies
  // above the requested tolerance (FP32 recurrences on ill-conditioned
  // systems); the iterate is returned as after the iteration limit.
  double best = -1.0;
  int best_at = 0;
  for (int done = 0; done < max_it; done += chunk) {
    NLE_HIP(c, hipGraphLaunch(c->gexec, c->stream));
    NLE_HIP(c, hipMemcpyAsync(c->hpin, flag, 8, hipMemcpyDeviceToHost, c->stream));
    NLE_HIP(c, hipMemcpyAsync(c->hpin + 1, c->dscal + 3, 8, hipMemcpyDeviceToHost, c->stream));
    NLE_HIP(c, hipStreamSynchronize(c->stream));
    int32_t f;
    std::memcpy(&f, c->hpin, 4);
    if (f != 0) break;
    const double rr = c->hpin[1];
    const int its = done + chunk;
    if (best < 0.0 || rr < 0.98 * best) {
      best = rr;
      best_at = its;
    } else if (its - best_at >= std::max(4000, its / 4)) {
      break;
    }
  }
  return NLE_OK;
}

// Solve J x = b (J = tangent at the current linearization, precision prec)
// from x = 0.  Converged when ||b - J x|| <= max(rtol ||b||, atol).
nle_status ksp_solve(Ctx *c, const KspOpts &o, int prec, const void *b, void *x, Carver &W,
                     KspResult *R, int64_t *n_jv) {
  const int64_t n = ndof(c);
  const size_t vb = size_t(n) * esz(prec);
  const void *dinv = nullptr;
  int pcb = 1;
  const bool amg = o.pc == NLE_PC_AMG;
  if (amg) {
    if (c->mixed && c->mx.n_p > 0 && o.type != NLE_KSP_GMRES)
      return fail(c, NLE_E_UNSUPPORTED, "with a pressure field the multigrid runs with GMRES");
    const nle_status sa = amg_prepare(c);
    if (sa != NLE_OK) return sa;
  }
  if (o.pc == NLE_PC_JACOBI) {
    dinv = prec == NLE_FP32 ? static_cast<const void *>(c->dinv32)
                            : static_cast<const void *>(c->dinv64);
  } else if (o.pc == NLE_PC_BJACOBI3) {
    const nle_status sb = ensure_block(c);
    if (sb != NLE_OK) return sb;
    dinv = prec == NLE_FP32 ? static_cast<const void *>(c->binv32)
                            : static_cast<const void *>(c->binv64);
    pcb = 3;
  }
  const void *ulin = prec == NLE_FP32 ? static_cast<const void *>(c->ulin32)
                                      : static_cast<const void *>(c->ulin64);
  int32_t *flag = c->dflag + 8;
  const int check = std::max(1, o.check_every);
  R->its = 0;
  R->flag = 0;
  const int cap = elem_red_capacity(c);
  double *red_a = c->red, *red_b = c->red + cap, *red_r = c->red + cap + 2 * VGRID_MAX;
  if (o.type == NLE_KSP_CG || o.type == NLE_KSP_MINRES) {
    // the loop runs on the library's own stream (graph capture needs a
    // non-default stream), ordered after and before the caller's stream
    hipStream_t user = c->stream;
    NLE_HIP(c, hipEventRecord(c->ev_a, user));
    NLE_HIP(c, hipStreamWaitEvent(c->kstream, c->ev_a, 0));
    c->stream = c->kstream;
    struct Restore {
      Ctx *c;
      hipStream_t user;
      ~Restore() {
        c->elem_skip = nullptr;
        c->cg.z = nullptr;
        c->ep.w = nullptr;
        c->ep.coef = nullptr;
        c->ep.red = nullptr;
        c->stream = user;
      }
    } restore{c, user};
    nle_status st = NLE_OK;
    hipError_t e = hipSuccess;
    if (o.type == NLE_KSP_CG) {
      CgArgs a;
      a.prec = prec;
      a.n = n;
      a.x = x;
      a.r = W.take(vb);
      a.z = W.take(vb);
      a.p = W.take(vb);
      a.Ap = W.take(vb);
      a.dinv = dinv;
      a.pcb = pcb;
      a.red_a = red_a;
      a.red_b = red_b;
      a.scal = c->dscal;
      a.flag = flag;
      a.np_a = 0;
      // with the multigrid the update also takes the cycle's first
      // Chebyshev step (the same arithmetic as the cycle's own kernel)
      bool first = false;
      if (amg) {
        // the cycle replaces z = p = M^-1 b and the r.z partials
        NLE_HIP(c, cg_start(c, a, b, o.rtol, o.atol, o.max_it, false));
        NLE_HIP(c, amg_apply(c, prec, a.r, a.z, red_b));
        NLE_HIP(c, hipMemcpyAsync(a.p, a.z, vb, hipMemcpyDeviceToDevice, c->stream));
        NLE_HIP(c, cg_start_finish(c, a, o.rtol, o.atol, o.max_it));
        first = amg_first_step(c, prec, &a.dinv, &a.cd, &a.cth);
      } else {
        NLE_HIP(c, cg_start(c, a, b, o.rtol, o.atol, o.max_it));
      }
      c->elem_skip = flag;
      c->ep.red = red_a;
      // three launches per iteration (the next direction and the stopping
      // test formed inside the Jacobian action) on request, where the element
      // kernels support it; four otherwise.  On the 64x64x4 Cook mesh both
      // take ~20 us per iteration with point Jacobi: the fused form saves a
      // launch but adds the partial sums to the Jacobian action's critical
      // path.  With the multigrid the cycle runs after the update and
      // overwrites z and the r.z partials that the next Jacobian action reads.
      const bool fuse = !c->mixed && c->surf.nsn == 0 && o.cg_launches == 3;
      if (fuse) {
        c->cg.z = a.z;
        c->cg.red = red_b;
        c->cg.np = vgrid(n);
        c->cg.scal = c->dscal;
        c->cg.flag = flag;
      }
      auto iter = [&]() -> hipError_t {
        hipError_t err;
        a.np_a = elem_apply(c, OP_JV, prec, ulin, a.p, a.Ap, nullptr, &err);
        if (err != hipSuccess) return err;
        err = cg_update(c, a, fuse);
        if (err != hipSuccess) return err;
        if (amg) {  // z = M^-1 r by one cycle (the update left z = r, or took its first
                    // step), with the r.z partials
          if ((err = amg_apply(c, prec, a.r, a.z, red_b, first)) != hipSuccess) return err;
        }
        return fuse ? hipSuccess : cg_direction(c, a);
      };
      std::vector<uint64_t> key = {1, uint64_t(prec), uint64_t(n), uint64_t(check),
                                   uint64_t(uintptr_t(x)), uint64_t(uintptr_t(a.r)),
                                   uint64_t(uintptr_t(dinv)), uint64_t(uintptr_t(ulin)),
                                   uint64_t(uintptr_t(c->red)), uint64_t(uintptr_t(c->m.xr32)),
                                   uint64_t(uintptr_t(c->m.nodes)), uint64_t(c->mat.kind),
                                   uint64_t(uintptr_t(c->mx.G32)), uint64_t(uintptr_t(c->mx.cu)),
                                   uint64_t(uintptr_t(c->lc_valid ? c->lc64 : nullptr)),
                                   uint64_t(pcb), uint64_t(fuse), uint64_t(amg),
                                   amg ? c->amg_gen : 0, uint64_t(first)};
      st = run_chunks(c, key, check, o.max_it, flag, iter);
    } else {
      MinresArgs a;
      a.prec = prec;
      a.n = n;
      a.x = x;
      a.r1 = W.take(vb);
      a.r2 = W.take(vb);
      a.y = W.take(vb);
      a.v = W.take(vb);
      a.av = W.take(vb);
      a.wa = W.take(vb);
      a.wb = W.take(vb);
      a.za = W.take(vb);
      a.zb = W.take(vb);
      a.r = W.take(vb);
      a.dinv = dinv;
      a.pcb = pcb;
      a.red_a = red_a;
      a.red_b = red_b;
      a.red_r = red_r;
      a.scal = c->dscal;
      a.flag = flag;
      a.np_a = 0;
      // with the multigrid the vector kernels apply the identity and one
      // cycle replaces y = M^-1 t and the t.y partials (the cycle is
      // symmetric; positive definite for a positive definite tangent)
      auto cycle = [](Ctx *cc, const MinresArgs &aa) -> hipError_t {
        return amg_apply(cc, aa.prec, aa.r2, aa.y, aa.red_b);
      };
      if (amg) {
        NLE_HIP(c, mr_start(c, a, b, o.rtol, o.atol, o.max_it, false));
        NLE_HIP(c, amg_apply(c, prec, a.r1, a.y, red_b));
        NLE_HIP(c, mr_start_finish(c, a, o.rtol, o.atol, o.max_it));
      } else {
        NLE_HIP(c, mr_start(c, a, b, o.rtol, o.atol, o.max_it));
      }
      c->elem_skip = flag;
      c->ep.w = a.r1;
      c->ep.coef = c->dscal + 20;  // M_COEF
      c->ep.red = red_a;
      auto iter = [&]() -> hipError_t {
        hipError_t err;
        a.np_a = elem_apply(c, OP_JV, prec, ulin, a.v, a.y, nullptr, &err);
        if (err != hipSuccess) return err;
        return mr_iterate(c, a, amg ? +cycle : nullptr);
      };
      std::vector<uint64_t> key = {2, uint64_t(prec), uint64_t(n), uint64_t(check),
                                   uint64_t(uintptr_t(x)), uint64_t(uintptr_t(a.r1)),
                                   uint64_t(uintptr_t(dinv)), uint64_t(uintptr_t(ulin)),
                                   uint64_t(uintptr_t(c->red)), uint64_t(uintptr_t(c->m.xr32)),
                                   uint64_t(uintptr_t(c->m.nodes)), uint64_t(c->mat.kind),
                                   uint64_t(uintptr_t(c->mx.G32)), uint64_t(uintptr_t(c->mx.cu)),
                                   uint64_t(uintptr_t(c->lc_valid ? c->lc64 : nullptr)),
                                   uint64_t(pcb), uint64_t(amg), amg ? c->amg_gen : 0};
      st = run_chunks(c, key, check, o.max_it, flag, iter);
    }
    if (st != NLE_OK) return st;
    (void)e;
    st = read_scalars(c, flag, 8);
    if (st != NLE_OK) return st;
    int32_t f[2];
    std::memcpy(f, c->hpin, 8);
    R->its = f[1];
    R->flag = f[0] == 5 ? 0 : f[0];
    *n_jv += f[1];
    NLE_HIP(c, hipEventRecord(c->ev_b, c->kstream));
    NLE_HIP(c, hipStreamWaitEvent(user, c->ev_b, 0));
    return NLE_OK;
  }
  // ---- GMRES (right preconditioned) -----------------------------------------
  const int m = o.restart > 0 ? std::min(o.restart, o.max_it) : o.max_it;
  GmresArgs a;
  a.prec = prec;
  a.n = n;
  a.m = m;
  a.Vp = static_cast<void **>(W.take(size_t(m + 1) * 8));
  a.Hp = static_cast<double **>(W.take(size_t(m + 1) * 8));
  a.Rp = static_cast<double **>(W.take(size_t(m + 1) * 8));
  a.w = W.take(vb);
  a.z = W.take(vb);
  a.x = x;
  a.dinv = dinv;
  a.pcb = pcb;
  a.rot = static_cast<double *>(W.take(size_t(4 * m + 4) * 8));
  a.redsq = static_cast<double *>(W.take(size_t(VGRID_MAX) * 8));
  a.scal = static_cast<double *>(W.take(size_t(8 + 2 * (m + 1)) * 8));
  a.flag = flag;
  // the first vectors of the basis; the pool grows as the cycle proceeds
  int filled = 0;
  {
    nle_status s = gmres_reserve(c, a, vb, std::min(m + 1, 64), &filled);
    if (s != NLE_OK) return s;
  }
  a.hV = c->gm_hv.data();
  a.hR = c->gm_hr.data();
  // the lower block-triangular (Schur) preconditioner of a displacement /
  // pressure tangent: two more work vectors, and the SIMPLE diagonal of this
  // linearization when asked for
  const int schur = (c->mixed && c->mx.n_p > 0) ? o.schur : 0;
  void *st1 = schur ? W.take(vb) : nullptr;
  void *st2 = schur ? W.take(vb) : nullptr;
  if (schur == NLE_SCHUR_LOWER_SIMPLE) NLE_HIP(c, mixed_simple_diag(c));
  auto precond = [&](const void *in, void *out) -> hipError_t {
    if (schur) return schur_lower_apply(c, prec, amg, schur, in, out, st1, st2);
    if (amg) return amg_apply(c, prec, in, out);
    if (dinv) return pc_apply(c, prec, pcb, dinv, in, out, n);
    return hipMemcpyAsync(out, in, vb, hipMemcpyDeviceToDevice, c->stream);
  };
  const int mgs = o.orth == NLE_ORTH_MGS;
  NLE_HIP(c, vec_fill(c, prec, x, 0.0, n));
  NLE_HIP(c, gmres_start(c, a, b, o.rtol, o.atol, 1));
  int total = 0;
  int32_t f[2] = {0, 0};
  c->elem_skip = flag;
  while (true) {
    int queued = 0;
    for (int j = 0; j < m && total + queued < o.max_it; ++j) {
      if (j + 2 > filled) {
        // column j writes basis vector j + 1
        nle_status s = gmres_reserve(c, a, vb, std::min(m + 1, j + 2), &filled);
        if (s != NLE_OK) {
          c->elem_skip = nullptr;
          return s;
        }
        a.hV = c->gm_hv.data();
        a.hR = c->gm_hr.data();
      }
      const void *vj = a.hV[j];
      hipError_t e = precond(vj, a.z);
      if (e == hipSuccess)
        elem_apply(c, OP_JV, prec,
                   prec == NLE_FP32 ? (const void *)c->ulin32 : (const void *)c->ulin64, a.z, a.w,
                   nullptr, &e);
      if (e == hipSuccess) {
        if (mgs) {
          for (int i = 0; i <= j && e == hipSuccess; ++i) e = gmres_mgs_step(c, a, i, j);
        } else {
          e = gmres_multidot(c, a, j);
          if (e == hipSuccess) e = gmres_subtract(c, a, j, 0, 0);
          if (e == hipSuccess) e = gmres_multidot(c, a, j);
          if (e == hipSuccess) e = gmres_subtract(c, a, j, 1, 1);
        }
      }
      if (e == hipSuccess) e = gmres_finish_col(c, a, j, mgs);
      if (e != hipSuccess) {
        c->elem_skip = nullptr;
        return fail(c, NLE_E_HIP, std::string("gmres: ") + hipGetErrorString(e));
      }
      ++queued;
      if (queued % check == 0) {
        nle_status s = read_scalars(c, flag, 8);
        if (s != NLE_OK) {
          c->elem_skip = nullptr;
          return s;
        }
        std::memcpy(f, c->hpin, 8);
        if (f[0] != 0) break;
      }
    }
    c->elem_skip = nullptr;
    if (amg || schur) {
      // x += M^-1 (V y): form V y in z, then one application into w
      GmresArgs t = a;
      t.x = a.z;
      t.dinv = nullptr;
      t.pcb = 1;
      NLE_HIP(c, vec_fill(c, prec, a.z, 0.0, n));
      NLE_HIP(c, gmres_update_x(c, t));
      NLE_HIP(c, precond(a.z, a.w));
      NLE_HIP(c, vec_axpy(c, prec, a.w, prec, x, 1.0, nullptr, n));
    } else {
      NLE_HIP(c, gmres_update_x(c, a));
    }
    nle_status s = read_scalars(c, flag, 8);
    if (s != NLE_OK) return s;
    std::memcpy(f, c->hpin, 8);
    total += f[1];
    *n_jv += f[1];
    if (f[0] == 1 || f[0] == 3 || total >= o.max_it || f[1] == 0) break;
    // restart: r = b - J x
    NLE_HIP(c, hipMemcpyAsync(a.w, b, vb, hipMemcpyDeviceToDevice, c->stream));
    s = jv(c, x, a.z, prec);
    if (s != NLE_OK) return s;
    *n_jv += 1;
    NLE_HIP(c, vec_axpy(c, prec, a.z, prec, a.w, -1.0, nullptr, n));
    NLE_HIP(c, gmres_start(c, a, a.w, o.rtol, o.atol, 0));
    c->elem_skip = flag;
  }
  R->its = total;
  R->flag = (f[0] == 1) ? 1 : (f[0] == 3 ? 3 : 0);
  return NLE_OK;
}

constexpr double kEtaMinFP32 = 1e-4;

double ew_eta(const nle_solver_opts &o, int k, double rn, double rn_prev, double linres_prev,
              double eta_prev) {
  if (k == 0) return std::min(o.ew_rtol0, o.ew_rtolmax);
  double eta, stol;
  if (o.ew_version == 2) {
    eta = o.ew_gamma * std::pow(rn / rn_prev, o.ew_alpha);
    stol = o.ew_gamma * std::pow(eta_prev, o.ew_alpha);
  } else {
    eta = std::fabs(rn - linres_prev) / rn_prev;
    stol = std::pow(eta_prev, o.ew_alpha2);
  }
  if (stol > o.ew_threshold) eta = std::max(eta, stol);
  eta = std::min(eta, o.ew_rtolmax);
  return std::max(eta, o.ew_rtolmin);
}

struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  Ctx *c;
  explicit Timer(Ctx *cc) : c(cc) {
    if (hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess)
      (void)hipEventRecord(a, c->stream);
  }
  double stop() {
    float ms = 0.f;
    if (a && b && hipEventRecord(b, c->stream) == hipSuccess &&
        hipEventSynchronize(b) == hipSuccess)
      (void)hipEventElapsedTime(&ms, a, b);
    return double(ms);
  }
  ~Timer() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

struct Report {
  nle_report *r;
  explicit Report(nle_report *rr) : r(rr) {
    if (r) {
      r->status = 0;
      r->nit = 0;
      r->lit_total = 0;
      r->n_jv = 0;
      r->n_residual = 0;
      r->bfgs_skipped = 0;
      r->cutbacks = 0;
      r->reserved = 0;
      r->rnorm0 = 0;
      r->rnorm_final = 0;
      r->t_ms = 0;
    }
  }
  void hist(int k, double rn, double eta, int lit) {
    if (!r || k < 0 || k >= r->hist_cap) return;
    if (r->rnorm_hist) r->rnorm_hist[k] = rn;
    if (r->eta_hist) r->eta_hist[k] = eta;
    if (r->lit_hist) r->lit_hist[k] = lit;
  }
};

nle_status check_ready(Ctx *c, double *u, const nle_solver_opts *o) {
  if (!c) return NLE_E_INVAL;
  if (!c->has_mesh) return fail(c, NLE_E_STATE, "no mesh uploaded");
  if (!c->has_mat) return fail(c, NLE_E_STATE, "no material set");
  if (need_fibres(c) != NLE_OK) return NLE_E_STATE;
  if (!u || !o) return fail(c, NLE_E_INVAL, "null argument");
  if (o->precision != NLE_PREC_FP64 && o->precision != NLE_PREC_MIXED)
    return fail(c, NLE_E_INVAL, "bad precision");
  if (o->ksp_type != NLE_KSP_CG && o->ksp_type != NLE_KSP_GMRES &&
      o->ksp_type != NLE_KSP_MINRES)
    return fail(c, NLE_E_INVAL, "bad ksp_type");
  if (o->pc != NLE_PC_JACOBI && o->pc != NLE_PC_NONE && o->pc != NLE_PC_BJACOBI3 &&
      o->pc != NLE_PC_AMG)
    return fail(c, NLE_E_INVAL, "bad pc");
  if (o->pc == NLE_PC_BJACOBI3 && c->mixed)
    return fail(c, NLE_E_UNSUPPORTED, "nodal block Jacobi needs a P1 mesh");
  if (o->pc == NLE_PC_AMG && c->mixed && c->mx.n_p > 0 && o->ksp_type != NLE_KSP_GMRES)
    return fail(c, NLE_E_UNSUPPORTED, "with a pressure field the multigrid runs with GMRES");
  if (o->ksp_max_it < 1 || o->snes_max_it < 0) return fail(c, NLE_E_INVAL, "bad iteration limits");
  if (o->cg_launches != 0 && o->cg_launches != 3 && o->cg_launches != 4)
    return fail(c, NLE_E_INVAL, "bad cg_launches");
  if (o->h0_refresh < 0) return fail(c, NLE_E_INVAL, "bad h0_refresh");
  if (o->jac_lag < 0) return fail(c, NLE_E_INVAL, "bad jac_lag");
  if (o->schur != NLE_SCHUR_DIAG && o->schur != NLE_SCHUR_LOWER_MASS &&
      o->schur != NLE_SCHUR_LOWER_SIMPLE)
    return fail(c, NLE_E_INVAL, "bad schur");
  if (o->schur != NLE_SCHUR_DIAG) {
    if (!(c->mixed && c->mx.n_p > 0))
      return fail(c, NLE_E_UNSUPPORTED, "the Schur forms need a displacement / pressure mesh");
    if (o->ksp_type != NLE_KSP_GMRES)
      return fail(c, NLE_E_UNSUPPORTED, "the lower block-triangular preconditioner needs GMRES");
    if (o->pc != NLE_PC_JACOBI && o->pc != NLE_PC_AMG)
      return fail(c, NLE_E_UNSUPPORTED, "the Schur forms take pc JACOBI or AMG for the "
                                        "displacement block");
    if (o->schur == NLE_SCHUR_LOWER_SIMPLE && c->mx.npe != 1)
      return fail(c, NLE_E_UNSUPPORTED, "SIMPLE is built for the constant-pressure pair");
  }
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, NLE_E_HIP, "hipSetDevice failed");
  return NLE_OK;
}

// Carry a change of the prescribed Dirichlet values into the interior before
// the Newton loop: with w = g - u on the Dirichlet dofs (0 elsewhere), solve
// K_ff d = -(r(u) + K w)_f with the tangent at the current u and set
// u += w + d (the first Newton step of the problem whose boundary increment
// is part of the unknown step).  Lifting u to g directly can invert the
// elements next to a rotated face.  Nothing is done when u already holds
// the prescribed values, or when r(u) shows an inverted element.  *imb
// receives ||(r(u) + K w)_f|| (the step's initial imbalance, 0 if skipped).
nle_status dirichlet_step(Ctx *c, double *u, const KspOpts &ko, int prec, double *w64, double *r,
                          void *b, void *dx, void *tmp, Carver &W, size_t ksp_off,
                          int64_t *n_jv, int64_t *lit_total, int64_t *n_res, double *imb) {
  *imb = 0.0;
  if (c->n_dir == 0) return NLE_OK;
  const int64_t n = ndof(c);
  NLE_HIP(c, vec_fill(c, NLE_FP64, w64, 0.0, n));
  NLE_HIP(c, vec_dir_delta(c, u, w64));
  hipError_t e;
  int np = vec_dot_partials(c, NLE_FP64, w64, w64, n, c->red, &e);
  if (e != hipSuccess) return fail(c, NLE_E_HIP, "Dirichlet step norm");
  NLE_HIP(c, reduce_scalar(c, c->red, np, c->dscal + 62));
  nle_status s = read_scalars(c, c->dscal + 62, 8);
  if (s != NLE_OK) return s;
  if (!(c->hpin[0] > 0.0)) return NLE_OK;
  double rn = 0.0;
  bool inv = false;
  s = residual_norm(c, u, r, &rn, &inv);
  if (s != NLE_OK) return s;
  ++*n_res;
  if (inv || !std::isfinite(rn)) return NLE_OK;
  s = linearize(c, u, prec);
  if (s != NLE_OK) return s;
  NLE_HIP(c, vec_cast_scale(c, NLE_FP64, w64, prec, dx, 1.0, n));
  c->jv_nomask = true;
  s = jv(c, dx, tmp, prec);
  c->jv_nomask = false;
  if (s != NLE_OK) return s;
  ++*n_jv;
  NLE_HIP(c, vec_axpy(c, prec, tmp, NLE_FP64, r, 1.0, nullptr, n));
  np = vec_dot_partials(c, NLE_FP64, r, r, n, c->red, &e);
  if (e != hipSuccess) return fail(c, NLE_E_HIP, "Dirichlet step norm");
  NLE_HIP(c, reduce_scalar(c, c->red, np, c->dscal + 62));
  s = read_scalars(c, c->dscal + 62, 8);
  if (s != NLE_OK) return s;
  const double bn = std::sqrt(c->hpin[0]);
  *imb = std::isfinite(bn) ? bn : 0.0;
  NLE_HIP(c, vec_axpy(c, NLE_FP64, w64, NLE_FP64, u, 1.0, nullptr, n));
  if (!(bn > 0.0) || !std::isfinite(bn)) return NLE_OK;
  NLE_HIP(c, vec_cast_scale(c, NLE_FP64, r, prec, b, -1.0 / bn, n));
  KspOpts kk = ko;
  kk.atol = ko.atol / bn;
  KspResult kr;
  W.off = ksp_off;
  s = ksp_solve(c, kk, prec, b, dx, W, &kr, n_jv);
  if (s != NLE_OK) return s;
  *lit_total += kr.its;
  if (kr.flag == 3) return NLE_OK;  // no usable interior step: the lift alone
  NLE_HIP(c, vec_axpy(c, prec, dx, NLE_FP64, u, bn, nullptr, n));
  return NLE_OK;
}

nle_status finish(Ctx *c, Report &rep, nle_status st, int nit, double rn0, double rn, Timer &t) {
  const double ms = t.stop();
  if (rep.r) {
    rep.r->status = st;
    rep.r->nit = nit;
    rep.r->rnorm0 = rn0;
    rep.r->rnorm_final = rn;
    rep.r->t_ms = ms;
  }
  if (st > 0 && c->err.empty()) c->err = "solver did not converge";
  return st;
}

nle_status newton(Ctx *c, double *u, const nle_solver_opts &o, nle_report *report, bool inexact) {
  Timer timer(c);
  Report rep(report);
  c->err.clear();
  const int prec = o.precision == NLE_PREC_MIXED ? NLE_FP32 : NLE_FP64;
  const int64_t n = ndof(c);
  KspOpts ko{o.ksp_type, o.orth, o.pc, o.restart, o.ksp_max_it, std::max(1, o.check_every),
             o.ksp_rtol, o.ksp_atol, o.cg_launches, o.schur};
  const size_t vb64 = (size_t(n) * 8 + 255) & ~size_t(255);
  const size_t vbp = (size_t(n) * esz(prec) + 255) & ~size_t(255);
  nle_status s = ensure_ws(c, 2 * vb64 + 3 * vbp + ksp_bytes(ko, n, prec));
  if (s != NLE_OK) return s;
  Carver W{static_cast<char *>(c->ws)};
  double *r = static_cast<double *>(W.take(vb64));
  double *w64 = static_cast<double *>(W.take(vb64));
  void *b = W.take(vbp);
  void *dx = W.take(vbp);
  void *tmp = W.take(vbp);
  const size_t ksp_off = W.off;
  int64_t n_jv = 0, n_res = 0, lit_total = 0;

  // the boundary increment is carried in at the NK tolerances (a loose
  // interior step can invert the elements next to a moved face)
  double imb = 0.0;
  s = dirichlet_step(c, u, ko, prec, w64, r, b, dx, tmp, W, ksp_off, &n_jv, &lit_total, &n_res,
                     &imb);
  if (s != NLE_OK) return s;
  NLE_HIP(c, vec_lift(c, u));
  double rn = 0.0;
  bool inv = false;
  s = residual_norm(c, u, r, &rn, &inv);
  if (s != NLE_OK) return s;
  ++n_res;
  // relative to the load step's initial imbalance when a boundary increment
  // was carried in (the residual after that step is already reduced)
  const double rn0 = imb > rn ? imb : rn;
  const double tol = std::max(o.snes_rtol * rn0, o.snes_atol);
  double rn_prev = 0.0, linres_prev = 0.0, eta_prev = 0.0;
  int k = 0;
  nle_status st = NLE_DIVERGED_MAXIT;
  auto fill_rep = [&]() {
    if (report) {
      report->lit_total = lit_total;
      report->n_jv = n_jv;
      report->n_residual = n_res;
    }
  };
  for (;; ++k) {
    if (inv) {
      st = fail(c, NLE_DIVERGED_INVERTED, "element with det F <= 0");
      break;
    }
    if (!std::isfinite(rn)) {
      st = fail(c, NLE_DIVERGED_NAN, "residual norm is not finite");
      break;
    }
    if (rn <= tol) {
      st = NLE_OK;
      rep.hist(k, rn, 0.0, 0);
      break;
    }
    if (k >= o.snes_max_it) {
      rep.hist(k, rn, 0.0, 0);
      break;
    }
    if (o.jac_lag <= 1 || k % o.jac_lag == 0) {  // else the lagged tangent is reused
      s = linearize(c, u, prec);
      if (s != NLE_OK) return s;
    }
    double eta = o.ksp_rtol, atol = o.ksp_atol;
    if (inexact) {
      eta = ew_eta(o, k, rn, rn_prev, linres_prev, eta_prev);
      // an FP32 Krylov solve cannot reach much below the single-precision
      // rounding level of its recurrences
      if (prec == NLE_FP32) eta = std::max(eta, kEtaMinFP32);
      atol = o.ink_ksp_atol;
    }
    // b = -r / ||r||: the solve is scaled to a unit right-hand side
    NLE_HIP(c, vec_cast_scale(c, NLE_FP64, r, prec, b, -1.0 / rn, n));
    KspOpts kk = ko;
    kk.rtol = eta;
    kk.atol = atol / rn;
    KspResult kr;
    W.off = ksp_off;
    s = ksp_solve(c, kk, prec, b, dx, W, &kr, &n_jv);
    if (s != NLE_OK) return s;
    lit_total += kr.its;
    rep.hist(k, rn, eta, kr.its);
    if (kr.flag == 3) {
      st = fail(c, NLE_DIVERGED_LINEAR, "Krylov solve produced NaN");
      break;
    }
    if (inexact) {  // ||r + J du|| = ||r|| ||J dx - b||, recomputed explicitly
      s = jv(c, dx, tmp, prec);
      if (s != NLE_OK) return s;
      ++n_jv;
      NLE_HIP(c, vec_axpy(c, prec, b, prec, tmp, -1.0, nullptr, n));
      hipError_t e;
      const int np = vec_dot_partials(c, prec, tmp, tmp, n, c->red, &e);
      if (e != hipSuccess) return fail(c, NLE_E_HIP, "linear residual");
      NLE_HIP(c, reduce_scalar(c, c->red, np, c->dscal + 62));
      s = read_scalars(c, c->dscal + 62, 8);
      if (s != NLE_OK) return s;
      linres_prev = rn * std::sqrt(c->hpin[0]);
      eta_prev = eta;
    }
    NLE_HIP(c, vec_axpy(c, prec, dx, NLE_FP64, u, rn, nullptr, n));
    rn_prev = rn;
    s = residual_norm(c, u, r, &rn, &inv);
    if (s != NLE_OK) return s;
    ++n_res;
  }
  fill_rep();
  return finish(c, rep, st, k, rn0, rn, timer);
}

nle_status bfgs(Ctx *c, double *u, const nle_solver_opts &o, nle_report *report) {
  Timer timer(c);
  Report rep(report);
  c->err.clear();
  const int prec = o.precision == NLE_PREC_MIXED ? NLE_FP32 : NLE_FP64;
  const int64_t n = ndof(c);
  const int m = std::max(1, o.qn_m);
  KspOpts ko{o.ksp_type, o.orth, o.pc, o.restart, o.ksp_max_it, std::max(1, o.check_every),
             o.h0_rtol, o.h0_atol, o.cg_launches, o.schur};
  const size_t vb64 = (size_t(n) * 8 + 255) & ~size_t(255);
  const size_t vbp = (size_t(n) * esz(prec) + 255) & ~size_t(255);
  size_t need = 3 * vb64 + size_t(2 * m + 5) * vbp + 8 * size_t(m + 8) + 4096;
  if (o.h0 == NLE_H0_KSP) need += ksp_bytes(ko, n, prec);
  nle_status s = ensure_ws(c, need);
  if (s != NLE_OK) return s;
  Carver W{static_cast<char *>(c->ws)};
  double *g = static_cast<double *>(W.take(vb64));
  double *gn = static_cast<double *>(W.take(vb64));
  double *y64 = static_cast<double *>(W.take(vb64));
  void *q = W.take(vbp);
  void *z = W.take(vbp);
  void *b = W.take(vbp);
  // m + 1 slots: the candidate pair of an iteration always has a free slot
  std::vector<void *> S(m + 1), Y(m + 1);
  for (int i = 0; i <= m; ++i) {
    S[i] = W.take(vbp);
    Y[i] = W.take(vbp);
  }
  double *alpha = static_cast<double *>(W.take(8 * size_t(m + 8)));
  const size_t ksp_off = W.off;
  int64_t n_jv = 0, n_res = 0, lit_total = 0;
  int skipped = 0;
  std::vector<double> rho(m + 1, 0.0);
  std::deque<int> pairs;      // slot ids of stored pairs, oldest first
  std::vector<int> free_slots;
  for (int i = m; i >= 0; --i) free_slots.push_back(i);

  double imb = 0.0;
  if (o.h0 == NLE_H0_KSP) {  // with a Krylov method configured for H0
    KspOpts kp = ko;
    kp.rtol = o.ksp_rtol;
    kp.atol = o.ksp_atol;
    s = dirichlet_step(c, u, kp, prec, y64, g, b, q, z, W, ksp_off, &n_jv, &lit_total, &n_res,
                       &imb);
    if (s != NLE_OK) return s;
  }
  NLE_HIP(c, vec_lift(c, u));
  double rn = 0.0;
  bool inv = false;
  s = residual_norm(c, u, g, &rn, &inv);
  if (s != NLE_OK) return s;
  ++n_res;
  const double rn0 = imb > rn ? imb : rn;
  const double tol = std::max(o.snes_rtol * rn0, o.snes_atol);
  if (rn > tol && std::isfinite(rn) && !inv) {
    s = linearize(c, u, prec);  // the single linearization of the step
    if (s != NLE_OK) return s;
    if (o.pc == NLE_PC_BJACOBI3 && o.h0 != NLE_H0_KSP) {
      s = ensure_block(c);
      if (s != NLE_OK) return s;
    }
  }
  const bool blk = o.pc == NLE_PC_BJACOBI3;
  const void *dinv = blk ? (prec == NLE_FP32 ? static_cast<const void *>(c->binv32)
                                             : static_cast<const void *>(c->binv64))
                         : (prec == NLE_FP32 ? static_cast<const void *>(c->dinv32)
                                             : static_cast<const void *>(c->dinv64));
  double *redA = c->red, *redB = c->red + VGRID_MAX;
  double rn_prev_it = rn, h0_eta_prev = o.h0_rtol;  // inexact-BFGS forcing state
  int k = 0;
  nle_status st = NLE_DIVERGED_MAXIT;
  for (;; ++k) {
    if (inv) {
      st = fail(c, NLE_DIVERGED_INVERTED, "element with det F <= 0");
      break;
    }
    if (!std::isfinite(rn)) {
      st = fail(c, NLE_DIVERGED_NAN, "residual norm is not finite");
      break;
    }
    if (rn <= tol) {
      st = NLE_OK;
      rep.hist(k, rn, 0.0, 0);
      break;
    }
    if (k >= o.snes_max_it) {
      rep.hist(k, rn, 0.0, 0);
      break;
    }
    if (o.h0_refresh > 0 && k > 0 && k % o.h0_refresh == 0) {
      // periodic reassembly: tangent, preconditioner and H0 at the current
      // iterate; the stored pairs refer to the old H0 and are dropped
      s = linearize(c, u, prec);
      if (s != NLE_OK) return s;
      if (blk && o.h0 != NLE_H0_KSP) {
        s = ensure_block(c);
        if (s != NLE_OK) return s;
      }
      while (!pairs.empty()) {
        free_slots.push_back(pairs.back());
        pairs.pop_back();
      }
    }
    // q = g / ||g||
    NLE_HIP(c, vec_cast_scale(c, NLE_FP64, g, prec, q, 1.0 / rn, n));
    const int np_pairs = int(pairs.size());
    // first loop, newest to oldest: alpha_i = rho_i s_i.q ; q -= alpha_i y_i
    int np = 0;
    if (np_pairs > 0) NLE_HIP(c, lbfgs_dot(c, prec, S[pairs.back()], q, n, redA, &np));
    for (int t = np_pairs - 1; t >= 0; --t) {
      const int i = pairs[t];
      const void *snext = t > 0 ? S[pairs[t - 1]] : nullptr;
      NLE_HIP(c, lbfgs_axpy_dot(c, prec, q, Y[i], redA, np, rho[i], alpha + i, snext,
                                snext ? redB : nullptr, n));
      std::swap(redA, redB);
    }
    // z = H0 q
    int lit = 0;
    double h0_eta = o.h0_rtol;
    if (o.h0 == NLE_H0_KSP && o.h0_ew && k > 0) {
      // Eisenstat-Walker choice 2 on the BFGS residual norms, capped at h0_rtol
      h0_eta = o.ew_gamma * std::pow(rn / rn_prev_it, o.ew_alpha);
      const double stol = o.ew_gamma * std::pow(h0_eta_prev, o.ew_alpha);
      if (stol > o.ew_threshold) h0_eta = std::max(h0_eta, stol);
      h0_eta = std::max(std::min(h0_eta, o.h0_rtol), o.ew_rtolmin);
      if (prec == NLE_FP32) h0_eta = std::max(h0_eta, kEtaMinFP32);
    }
    h0_eta_prev = h0_eta;
    if (o.h0 == NLE_H0_KSP) {
      KspResult kr;
      W.off = ksp_off;
      KspOpts kh = ko;
      kh.rtol = h0_eta;
      s = ksp_solve(c, kh, prec, q, z, W, &kr, &n_jv);
      if (s != NLE_OK) return s;
      lit = kr.its;
      lit_total += kr.its;
      if (kr.flag == 3) {
        st = fail(c, NLE_DIVERGED_LINEAR, "H0 Krylov solve produced NaN");
        break;
      }
    } else if (o.pc == NLE_PC_AMG) {
      // BFGS-preonly with one V-cycle as H0 (App. A)
      s = amg_prepare(c);
      if (s != NLE_OK) return s;
      NLE_HIP(c, amg_apply(c, prec, q, z));
    } else if (o.pc == NLE_PC_JACOBI || blk) {
      NLE_HIP(c, pc_apply(c, prec, blk ? 3 : 1, dinv, q, z, n));
    } else {
      NLE_HIP(c, hipMemcpyAsync(z, q, size_t(n) * esz(prec), hipMemcpyDeviceToDevice, c->stream));
    }
    // second loop, oldest to newest: beta = rho_i y_i.z ; z += (alpha_i - beta) s_i
    if (np_pairs > 0) NLE_HIP(c, lbfgs_dot(c, prec, Y[pairs.front()], z, n, redA, &np));
    for (int t = 0; t < np_pairs; ++t) {
      const int i = pairs[t];
      const void *ynext = t + 1 < np_pairs ? Y[pairs[t + 1]] : nullptr;
      NLE_HIP(c, lbfgs_axpy2_dot(c, prec, z, S[i], redA, np, rho[i], alpha + i, ynext,
                                 ynext ? redB : nullptr, n));
      std::swap(redA, redB);
    }
    rep.hist(k, rn, o.h0 == NLE_H0_KSP ? h0_eta : 0.0, lit);
    // step p = -||g|| z ; u += p ; s = p
    const int slot = free_slots.back();
    free_slots.pop_back();
    NLE_HIP(c, vec_cast_scale(c, prec, z, prec, S[slot], -rn, n));
    NLE_HIP(c, vec_axpy(c, prec, z, NLE_FP64, u, -rn, nullptr, n));
    // new gradient, y = g_new - g
    const double rn_old = rn;
    rn_prev_it = rn;
    hipError_t e;
    NLE_HIP(c, hipMemsetAsync(c->dflag, 0, 4, c->stream));
    const int npr = elem_apply(c, OP_RES, NLE_FP64, u, nullptr, gn, c->red + 4 * VGRID_MAX, &e);
    if (e != hipSuccess) return fail(c, NLE_E_HIP, "residual");
    ++n_res;
    NLE_HIP(c, reduce_scalar(c, c->red + 4 * VGRID_MAX, npr, c->dscal + 40));
    NLE_HIP(c, vec_cast_scale(c, NLE_FP64, gn, NLE_FP64, y64, 1.0, n));
    NLE_HIP(c, vec_axpy(c, NLE_FP64, g, NLE_FP64, y64, -1.0, nullptr, n));
    NLE_HIP(c, vec_cast_scale(c, NLE_FP64, y64, prec, Y[slot], 1.0, n));
    int n1 = vec_dot_partials(c, prec, S[slot], Y[slot], n, c->red, &e);
    vec_dot_partials(c, prec, S[slot], S[slot], n, c->red + VGRID_MAX, &e);
    vec_dot_partials(c, prec, Y[slot], Y[slot], n, c->red + 2 * VGRID_MAX, &e);
    if (e != hipSuccess) return fail(c, NLE_E_HIP, "curvature dots");
    NLE_HIP(c, reduce_scalars(c, c->red, n1, 3, c->dscal + 41));
    NLE_HIP(c, hipMemcpyAsync(c->hpin, c->dscal + 40, 32, hipMemcpyDeviceToHost, c->stream));
    NLE_HIP(c, hipMemcpyAsync(c->hpin + 4, c->dflag, 4, hipMemcpyDeviceToHost, c->stream));
    NLE_HIP(c, hipStreamSynchronize(c->stream));
    rn = std::sqrt(c->hpin[0]);
    const double sy = c->hpin[1], ss = c->hpin[2], yy = c->hpin[3];
    int32_t fl;
    std::memcpy(&fl, c->hpin + 4, 4);
    inv = fl != 0;
    (void)rn_old;
    if (sy > o.curvature_eps * std::sqrt(ss * yy) && std::isfinite(sy)) {
      rho[slot] = 1.0 / sy;
      pairs.push_back(slot);
      if (int(pairs.size()) > m) {
        free_slots.push_back(pairs.front());
        pairs.pop_front();
      }
    } else {
      ++skipped;
      free_slots.push_back(slot);
    }
    std::swap(g, gn);
  }
  if (report) {
    report->lit_total = lit_total;
    report->n_jv = n_jv;
    report->n_residual = n_res;
    report->bfgs_skipped = skipped;
  }
  return finish(c, rep, st, k, rn0, rn, timer);
}

}  // namespace

}  // namespace nle

using namespace nle;

extern "C" {

void nle_default_opts(int32_t method, nle_solver_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = NLE_PREC_FP64;
  o->ksp_type = NLE_KSP_CG;
  o->orth = NLE_ORTH_CGS2;
  o->pc = NLE_PC_JACOBI;
  o->restart = 0;
  o->ksp_max_it = 100000;
  o->snes_max_it = 50;
  o->ew_version = 1;
  o->qn_m = 50;
  o->h0 = NLE_H0_KSP;
  o->check_every = 32;
  o->ksp_rtol = 1e-6;
  o->ksp_atol = 1e-10;
  o->ew_rtol0 = 0.1;
  o->ew_rtolmax = 0.1;
  o->ew_rtolmin = 0.0;
  o->ew_gamma = 1.0;
  o->ew_alpha = GOLDEN;
  o->ew_alpha2 = GOLDEN;
  o->ew_threshold = 0.1;
  o->ink_ksp_atol = 1e-14;
  o->snes_rtol = 1e-8;
  o->snes_atol = 0.0;
  o->h0_rtol = 1e-2;
  o->h0_atol = 1e-14;
  o->curvature_eps = 1e-12;
  if (method == NLE_BFGS) o->snes_max_it = 1000;
}

nle_status nle_solve_nk(nle_ctx *ctx, double *u, const nle_solver_opts *o, nle_report *rep) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  nle_status s = check_ready(c, u, o);
  if (s != NLE_OK) return s;
  try {
    return newton(c, u, *o, rep, false);
  } catch (...) {
    c->elem_skip = nullptr;
    return fail(c, NLE_E_OOM, "host exception in solver");
  }
}

nle_status nle_solve_ink(nle_ctx *ctx, double *u, const nle_solver_opts *o, nle_report *rep) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  nle_status s = check_ready(c, u, o);
  if (s != NLE_OK) return s;
  try {
    return newton(c, u, *o, rep, true);
  } catch (...) {
    c->elem_skip = nullptr;
    return fail(c, NLE_E_OOM, "host exception in solver");
  }
}

nle_status nle_solve_bfgs(nle_ctx *ctx, double *u, const nle_solver_opts *o, nle_report *rep) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  nle_status s = check_ready(c, u, o);
  if (s != NLE_OK) return s;
  try {
    return bfgs(c, u, *o, rep);
  } catch (...) {
    c->elem_skip = nullptr;
    return fail(c, NLE_E_OOM, "host exception in solver");
  }
}

}  // extern "C"
