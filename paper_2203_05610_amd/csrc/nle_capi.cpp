// C-ABI entry points: context, problem data and single-operator calls.
#include <cmath>
#include <cstring>
#include <exception>
#include <new>
#include <unordered_map>
#include <algorithm>

#include "nle_internal.hpp"

namespace nle {

nle_status fail(Ctx *c, nle_status code, const std::string &msg) {
  if (c) c->err = msg;
  return code;
}

void *dalloc(Ctx *c, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (c->custom_alloc) return c->al.alloc(bytes, c->al.user);
  void *p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void dfree(Ctx *c, void *p) {
  if (!p) return;
  if (c->custom_alloc)
    c->al.free(p, c->al.user);
  else
    (void)hipFree(p);
}

namespace {

nle_status need_mesh(Ctx *c) {
  if (!c) return NLE_E_INVAL;
  if (!c->has_mesh) return fail(c, NLE_E_STATE, "no mesh uploaded");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, NLE_E_HIP, "hipSetDevice failed");
  return NLE_OK;
}

nle_status rebuild_fext(Ctx *c) {
  const int64_t n = 3 * c->m.n_nodes;
  std::vector<double> f(n);
  for (int64_t i = 0; i < n; ++i) f[i] = c->h_ftrac[i] + c->h_fbody[i];
  NLE_HIP(c, hipMemcpyAsync(c->fext, f.data(), n * 8, hipMemcpyHostToDevice, c->stream));
  NLE_HIP(c, hipStreamSynchronize(c->stream));
  return NLE_OK;
}

template <typename F>
nle_status guarded(Ctx *c, F &&f) {
  try {
    return f();
  } catch (const std::bad_alloc &) {
    return fail(c, NLE_E_OOM, "host allocation failed");
  } catch (const std::exception &e) {
    return fail(c, NLE_E_INVAL, e.what());
  } catch (...) {
    return fail(c, NLE_E_INVAL, "unknown error");
  }
}

}  // namespace

// ---- readback helper used by the solvers --------------------------------
nle_status read_scalars(Ctx *c, const void *dev, size_t bytes) {
  NLE_HIP(c, hipMemcpyAsync(c->hpin, dev, bytes, hipMemcpyDeviceToHost, c->stream));
  NLE_HIP(c, hipStreamSynchronize(c->stream));
  return NLE_OK;
}

// r = R(u), ||r|| -> *rn (synchronising); inverted -> *inv
nle_status residual_norm(Ctx *c, const double *u, double *r, double *rn, bool *inv) {
  NLE_HIP(c, hipMemsetAsync(c->dflag, 0, sizeof(int32_t), c->stream));
  hipError_t e;
  int np = elem_apply(c, OP_RES, NLE_FP64, u, nullptr, r, c->red, &e);
  if (e != hipSuccess) return fail(c, NLE_E_HIP, std::string("residual: ") + hipGetErrorString(e));
  NLE_HIP(c, reduce_scalar(c, c->red, np, c->dscal + 63));
  NLE_HIP(c, hipMemcpyAsync(c->hpin, c->dscal + 63, 8, hipMemcpyDeviceToHost, c->stream));
  NLE_HIP(c, hipMemcpyAsync(c->hpin + 1, c->dflag, 4, hipMemcpyDeviceToHost, c->stream));
  NLE_HIP(c, hipStreamSynchronize(c->stream));
  *rn = std::sqrt(c->hpin[0]);
  int32_t f;
  std::memcpy(&f, c->hpin + 1, 4);
  *inv = f != 0;
  return NLE_OK;
}

nle_status linearize(Ctx *c, const double *u, int prec) {
  const int64_t n = ndof(c);
  NLE_HIP(c, surf_set_linear_pressure(c));
  c->lc_valid = false;
  if (!c->mixed) {  // room for the per-element tangent coefficients
    const int nk = c->mat.kind == NLE_MAT_M1 ? 1
                   : (c->mat.kind == NLE_MAT_M2 ? 3 : (c->mat.kind == NLE_MAT_M6 ? 4 : 7));
    const int64_t need = int64_t(nk) * c->m.n_elems;
    if (need > c->lc_cap) {
      drop_graph(c);
      NLE_HIP(c, hipStreamSynchronize(c->stream));
      dfree(c, c->lc64);
      dfree(c, c->lc32);
      c->lc64 = static_cast<double *>(dalloc(c, size_t(need) * 8));
      c->lc32 = static_cast<float *>(dalloc(c, size_t(need) * 4));
      c->lc_cap = (c->lc64 && c->lc32) ? need : 0;
      if (!c->lc_cap) {
        dfree(c, c->lc64);
        dfree(c, c->lc32);
        c->lc64 = nullptr;
        c->lc32 = nullptr;
        return fail(c, NLE_E_OOM, "device allocation failed (linearization cache)");
      }
    }
  }
  if (u != c->ulin64)
    NLE_HIP(c, hipMemcpyAsync(c->ulin64, u, n * 8, hipMemcpyDeviceToDevice, c->stream));
  hipError_t e;
  elem_apply(c, OP_DIAG, NLE_FP64, c->ulin64, nullptr, c->diag64, nullptr, &e);
  if (e != hipSuccess) return fail(c, NLE_E_HIP, std::string("diag: ") + hipGetErrorString(e));
  NLE_HIP(c, vec_recip(c, c->diag64, c->dinv64, n));
  c->blk_valid = false;
  amg_invalidate(c);
  c->lc_valid = !c->mixed && c->lc64 != nullptr;
  c->lin64 = true;
  c->lin32 = false;
  if (prec == NLE_FP32) {
    NLE_HIP(c, vec_cast_scale(c, NLE_FP64, c->ulin64, NLE_FP32, c->ulin32, 1.0, n));
    NLE_HIP(c, vec_cast_scale(c, NLE_FP64, c->dinv64, NLE_FP32, c->dinv32, 1.0, n));
    c->lin32 = true;
  }
  return NLE_OK;
}

// Nodal 3x3 diagonal blocks of the tangent at the current linearization and
// their inverses (binv64 / binv32), computed once per linearization.
nle_status ensure_block(Ctx *c) {
  if (c->mixed) return fail(c, NLE_E_UNSUPPORTED, "nodal block Jacobi needs a P1 mesh");
  if (c->mat.kind == NLE_MAT_M6)
    return fail(c, NLE_E_UNSUPPORTED, "nodal block Jacobi is not offered for law M6");
  if (!c->lin64) return fail(c, NLE_E_STATE, "not linearized");
  if (c->blk_valid) return NLE_OK;
  const int64_t nn = c->m.n_nodes;
  if (!c->odiag64) {
    c->odiag64 = static_cast<double *>(dalloc(c, size_t(3 * nn) * 8));
    c->binv64 = static_cast<double *>(dalloc(c, size_t(6 * nn) * 8));
    c->binv32 = static_cast<float *>(dalloc(c, size_t(6 * nn) * 4));
    for (void *p : {(void *)c->odiag64, (void *)c->binv64, (void *)c->binv32})
      if (p) c->mesh_allocs.push_back(p);
    if (!c->odiag64 || !c->binv64 || !c->binv32) {
      for (void *p : {(void *)c->odiag64, (void *)c->binv64, (void *)c->binv32}) {
        if (!p) continue;
        dfree(c, p);
        c->mesh_allocs.erase(std::find(c->mesh_allocs.begin(), c->mesh_allocs.end(), p));
      }
      c->odiag64 = c->binv64 = nullptr;
      c->binv32 = nullptr;
      return fail(c, NLE_E_OOM, "device allocation failed (block preconditioner)");
    }
  }
  hipError_t e;
  elem_apply(c, OP_ODIAG, NLE_FP64, c->ulin64, nullptr, c->odiag64, nullptr, &e);
  if (e != hipSuccess) return fail(c, NLE_E_HIP, std::string("block diag: ") + hipGetErrorString(e));
  NLE_HIP(c, block_inverse(c, nn));
  c->blk_valid = true;
  return NLE_OK;
}

nle_status jv(Ctx *c, const void *v, void *y, int prec) {
  hipError_t e;
  const void *ul = prec == NLE_FP32 ? static_cast<const void *>(c->ulin32)
                                    : static_cast<const void *>(c->ulin64);
  elem_apply(c, OP_JV, prec, ul, v, y, nullptr, &e);
  if (e != hipSuccess) return fail(c, NLE_E_HIP, std::string("jv: ") + hipGetErrorString(e));
  return NLE_OK;
}

}  // namespace nle

using namespace nle;

extern "C" {

const char *nle_version(void) { return "nlelast 0.1.0 (gfx950)"; }

const char *nle_last_error(const nle_ctx *ctx) {
  if (!ctx) return "null context";
  return reinterpret_cast<const Ctx *>(ctx)->err.c_str();
}

nle_status nle_create(nle_ctx **out, int32_t device, void *stream, const nle_allocator *alloc) {
  if (!out) return NLE_E_INVAL;
  *out = nullptr;
  Ctx *c = new (std::nothrow) Ctx();
  if (!c) return NLE_E_OOM;
  c->device = device;
  c->stream = static_cast<hipStream_t>(stream);
  if (alloc && alloc->alloc && alloc->free) {
    c->al = *alloc;
    c->custom_alloc = true;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    delete c;
    return NLE_E_HIP;
  }
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    return NLE_E_HIP;
  }
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess &&
      lds > 0)
    c->lds_limit = size_t(lds);
  if (hipStreamCreateWithFlags(&c->kstream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_a, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_b, hipEventDisableTiming) != hipSuccess) {
    delete c;
    return NLE_E_HIP;
  }
  // the fixed workspace of nle_jv_noalloc, looked up with the device current
  if (noalloc_scratch_init(device, &c->noalloc_ws) != hipSuccess) {
    (void)hipStreamDestroy(c->kstream);
    (void)hipEventDestroy(c->ev_a);
    (void)hipEventDestroy(c->ev_b);
    delete c;
    return NLE_E_HIP;
  }
  c->dscal = static_cast<double *>(dalloc(c, 64 * 8));
  c->dflag = static_cast<int32_t *>(dalloc(c, 64 * 4));
  if (!c->dscal || !c->dflag || hipHostMalloc(&c->hpin, 4096) != hipSuccess) {
    dfree(c, c->dscal);
    dfree(c, c->dflag);
    delete c;
    return NLE_E_OOM;
  }
  if (hipMemsetAsync(c->dflag, 0, 64 * 4, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    dfree(c, c->dscal);
    dfree(c, c->dflag);
    (void)hipHostFree(c->hpin);
    delete c;
    return NLE_E_HIP;
  }
  *out = reinterpret_cast<nle_ctx *>(c);
  return NLE_OK;
}

void nle_destroy(nle_ctx *ctx) {
  if (!ctx) return;
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  if (c->kstream) (void)hipStreamSynchronize(c->kstream);
  drop_graph(c);
  amg_release(c);
  gmres_pool_release(c);
  for (void *p : c->mesh_allocs) dfree(c, p);
  for (void *p : c->ws_allocs) dfree(c, p);
  dfree(c, c->red);
  dfree(c, c->dscal);
  dfree(c, c->dflag);
  dfree(c, c->dir_dofs);
  dfree(c, c->dir_vals);
  dfree(c, c->lc64);
  dfree(c, c->lc32);
  for (void *p : c->fib_allocs) dfree(c, p);
  free_surface(c);
  if (c->hpin) (void)hipHostFree(c->hpin);
  if (c->ev_a) (void)hipEventDestroy(c->ev_a);
  if (c->ev_b) (void)hipEventDestroy(c->ev_b);
  if (c->kstream) {
    (void)hipStreamSynchronize(c->kstream);
    (void)hipStreamDestroy(c->kstream);
  }
  delete c;
}

nle_status nle_set_block_size(nle_ctx *ctx, int32_t be) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!c) return NLE_E_INVAL;
  if (be < 64 || be > 4096) return fail(c, NLE_E_INVAL, "block size must be in [64, 4096]");
  c->be_req = be;
  return NLE_OK;
}

nle_status nle_upload_mesh(nle_ctx *ctx, int64_t n_nodes, const double *X, int64_t n_elems,
                           int32_t npe, const int32_t *conn) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!c) return NLE_E_INVAL;
  if (npe == 10)  // second-order displacement elements (no pressure field)
    return nle_upload_mesh_mixed(ctx, n_nodes, X, n_elems, conn, 0, nullptr);
  return guarded(c, [&]() -> nle_status {
    if (npe != 4) return fail(c, NLE_E_UNSUPPORTED, "nodes_per_elem must be 4 or 10");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, NLE_E_HIP, "hipSetDevice failed");
    c->has_mesh = false;
    drop_graph(c);
    dfree(c, c->lc64);
    dfree(c, c->lc32);
    c->lc64 = nullptr;
    c->lc32 = nullptr;
    c->lc_cap = 0;
    nle_status s = build_mesh(c, n_nodes, X, n_elems, conn);
    if (s != NLE_OK) return s;
    // per-element and per-face data of the previous mesh no longer apply
    for (void *p : c->fib_allocs) dfree(c, p);
    c->fib_allocs.clear();
    c->fib64 = nullptr;
    c->fib32 = nullptr;
    c->sh64 = nullptr;
    c->sh32 = nullptr;
    free_surface(c);
    c->surf.h_ptri.clear();
    c->surf.h_rtri.clear();
    dfree(c, c->dir_dofs);
    dfree(c, c->dir_vals);
    c->dir_dofs = nullptr;
    c->dir_vals = nullptr;
    return upload_node_masks(c);
  });
}

namespace {
nle_status upload_mixed(Ctx *c, int64_t n_nodes, const double *X, int64_t n_elems,
                        const int32_t *conn, int64_t n_pnodes, const int32_t *pconn, int npe);
}  // namespace

nle_status nle_upload_mesh_mixed(nle_ctx *ctx, int64_t n_nodes, const double *X, int64_t n_elems,
                                 const int32_t *conn, int64_t n_pnodes, const int32_t *pconn) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!c) return NLE_E_INVAL;
  return upload_mixed(c, n_nodes, X, n_elems, conn, n_pnodes, pconn, 4);
}

nle_status nle_upload_mesh_mixed_p0(nle_ctx *ctx, int64_t n_nodes, const double *X,
                                    int64_t n_elems, const int32_t *conn) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!c) return NLE_E_INVAL;
  if (n_elems <= 0 || n_elems >= (int64_t(1) << 28))
    return fail(c, NLE_E_INVAL, "bad element count");
  // the pressure unknown of element e is p[e]
  std::vector<int32_t> pc(static_cast<size_t>(n_elems));
  for (int64_t e = 0; e < n_elems; ++e) pc[size_t(e)] = int32_t(e);
  return upload_mixed(c, n_nodes, X, n_elems, conn, n_elems, pc.data(), 1);
}

namespace {
nle_status upload_mixed(Ctx *c, int64_t n_nodes, const double *X, int64_t n_elems,
                        const int32_t *conn, int64_t n_pnodes, const int32_t *pconn, int npe) {
  return guarded(c, [&]() -> nle_status {
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, NLE_E_HIP, "hipSetDevice failed");
    c->has_mesh = false;
    drop_graph(c);
    NLE_HIP(c, hipStreamSynchronize(c->stream));
    for (void *p : c->fib_allocs) dfree(c, p);
    c->fib_allocs.clear();
    c->fib64 = nullptr;
    c->fib32 = nullptr;
    c->sh64 = nullptr;
    c->sh32 = nullptr;
    free_surface(c);
    c->surf.h_ptri.clear();
    c->surf.h_rtri.clear();
    nle_status s = build_mixed_mesh(c, n_nodes, X, n_elems, conn, n_pnodes, pconn, npe);
    if (s != NLE_OK) return s;
    dfree(c, c->dir_dofs);
    dfree(c, c->dir_vals);
    c->dir_dofs = nullptr;
    c->dir_vals = nullptr;
    return NLE_OK;
  });
}
}  // namespace

nle_status nle_set_material(nle_ctx *ctx, int32_t kind, const double *p, int32_t np) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!c) return NLE_E_INVAL;
  if (!p) return fail(c, NLE_E_INVAL, "null parameter array");
  MatParams m{};
  if (kind == NLE_MAT_M3) {
    if (np != 1) return fail(c, NLE_E_INVAL, "M3 takes (mu)");
    if (!(p[0] > 0.0) || !std::isfinite(p[0])) return fail(c, NLE_E_INVAL, "M3 needs mu > 0");
    m.kind = kind;
    m.mu = p[0];
    m.lam = 0.0;
    m.cvol = 0.25;
    m.kappa = 0.0;
    drop_graph(c);
    c->mat = m;
    c->has_mat = true;
    c->lin64 = c->lin32 = c->lc_valid = false;
    return NLE_OK;
  } else if (kind == NLE_MAT_M5) {
    if (np != 4) return fail(c, NLE_E_INVAL, "M5 takes (alpha_p, beta_p, alpha_s, beta_s)");
    for (int i = 0; i < 4; ++i)
      if (!std::isfinite(p[i]) || !(p[i] >= 0.0))
        return fail(c, NLE_E_INVAL, "M5 needs finite non-negative constants");
    if (!(p[0] + p[1] > 0.0)) return fail(c, NLE_E_INVAL, "M5 needs alpha_p + beta_p > 0");
    m.kind = kind;
    m.a_iso = p[0];                 // alpha_p
    m.b_iso = p[1];                 // beta_p
    m.a_f = 4.0 * p[3] + 2.0 * p[2];  // the logarithmic term's 4 beta_s + 2 alpha_s
    m.b_f = 0.0;
    m.mu = 2.0 * (p[0] + p[1]);     // small-strain shear modulus
    m.lam = 4.0 * p[1];
    m.cvol = 0.25;
    m.kappa = 0.0;
    drop_graph(c);
    c->mat = m;
    c->has_mat = true;
    c->lin64 = c->lin32 = c->lc_valid = false;
    return NLE_OK;
  } else if (kind == NLE_MAT_M6) {
    if (np != 8)
      return fail(c, NLE_E_INVAL, "M6 takes (C, b_ff, b_ss, b_nn, b_fs, b_fn, b_sn, B)");
    for (int i = 0; i < 8; ++i)
      if (!std::isfinite(p[i]) || !(p[i] >= 0.0))
        return fail(c, NLE_E_INVAL, "M6 needs finite non-negative constants");
    if (!(p[0] > 0.0) || !(p[7] > 0.0)) return fail(c, NLE_E_INVAL, "M6 needs C > 0 and B > 0");
    m.kind = kind;
    for (int i = 0; i < 8; ++i) m.g6[i] = p[i];
    m.gamma = c->mat.gamma;
    m.mu = 0.5 * p[0] * p[1];  // a reported small-strain shear scale (C b_ff / 2)
    m.lam = p[7];
    m.cvol = 0.25;
    m.kappa = p[7];
    drop_graph(c);
    c->mat = m;
    c->has_mat = true;
    c->lin64 = c->lin32 = c->lc_valid = false;
    return NLE_OK;
  } else if (kind == NLE_MAT_M1) {
    if (np != 2) return fail(c, NLE_E_INVAL, "M1 takes (mu, lambda)");
    m.kind = kind;
    m.mu = p[0];
    m.lam = p[1];
    m.cvol = 0.25;
  } else if (kind == NLE_MAT_M2) {
    if (np != 2 && np != 3) return fail(c, NLE_E_INVAL, "M2 takes (mu, lambda[, c_vol])");
    m.kind = kind;
    m.mu = p[0];
    m.lam = p[1];
    m.cvol = np == 3 ? p[2] : 0.25;
  } else if (kind == NLE_MAT_M4) {
    if (np != 5) return fail(c, NLE_E_INVAL, "M4 takes (a, b, a_f, b_f, kappa)");
    for (int i = 0; i < 5; ++i)
      if (!std::isfinite(p[i])) return fail(c, NLE_E_INVAL, "non-finite material parameter");
    if (!(p[0] > 0.0) || !(p[1] > 0.0) || !(p[2] >= 0.0) || !(p[3] > 0.0) || !(p[4] > 0.0))
      return fail(c, NLE_E_INVAL, "M4 needs a, b, b_f, kappa > 0 and a_f >= 0");
    m.kind = kind;
    m.a_iso = p[0];
    m.b_iso = p[1];
    m.a_f = p[2];
    m.b_f = p[3];
    m.kappa = p[4];
    m.gamma = c->mat.gamma;
    m.mu = p[0];  // small-strain shear modulus (used only for reporting)
    m.lam = p[4] - 2.0 * p[0] / 3.0;
    m.cvol = 0.25;
    drop_graph(c);
    c->mat = m;
    c->has_mat = true;
    c->lin64 = c->lin32 = c->lc_valid = false;
    return NLE_OK;
  } else {
    return fail(c, NLE_E_UNSUPPORTED, "unknown material kind");
  }
  if (!(m.mu > 0.0) || !std::isfinite(m.lam) || !std::isfinite(m.cvol))
    return fail(c, NLE_E_INVAL, "material parameters must be finite with mu > 0");
  m.kappa = m.lam + 2.0 * m.mu / 3.0;
  m.gamma = c->mat.gamma;
  drop_graph(c);
  c->mat = m;
  c->has_mat = true;
  c->lin64 = c->lin32 = c->lc_valid = false;
  return NLE_OK;
}

nle_status nle_set_dirichlet(nle_ctx *ctx, int64_t n, const int64_t *dofs, const double *vals) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  nle_status s = need_mesh(c);
  if (s != NLE_OK) return s;
  return guarded(c, [&]() -> nle_status {
    if (n < 0 || (n > 0 && (!dofs || !vals))) return fail(c, NLE_E_INVAL, "bad Dirichlet arrays");
    const int64_t ndof = 3 * c->m.n_nodes;
    std::vector<uint8_t> mask(c->m.n_nodes, 0);
    for (int64_t k = 0; k < n; ++k) {
      const int64_t d = dofs[k];
      if (d < 0 || d >= ndof) return fail(c, NLE_E_INVAL, "Dirichlet dof out of range");
      const uint8_t bit = uint8_t(1u << (d % 3));
      if (mask[d / 3] & bit) return fail(c, NLE_E_INVAL, "repeated Dirichlet dof");
      if (!std::isfinite(vals[k])) return fail(c, NLE_E_INVAL, "non-finite Dirichlet value");
      mask[d / 3] |= bit;
    }
    // the new arrays are allocated before the old ones are released, so a
    // failed allocation leaves the previous Dirichlet set intact and usable
    int64_t *nd = nullptr;
    double *nv = nullptr;
    if (n > 0) {
      nd = static_cast<int64_t *>(dalloc(c, n * 8));
      nv = static_cast<double *>(dalloc(c, n * 8));
      if (!nd || !nv) {
        dfree(c, nd);
        dfree(c, nv);
        return fail(c, NLE_E_OOM, "device allocation failed");
      }
    }
    NLE_HIP(c, hipStreamSynchronize(c->stream));  // no queued kernel reads the old arrays
    dfree(c, c->dir_dofs);
    dfree(c, c->dir_vals);
    c->dir_dofs = nd;
    c->dir_vals = nv;
    c->n_dir = n;
    if (n > 0) {
      NLE_HIP(c, hipMemcpyAsync(c->dir_dofs, dofs, n * 8, hipMemcpyHostToDevice, c->stream));
      NLE_HIP(c, hipMemcpyAsync(c->dir_vals, vals, n * 8, hipMemcpyHostToDevice, c->stream));
    }
    const bool changed = mask != c->h_mask;
    c->h_mask = mask;
    if (changed) {
      c->lin64 = c->lin32 = c->lc_valid = false;
      amg_release(c);  // its candidates vanish on Dirichlet dofs
      return upload_node_masks(c);
    }
    NLE_HIP(c, hipStreamSynchronize(c->stream));
    return NLE_OK;
  });
}

nle_status nle_set_traction(nle_ctx *ctx, int64_t nf, const int32_t *tri, const double *t) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  nle_status s = need_mesh(c);
  if (s != NLE_OK) return s;
  return guarded(c, [&]() -> nle_status {
    if (nf < 0 || (nf > 0 && (!tri || !t))) return fail(c, NLE_E_INVAL, "bad traction arrays");
    std::vector<double> f(3 * c->m.n_nodes, 0.0);
    const double *X = c->m.h_X.data();
    if (c->mixed) {
      // flat 6-node faces: the quadratic shape functions integrate to 0 at
      // the vertices and to A/3 at each edge midpoint
      std::unordered_map<uint64_t, int32_t> mid;
      const std::vector<int32_t> &cn = c->mx.h_conn;
      static const int ea[6] = {0, 1, 0, 0, 1, 2}, eb[6] = {1, 2, 2, 3, 3, 3};
      for (size_t e = 0; e + 9 < cn.size(); e += 10)
        for (int q = 0; q < 6; ++q) {
          const uint32_t va = uint32_t(cn[e + ea[q]]), vb = uint32_t(cn[e + eb[q]]);
          mid[(uint64_t(std::min(va, vb)) << 32) | std::max(va, vb)] = cn[e + 4 + q];
        }
      for (int64_t k = 0; k < nf; ++k) {
        const int32_t *v = tri + 3 * k;
        for (int a = 0; a < 3; ++a)
          if (v[a] < 0 || v[a] >= c->m.n_nodes) return fail(c, NLE_E_INVAL, "face node out of range");
        double e1[3], e2[3];
        for (int i = 0; i < 3; ++i) {
          e1[i] = X[3 * v[1] + i] - X[3 * v[0] + i];
          e2[i] = X[3 * v[2] + i] - X[3 * v[0] + i];
        }
        const double cx = e1[1] * e2[2] - e1[2] * e2[1];
        const double cy = e1[2] * e2[0] - e1[0] * e2[2];
        const double cz = e1[0] * e2[1] - e1[1] * e2[0];
        const double area = 0.5 * std::sqrt(cx * cx + cy * cy + cz * cz);
        static const int fa[3] = {0, 1, 0}, fb[3] = {1, 2, 2};
        for (int q = 0; q < 3; ++q) {
          const uint32_t va = uint32_t(v[fa[q]]), vb = uint32_t(v[fb[q]]);
          auto it = mid.find((uint64_t(std::min(va, vb)) << 32) | std::max(va, vb));
          if (it == mid.end()) return fail(c, NLE_E_INVAL, "face edge is not an element edge");
          for (int i = 0; i < 3; ++i) f[3 * int64_t(it->second) + i] += t[i] * area / 3.0;
        }
      }
      c->h_ftrac = f;
      return rebuild_fext(c);
    }
    for (int64_t k = 0; k < nf; ++k) {
      const int32_t *v = tri + 3 * k;
      for (int a = 0; a < 3; ++a)
        if (v[a] < 0 || v[a] >= c->m.n_nodes) return fail(c, NLE_E_INVAL, "face node out of range");
      double e1[3], e2[3];
      for (int i = 0; i < 3; ++i) {
        e1[i] = X[3 * v[1] + i] - X[3 * v[0] + i];
        e2[i] = X[3 * v[2] + i] - X[3 * v[0] + i];
      }
      const double cx = e1[1] * e2[2] - e1[2] * e2[1];
      const double cy = e1[2] * e2[0] - e1[0] * e2[2];
      const double cz = e1[0] * e2[1] - e1[1] * e2[0];
      const double area = 0.5 * std::sqrt(cx * cx + cy * cy + cz * cz);
      for (int a = 0; a < 3; ++a)
        for (int i = 0; i < 3; ++i) f[3 * int64_t(v[a]) + i] += t[i] * area / 3.0;
    }
    c->h_ftrac = f;
    return rebuild_fext(c);
  });
}

nle_status nle_set_body_force(nle_ctx *ctx, const double *fb) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  nle_status s = need_mesh(c);
  if (s != NLE_OK) return s;
  if (c->mixed) return fail(c, NLE_E_UNSUPPORTED, "not available on mixed meshes");
  if (!fb) return fail(c, NLE_E_INVAL, "null body force");
  return guarded(c, [&]() -> nle_status {
    std::vector<double> f(3 * c->m.n_nodes, 0.0);
    for (int64_t e = 0; e < c->m.n_elems; ++e)
      for (int a = 0; a < 4; ++a)
        for (int i = 0; i < 3; ++i)
          f[3 * int64_t(c->m.h_conn[4 * e + a]) + i] += fb[i] * c->m.h_V[e] / 4.0;
    c->h_fbody = f;
    return rebuild_fext(c);
  });
}

nle_status nle_set_load_scale(nle_ctx *ctx, double s) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!c) return NLE_E_INVAL;
  if (!std::isfinite(s)) return fail(c, NLE_E_INVAL, "non-finite load scale");
  c->load_scale = s;
  return NLE_OK;
}

namespace {
// Per-element unit fibres (and, when sheet is given, sheet directions
// orthogonal to them), reordered into the element partition's order.
nle_status set_frame(Ctx *c, const double *fib, const double *sheet) {
  nle_status s = need_mesh(c);
  if (s != NLE_OK) return s;
  if (c->mixed && c->mx.n_p > 0)
    return fail(c, NLE_E_UNSUPPORTED, "fibres belong to meshes without a pressure field");
  if (!fib) return fail(c, NLE_E_INVAL, "null fibre array");
  return guarded(c, [&]() -> nle_status {
    // P1 meshes store per-element data in the block order, quadratic
    // displacement meshes in the caller's element order
    const int64_t ne = c->mixed ? c->mx.n_e : c->m.n_elems;
    const int nv = sheet ? 2 : 1;
    std::vector<double> f64(3 * nv * ne);
    std::vector<float> f32(3 * nv * ne);
    for (int64_t k = 0; k < ne; ++k) {
      const int64_t e = c->mixed ? k : c->m.h_perm[k];
      for (int v = 0; v < nv; ++v) {
        const double *f = (v == 0 ? fib : sheet) + 3 * e;
        const double l2 = f[0] * f[0] + f[1] * f[1] + f[2] * f[2];
        if (!std::isfinite(l2) || !(std::fabs(l2 - 1.0) <= 1e-6))
          return fail(c, NLE_E_INVAL, "fibres and sheets must be finite unit vectors");
        for (int j = 0; j < 3; ++j) {
          f64[(3 * v + j) * ne + k] = f[j];
          f32[(3 * v + j) * ne + k] = float(f[j]);
        }
      }
      if (sheet) {
        const double *f = fib + 3 * e, *sh = sheet + 3 * e;
        if (!(std::fabs(f[0] * sh[0] + f[1] * sh[1] + f[2] * sh[2]) <= 1e-6))
          return fail(c, NLE_E_INVAL, "sheets must be orthogonal to the fibres");
      }
    }
    drop_graph(c);
    NLE_HIP(c, hipStreamSynchronize(c->stream));
    for (void *p : c->fib_allocs) dfree(c, p);
    c->fib_allocs.clear();
    c->fib64 = static_cast<double *>(dalloc(c, f64.size() * 8));
    c->fib32 = static_cast<float *>(dalloc(c, f32.size() * 4));
    c->fib_allocs = {c->fib64, c->fib32};
    if (!c->fib64 || !c->fib32) {
      c->fib64 = nullptr;
      c->fib32 = nullptr;
      c->sh64 = nullptr;
      c->sh32 = nullptr;
      return fail(c, NLE_E_OOM, "device allocation failed");
    }
    c->sh64 = sheet ? c->fib64 + 3 * ne : nullptr;
    c->sh32 = sheet ? c->fib32 + 3 * ne : nullptr;
    NLE_HIP(c, hipMemcpyAsync(c->fib64, f64.data(), f64.size() * 8, hipMemcpyHostToDevice, c->stream));
    NLE_HIP(c, hipMemcpyAsync(c->fib32, f32.data(), f32.size() * 4, hipMemcpyHostToDevice, c->stream));
    NLE_HIP(c, hipStreamSynchronize(c->stream));
    c->lin64 = c->lin32 = c->lc_valid = false;
    return NLE_OK;
  });
}
}  // namespace

nle_status nle_set_fibres(nle_ctx *ctx, const double *fib) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!c) return NLE_E_INVAL;
  return set_frame(c, fib, nullptr);
}

nle_status nle_set_fibre_frame(nle_ctx *ctx, const double *fib, const double *sheet) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!c) return NLE_E_INVAL;
  if (!sheet) return fail(c, NLE_E_INVAL, "null sheet array");
  return set_frame(c, fib, sheet);
}

nle_status nle_set_active_tension(nle_ctx *ctx, double gamma) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  if (!c) return NLE_E_INVAL;
  if (!std::isfinite(gamma)) return fail(c, NLE_E_INVAL, "non-finite active tension");
  if (gamma != c->mat.gamma) {
    drop_graph(c);
    c->mat.gamma = gamma;
    c->lin64 = c->lin32 = c->lc_valid = false;
  }
  return NLE_OK;
}

namespace {
nle_status check_tri(Ctx *c, int64_t nf, const int32_t *tri, std::vector<int32_t> *out) {
  if (nf < 0 || (nf > 0 && !tri)) return fail(c, NLE_E_INVAL, "bad face arrays");
  out->assign(tri, tri + 3 * nf);
  for (int32_t v : *out)
    if (v < 0 || v >= c->m.n_nodes) return fail(c, NLE_E_INVAL, "face node out of range");
  return NLE_OK;
}
}  // namespace

nle_status nle_set_pressure(nle_ctx *ctx, int64_t nf, const int32_t *tri, double p) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  nle_status s = need_mesh(c);
  if (s != NLE_OK) return s;
  if (c->mixed && c->mx.n_p > 0)
    return fail(c, NLE_E_UNSUPPORTED, "surface loads need a mesh without a pressure field");
  if (!std::isfinite(p)) return fail(c, NLE_E_INVAL, "non-finite pressure");
  return guarded(c, [&]() -> nle_status {
    std::vector<int32_t> t;
    nle_status st = check_tri(c, nf, tri, &t);
    if (st != NLE_OK) return st;
    c->surf.p = p;
    c->lin64 = c->lin32 = c->lc_valid = false;
    if (t == c->surf.h_ptri) return NLE_OK;
    c->surf.h_ptri = t;
    return build_surface(c);
  });
}

nle_status nle_set_traction_follower(nle_ctx *ctx, int64_t nf, const int32_t *tri, const double *t) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  nle_status s = need_mesh(c);
  if (s != NLE_OK) return s;
  if (c->mixed) return fail(c, NLE_E_UNSUPPORTED, "not available on mixed meshes");
  if (!t) return fail(c, NLE_E_INVAL, "null traction");
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(t[i])) return fail(c, NLE_E_INVAL, "non-finite traction");
  return guarded(c, [&]() -> nle_status {
    std::vector<int32_t> tv;
    nle_status st = check_tri(c, nf, tri, &tv);
    if (st != NLE_OK) return st;
    for (int i = 0; i < 3; ++i) c->surf.tf[i] = t[i];
    drop_graph(c);  // the traction is a kernel argument of captured chunks
    c->lin64 = c->lin32 = c->lc_valid = false;
    if (tv == c->surf.h_ttri) return NLE_OK;
    c->surf.h_ttri = tv;
    return build_surface(c);
  });
}

nle_status nle_set_inertia(nle_ctx *ctx, double rho, double coef, const double *ut) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  nle_status s = need_mesh(c);
  if (s != NLE_OK) return s;
  if (c->mixed) return fail(c, NLE_E_UNSUPPORTED, "not available on mixed meshes");
  if (!std::isfinite(rho) || !std::isfinite(coef) || rho < 0.0 || coef < 0.0)
    return fail(c, NLE_E_INVAL, "rho and the coefficient must be finite and >= 0");
  return guarded(c, [&]() -> nle_status {
    const bool on = rho > 0.0 && coef > 0.0;
    if (on && !ut) return fail(c, NLE_E_INVAL, "null u_tilde");
    const int64_t nn = c->m.n_nodes, n = 3 * nn;
    if (on != c->inr.on) drop_graph(c);  // the inertia pointers are kernel arguments
    if (on && !c->inr.cm64) {
      c->inr.cm64 = static_cast<double *>(dalloc(c, size_t(n) * 8));
      c->inr.cm32 = static_cast<float *>(dalloc(c, size_t(n) * 4));
      c->inr.ut = static_cast<double *>(dalloc(c, size_t(n) * 8));
      for (void *p : {(void *)c->inr.cm64, (void *)c->inr.cm32, (void *)c->inr.ut})
        if (p) c->mesh_allocs.push_back(p);
      if (!c->inr.cm64 || !c->inr.cm32 || !c->inr.ut) {
        for (void *p : {(void *)c->inr.cm64, (void *)c->inr.cm32, (void *)c->inr.ut}) {
          if (!p) continue;
          dfree(c, p);
          c->mesh_allocs.erase(std::find(c->mesh_allocs.begin(), c->mesh_allocs.end(), p));
        }
        c->inr = decltype(c->inr)();
        return fail(c, NLE_E_OOM, "device allocation failed (inertia)");
      }
      c->inr.rho = c->inr.c = -1.0;  // force the mass upload below
    }
    c->inr.on = on;
    c->lin64 = c->lin32 = c->lc_valid = false;
    if (!on) return NLE_OK;
    if (rho != c->inr.rho || coef != c->inr.c) {
      // row-sum lumped P1 mass: rho V / 4 per element vertex, times coef
      std::vector<double> m(nn, 0.0);
      for (int64_t e = 0; e < c->m.n_elems; ++e)
        for (int a = 0; a < 4; ++a) m[c->m.h_conn[4 * e + a]] += rho * c->m.h_V[e] / 4.0;
      std::vector<double> cm(n);
      std::vector<float> cm32(n);
      for (int64_t k = 0; k < n; ++k) {
        cm[k] = coef * m[k / 3];
        cm32[k] = float(cm[k]);
      }
      NLE_HIP(c, hipMemcpyAsync(c->inr.cm64, cm.data(), n * 8, hipMemcpyHostToDevice, c->stream));
      NLE_HIP(c, hipMemcpyAsync(c->inr.cm32, cm32.data(), n * 4, hipMemcpyHostToDevice, c->stream));
      NLE_HIP(c, hipStreamSynchronize(c->stream));
      c->inr.rho = rho;
      c->inr.c = coef;
    }
    NLE_HIP(c, hipMemcpyAsync(c->inr.ut, ut, n * 8, hipMemcpyDeviceToDevice, c->stream));
    return NLE_OK;
  });
}

nle_status nle_newmark_predict(nle_ctx *ctx, double dt, double beta, double gamma,
                               const double *u, const double *v, const double *a, double *ut,
                               double *vt) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  nle_status s = need_mesh(c);
  if (s != NLE_OK) return s;
  if (!u || !v || !a || !ut) return fail(c, NLE_E_INVAL, "null vector");
  if (!(dt > 0.0) || !(beta > 0.0)) return fail(c, NLE_E_INVAL, "dt and beta must be positive");
  if (!std::isfinite(gamma)) return fail(c, NLE_E_INVAL, "non-finite gamma");
  NLE_HIP(c, newmark_predict(c, u, v, a, ut, vt, dt, beta, gamma, ndof(c)));
  return NLE_OK;
}

nle_status nle_set_robin_damping(nle_ctx *ctx, double c_perp, double c_par) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  nle_status s = need_mesh(c);
  if (s != NLE_OK) return s;
  if (c->mixed && c->mx.n_p > 0)
    return fail(c, NLE_E_UNSUPPORTED, "surface loads need a mesh without a pressure field");
  if (!std::isfinite(c_perp) || !std::isfinite(c_par) || c_perp < 0.0 || c_par < 0.0)
    return fail(c, NLE_E_INVAL, "dashpot coefficients must be finite and >= 0");
  drop_graph(c);  // kernel arguments of captured chunks
  c->surf.cperp = c_perp;
  c->surf.cpar = c_par;
  c->lin64 = c->lin32 = c->lc_valid = false;
  return NLE_OK;
}

nle_status nle_set_step_velocity(nle_ctx *ctx, double cv, const double *vt) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  nle_status s = need_mesh(c);
  if (s != NLE_OK) return s;
  if (c->mixed) return fail(c, NLE_E_UNSUPPORTED, "not available on mixed meshes");
  if (!std::isfinite(cv) || cv < 0.0) return fail(c, NLE_E_INVAL, "cv must be finite and >= 0");
  if (cv > 0.0 && !vt) return fail(c, NLE_E_INVAL, "null v_tilde");
  return guarded(c, [&]() -> nle_status {
    const int64_t n = 3 * c->m.n_nodes;
    if (cv > 0.0 && !c->inr.vt) {
      c->inr.vt = static_cast<double *>(dalloc(c, size_t(n) * 8));
      if (!c->inr.vt) return fail(c, NLE_E_OOM, "device allocation failed (step velocity)");
      c->mesh_allocs.push_back(c->inr.vt);
    }
    if (cv != c->inr.cv) drop_graph(c);  // a kernel argument of captured chunks
    c->inr.cv = cv;
    c->lin64 = c->lin32 = c->lc_valid = false;
    if (cv > 0.0)
      NLE_HIP(c, hipMemcpyAsync(c->inr.vt, vt, n * 8, hipMemcpyDeviceToDevice, c->stream));
    return NLE_OK;
  });
}

nle_status nle_newmark_correct(nle_ctx *ctx, double dt, double beta, double gamma,
                               const double *u, const double *ut, double *v, double *a) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  nle_status s = need_mesh(c);
  if (s != NLE_OK) return s;
  if (!u || !ut || !v || !a) return fail(c, NLE_E_INVAL, "null vector");
  if (!(dt > 0.0) || !(beta > 0.0)) return fail(c, NLE_E_INVAL, "dt and beta must be positive");
  if (!std::isfinite(dt) || !std::isfinite(beta) || !std::isfinite(gamma))
    return fail(c, NLE_E_INVAL, "dt, beta and gamma must be finite");
  NLE_HIP(c, newmark_correct(c, u, ut, v, a, dt, beta, gamma, ndof(c)));
  return NLE_OK;
}

nle_status nle_set_robin(nle_ctx *ctx, int64_t nf, const int32_t *tri, double k_perp, double k_par) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  nle_status s = need_mesh(c);
  if (s != NLE_OK) return s;
  if (c->mixed && c->mx.n_p > 0)
    return fail(c, NLE_E_UNSUPPORTED, "surface loads need a mesh without a pressure field");
  if (!std::isfinite(k_perp) || !std::isfinite(k_par))
    return fail(c, NLE_E_INVAL, "non-finite spring constants");
  return guarded(c, [&]() -> nle_status {
    std::vector<int32_t> t;
    nle_status st = check_tri(c, nf, tri, &t);
    if (st != NLE_OK) return st;
    if (k_perp != c->surf.kperp || k_par != c->surf.kpar) drop_graph(c);
    c->surf.kperp = k_perp;
    c->surf.kpar = k_par;
    c->lin64 = c->lin32 = c->lc_valid = false;
    if (t == c->surf.h_rtri) return NLE_OK;
    c->surf.h_rtri = t;
    return build_surface(c);
  });
}

nle_status nle_lift(nle_ctx *ctx, double *u) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  nle_status s = need_mesh(c);
  if (s != NLE_OK) return s;
  if (!u) return fail(c, NLE_E_INVAL, "null vector");
  NLE_HIP(c, vec_lift(c, u));
  return NLE_OK;
}

nle_status nle_residual(nle_ctx *ctx, const double *u, double *r, double *rn) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  nle_status s = need_mesh(c);
  if (s != NLE_OK) return s;
  if (!c->has_mat) return fail(c, NLE_E_STATE, "no material set");
  if (!u || !r) return fail(c, NLE_E_INVAL, "null vector");
  s = need_fibres(c);
  if (s != NLE_OK) return s;
  if (rn) {
    bool inv = false;
    s = residual_norm(c, u, r, rn, &inv);
    if (s != NLE_OK) return s;
    return inv ? fail(c, NLE_DIVERGED_INVERTED, "element with det F <= 0") : NLE_OK;
  }
  hipError_t e;
  elem_apply(c, OP_RES, NLE_FP64, u, nullptr, r, c->red, &e);
  if (e != hipSuccess) return fail(c, NLE_E_HIP, std::string("residual: ") + hipGetErrorString(e));
  return NLE_OK;
}

nle_status nle_linearize(nle_ctx *ctx, const double *u, int32_t prec) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  nle_status s = need_mesh(c);
  if (s != NLE_OK) return s;
  if (!c->has_mat) return fail(c, NLE_E_STATE, "no material set");
  if (!u) return fail(c, NLE_E_INVAL, "null vector");
  if (prec != NLE_FP64 && prec != NLE_FP32) return fail(c, NLE_E_INVAL, "bad precision");
  s = need_fibres(c);
  if (s != NLE_OK) return s;
  return linearize(c, u, prec);
}

nle_status nle_jv(nle_ctx *ctx, const void *v, void *y, int32_t prec) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  nle_status s = need_mesh(c);
  if (s != NLE_OK) return s;
  if (!v || !y) return fail(c, NLE_E_INVAL, "null vector");
  if (prec != NLE_FP64 && prec != NLE_FP32) return fail(c, NLE_E_INVAL, "bad precision");
  if ((prec == NLE_FP64 && !c->lin64) || (prec == NLE_FP32 && !c->lin32))
    return fail(c, NLE_E_STATE, "nle_jv needs nle_linearize in this precision first");
  return jv(c, v, y, prec);
}

nle_status nle_jv_noalloc(nle_ctx *ctx, const void *v, void *y, int32_t prec) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  nle_status s = need_mesh(c);
  if (s != NLE_OK) return s;
  if (!v || !y) return fail(c, NLE_E_INVAL, "null vector");
  if (prec != NLE_FP64 && prec != NLE_FP32) return fail(c, NLE_E_INVAL, "bad precision");
  if ((prec == NLE_FP64 && !c->lin64) || (prec == NLE_FP32 && !c->lin32))
    return fail(c, NLE_E_STATE, "nle_jv_noalloc needs nle_linearize in this precision first");
  if (c->mixed)
    return fail(c, NLE_E_UNSUPPORTED, "nle_jv_noalloc takes P1 meshes (the partial sums of "
                                      "shared nodes are its workspace)");
  if (!c->noalloc_ws) return fail(c, NLE_E_STATE, "no fixed workspace on this device");
  const size_t need = size_t(c->m.n_fx) * 3 * (prec == NLE_FP32 ? 4 : 8);
  if (need > NOALLOC_SCRATCH_BYTES)
    return fail(c, NLE_E_INVAL, "nle_jv_noalloc: the mesh's shared-slot partial sums need " +
                                    std::to_string(need) + " bytes, more than the fixed " +
                                    std::to_string(NOALLOC_SCRATCH_BYTES) + "-byte workspace");
  // same kernels as nle_jv, with the partial sums in the fixed workspace
  void *own = c->partial;
  c->partial = c->noalloc_ws;
  const nle_status r = jv(c, v, y, prec);
  c->partial = own;
  return r;
}

nle_status nle_diag(nle_ctx *ctx, double *d) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  nle_status s = need_mesh(c);
  if (s != NLE_OK) return s;
  if (!d) return fail(c, NLE_E_INVAL, "null vector");
  if (!c->lin64) return fail(c, NLE_E_STATE, "nle_diag needs nle_linearize first");
  NLE_HIP(c, hipMemcpyAsync(d, c->diag64, ndof(c) * 8, hipMemcpyDeviceToDevice, c->stream));
  return NLE_OK;
}

nle_status nle_block_diag(nle_ctx *ctx, double *b) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  nle_status s = need_mesh(c);
  if (s != NLE_OK) return s;
  if (!b) return fail(c, NLE_E_INVAL, "null vector");
  if (!c->lin64) return fail(c, NLE_E_STATE, "nle_block_diag needs nle_linearize first");
  s = ensure_block(c);
  if (s != NLE_OK) return s;
  const size_t nn = size_t(c->m.n_nodes);
  NLE_HIP(c, hipMemcpy2DAsync(b, 48, c->diag64, 24, 24, nn, hipMemcpyDeviceToDevice, c->stream));
  NLE_HIP(c, hipMemcpy2DAsync(b + 3, 48, c->odiag64, 24, 24, nn, hipMemcpyDeviceToDevice,
                              c->stream));
  return NLE_OK;
}

nle_status nle_pc_apply(nle_ctx *ctx, int32_t pc, int32_t prec, const void *x, void *y) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  nle_status s = need_mesh(c);
  if (s != NLE_OK) return s;
  if (!x || !y) return fail(c, NLE_E_INVAL, "null vector");
  if (prec != NLE_FP64 && prec != NLE_FP32) return fail(c, NLE_E_INVAL, "bad precision");
  if (pc != NLE_PC_NONE && pc != NLE_PC_JACOBI && pc != NLE_PC_BJACOBI3 && pc != NLE_PC_AMG)
    return fail(c, NLE_E_INVAL, "bad pc");
  if (!(prec == NLE_FP32 ? c->lin32 : c->lin64))
    return fail(c, NLE_E_STATE, "nle_pc_apply needs nle_linearize at this precision first");
  const int64_t n = ndof(c);
  if (pc == NLE_PC_AMG) {
    if (x == y) return fail(c, NLE_E_INVAL, "the multigrid cycle cannot run in place");
    s = amg_prepare(c);
    if (s != NLE_OK) return s;
    NLE_HIP(c, amg_apply(c, prec, x, y));
    return NLE_OK;
  }
  if (pc == NLE_PC_NONE) {
    NLE_HIP(c, hipMemcpyAsync(y, x, size_t(n) * (prec == NLE_FP32 ? 4 : 8),
                              hipMemcpyDeviceToDevice, c->stream));
    return NLE_OK;
  }
  const void *d;
  int pcb = 1;
  if (pc == NLE_PC_BJACOBI3) {
    s = ensure_block(c);
    if (s != NLE_OK) return s;
    d = prec == NLE_FP32 ? static_cast<const void *>(c->binv32) : static_cast<const void *>(c->binv64);
    pcb = 3;
  } else {
    d = prec == NLE_FP32 ? static_cast<const void *>(c->dinv32) : static_cast<const void *>(c->dinv64);
  }
  NLE_HIP(c, pc_apply(c, prec, pcb, d, x, y, n));
  return NLE_OK;
}

nle_status nle_schur_apply(nle_ctx *ctx, int32_t pc, int32_t schur, int32_t prec, const void *x,
                           void *y) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  nle_status s = need_mesh(c);
  if (s != NLE_OK) return s;
  if (!x || !y) return fail(c, NLE_E_INVAL, "null vector");
  if (x == y) return fail(c, NLE_E_INVAL, "the Schur preconditioner cannot run in place");
  if (prec != NLE_FP64 && prec != NLE_FP32) return fail(c, NLE_E_INVAL, "bad precision");
  if (pc != NLE_PC_JACOBI && pc != NLE_PC_AMG) return fail(c, NLE_E_INVAL, "bad pc");
  if (schur != NLE_SCHUR_LOWER_MASS && schur != NLE_SCHUR_LOWER_SIMPLE)
    return fail(c, NLE_E_INVAL, "bad schur");
  if (!(c->mixed && c->mx.n_p > 0))
    return fail(c, NLE_E_UNSUPPORTED, "the Schur forms need a displacement / pressure mesh");
  if (schur == NLE_SCHUR_LOWER_SIMPLE && c->mx.npe != 1)
    return fail(c, NLE_E_UNSUPPORTED, "SIMPLE is built for the constant-pressure pair");
  if (!(prec == NLE_FP32 ? c->lin32 : c->lin64))
    return fail(c, NLE_E_STATE, "nle_schur_apply needs nle_linearize at this precision first");
  if (pc == NLE_PC_AMG) {
    s = amg_prepare(c);
    if (s != NLE_OK) return s;
  }
  if (schur == NLE_SCHUR_LOWER_SIMPLE) NLE_HIP(c, mixed_simple_diag(c));
  const size_t vb = size_t(ndof(c)) * (prec == NLE_FP32 ? 4 : 8);
  void *t1 = dalloc(c, vb), *t2 = dalloc(c, vb);
  if (!t1 || !t2) {
    dfree(c, t1);
    dfree(c, t2);
    return fail(c, NLE_E_OOM, "device allocation failed");
  }
  const hipError_t e = schur_lower_apply(c, prec, pc == NLE_PC_AMG, schur, x, y, t1, t2);
  const hipError_t e2 = hipStreamSynchronize(c->stream);
  dfree(c, t1);
  dfree(c, t2);
  if (e != hipSuccess || e2 != hipSuccess)
    return fail(c, NLE_E_HIP, std::string("schur apply: ") +
                                  hipGetErrorString(e != hipSuccess ? e : e2));
  return NLE_OK;
}

nle_status nle_simple_diag(nle_ctx *ctx, double *s_dev) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  nle_status s = need_mesh(c);
  if (s != NLE_OK) return s;
  if (!s_dev) return fail(c, NLE_E_INVAL, "null vector");
  if (!(c->mixed && c->mx.n_p > 0 && c->mx.npe == 1))
    return fail(c, NLE_E_UNSUPPORTED, "SIMPLE is built for the constant-pressure pair");
  if (!c->lin64) return fail(c, NLE_E_STATE, "nle_simple_diag needs nle_linearize first");
  NLE_HIP(c, mixed_simple_diag(c, s_dev));
  return NLE_OK;
}

nle_status nle_energy(nle_ctx *ctx, const double *u, double *pi) {
  Ctx *c = reinterpret_cast<Ctx *>(ctx);
  nle_status s = need_mesh(c);
  if (s != NLE_OK) return s;
  if (!c->has_mat) return fail(c, NLE_E_STATE, "no material set");
  if (!u || !pi) return fail(c, NLE_E_INVAL, "null argument");
  if (c->surf.npf + c->surf.ntf > 0)
    return fail(c, NLE_E_UNSUPPORTED, "a follower load has no potential");
  if (damping_on(c)) return fail(c, NLE_E_UNSUPPORTED, "dashpots have no potential here");
  s = need_fibres(c);
  if (s != NLE_OK) return s;
  hipError_t e;
  const int np = elem_apply(c, OP_ENERGY, NLE_FP64, u, nullptr, nullptr, c->red, &e);
  if (e != hipSuccess) return fail(c, NLE_E_HIP, std::string("energy: ") + hipGetErrorString(e));
  NLE_HIP(c, reduce_scalar(c, c->red, np, c->dscal + 60));
  double *red2 = c->red + np;
  const int np2 = vec_dot_partials(c, NLE_FP64, c->fext, u, 3 * c->m.n_nodes, red2, &e);
  if (e != hipSuccess) return fail(c, NLE_E_HIP, "energy dot");
  NLE_HIP(c, reduce_scalar(c, red2, np2, c->dscal + 61));
  int np3 = 0;
  double *red3 = red2 + np2;
  const int64_t nsg = (c->surf.nsn + NT - 1) / NT;
  if (np + np2 + nsg > c->red_cap) return fail(c, NLE_E_UNSUPPORTED, "too many face nodes");
  surf_apply(c, OP_ENERGY, NLE_FP64, u, nullptr, &np3, &e, red3);
  if (e != hipSuccess) return fail(c, NLE_E_HIP, "spring energy");
  if (np3 > 0) {
    NLE_HIP(c, reduce_scalar(c, red3, np3, c->dscal + 62));
  } else {
    NLE_HIP(c, hipMemsetAsync(c->dscal + 62, 0, 8, c->stream));
  }
  // inertia of the time step: c/2 (u - u~)^T M (u - u~)
  if (c->inr.on) {
    double *red4 = red3 + np3;
    const int64_t n = 3 * c->m.n_nodes;
    if (np + np2 + nsg + vgrid(n) > c->red_cap)
      return fail(c, NLE_E_UNSUPPORTED, "reduction space");
    const int np4 = vec_wdiff2_partials(c, c->inr.cm64, u, c->inr.ut, n, red4, &e);
    if (e != hipSuccess) return fail(c, NLE_E_HIP, "inertia energy");
    NLE_HIP(c, reduce_scalar(c, red4, np4, c->dscal + 63));
  } else {
    NLE_HIP(c, hipMemsetAsync(c->dscal + 63, 0, 8, c->stream));
  }
  s = read_scalars(c, c->dscal + 60, 32);
  if (s != NLE_OK) return s;
  *pi = c->hpin[0] - c->load_scale * c->hpin[1] + c->hpin[2] + 0.5 * c->hpin[3];
  return NLE_OK;
}

nle_status nle_amg_levels(const nle_ctx *ctx, int32_t *n_levels, int64_t *sizes, int32_t cap) {
  const Ctx *c = reinterpret_cast<const Ctx *>(ctx);
  if (!c || !n_levels || (cap > 0 && !sizes) || cap < 0) return NLE_E_INVAL;
  *n_levels = amg_levels(c, sizes, cap);
  return NLE_OK;
}

nle_status nle_partition_info(const nle_ctx *ctx, int64_t *info) {
  const Ctx *c = reinterpret_cast<const Ctx *>(ctx);
  if (!c || !info) return NLE_E_INVAL;
  if (!c->has_mesh) return NLE_E_STATE;
  if (c->mixed) return NLE_E_UNSUPPORTED;
  const Mesh &M = c->m;
  info[0] = M.nblk;
  info[1] = M.be_max;
  info[2] = M.nl_max;
  info[3] = M.n_slots;
  info[4] = M.n_shared;
  info[5] = M.n_fx;
  info[6] = int64_t(9 * M.nl_max + 12 * M.be_max) * 8;
  info[7] = int64_t(9 * M.nl_max + 12 * M.be_max) * 4;
  return NLE_OK;
}

}  // extern "C"
