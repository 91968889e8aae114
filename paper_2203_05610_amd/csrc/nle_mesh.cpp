// Host-side mesh preparation: validation, P1 geometry, element partition into
// blocks, block-local connectivity / contribution lists and the merge lists of
// nodes shared between blocks.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "nle_internal.hpp"

namespace nle {

namespace {

// Recursive coordinate bisection of elements into blocks of exactly `be`
// elements (the last block may be smaller).  Each split puts a multiple of
// `be` elements on the lower side along the longest extent of the centroids.
void rcb(std::vector<int64_t> &idx, int64_t lo, int64_t hi, const std::vector<double> &cen,
         int64_t be, std::vector<int64_t> &starts) {
  const int64_t n = hi - lo;
  if (n <= be) {
    starts.push_back(lo);
    return;
  }
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t k = lo; k < hi; ++k)
    for (int d = 0; d < 3; ++d) {
      double v = cen[3 * idx[k] + d];
      mn[d] = std::min(mn[d], v);
      mx[d] = std::max(mx[d], v);
    }
  int ax = 0;
  for (int d = 1; d < 3; ++d)
    if (mx[d] - mn[d] > mx[ax] - mn[ax]) ax = d;
  const int64_t nb = (n + be - 1) / be;
  const int64_t nl = (nb / 2) * be;
  auto cmp = [&](int64_t a, int64_t b) {
    double va = cen[3 * a + ax], vb = cen[3 * b + ax];
    return va < vb || (va == vb && a < b);
  };
  std::nth_element(idx.begin() + lo, idx.begin() + lo + nl, idx.begin() + hi, cmp);
  rcb(idx, lo, lo + nl, cen, be, starts);
  rcb(idx, lo + nl, hi, cen, be, starts);
}

template <typename T>
T *upload(Ctx *c, const std::vector<T> &h, hipError_t *e) {
  if (h.empty()) return nullptr;
  T *d = static_cast<T *>(dalloc(c, h.size() * sizeof(T)));
  if (!d) {
    *e = hipErrorOutOfMemory;
    return nullptr;
  }
  c->mesh_allocs.push_back(d);
  hipError_t r = hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, c->stream);
  if (r != hipSuccess) *e = r;
  return d;
}

}  // namespace

nle_status build_mesh(Ctx *c, int64_t nn, const double *X, int64_t ne, const int32_t *conn,
                      const std::vector<int64_t> *inst_elem, const std::vector<int64_t> *inst_node) {
  std::vector<int64_t> ie = inst_elem ? *inst_elem : std::vector<int64_t>{0, ne};
  std::vector<int64_t> in = inst_node ? *inst_node : std::vector<int64_t>{0, nn};
  const int32_t n_inst = int32_t(ie.size()) - 1;
  if (nn <= 0 || ne <= 0) return fail(c, NLE_E_INVAL, "mesh needs n_nodes > 0 and n_elems > 0");
  if (nn >= (int64_t(1) << 28)) return fail(c, NLE_E_UNSUPPORTED, "n_nodes must be < 2^28");
  if (!X || !conn) return fail(c, NLE_E_INVAL, "null mesh array");
  // ---- validation and geometry (FP64) ------------------------------------
  std::vector<double> G(9 * ne), V(ne), cen(3 * ne);
  for (int64_t e = 0; e < ne; ++e) {
    const int32_t *v = conn + 4 * e;
    for (int a = 0; a < 4; ++a) {
      if (v[a] < 0 || v[a] >= nn)
        return fail(c, NLE_E_BADMESH, "element " + std::to_string(e) + ": node index out of range");
      for (int b = 0; b < a; ++b)
        if (v[a] == v[b])
          return fail(c, NLE_E_BADMESH, "element " + std::to_string(e) + ": repeated node");
    }
    const double *x0 = X + 3 * int64_t(v[0]);
    double D[3][3];  // columns X_a - X_0
    for (int a = 1; a < 4; ++a) {
      const double *xa = X + 3 * int64_t(v[a]);
      for (int i = 0; i < 3; ++i) D[i][a - 1] = xa[i] - x0[i];
    }
    // cofactors of D; D^-1 = cof(D)^T / det D
    double C[3][3];
    C[0][0] = D[1][1] * D[2][2] - D[1][2] * D[2][1];
    C[0][1] = D[1][2] * D[2][0] - D[1][0] * D[2][2];
    C[0][2] = D[1][0] * D[2][1] - D[1][1] * D[2][0];
    C[1][0] = D[0][2] * D[2][1] - D[0][1] * D[2][2];
    C[1][1] = D[0][0] * D[2][2] - D[0][2] * D[2][0];
    C[1][2] = D[0][1] * D[2][0] - D[0][0] * D[2][1];
    C[2][0] = D[0][1] * D[1][2] - D[0][2] * D[1][1];
    C[2][1] = D[0][2] * D[1][0] - D[0][0] * D[1][2];
    C[2][2] = D[0][0] * D[1][1] - D[0][1] * D[1][0];
    const double det = D[0][0] * C[0][0] + D[0][1] * C[0][1] + D[0][2] * C[0][2];
    double scale = 0.0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) scale = std::max(scale, std::fabs(D[i][j]));
    if (!(det > 1e-14 * scale * scale * scale))
      return fail(c, NLE_E_BADMESH,
                  "element " + std::to_string(e) + ": non-positive or degenerate volume");
    // grad N_a (a = 1..3) = row a-1 of D^-1 = column a-1 of cof(D) / det
    for (int a = 0; a < 3; ++a)
      for (int J = 0; J < 3; ++J) G[(3 * a + J) * ne + e] = C[J][a] / det;
    V[e] = det / 6.0;
    for (int i = 0; i < 3; ++i) {
      double s = 0.0;
      for (int a = 0; a < 4; ++a) s += X[3 * int64_t(v[a]) + i];
      cen[3 * e + i] = 0.25 * s;
    }
  }

  // ---- partition -------------------------------------------------------------
  const int64_t be = c->be_req;
  std::vector<int64_t> perm(ne);
  std::iota(perm.begin(), perm.end(), int64_t(0));
  std::vector<int64_t> starts;
  std::vector<int32_t> inst_blk(n_inst + 1, 0);
  for (int32_t i = 0; i < n_inst; ++i) {  // blocks never span two instances
    const size_t s0 = starts.size();
    rcb(perm, ie[i], ie[i + 1], cen, be, starts);
    std::sort(starts.begin() + s0, starts.end());
    inst_blk[i + 1] = int32_t(starts.size());
  }
  const int32_t nblk = int32_t(starts.size());
  std::vector<int32_t> blk_elem(nblk + 1), blk_inst(nblk);
  for (int32_t b = 0; b < nblk; ++b) blk_elem[b] = int32_t(starts[b]);
  blk_elem[nblk] = int32_t(ne);
  for (int32_t i = 0; i < n_inst; ++i)
    for (int32_t b = inst_blk[i]; b < inst_blk[i + 1]; ++b) blk_inst[b] = i;
  for (int32_t b = 0; b < nblk; ++b)  // elements of a block in user order
    std::sort(perm.begin() + blk_elem[b], perm.begin() + blk_elem[b + 1]);

  // ---- per-block node slots, local connectivity, contribution lists ---------
  std::vector<int32_t> blk_node(nblk + 1, 0);
  std::vector<uint32_t> nodes;
  nodes.reserve(size_t(ne));
  std::vector<uint16_t> lcp(8 * ne), csr_end;
  std::vector<int32_t> loc(nn, -1), touch(nn, 0);
  std::vector<int32_t> cnt;
  int32_t be_max = 0, nl_max = 0;
  for (int32_t b = 0; b < nblk; ++b) {
    const int64_t e0 = blk_elem[b], e1 = blk_elem[b + 1];
    std::vector<int32_t> bn;
    bn.reserve(4 * (e1 - e0));
    for (int64_t k = e0; k < e1; ++k)
      for (int a = 0; a < 4; ++a) bn.push_back(conn[4 * perm[k] + a]);
    std::sort(bn.begin(), bn.end());
    bn.erase(std::unique(bn.begin(), bn.end()), bn.end());
    const int32_t nl = int32_t(bn.size());
    if (nl > 65535) return fail(c, NLE_E_UNSUPPORTED, "block touches more than 65535 nodes");
    // slots in decreasing order of their contribution counts (then by node
    // id): the node sums of one wave then run loops of similar length
    {
      for (int32_t l = 0; l < nl; ++l) loc[bn[l]] = l;
      std::vector<int32_t> nc(nl, 0);
      for (int64_t k = e0; k < e1; ++k)
        for (int a = 0; a < 4; ++a) nc[loc[conn[4 * perm[k] + a]]] += 1;
      std::vector<int32_t> ord(nl);
      std::iota(ord.begin(), ord.end(), 0);
      std::stable_sort(ord.begin(), ord.end(),
                       [&](int32_t x, int32_t y) { return nc[x] > nc[y]; });
      std::vector<int32_t> sorted(nl);
      for (int32_t l = 0; l < nl; ++l) sorted[l] = bn[ord[l]];
      bn.swap(sorted);
    }
    for (int32_t l = 0; l < nl; ++l) {
      loc[bn[l]] = l;
      touch[bn[l]] += 1;
    }
    blk_node[b] = int32_t(nodes.size());
    for (int32_t l = 0; l < nl; ++l) nodes.push_back(uint32_t(bn[l]));
    cnt.assign(nl + 1, 0);
    for (int64_t k = e0; k < e1; ++k)
      for (int a = 0; a < 4; ++a) {
        int32_t l = loc[conn[4 * perm[k] + a]];
        lcp[8 * k + a] = uint16_t(l);
        cnt[l + 1] += 1;
      }
    for (int32_t l = 0; l < nl; ++l) cnt[l + 1] += cnt[l];
    for (int32_t l = 0; l < nl; ++l) csr_end.push_back(uint16_t(cnt[l + 1]));
    // position of contribution (element, vertex) in the block's slot-sorted
    // order; within a slot, increasing (element, vertex) order
    std::vector<int32_t> fillp(cnt.begin(), cnt.end() - 1);
    for (int64_t k = e0; k < e1; ++k)
      for (int a = 0; a < 4; ++a) {
        int32_t l = loc[conn[4 * perm[k] + a]];
        lcp[8 * k + 4 + a] = uint16_t(fillp[l]++);
      }
    for (int32_t l = 0; l < nl; ++l) loc[bn[l]] = -1;
    be_max = std::max<int32_t>(be_max, int32_t(e1 - e0));
    nl_max = std::max(nl_max, nl);
  }
  blk_node[nblk] = int32_t(nodes.size());
  const int64_t n_slots = int64_t(nodes.size());
  // slot coordinates relative to the block's first slot: small numbers, so
  // their FP32 copy resolves element edges to ~1e-6 of the edge length
  std::vector<double> xr64(3 * n_slots);
  std::vector<float> xr32(3 * n_slots);
  for (int32_t b = 0; b < nblk; ++b) {
    const double *x0 = X + 3 * int64_t(nodes[blk_node[b]]);
    for (int64_t p = blk_node[b]; p < blk_node[b + 1]; ++p) {
      const double *x = X + 3 * int64_t(nodes[p]);
      for (int i = 0; i < 3; ++i) {
        xr64[3 * p + i] = x[i] - x0[i];
        xr32[3 * p + i] = float(x[i] - x0[i]);
      }
    }
  }

  // ---- shared nodes and their merge lists (slots in block order) -------------
  // With several instances each instance's shared nodes start on a whole
  // merge workgroup (padding entries: id 0xFFFFFFFF, empty slot range).
  std::vector<int32_t> fx_id(nn, -1);
  std::vector<uint32_t> fx_node;
  std::vector<int32_t> inst_mwg(n_inst + 1, 0);
  for (int32_t i = 0; i < n_inst; ++i) {
    for (int64_t g = in[i]; g < in[i + 1]; ++g)
      if (touch[g] >= 2) {
        fx_id[g] = int32_t(fx_node.size());
        fx_node.push_back(uint32_t(g));
      }
    if (n_inst > 1)
      while (fx_node.size() % NT != 0) fx_node.push_back(0xFFFFFFFFu);
    inst_mwg[i + 1] = int32_t((fx_node.size() + NT - 1) / NT);
  }
  const int64_t n_sh = int64_t(fx_node.size());
  std::vector<int32_t> mwg_inst(inst_mwg[n_inst]);
  for (int32_t i = 0; i < n_inst; ++i)
    for (int32_t w = inst_mwg[i]; w < inst_mwg[i + 1]; ++w) mwg_inst[w] = i;
  std::vector<int32_t> fx_ptr(n_sh + 1, 0), fx_slot;
  for (int64_t p = 0; p < n_slots; ++p) {
    int32_t f = fx_id[nodes[p]];
    if (f >= 0) {
      fx_ptr[f + 1] += 1;
      nodes[p] |= 0x80000000u;
    }
  }
  for (int64_t k = 0; k < n_sh; ++k) fx_ptr[k + 1] += fx_ptr[k];
  fx_slot.resize(fx_ptr[n_sh]);
  // mpos[p]: where a shared slot writes its partial sum, so that each shared
  // node's partials are contiguous (in block order) for the merge
  std::vector<int32_t> mpos(n_slots, -1);
  {
    std::vector<int32_t> fp(fx_ptr.begin(), fx_ptr.end() - 1);
    for (int64_t p = 0; p < n_slots; ++p) {  // slots are in block order
      int32_t f = fx_id[nodes[p] & NODE_MASK];
      if (f >= 0) {
        mpos[p] = fp[f];
        fx_slot[fp[f]++] = int32_t(p);
      }
    }
  }
  for (int64_t g = 0; g < nn; ++g)
    if (touch[g] == 0)
      return fail(c, NLE_E_BADMESH, "node " + std::to_string(g) + " belongs to no element");

  // ---- LDS budget ---------------------------------------------------------------
  // see the element kernel: nodal state, contributions, reduction scratch
  const size_t lds64 = size_t(9 * nl_max + 12 * be_max) * 8 + 512 / 64 * 8;
  if (lds64 > c->lds_limit)
    return fail(c, NLE_E_UNSUPPORTED,
                "element block needs " + std::to_string(lds64) + " B of LDS (limit " +
                    std::to_string(c->lds_limit) + "); use a smaller block size");

  // ---- upload ---------------------------------------------------------------------
  for (void *p : c->mesh_allocs) dfree(c, p);
  c->mesh_allocs.clear();
  c->odiag64 = c->binv64 = nullptr;
  c->binv32 = nullptr;
  c->blk_valid = false;
  c->inr = decltype(c->inr)();
  amg_release(c);
  Mesh &M = c->m;
  M = Mesh();
  M.n_nodes = nn;
  M.n_elems = ne;
  M.nblk = nblk;
  M.be_max = be_max;
  M.nl_max = nl_max;
  M.n_slots = n_slots;
  M.n_shared = n_sh;
  M.n_fx = int64_t(fx_slot.size());
  hipError_t herr = hipSuccess;
  M.xr64 = upload(c, xr64, &herr);
  M.xr32 = upload(c, xr32, &herr);
  M.lcp = reinterpret_cast<uint4 *>(upload(c, lcp, &herr));
  M.csr_end = upload(c, csr_end, &herr);
  M.nodes = upload(c, nodes, &herr);
  M.mpos = upload(c, mpos, &herr);
  M.blk_elem = upload(c, blk_elem, &herr);
  M.blk_node = upload(c, blk_node, &herr);
  M.n_inst = n_inst;
  M.n_mwg = inst_mwg[n_inst];
  M.h_inst_elem = ie;
  M.h_inst_node = in;
  M.h_inst_blk = inst_blk;
  M.h_inst_mwg = inst_mwg;
  if (n_inst > 1) {
    M.blk_inst = upload(c, blk_inst, &herr);
    if (!mwg_inst.empty()) M.mwg_inst = upload(c, mwg_inst, &herr);
  }
  if (n_sh > 0) {
    M.fx_node = upload(c, fx_node, &herr);
    M.fx_ptr = upload(c, fx_ptr, &herr);
  }
  void *part = dalloc(c, size_t(n_slots) * 3 * sizeof(double));
  if (!part) herr = hipErrorOutOfMemory;
  c->mesh_allocs.push_back(part);
  c->partial = part;
  double *fext = static_cast<double *>(dalloc(c, size_t(3 * nn) * sizeof(double)));
  if (!fext) herr = hipErrorOutOfMemory;
  c->mesh_allocs.push_back(fext);
  c->fext = fext;
  // linearization buffers
  c->ulin64 = static_cast<double *>(dalloc(c, size_t(3 * nn) * 8));
  c->ulin32 = static_cast<float *>(dalloc(c, size_t(3 * nn) * 4));
  c->diag64 = static_cast<double *>(dalloc(c, size_t(3 * nn) * 8));
  c->dinv64 = static_cast<double *>(dalloc(c, size_t(3 * nn) * 8));
  c->dinv32 = static_cast<float *>(dalloc(c, size_t(3 * nn) * 4));
  for (void *p : {(void *)c->ulin64, (void *)c->ulin32, (void *)c->diag64, (void *)c->dinv64,
                  (void *)c->dinv32}) {
    if (!p) herr = hipErrorOutOfMemory;
    c->mesh_allocs.push_back(p);
  }
  // reduction buffer sized for the largest element grid plus vector grids
  int64_t need = int64_t(elem_red_capacity(c)) + 64 * int64_t(VGRID_MAX) + 64;
  if (need > c->red_cap) {
    if (c->red) dfree(c, c->red);
    c->red = static_cast<double *>(dalloc(c, size_t(need) * 8));
    if (!c->red) herr = hipErrorOutOfMemory;
    c->red_cap = need;
  }
  if (herr == hipErrorOutOfMemory) return fail(c, NLE_E_OOM, "device allocation failed");
  if (herr != hipSuccess) return fail(c, NLE_E_HIP, std::string("upload: ") + hipGetErrorString(herr));
  NLE_HIP(c, hipMemsetAsync(fext, 0, size_t(3 * nn) * 8, c->stream));

  M.h_nodes = nodes;
  M.h_fx_node = fx_node;
  M.h_conn.assign(conn, conn + 4 * ne);
  M.h_V = V;
  M.h_perm = perm;
  M.h_X.assign(X, X + 3 * nn);
  c->h_mask.assign(nn, 0);
  c->h_ftrac.assign(3 * nn, 0.0);
  c->h_fbody.assign(3 * nn, 0.0);
  c->n_dir = 0;
  c->lin64 = c->lin32 = c->lc_valid = false;
  c->load_scale = 1.0;
  NLE_HIP(c, hipStreamSynchronize(c->stream));
  c->mixed = false;
  c->has_mesh = true;
  return NLE_OK;
}

// Re-write the Dirichlet mask bits of the block-node and merge-node words.
nle_status upload_node_masks(Ctx *c) {
  if (c->mixed) return upload_mixed_masks(c);
  Mesh &M = c->m;
  std::vector<uint32_t> nodes(M.h_nodes), fx(M.h_fx_node);
  for (auto &w : nodes) w |= uint32_t(c->h_mask[w & NODE_MASK] & 7u) << 28;
  for (auto &w : fx)
    if (w != 0xFFFFFFFFu) w |= uint32_t(c->h_mask[w] & 7u) << 28;
  NLE_HIP(c, hipMemcpyAsync(M.nodes, nodes.data(), nodes.size() * 4, hipMemcpyHostToDevice, c->stream));
  if (!fx.empty())
    NLE_HIP(c, hipMemcpyAsync(M.fx_node, fx.data(), fx.size() * 4, hipMemcpyHostToDevice, c->stream));
  NLE_HIP(c, hipStreamSynchronize(c->stream));
  return upload_surface_masks(c);
}

}  // namespace nle
