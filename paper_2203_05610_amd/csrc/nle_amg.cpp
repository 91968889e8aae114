// Aggregation multigrid preconditioner (the AMG of Sec. 4 and App. A, whose
// construction the paper leaves to its library): rigid-body candidates,
// two-pass greedy aggregation, orthonormal tentative prolongators by
// modified Gram-Schmidt, Galerkin coarse operators, a degree-2 Chebyshev
// smoother on the finest level and damped Jacobi below (both scaled by
// power-iteration estimates), one V(1,1)-cycle per application.
//
// What depends on the mesh and the Dirichlet set only (graphs, aggregates,
// prolongators, operator patterns, probing tasks) is built once, on the host.
// Per linearization: the finest level's Jacobi weight by a power iteration
// with the matrix-free Jacobian action; the level-1 operator P0^T J P0 by
// probing, i.e. J applied to sums of prolongator columns of aggregates
// whose node neighbourhoods are disjoint (one colour), read off per
// (aggregate, aggregate) pair by a GPU kernel; the small coarser operators
// (a few percent of the fine size) on the host; the coarsest level inverted
// densely.  The cycle itself runs on the GPU, in the Krylov loop's precision.
//
// With a pressure field (the mixed displacement-pressure meshes) the
// hierarchy is built for the displacement block and the preconditioner is
// the block-diagonal field split: the cycle on the displacements, the
// pressure block's diagonal on the pressures.

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <thread>
#include <vector>

#include "nle_amg.hpp"

namespace nle {
namespace {

constexpr int POWER_ITS = 15;
// finest-level Chebyshev smoother: degree, interval [hi / RATIO, hi], hi = SAFETY rho
constexpr int CHEB_DEGREE = 2;
constexpr double CHEB_RATIO = 30.0, CHEB_SAFETY = 1.2;
constexpr int64_t N_COARSE = 300;
constexpr int MAX_LEVELS = 10;
constexpr double DROP_TOL = 1e-8;
constexpr int64_t MAX_DENSE = 4000;

struct Level {
  int64_t n = 0, nv = 0;             // dofs, vertices
  std::vector<int64_t> vbeg;         // [nv+1] first dof of each vertex
  std::vector<int64_t> adjp;         // vertex graph (CSR, sorted, no self)
  std::vector<int32_t> adji;
  // operator (levels >= 1)
  std::vector<int32_t> rp, ci;
  std::vector<double> val, dinv;
  double w = 0.0;
  // transfer to the next level
  std::vector<int32_t> poff, pk, rs, re, ri, arows;
  std::vector<double> pv;
  // device
  int32_t *d_rp = nullptr, *d_ci = nullptr;
  double *d_v64 = nullptr, *d_dinv64 = nullptr, *d_pv64 = nullptr;
  float *d_v32 = nullptr, *d_dinv32 = nullptr, *d_pv32 = nullptr;
  int32_t *d_poff = nullptr, *d_pk = nullptr, *d_rs = nullptr, *d_re = nullptr, *d_ri = nullptr,
          *d_arows = nullptr;
  double *d_b = nullptr, *d_x = nullptr, *d_r = nullptr;  // work vectors (FP32 uses the front)
};

struct Amg {
  std::vector<Level> L;
  std::vector<double> inv;  // coarsest inverse, row-major
  double *d_inv64 = nullptr;
  float *d_inv32 = nullptr;
  // probing of the level-1 operator
  int ncol = 0;
  std::vector<int32_t> tc;  // [ncol+1] task ranges
  int32_t *d_tbeg = nullptr, *d_tend = nullptr, *d_tkp = nullptr, *d_tka = nullptr,
          *d_nodes = nullptr, *d_dcol = nullptr;
  int64_t *d_tdest = nullptr;
  double *d_z = nullptr, *d_y = nullptr, *d_t = nullptr, *d_red = nullptr, *d_s = nullptr;
  double *d_cd = nullptr;  // the Chebyshev direction on the finest level
  // Chebyshev steps j = 1 .. CHEB_DEGREE: d <- cd[j] d + cr[j] D^-1 (b - A x)
  double cheb_cd[CHEB_DEGREE] = {}, cheb_cr[CHEB_DEGREE] = {};
  std::vector<int32_t> agg0, keep0;  // finest aggregation: node -> aggregate -> level-1 vertex
  bool valid = false;
  std::vector<void *> allocs;
};

Amg *state(Ctx *c) { return static_cast<Amg *>(c->amg); }

template <typename P>
bool alloc(Ctx *c, Amg *A, P **p, size_t count) {
  *p = static_cast<P *>(dalloc(c, count * sizeof(P)));
  if (*p) A->allocs.push_back(*p);
  return *p != nullptr;
}

template <typename P>
bool upload(Ctx *c, Amg *A, P **p, const std::vector<P> &h) {
  if (!alloc(c, A, p, std::max<size_t>(h.size(), 1))) return false;
  if (!h.empty() &&
      hipMemcpyAsync(*p, h.data(), h.size() * sizeof(P), hipMemcpyHostToDevice, c->stream) !=
          hipSuccess)
    return false;
  return true;
}

std::vector<float> to32(const std::vector<double> &v) {
  std::vector<float> f(v.size());
  for (size_t i = 0; i < v.size(); ++i) f[i] = float(v[i]);
  return f;
}

// x_i = frac(i * 2654435761 / 2^32) - 1/2
std::vector<double> start_vector(int64_t n) {
  std::vector<double> x(n);
  for (int64_t i = 0; i < n; ++i) {
    const uint64_t h = (uint64_t(i) * 2654435761ull) & 0xFFFFFFFFull;
    x[i] = double(h) / 4294967296.0 - 0.5;
  }
  return x;
}

// two-pass greedy aggregation of a CSR graph
int64_t aggregate(const Level &G, std::vector<int32_t> &agg) {
  const int64_t nv = G.nv;
  agg.assign(nv, -1);
  int64_t na = 0;
  for (int64_t v = 0; v < nv; ++v) {
    if (agg[v] >= 0) continue;
    bool free_nb = true;
    for (int64_t q = G.adjp[v]; q < G.adjp[v + 1] && free_nb; ++q) free_nb = agg[G.adji[q]] < 0;
    if (!free_nb) continue;
    agg[v] = int32_t(na);
    for (int64_t q = G.adjp[v]; q < G.adjp[v + 1]; ++q) agg[G.adji[q]] = int32_t(na);
    ++na;
  }
  const std::vector<int32_t> first = agg;
  for (int64_t v = 0; v < nv; ++v) {
    if (agg[v] >= 0) continue;
    int32_t best = -1;  // lowest-numbered neighbour aggregated in pass 1
    for (int64_t q = G.adjp[v]; q < G.adjp[v + 1]; ++q)
      if (first[G.adji[q]] >= 0) {
        best = G.adji[q];
        break;  // neighbour lists are sorted
      }
    if (best < 0) {  // cannot happen (v would have been a root); keep it alone
      agg[v] = int32_t(na++);
    } else {
      agg[v] = first[best];
    }
  }
  return na;
}

// Gauss-Jordan inverse with partial pivoting; false if singular
bool invert(std::vector<double> &a, int64_t n, std::vector<double> &inv) {
  inv.assign(size_t(n * n), 0.0);
  for (int64_t i = 0; i < n; ++i) inv[i * n + i] = 1.0;
  for (int64_t k = 0; k < n; ++k) {
    int64_t p = k;
    for (int64_t i = k + 1; i < n; ++i)
      if (std::fabs(a[i * n + k]) > std::fabs(a[p * n + k])) p = i;
    if (!(std::fabs(a[p * n + k]) > 0.0)) return false;
    if (p != k)
      for (int64_t j = 0; j < n; ++j) {
        std::swap(a[k * n + j], a[p * n + j]);
        std::swap(inv[k * n + j], inv[p * n + j]);
      }
    const double d = 1.0 / a[k * n + k];
    for (int64_t j = 0; j < n; ++j) {
      a[k * n + j] *= d;
      inv[k * n + j] *= d;
    }
    for (int64_t i = 0; i < n; ++i) {
      if (i == k) continue;
      const double f = a[i * n + k];
      if (f == 0.0) continue;
      for (int64_t j = 0; j < n; ++j) {
        a[i * n + j] -= f * a[k * n + j];
        inv[i * n + j] -= f * inv[k * n + j];
      }
    }
  }
  return true;
}

double host_power(const Level &l) {
  std::vector<double> x = start_vector(l.n), y(l.n);
  double lam = 0.0;
  for (int it = 0; it < POWER_ITS; ++it) {
    double ny = 0.0, nx = 0.0;
    for (int64_t i = 0; i < l.n; ++i) {
      double s = 0.0;
      for (int32_t q = l.rp[i]; q < l.rp[i + 1]; ++q) s += l.val[q] * x[l.ci[q]];
      y[i] = s * l.dinv[i];
      ny += y[i] * y[i];
      nx += x[i] * x[i];
    }
    lam = std::sqrt(ny) / std::sqrt(nx);
    const double f = 1.0 / std::sqrt(ny);
    for (int64_t i = 0; i < l.n; ++i) x[i] = y[i] * f;
  }
  return lam;
}

// ---- structure (mesh + Dirichlet set) ---------------------------------------------
nle_status build_structure(Ctx *c, Amg *A) {
  const Mesh &M = c->m;
  const int64_t nn = M.n_nodes;
  A->L.clear();
  A->L.emplace_back();
  {
    Level &l0 = A->L[0];
    l0.nv = nn;
    l0.n = 3 * nn;
    l0.vbeg.resize(nn + 1);
    for (int64_t v = 0; v <= nn; ++v) l0.vbeg[v] = 3 * v;
    // nodes sharing an element (all ten nodes of a quadratic element)
    const int npe = c->mixed ? 10 : 4;
    const std::vector<int32_t> &conn = c->mixed ? c->mx.h_conn : M.h_conn;
    std::vector<uint64_t> pairs;
    pairs.reserve(size_t(M.n_elems) * npe * (npe - 1));
    for (int64_t e = 0; e < M.n_elems; ++e)
      for (int a = 0; a < npe; ++a)
        for (int b = 0; b < npe; ++b)
          if (a != b)
            pairs.push_back((uint64_t(uint32_t(conn[npe * e + a])) << 32) |
                            uint32_t(conn[npe * e + b]));
    std::sort(pairs.begin(), pairs.end());
    pairs.erase(std::unique(pairs.begin(), pairs.end()), pairs.end());
    l0.adjp.assign(nn + 1, 0);
    l0.adji.resize(pairs.size());
    for (size_t q = 0; q < pairs.size(); ++q) {
      ++l0.adjp[(pairs[q] >> 32) + 1];
      l0.adji[q] = int32_t(pairs[q] & 0xFFFFFFFFu);
    }
    for (int64_t v = 0; v < nn; ++v) l0.adjp[v + 1] += l0.adjp[v];
  }
  // candidates: translations and rotations e_k x X, zero on Dirichlet dofs
  std::vector<double> B(size_t(3 * nn) * 6, 0.0);
  for (int64_t v = 0; v < nn; ++v) {
    const double x = M.h_X[3 * v], y = M.h_X[3 * v + 1], z = M.h_X[3 * v + 2];
    const double rows[3][6] = {{1, 0, 0, 0, z, -y}, {0, 1, 0, -z, 0, x}, {0, 0, 1, y, -x, 0}};
    for (int d = 0; d < 3; ++d) {
      const bool fixed = (c->h_mask[v] >> d) & 1u;
      for (int k = 0; k < 6; ++k) B[(3 * v + d) * 6 + k] = fixed ? 0.0 : rows[d][k];
    }
  }
  while (A->L.back().n > N_COARSE && int(A->L.size()) < MAX_LEVELS) {
    Level &l = A->L.back();
    std::vector<int32_t> agg;
    const int64_t na = aggregate(l, agg);
    if (na >= l.nv) break;
    // members of each aggregate in increasing order
    std::vector<int64_t> mp(na + 1, 0);
    for (int64_t v = 0; v < l.nv; ++v) ++mp[agg[v] + 1];
    for (int64_t a = 0; a < na; ++a) mp[a + 1] += mp[a];
    std::vector<int32_t> mem(l.nv);
    {
      std::vector<int64_t> fill(mp.begin(), mp.end() - 1);
      for (int64_t v = 0; v < l.nv; ++v) mem[fill[agg[v]]++] = int32_t(v);
    }
    // modified Gram-Schmidt per aggregate
    l.poff.assign(l.n, 0);
    l.pk.assign(l.n, 0);
    l.pv.assign(size_t(l.n) * 6, 0.0);
    std::vector<int32_t> kc(na, 0);
    std::vector<double> Bn;
    std::vector<int32_t> keep_id(na, -1);
    std::vector<int64_t> cbeg;  // first coarse dof of each kept aggregate
    int64_t ncd = 0;
    l.arows.clear();
    std::vector<int64_t> abeg(na + 1, 0);
    for (int64_t a = 0; a < na; ++a) {
      std::vector<int32_t> rows;
      for (int64_t q = mp[a]; q < mp[a + 1]; ++q)
        for (int64_t r = l.vbeg[mem[q]]; r < l.vbeg[mem[q] + 1]; ++r) rows.push_back(int32_t(r));
      abeg[a] = int64_t(l.arows.size());
      l.arows.insert(l.arows.end(), rows.begin(), rows.end());
      const size_t m = rows.size();
      std::vector<std::vector<double>> qs;
      for (int k = 0; k < 6; ++k) {
        std::vector<double> v(m);
        double nb = 0.0;
        for (size_t i = 0; i < m; ++i) {
          v[i] = B[size_t(rows[i]) * 6 + k];
          nb += v[i] * v[i];
        }
        nb = std::sqrt(nb);
        for (const auto &q : qs) {
          double d = 0.0;
          for (size_t i = 0; i < m; ++i) d += q[i] * v[i];
          for (size_t i = 0; i < m; ++i) v[i] -= d * q[i];
        }
        double nv = 0.0;
        for (size_t i = 0; i < m; ++i) nv += v[i] * v[i];
        nv = std::sqrt(nv);
        if (nb > 0.0 && nv > DROP_TOL * nb) {
          for (size_t i = 0; i < m; ++i) v[i] /= nv;
          qs.push_back(std::move(v));
        }
      }
      kc[a] = int32_t(qs.size());
      if (qs.empty()) continue;
      keep_id[a] = int32_t(cbeg.size());
      cbeg.push_back(ncd);
      for (size_t i = 0; i < qs.size(); ++i) {
        for (int k = 0; k < 6; ++k) {
          double d = 0.0;
          for (size_t t = 0; t < m; ++t) d += qs[i][t] * B[size_t(rows[t]) * 6 + k];
          Bn.push_back(d);
        }
        for (size_t t = 0; t < m; ++t) l.pv[size_t(rows[t]) * 6 + i] = qs[i][t];
      }
      for (size_t t = 0; t < m; ++t) {
        l.poff[rows[t]] = int32_t(ncd);
        l.pk[rows[t]] = kc[a];
      }
      ncd += int64_t(qs.size());
    }
    abeg[na] = int64_t(l.arows.size());
    if (ncd == 0) break;
    if (A->L.size() == 1) {
      A->agg0 = agg;
      A->keep0 = keep_id;
    }
    l.rs.resize(ncd);
    l.re.resize(ncd);
    l.ri.resize(ncd);
    for (int64_t a = 0; a < na; ++a) {
      if (keep_id[a] < 0) continue;
      for (int i = 0; i < kc[a]; ++i) {
        const int64_t R = cbeg[keep_id[a]] + i;
        l.rs[R] = int32_t(abeg[a]);
        l.re[R] = int32_t(abeg[a + 1]);
        l.ri[R] = i;
      }
    }
    // next level: kept aggregates, adjacency through members
    Level nx;
    nx.nv = int64_t(cbeg.size());
    nx.n = ncd;
    nx.vbeg.resize(nx.nv + 1);
    for (int64_t a = 0; a < nx.nv; ++a) nx.vbeg[a] = cbeg[a];
    nx.vbeg[nx.nv] = ncd;
    std::vector<std::vector<int32_t>> nb(nx.nv);
    for (int64_t v = 0; v < l.nv; ++v) {
      const int32_t a = keep_id[agg[v]];
      if (a < 0) continue;
      for (int64_t q = l.adjp[v]; q < l.adjp[v + 1]; ++q) {
        const int32_t b = keep_id[agg[l.adji[q]]];
        if (b >= 0 && b != a) nb[a].push_back(b);
      }
    }
    nx.adjp.assign(nx.nv + 1, 0);
    for (int64_t a = 0; a < nx.nv; ++a) {
      std::sort(nb[a].begin(), nb[a].end());
      nb[a].erase(std::unique(nb[a].begin(), nb[a].end()), nb[a].end());
      nx.adjp[a + 1] = nx.adjp[a] + int64_t(nb[a].size());
    }
    nx.adji.reserve(nx.adjp[nx.nv]);
    for (int64_t a = 0; a < nx.nv; ++a) nx.adji.insert(nx.adji.end(), nb[a].begin(), nb[a].end());
    // operator pattern: every dof of vertex a couples to the dofs of a and its neighbours
    nx.rp.assign(nx.n + 1, 0);
    for (int64_t a = 0; a < nx.nv; ++a) {
      std::vector<int32_t> vs(nb[a]);
      vs.push_back(int32_t(a));
      std::sort(vs.begin(), vs.end());
      int64_t w = 0;
      for (int32_t b : vs) w += nx.vbeg[b + 1] - nx.vbeg[b];
      if (int64_t(nx.rp[nx.vbeg[a]]) + w * (nx.vbeg[a + 1] - nx.vbeg[a]) > INT32_MAX)
        return fail(c, NLE_E_UNSUPPORTED, "multigrid: a coarse operator exceeds 2^31 entries");
      for (int64_t R = nx.vbeg[a]; R < nx.vbeg[a + 1]; ++R) {
        nx.rp[R + 1] = int32_t(nx.rp[R] + w);
        for (int32_t b : vs)
          for (int64_t C = nx.vbeg[b]; C < nx.vbeg[b + 1]; ++C) nx.ci.push_back(int32_t(C));
      }
    }
    B = std::move(Bn);
    A->L.push_back(std::move(nx));
  }
  const int64_t nco = A->L.back().n;
  if (nco > MAX_DENSE)
    return fail(c, NLE_E_UNSUPPORTED, "multigrid: the coarsest level stays too large");

  // probing tasks of the level-1 operator: colour the level-1 vertices so that
  // the node neighbourhoods of one colour's aggregates are disjoint
  A->tc.assign(1, 0);
  A->ncol = 0;
  std::vector<int32_t> tbeg, tend, tkp, tka, nodes, dcol(3 * nn, -1);
  std::vector<int64_t> tdest;
  if (A->L.size() >= 2) {
    const Level &l0 = A->L[0];
    const Level &l1 = A->L[1];
    std::vector<int32_t> v1(nn, -1);  // level-1 vertex of each node (or -1)
    for (int64_t v = 0; v < nn; ++v) v1[v] = A->keep0[A->agg0[v]];
    std::vector<std::vector<int32_t>> members(l1.nv);
    for (int64_t v = 0; v < nn; ++v)
      if (v1[v] >= 0) members[v1[v]].push_back(int32_t(v));
    std::vector<std::vector<int32_t>> owner;
    std::vector<int32_t> colour(l1.nv, -1);
    std::vector<int32_t> nbh;
    for (int64_t a = 0; a < l1.nv; ++a) {
      nbh.clear();
      for (int32_t v : members[a]) {
        nbh.push_back(v);
        for (int64_t q = l0.adjp[v]; q < l0.adjp[v + 1]; ++q) nbh.push_back(l0.adji[q]);
      }
      std::sort(nbh.begin(), nbh.end());
      nbh.erase(std::unique(nbh.begin(), nbh.end()), nbh.end());
      int cc = 0;
      for (;; ++cc) {
        if (cc == int(owner.size())) owner.emplace_back(nn, -1);
        bool ok = true;
        for (int32_t v : nbh)
          if (owner[cc][v] >= 0) {
            ok = false;
            break;
          }
        if (ok) break;
      }
      colour[a] = cc;
      for (int32_t v : nbh) owner[cc][v] = int32_t(a);
    }
    A->ncol = int(owner.size());
    for (int64_t v = 0; v < nn; ++v)
      if (v1[v] >= 0)
        for (int d = 0; d < 3; ++d) dcol[3 * v + d] = colour[v1[v]];
    for (int cc = 0; cc < A->ncol; ++cc) {
      std::map<std::pair<int32_t, int32_t>, std::vector<int32_t>> pairs;  // (row vertex, col vertex)
      for (int64_t v = 0; v < nn; ++v) {
        const int32_t a = owner[cc][v];
        if (a < 0 || v1[v] < 0) continue;
        pairs[{v1[v], a}].push_back(int32_t(v));
      }
      for (const auto &kv : pairs) {
        if (nodes.size() + kv.second.size() > size_t(INT32_MAX) ||
            tbeg.size() + 6 > size_t(INT32_MAX))
          return fail(c, NLE_E_UNSUPPORTED, "multigrid: probing lists exceed 2^31 entries");
        const int32_t b = kv.first.first, a = kv.first.second;
        const int32_t nb0 = int32_t(nodes.size());
        nodes.insert(nodes.end(), kv.second.begin(), kv.second.end());
        const int32_t nb1 = int32_t(nodes.size());
        const int32_t ka = int32_t(l1.vbeg[a + 1] - l1.vbeg[a]);
        for (int64_t R = l1.vbeg[b]; R < l1.vbeg[b + 1]; ++R) {
          const int32_t *lo = l1.ci.data() + l1.rp[R], *hi = l1.ci.data() + l1.rp[R + 1];
          const int32_t *p = std::lower_bound(lo, hi, int32_t(l1.vbeg[a]));
          if (p == hi || *p != l1.vbeg[a])
            return fail(c, NLE_E_STATE, "multigrid: probing pattern mismatch");
          tbeg.push_back(nb0);
          tend.push_back(nb1);
          tkp.push_back(int32_t(R - l1.vbeg[b]));
          tka.push_back(ka);
          tdest.push_back(int64_t(p - l1.ci.data()));
        }
      }
      A->tc.push_back(int32_t(tbeg.size()));
    }
  }

  // ---- device copies ----------------------------------------------------------------
  bool ok = true;
  const int64_t n0 = A->L[0].n;
  for (size_t li = 0; li < A->L.size() && ok; ++li) {
    Level &l = A->L[li];
    if (li >= 1) {
      ok = ok && upload(c, A, &l.d_rp, l.rp) && upload(c, A, &l.d_ci, l.ci);
      ok = ok && alloc(c, A, &l.d_v64, l.ci.size() + 1) && alloc(c, A, &l.d_v32, l.ci.size() + 1);
      ok = ok && alloc(c, A, &l.d_dinv64, size_t(l.n)) && alloc(c, A, &l.d_dinv32, size_t(l.n));
      ok = ok && alloc(c, A, &l.d_b, size_t(l.n)) && alloc(c, A, &l.d_x, size_t(l.n)) &&
           alloc(c, A, &l.d_r, size_t(l.n));
    }
    if (li + 1 < A->L.size()) {
      ok = ok && upload(c, A, &l.d_poff, l.poff) && upload(c, A, &l.d_pk, l.pk) &&
           upload(c, A, &l.d_rs, l.rs) && upload(c, A, &l.d_re, l.re) &&
           upload(c, A, &l.d_ri, l.ri) && upload(c, A, &l.d_arows, l.arows) &&
           upload(c, A, &l.d_pv64, l.pv);
      if (ok) {
        const std::vector<float> p32 = to32(l.pv);
        ok = upload(c, A, &l.d_pv32, p32);
        if (ok) ok = hipStreamSynchronize(c->stream) == hipSuccess;  // p32 leaves scope
      }
    }
  }
  ok = ok && alloc(c, A, &A->d_inv64, size_t(nco * nco)) &&
       alloc(c, A, &A->d_inv32, size_t(nco * nco));
  ok = ok && upload(c, A, &A->d_tbeg, tbeg) && upload(c, A, &A->d_tend, tend) &&
       upload(c, A, &A->d_tkp, tkp) && upload(c, A, &A->d_tka, tka) &&
       upload(c, A, &A->d_tdest, tdest) && upload(c, A, &A->d_nodes, nodes) &&
       upload(c, A, &A->d_dcol, dcol);
  // vectors the Jacobian action reads or writes span all unknowns (a pressure
  // field's entries stay zero in the inputs)
  const int64_t nfull = ndof(c);
  ok = ok && alloc(c, A, &A->d_z, size_t(nfull)) && alloc(c, A, &A->d_y, size_t(nfull)) &&
       alloc(c, A, &A->d_t, size_t(nfull)) && alloc(c, A, &A->d_red, size_t(2 * VGRID_MAX)) &&
       alloc(c, A, &A->d_s, 8) && alloc(c, A, &A->d_cd, size_t(n0));
  ok = ok && hipMemsetAsync(A->d_z, 0, size_t(nfull) * 8, c->stream) == hipSuccess;
  if (ok) ok = hipStreamSynchronize(c->stream) == hipSuccess;
  if (!ok) return fail(c, NLE_E_OOM, "multigrid: device allocation or copy failed");
  return NLE_OK;
}

// Rows of the coarse vertices a = t, t + nth, ... of nx.val = P^T l.val P
// (*bad = 1 on a pattern mismatch).
void galerkin_chunk(const Level &l, Level &nx, int t, int nth, char *bad) {
  const int64_t nagg = nx.nv;
  std::vector<int32_t> marker(size_t(nx.n), -1);
  std::vector<double> tr, acc;
  for (int64_t a = t; a < nagg; a += nth) {
    const int64_t R0 = nx.vbeg[a], ka = nx.vbeg[a + 1] - R0;
    const int32_t p0 = nx.rp[R0], width = nx.rp[R0 + 1] - p0;
    for (int32_t q = 0; q < width; ++q) marker[nx.ci[p0 + q]] = q;
    acc.assign(size_t(ka * width), 0.0);
    tr.resize(width);
    for (int32_t q = l.rs[R0]; q < l.re[R0]; ++q) {
      const int32_t r = l.arows[q];
      std::fill(tr.begin(), tr.end(), 0.0);
      for (int32_t e2 = l.rp[r]; e2 < l.rp[r + 1]; ++e2) {
        const int32_t s = l.ci[e2];
        const double av = l.val[e2];
        for (int j = 0; j < l.pk[s]; ++j) {
          const int32_t m = marker[l.poff[s] + j];
          if (m < 0) {
            *bad = 1;
            return;
          }
          tr[m] += av * l.pv[size_t(s) * 6 + j];
        }
      }
      for (int64_t i = 0; i < ka; ++i) {
        const double p = l.pv[size_t(r) * 6 + i];
        if (p == 0.0) continue;
        for (int32_t q2 = 0; q2 < width; ++q2) acc[size_t(i * width + q2)] += p * tr[q2];
      }
    }
    for (int64_t i = 0; i < ka; ++i)
      std::memcpy(nx.val.data() + nx.rp[R0 + i], acc.data() + i * width, size_t(width) * 8);
    for (int32_t q = 0; q < width; ++q) marker[nx.ci[p0 + q]] = -1;
  }
}

// nx.val = P^T l.val P for the coarse operator pattern of nx.  Each coarse
// vertex's rows are formed by one host thread in the same order whatever the
// thread count, so the values are the same bit for bit.
nle_status galerkin(Ctx *c, const Level &l, Level &nx) {
  nx.val.assign(nx.ci.size(), 0.0);
  const int64_t nagg = nx.nv;
  const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const int nth = int(std::max<int64_t>(1, std::min<int64_t>(nagg, hw)));
  std::vector<char> bad(size_t(nth), 0);  // 1: pattern mismatch, 2: host allocation failed
  auto work = [&](int t) noexcept {
    try {
      galerkin_chunk(l, nx, t, nth, &bad[size_t(t)]);
    } catch (...) {
      bad[size_t(t)] = 2;
    }
  };
  // chunk t (coarse vertices a = t mod nth) runs on thread t; chunks whose
  // thread could not be started run on this one
  std::vector<std::thread> th;
  int started = 1;
  try {
    for (int t = 1; t < nth; ++t) {
      th.emplace_back(work, t);
      started = t + 1;
    }
  } catch (...) {
  }
  work(0);
  for (int t = started; t < nth; ++t) work(t);
  for (std::thread &x : th) x.join();
  for (char b : bad) {
    if (b == 1) return fail(c, NLE_E_STATE, "multigrid: Galerkin pattern mismatch");
    if (b == 2) return fail(c, NLE_E_OOM, "multigrid: host allocation failed");
  }
  return NLE_OK;
}

// ---- values of the current linearization ----------------------------------------
nle_status build_values(Ctx *c, Amg *A) {
  const int64_t n0 = A->L[0].n;
  hipError_t e = hipSuccess;
  if (A->L.size() == 1) {
    // one level: the tangent itself, column by column
    std::vector<double> K(size_t(n0 * n0)), col(n0);
    for (int64_t j = 0; j < n0; ++j) {
      NLE_HIP(c, hipMemsetAsync(A->d_z, 0, size_t(ndof(c)) * 8, c->stream));
      const double one = 1.0;
      NLE_HIP(c, hipMemcpyAsync(A->d_z + j, &one, 8, hipMemcpyHostToDevice, c->stream));
      elem_apply(c, OP_JV, NLE_FP64, c->ulin64, A->d_z, A->d_y, nullptr, &e);
      if (e != hipSuccess) return fail(c, NLE_E_HIP, "multigrid: Jacobian action");
      NLE_HIP(c, hipMemcpyAsync(col.data(), A->d_y, size_t(n0) * 8, hipMemcpyDeviceToHost,
                                c->stream));
      NLE_HIP(c, hipStreamSynchronize(c->stream));
      for (int64_t i = 0; i < n0; ++i) K[size_t(i * n0 + j)] = col[i];
    }
    if (!invert(K, n0, A->inv)) return fail(c, NLE_E_STATE, "multigrid: singular tangent");
  } else {
    // finest level: power iteration for the Jacobi weight
    {
      const std::vector<double> x0 = start_vector(n0);
      NLE_HIP(c, hipMemcpyAsync(A->d_z, x0.data(), size_t(n0) * 8, hipMemcpyHostToDevice,
                                c->stream));
      for (int it = 0; it < POWER_ITS; ++it) {
        elem_apply(c, OP_JV, NLE_FP64, c->ulin64, A->d_z, A->d_t, nullptr, &e);
        if (e != hipSuccess) return fail(c, NLE_E_HIP, "multigrid: Jacobian action");
        const int np = amg_power_partials(c, A->d_t, c->dinv64, A->d_z, A->d_y, n0, A->d_red, &e);
        if (e != hipSuccess) return fail(c, NLE_E_HIP, "multigrid: power iteration");
        NLE_HIP(c, reduce_scalars(c, A->d_red, np, 2, A->d_s));
        if (it + 1 < POWER_ITS) NLE_HIP(c, amg_power_scale(c, A->d_y, A->d_s, A->d_z, n0));
      }
      double s[2];
      NLE_HIP(c, hipMemcpyAsync(s, A->d_s, 16, hipMemcpyDeviceToHost, c->stream));
      NLE_HIP(c, hipStreamSynchronize(c->stream));
      const double lam = std::sqrt(s[0]) / std::sqrt(s[1]);
      if (!(lam > 0.0) || !std::isfinite(lam))
        return fail(c, NLE_E_STATE, "multigrid: bad spectral radius estimate");
      A->L[0].w = 1.0 / lam;
      // Chebyshev coefficients on [hi / RATIO, hi]
      const double hi = CHEB_SAFETY * lam, lo = hi / CHEB_RATIO;
      const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
      A->cheb_cd[0] = 0.0;
      A->cheb_cr[0] = 1.0 / theta;
      double rho_prev = 1.0 / sigma;
      for (int j = 1; j < CHEB_DEGREE; ++j) {
        const double rho_j = 1.0 / (2.0 * sigma - rho_prev);
        A->cheb_cd[j] = rho_j * rho_prev;
        A->cheb_cr[j] = 2.0 * rho_j / delta;
        rho_prev = rho_j;
      }
    }
    // level 1 by probing
    Level &l1 = A->L[1];
    NLE_HIP(c, hipMemsetAsync(l1.d_v64, 0, l1.ci.size() * 8, c->stream));
    for (int cc = 0; cc < A->ncol; ++cc) {
      AmgTasks t{A->d_tbeg + A->tc[cc], A->d_tend + A->tc[cc], A->d_tkp + A->tc[cc],
                 A->d_tka + A->tc[cc], A->d_tdest + A->tc[cc], A->d_nodes,
                 A->tc[cc + 1] - A->tc[cc]};
      for (int k = 0; k < 6; ++k) {
        NLE_HIP(c, amg_probe_vec(c, A->d_z, A->L[0].d_pv64, A->L[0].d_pk, A->d_dcol, cc, k, n0));
        elem_apply(c, OP_JV, NLE_FP64, c->ulin64, A->d_z, A->d_y, nullptr, &e);
        if (e != hipSuccess) return fail(c, NLE_E_HIP, "multigrid: probing");
        NLE_HIP(c, amg_extract(c, A->d_y, A->L[0].d_pv64, t, k, l1.d_v64));
      }
    }
    l1.val.resize(l1.ci.size());
    NLE_HIP(c, hipMemcpyAsync(l1.val.data(), l1.d_v64, l1.ci.size() * 8, hipMemcpyDeviceToHost,
                              c->stream));
    NLE_HIP(c, hipStreamSynchronize(c->stream));
    // coarser levels on the host; level 1's Jacobi weight by a power
    // iteration on the GPU (its operator is there already), queued before
    // the host forms the coarser Galerkin products and read back after them
    const std::vector<double> x1 = start_vector(A->L[1].n);
    bool gpu_power = false;
    for (size_t li = 1; li < A->L.size(); ++li) {
      Level &l = A->L[li];
      l.dinv.assign(l.n, 0.0);
      for (int64_t i = 0; i < l.n; ++i) {
        double d = 0.0;
        for (int32_t q = l.rp[i]; q < l.rp[i + 1]; ++q)
          if (l.ci[q] == i) d = l.val[q];
        if (!(d != 0.0) || !std::isfinite(d))
          return fail(c, NLE_E_STATE, "multigrid: zero coarse diagonal");
        l.dinv[i] = 1.0 / d;
      }
      if (li + 1 == A->L.size()) break;
      if (li == 1) {
        NLE_HIP(c, hipMemcpyAsync(l.d_dinv64, l.dinv.data(), size_t(l.n) * 8,
                                  hipMemcpyHostToDevice, c->stream));
        NLE_HIP(c, hipMemcpyAsync(A->d_z, x1.data(), size_t(l.n) * 8, hipMemcpyHostToDevice,
                                  c->stream));
        for (int it = 0; it < POWER_ITS; ++it) {
          NLE_HIP(c, amg_csr_mv(c, A->d_t, A->d_z, l.d_rp, l.d_ci, l.d_v64, l.n));
          const int np = amg_power_partials(c, A->d_t, l.d_dinv64, A->d_z, A->d_y, l.n, A->d_red, &e);
          if (e != hipSuccess) return fail(c, NLE_E_HIP, "multigrid: power iteration");
          NLE_HIP(c, reduce_scalars(c, A->d_red, np, 2, A->d_s));
          if (it + 1 < POWER_ITS) NLE_HIP(c, amg_power_scale(c, A->d_y, A->d_s, A->d_z, l.n));
        }
        gpu_power = true;
      } else {
        l.w = 1.0 / host_power(l);
      }
      const nle_status sg = galerkin(c, l, A->L[li + 1]);
      if (sg != NLE_OK) return sg;
    }
    if (gpu_power) {
      double s[2];
      NLE_HIP(c, hipMemcpyAsync(s, A->d_s, 16, hipMemcpyDeviceToHost, c->stream));
      NLE_HIP(c, hipStreamSynchronize(c->stream));
      const double lam = std::sqrt(s[0]) / std::sqrt(s[1]);
      if (!(lam > 0.0) || !std::isfinite(lam))
        return fail(c, NLE_E_STATE, "multigrid: bad spectral radius estimate");
      A->L[1].w = 1.0 / lam;
    }
    const Level &lc = A->L.back();
    std::vector<double> D(size_t(lc.n * lc.n), 0.0);
    for (int64_t i = 0; i < lc.n; ++i)
      for (int32_t q = lc.rp[i]; q < lc.rp[i + 1]; ++q) D[size_t(i * lc.n + lc.ci[q])] = lc.val[q];
    if (!invert(D, lc.n, A->inv)) return fail(c, NLE_E_STATE, "multigrid: singular coarsest level");
    // upload operator values
    for (size_t li = 1; li < A->L.size(); ++li) {
      Level &l = A->L[li];
      const std::vector<float> v32 = to32(l.val), d32 = to32(l.dinv);
      NLE_HIP(c, hipMemcpyAsync(l.d_v64, l.val.data(), l.val.size() * 8, hipMemcpyHostToDevice,
                                c->stream));
      NLE_HIP(c, hipMemcpyAsync(l.d_v32, v32.data(), v32.size() * 4, hipMemcpyHostToDevice,
                                c->stream));
      NLE_HIP(c, hipMemcpyAsync(l.d_dinv64, l.dinv.data(), l.dinv.size() * 8,
                                hipMemcpyHostToDevice, c->stream));
      NLE_HIP(c, hipMemcpyAsync(l.d_dinv32, d32.data(), d32.size() * 4, hipMemcpyHostToDevice,
                                c->stream));
      NLE_HIP(c, hipStreamSynchronize(c->stream));
    }
  }
  const std::vector<float> i32 = to32(A->inv);
  NLE_HIP(c, hipMemcpyAsync(A->d_inv64, A->inv.data(), A->inv.size() * 8, hipMemcpyHostToDevice,
                            c->stream));
  NLE_HIP(c, hipMemcpyAsync(A->d_inv32, i32.data(), i32.size() * 4, hipMemcpyHostToDevice,
                            c->stream));
  NLE_HIP(c, hipStreamSynchronize(c->stream));
  return NLE_OK;
}

AmgXfer<void> xfer(const Level &l, const Level &nx, int prec) {
  return AmgXfer<void>{l.d_poff, l.d_pk,
                       prec == NLE_FP32 ? static_cast<const void *>(l.d_pv32)
                                        : static_cast<const void *>(l.d_pv64),
                       l.d_rs, l.d_re, l.d_ri, l.d_arows, l.n, nx.n};
}

// One V-cycle at level li for b.  Level 0 leaves the result in x; a coarser
// level returns in *res where its result is (x, or its residual buffer, which
// the fused post-smoother writes to).
hipError_t cycle(Ctx *c, Amg *A, int prec, size_t li, const void *b, void *x,
                 const void **res, double *red_dot, bool first_done = false) {
  const Level &l = A->L[li];
  const bool f32 = prec == NLE_FP32;
  *res = x;
  if (li + 1 == A->L.size())
    return amg_dense_mv(c, prec, x, f32 ? static_cast<const void *>(A->d_inv32) : A->d_inv64, b,
                        l.n);
  const Level &nx = A->L[li + 1];
  const AmgXfer<void> X = xfer(l, nx, prec);
  hipError_t e;
  if (li == 0) {
    // finest level: Chebyshev smoothing with the matrix-free Jacobian action
    const void *dinv = f32 ? static_cast<const void *>(c->dinv32) : c->dinv64;
    const void *ulin = f32 ? static_cast<const void *>(c->ulin32) : c->ulin64;
    if (!first_done &&
        (e = amg_cheb_first(c, prec, x, A->d_cd, b, dinv, A->cheb_cr[0], l.n)) != hipSuccess)
      return e;
    for (int j = 1; j < CHEB_DEGREE; ++j) {
      elem_apply(c, OP_JV, prec, ulin, x, A->d_t, nullptr, &e);
      if (e != hipSuccess) return e;
      amg_cheb_step(c, prec, x, A->d_cd, b, A->d_t, dinv, A->cheb_cd[j], A->cheb_cr[j], l.n,
                    nullptr, &e);
      if (e != hipSuccess) return e;
    }
    elem_apply(c, OP_JV, prec, ulin, x, A->d_t, nullptr, &e);
    if (e != hipSuccess) return e;
    if ((e = amg_restrict(c, prec, nx.d_b, b, A->d_t, X)) != hipSuccess) return e;
    const void *xc = nullptr;
    if ((e = cycle(c, A, prec, 1, nx.d_b, nx.d_x, &xc, nullptr)) != hipSuccess) return e;
    if ((e = amg_prolong_add(c, prec, x, xc, X)) != hipSuccess) return e;
    for (int j = 0; j < CHEB_DEGREE; ++j) {  // the recurrence restarts (cd[0] = 0)
      elem_apply(c, OP_JV, prec, ulin, x, A->d_t, nullptr, &e);
      if (e != hipSuccess) return e;
      amg_cheb_step(c, prec, x, A->d_cd, b, A->d_t, dinv, A->cheb_cd[j], A->cheb_cr[j], l.n,
                    j + 1 == CHEB_DEGREE ? red_dot : nullptr, &e);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  const void *dinv = f32 ? static_cast<const void *>(l.d_dinv32) : l.d_dinv64;
  const void *v = f32 ? static_cast<const void *>(l.d_v32) : l.d_v64;
  if ((e = amg_csr_pre(c, prec, x, l.d_r, b, dinv, l.w, l.d_rp, l.d_ci, v, l.n)) != hipSuccess)
    return e;
  if ((e = amg_restrict(c, prec, nx.d_b, l.d_r, nullptr, X)) != hipSuccess) return e;
  const void *xc = nullptr;
  if ((e = cycle(c, A, prec, li + 1, nx.d_b, nx.d_x, &xc, nullptr)) != hipSuccess) return e;
  if ((e = amg_prolong_add(c, prec, x, xc, X)) != hipSuccess) return e;
  // the restriction has consumed the residual buffer: the post-smoothed
  // iterate goes there
  *res = l.d_r;
  return amg_csr_post(c, prec, l.d_r, x, b, dinv, l.w, l.d_rp, l.d_ci, v, l.n);
}

}  // namespace

void amg_release(Ctx *c) {
  Amg *A = state(c);
  if (!A) return;
  (void)hipStreamSynchronize(c->stream);
  for (void *p : A->allocs) dfree(c, p);
  delete A;
  c->amg = nullptr;
}

void amg_invalidate(Ctx *c) {
  if (Amg *A = state(c)) A->valid = false;
}

nle_status amg_prepare(Ctx *c) {
  if (!c->lin64) return fail(c, NLE_E_STATE, "multigrid needs a linearization");
  Amg *A = state(c);
  if (A && A->valid) return NLE_OK;
  if (!A) {
    A = new Amg();
    c->amg = A;
    const nle_status s = build_structure(c, A);
    if (s != NLE_OK) {
      amg_release(c);
      return s;
    }
  }
  const nle_status s = build_values(c, A);
  if (s != NLE_OK) return s;
  A->valid = true;
  ++c->amg_gen;
  return NLE_OK;
}

bool amg_first_step(Ctx *c, int prec, const void **dinv, void **d, double *inv_theta) {
  Amg *A = state(c);
  if (!A || !A->valid || A->L.size() < 2 || (c->mixed && c->mx.n_p > 0)) return false;
  *dinv = prec == NLE_FP32 ? static_cast<const void *>(c->dinv32) : c->dinv64;
  *d = A->d_cd;
  *inv_theta = A->cheb_cr[0];
  return true;
}

hipError_t amg_apply(Ctx *c, int prec, const void *b, void *x, double *red_dot, bool first_done) {
  Amg *A = state(c);
  if (!A || !A->valid) return hipErrorNotReady;
  if (first_done && (A->L.size() < 2 || (c->mixed && c->mx.n_p > 0))) return hipErrorInvalidValue;
  // the smoother's Jacobian actions are the plain tangent: a Krylov loop's
  // epilogue (MINRES: y = J v - coef w with v.y partials) or fused CG
  // direction must not act inside the cycle
  struct Plain {
    Ctx *c;
    decltype(Ctx::ep) ep;
    const void *cgz;
    explicit Plain(Ctx *cc) : c(cc), ep(cc->ep), cgz(cc->cg.z) {
      c->ep.w = nullptr;
      c->ep.coef = nullptr;
      c->ep.red = nullptr;
      c->cg.z = nullptr;
    }
    ~Plain() {
      c->ep = ep;
      c->cg.z = cgz;
    }
  } plain(c);
  const void *res = nullptr;
  if (c->mixed && c->mx.n_p > 0) {
    // field split: the cycle on the displacements (whose Jacobian actions
    // see zero pressures), the pressure block's diagonal on the pressures
    if (red_dot) return hipErrorInvalidValue;
    const int64_t n0 = A->L[0].n, np = c->mx.n_p;
    const size_t es = prec == NLE_FP32 ? 4 : 8;
    void *xp = static_cast<char *>(x) + size_t(n0) * es;
    const void *bp = static_cast<const char *>(b) + size_t(n0) * es;
    const void *dp = prec == NLE_FP32 ? static_cast<const void *>(c->dinv32 + n0)
                                      : static_cast<const void *>(c->dinv64 + n0);
    hipError_t e = vec_fill(c, prec, xp, 0.0, np);
    if (e != hipSuccess) return e;
    if ((e = cycle(c, A, prec, 0, b, x, &res, nullptr)) != hipSuccess) return e;
    return pc_apply(c, prec, 1, dp, bp, xp, np);
  }
  if (red_dot && A->L.size() == 1) {  // one level: the dense solve, then the dot
    hipError_t e = cycle(c, A, prec, 0, b, x, &res, nullptr);
    if (e != hipSuccess) return e;
    vec_dot_partials(c, prec, b, x, A->L[0].n, red_dot, &e);
    return e;
  }
  return cycle(c, A, prec, 0, b, x, &res, red_dot, first_done);  // level 0 works in place
}

int amg_levels(const Ctx *c, int64_t *sizes, int cap) {
  const Amg *A = static_cast<const Amg *>(c->amg);
  if (!A) return 0;
  const int L = int(A->L.size());
  for (int i = 0; i < L && i < cap; ++i) sizes[i] = A->L[i].n;
  return L;
}

}  // namespace nle
