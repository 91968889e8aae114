// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "nlelast.h"

namespace nle {

constexpr int NT = 256;            // threads per workgroup (four wave64)
constexpr int VGRID_MAX = 1024;    // workgroups of the streaming vector kernels
constexpr uint32_t NODE_MASK = 0x0FFFFFFFu;  // node id bits of a block-node word
// Size of the fixed per-device workspace of nle_jv_noalloc (shared-slot
// partial sums: 3 values per shared block-node slot), and the devices it
// is set up for.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;

// Device scalar slots of the CG loop (shared by the vector kernels and the
// element kernels that form the CG direction).
namespace cgslot {
enum { RZ = 0, RZOLD = 1, TOL2 = 2, RR = 3, B2 = 4, MAXIT = 5, BETA = 6 };
}

// Element kernel operations.
// OP_ODIAG: the off-diagonal entries (xy, yz, xz) of each node's diagonal
// 3x3 tangent block (FP64, P1 meshes only).
enum ElemOp : int { OP_RES = 0, OP_JV = 1, OP_DIAG = 2, OP_ENERGY = 3, OP_ODIAG = 4 };

struct MatParams {
  int32_t kind;   // NLE_MAT_M1 .. NLE_MAT_M6
  double mu, lam, cvol, kappa;
  double a_iso, b_iso, a_f, b_f, gamma;  // law M4 (kappa shared)
  // law M6 (Guccione): C, b_ff, b_ss, b_nn, b_fs, b_fn, b_sn, B
  double g6[8];
};

// Element partition and geometry on the device.  Elements are renumbered
// into blocks (contiguous ranges); every block owns a sorted list of the
// nodes it touches ("slots") and a block-local connectivity.  Each
// (element, vertex) contribution has a position in the block's slot-sorted
// order (stored with the local ids), so the contributions of slot l occupy the contiguous range
// [csr_end[l-1], csr_end[l]) of the block's contribution array.
struct Mesh {
  int64_t n_nodes = 0, n_elems = 0;
  int32_t nblk = 0, be_max = 0, nl_max = 0;
  int64_t n_slots = 0, n_shared = 0, n_fx = 0;
  // [n_slots][3] coordinates of each slot's node relative to the block's
  // first slot (the element kernels form grad N and V from them)
  double *xr64 = nullptr; float *xr32 = nullptr;
  uint4 *lcp = nullptr;   // [n_elems] 4 slot-local vertex ids, 4 slot-sorted positions (u16)
  uint16_t *csr_end = nullptr;                  // [n_slots] end of the slot's range
  uint32_t *nodes = nullptr;                    // [n_slots] id | mask<<28 | shared<<31
  int32_t *blk_elem = nullptr, *blk_node = nullptr;  // [nblk+1]
  // batched meshes (disjoint union of instances): instance of each block and
  // of each merge workgroup (each instance's shared nodes start on a whole
  // merge workgroup), and per-instance ranges
  int32_t *blk_inst = nullptr, *mwg_inst = nullptr;
  int32_t n_inst = 1, n_mwg = 0;
  std::vector<int64_t> h_inst_node, h_inst_elem;   // [n_inst+1] offsets
  std::vector<int32_t> h_inst_blk, h_inst_mwg;     // [n_inst+1] block / merge-WG offsets
  uint32_t *fx_node = nullptr;                  // [n_shared] id | mask<<28
  int32_t *fx_ptr = nullptr;  // [n_shared+1] ranges of each shared node's partials
  int32_t *mpos = nullptr;    // [n_slots] partial position of a shared slot
  // host mirrors needed later
  std::vector<uint32_t> h_nodes, h_fx_node;     // ids and shared bit, no mask
  std::vector<int32_t> h_conn;                  // user connectivity (user order)
  std::vector<double> h_V;                      // volumes (user order)
  std::vector<int64_t> h_perm;                  // user element of each renumbered element
  std::vector<double> h_X;
};

// Mixed quadratic-displacement / linear-pressure mesh (twist test): element
// data in user element order, node-centred gather lists.
struct MixedMesh {
  int64_t n_u = 0, n_p = 0, n_e = 0;
  int32_t npe = 0;            // pressure values per element: 4 (linear), 1 (constant), 0
  int32_t *conn = nullptr;    // [10][n_e] displacement nodes
  int32_t *pconn = nullptr;   // [npe][n_e] pressure nodes
  double *G64 = nullptr;      // [9][n_e] grad lambda_1..3
  float *G32 = nullptr;
  double *V64 = nullptr;      // [n_e]
  float *V32 = nullptr;
  int32_t *u_ptr = nullptr, *u_ent = nullptr;  // per u node: entries e*10 + a
  int32_t *p_ptr = nullptr, *p_ent = nullptr;  // per p node: entries e*4 + b
  uint8_t *umask = nullptr;   // [n_u] Dirichlet bits
  double *mlump = nullptr;    // [n_p] lumped pressure mass
  void *cu = nullptr;         // [n_e*10][4] element contributions (double or float)
  void *cp = nullptr;         // [n_e*npe]
  // constant pressure: the SIMPLE Schur diagonal s_e and its inverse (per
  // linearization, computed on first use)
  double *s64 = nullptr, *sinv64 = nullptr;
  float *sinv32 = nullptr;
  std::vector<int32_t> h_conn;  // [n_e][10] (host, for the face loads)
};

struct Ctx;

// Device memory through the optional caller allocator.
void *dalloc(Ctx *c, size_t bytes);
void dfree(Ctx *c, void *p);

struct Ctx {
  int32_t device = 0;
  hipStream_t stream = nullptr;   // the caller's stream (current launch stream)
  hipStream_t kstream = nullptr;  // library stream for captured Krylov loops
  hipEvent_t ev_a = nullptr, ev_b = nullptr;
  nle_allocator al{};
  bool custom_alloc = false;
  std::string err;
  int32_t be_req = 512;
  int32_t xcd_remap = 1;
  size_t lds_limit = 65536;

  Mesh m;
  bool has_mesh = false;
  bool mixed = false;        // quadratic / linear mixed mesh (law M3)
  MixedMesh mx;
  std::vector<void *> mesh_allocs;  // freed on re-upload

  MatParams mat{NLE_MAT_M1, 1.0, 1.0, 0.25, 1.0 + 2.0 / 3.0};
  bool has_mat = false;

  // Dirichlet data
  int64_t n_dir = 0;
  int64_t *dir_dofs = nullptr;
  double *dir_vals = nullptr;
  std::vector<uint8_t> h_mask;  // per node, bit i = component i prescribed

  // loads
  std::vector<double> h_ftrac, h_fbody;
  double *fext = nullptr;
  double load_scale = 1.0;

  // linearization cache: per-element tangent coefficients at u_lin ([k][n_e],
  // k < 7), written by the diagonal pass of nle_linearize, read by the
  // Jacobian action of P1 meshes; lc_valid while they match u_lin
  double *lc64 = nullptr;
  float *lc32 = nullptr;
  int64_t lc_cap = 0;   // elements x coefficients allocated
  bool lc_valid = false;

  // laws M4, M6: unit fibre per element, [3][n_elems] in the renumbered
  // order; law M6 also the sheet direction (n = f x s)
  double *fib64 = nullptr;
  float *fib32 = nullptr;
  double *sh64 = nullptr;
  float *sh32 = nullptr;
  std::vector<void *> fib_allocs;

  // surface loads: follower pressure (scaled by the load scale) and elastic
  // springs, evaluated node by node over the incident faces
  struct Surf {
    int64_t nsn = 0;             // face nodes
    // pressure faces, follower-traction faces, spring faces (numbered in that order)
    int32_t npf = 0, ntf = 0, nrf = 0;
    int32_t *node = nullptr;     // [nsn] node ids
    int32_t *ptr = nullptr;      // [nsn+1] incident-face ranges
    int32_t *ent = nullptr;      // incident faces, increasing
    int32_t fv = 3;              // nodes per face: 3, or 6 on quadratic meshes
    int32_t *tri = nullptr;      // [npf+ntf+nrf][fv]
    uint32_t *fmask = nullptr;   // [npf+ntf+nrf] Dirichlet bits of the fv nodes (3 each)
    double *pgeo64 = nullptr;    // [npf+ntf][3 fv] reference node coordinates
    float *pgeo32 = nullptr;
    double *rgeo64 = nullptr;    // [nrf][4] reference unit normal, area
    float *rgeo32 = nullptr;
    double *plin = nullptr;      // device: [0] effective pressure, [1] load scale, at the linearization
    double *fs64 = nullptr;      // [3 n_nodes] contributions (zero off the face nodes)
    float *fs32 = nullptr;
    double p = 0.0, kperp = 0.0, kpar = 0.0;
    double cperp = 0.0, cpar = 0.0;  // dashpots on the spring faces
    double tf[3] = {0.0, 0.0, 0.0};  // follower traction per unit current area
    std::vector<int32_t> h_ptri, h_ttri, h_rtri, h_tri;
    std::vector<void *> allocs;
  } surf;

  // batched mode: per-instance load scale, material (mu, lam, cvol, kappa)
  // and done mask on the device (null for a single problem)
  double *inst_s = nullptr;
  double *inst_mat = nullptr;
  int32_t *inst_done = nullptr;
  int32_t *inst_inv = nullptr;  // per-instance "some det F <= 0" flags
  // aggregation multigrid (nle_amg.cpp), built on first use; amg_gen counts
  // its operator builds (captured Krylov chunks hold its smoother weights)
  void *amg = nullptr;
  uint64_t amg_gen = 0;

  // inertia of an implicit time step: c M (u - u_tilde) in the residual,
  // c M in the tangent (M the row-sum lumped P1 mass of density rho)
  struct {
    bool on = false;
    double rho = 0.0, c = 0.0;
    double *cm64 = nullptr;  // [3 n_nodes] c * m per dof
    float *cm32 = nullptr;
    double *ut = nullptr;    // [3 n_nodes] u_tilde
    // the step's velocity v(u) = vt + cv (u - ut), which the dashpots act on
    double cv = 0.0;
    double *vt = nullptr;    // [3 n_nodes]
  } inr;

  // batched mode: when set, the element kernels run only the listed blocks
  // and merge workgroups (those of the instances still iterating)
  const int32_t *blk_list = nullptr, *mwg_list = nullptr;
  int32_t n_blist = 0, n_mlist = 0;

  // linearization
  bool lin64 = false, lin32 = false;
  double *ulin64 = nullptr;
  float *ulin32 = nullptr;
  double *diag64 = nullptr;
  double *dinv64 = nullptr;
  float *dinv32 = nullptr;
  // nodal block Jacobi (computed on first use after each linearization):
  // odiag64 [3 n_n] off-diagonals of the diagonal blocks, binv [6][n_n] the
  // symmetric block inverses (xx, yy, zz, xy, yz, xz), component-major
  bool blk_valid = false;
  double *odiag64 = nullptr;
  double *binv64 = nullptr;
  float *binv32 = nullptr;

  // scratch
  void *partial = nullptr;   // [n_slots][3] doubles (shared-slot partial sums)
  void *noalloc_ws = nullptr;  // this device's fixed workspace (nle_jv_noalloc)
  double *red = nullptr;     // reduction partials, RED_CAP doubles
  int64_t red_cap = 0;
  double *dscal = nullptr;   // device scalars
  int32_t *dflag = nullptr;  // device flags: [0] inverted element
  const int32_t *elem_skip = nullptr;  // Krylov done flag seen by element kernels
  // CG with the direction formed inside the Jacobian action (three launches
  // per iteration): when cg.z is set, the element kernels use the direction
  // v = z + beta p (p = their v argument), where every element workgroup
  // forms beta = (r.z) / scal[S_RZOLD] and the stopping test from the
  // previous update's partials (red: r.z at [0, np), r.r at [VGRID_MAX, ...))
  struct {
    const void *z = nullptr;
    const double *red = nullptr;
    int np = 0;
    double *scal = nullptr;
    int32_t *flag = nullptr;
  } cg;
  // Jacobian action with the Dirichlet columns kept and the Dirichlet rows
  // zero: y = (K w) on free rows, the coupling a change of prescribed values
  // induces (used by the step that carries such a change into the interior)
  bool jv_nomask = false;
  // Jv epilogue used by the Krylov loops: out = J v - (*coef) w; partial sums
  // of v.out to red (block partials, then merge partials)
  struct {
    const void *w = nullptr;
    const double *coef = nullptr;
    double *red = nullptr;
  } ep;
  double *hpin = nullptr;    // pinned host scalars
  std::vector<void *> ctx_allocs;

  // captured Krylov chunk (see drop_graph)
  std::vector<uint64_t> gkey;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;

  // solver workspace (grown on demand)
  std::vector<void *> ws_allocs;
  size_t ws_bytes = 0;
  void *ws = nullptr;

  // GMRES basis pool: segments of basis vectors (vector stride gm_vb), their
  // Hessenberg columns and partial rows, kept across solves
  struct GmSeg {
    void *p;
    int v0, nv;
    void *vbase;
    double *hbase, *rbase;
  };
  std::vector<GmSeg> gm_segs;
  size_t gm_vb = 0;
  std::vector<void *> gm_hv;
  std::vector<double *> gm_hr;
};

// Release the GMRES basis pool (waits for the stream first).
void gmres_pool_release(Ctx *c);

nle_status fail(Ctx *c, nle_status code, const std::string &msg);
// Length of the unknown vector: 3 per node, plus one per pressure node.
inline int64_t ndof(const Ctx *c) { return 3 * c->m.n_nodes + (c->mixed ? c->mx.n_p : 0); }
// The material must suit the mesh (M3 on mixed meshes only), and M4 needs fibres.
inline nle_status need_fibres(Ctx *c) {
  if (c->mixed && c->mx.n_p == 0) {
    if (c->mat.kind == NLE_MAT_M3 || c->mat.kind == NLE_MAT_M5)
      return fail(c, NLE_E_STATE, "laws M3 and M5 need a pressure field");
  } else if ((c->mat.kind == NLE_MAT_M3 || c->mat.kind == NLE_MAT_M5) != c->mixed) {
    return fail(c, NLE_E_STATE,
                "laws M3 and M5 go with a mixed mesh, the other laws with P1 meshes");
  }
  if (c->mat.kind == NLE_MAT_M4 && !c->fib64)
    return fail(c, NLE_E_STATE, "law M4 needs nle_set_fibres");
  if (c->mat.kind == NLE_MAT_M6 && (!c->fib64 || !c->sh64))
    return fail(c, NLE_E_STATE, "law M6 needs nle_set_fibre_frame");
  return NLE_OK;
}
void drop_graph(Ctx *c);
#define NLE_HIP(c, call)                                                        \
  do {                                                                          \
    hipError_t e_ = (call);                                                     \
    if (e_ != hipSuccess)                                                       \
      return ::nle::fail((c), NLE_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// mesh preparation (host)
// inst_elem / inst_node: instance offsets (size n_inst + 1) of a disjoint
// union of meshes (element and node ranges); null for a single mesh.
nle_status build_mesh(Ctx *c, int64_t n_nodes, const double *X, int64_t n_elems, const int32_t *conn,
                      const std::vector<int64_t> *inst_elem = nullptr,
                      const std::vector<int64_t> *inst_node = nullptr);
nle_status upload_node_masks(Ctx *c);

// ---- surface loads (nle_surf.hip) ------------------------------------------
// (Re)build the face-node structure from surf.h_ptri / h_rtri and the mesh.
nle_status build_surface(Ctx *c);
// Re-write the per-face Dirichlet bits after the Dirichlet set changed.
nle_status upload_surface_masks(Ctx *c);
void free_surface(Ctx *c);
// Evaluate the surface contributions of op (OP_RES at u, OP_JV of v at the
// linearization state u, OP_DIAG at u) into surf.fs64 / fs32 and return that
// buffer; OP_ENERGY writes per-workgroup partials of the spring energy to red
// and returns their count through *n_red.
void *surf_apply(Ctx *c, int op, int prec, const void *u, const void *v, int *n_red,
                 hipError_t *err, double *red = nullptr);
// Store s * p as the pressure seen by the Jacobian action.
hipError_t surf_set_linear_pressure(Ctx *c);

// ---- mixed quadratic / linear elements (nle_mixed.hip) --------------------
nle_status build_mixed_mesh(Ctx *c, int64_t n_u, const double *X, int64_t n_e, const int32_t *conn,
                            int64_t n_p, const int32_t *pconn, int npe = 4);
// shear modulus of the mixed law's small-strain limit (pressure-mass scaling)
double mixed_mu_eff(const Ctx *c);
// the SIMPLE Schur diagonal of the constant-pressure pair at the current
// linearization (into mx.s64 or s_out, inverses into mx.sinv64 / sinv32)
hipError_t mixed_simple_diag(Ctx *c, double *s_out = nullptr);
nle_status upload_mixed_masks(Ctx *c);
int mixed_apply(Ctx *c, int op, int prec, const void *x, const void *v, void *out, double *red,
                hipError_t *err);
int mixed_red_capacity(const Ctx *c);

// ---- element kernels (nle_elem.hip) ---------------------------------------
// Launch the block and merge kernels of `op` in precision prec.
//  OP_RES: u = double state, out = r, red gets per-workgroup sum r.r
//  OP_JV : u = linearization state (prec), v = direction, out = J v
//  OP_DIAG: u = ulin64, out = diag (double)
//  OP_ENERGY: u = double state, red gets per-workgroup sum V Psi
// Returns the number of reduction partials written to red (0 if none); for
// OP_JV with c->ep.red set, the number of v.(Jv) partials written there.
int elem_apply(Ctx *c, int op, int prec, const void *u, const void *v, void *out, double *red,
               hipError_t *err);
// Address of the fixed workspace of the allocation-free Jacobian action on
// `device` (must be the current device), looked up once per device.
hipError_t noalloc_scratch_init(int device, void **out);
int elem_red_capacity(const Ctx *c);

// ---- vector kernels (nle_vec.hip) ------------------------------------------
int vgrid(int64_t n);
hipError_t vec_fill(Ctx *c, int prec, void *x, double val, int64_t n);
hipError_t vec_cast_scale(Ctx *c, int px, const void *x, int py, void *y, double scale, int64_t n);
// y = y + a * x   (x in precision px, y in precision py); a taken from a
// device scalar *a_dev times a_host (a_dev may be null).
hipError_t vec_axpy(Ctx *c, int px, const void *x, int py, void *y, double a_host,
                    const double *a_dev, int64_t n);
hipError_t vec_lift(Ctx *c, double *u);
// w[d] = (prescribed value - u[d]) on the Dirichlet dofs; other entries untouched
hipError_t vec_dir_delta(Ctx *c, const double *u, double *w);
// partials of sum_i a_i b_i (and sum b_i^2 if sq != 0) -> red; returns count
int vec_dot_partials(Ctx *c, int prec, const void *a, const void *b, int64_t n, double *red,
                     hipError_t *err);
// single-workgroup fixed-order sum of red[0..np) (stride 1) -> out[0]
hipError_t reduce_scalar(Ctx *c, const double *red, int np, double *out);
hipError_t reduce_scalars(Ctx *c, const double *red, int np, int count, double *out);
hipError_t vec_recip(Ctx *c, const double *d, double *dinv, int64_t n);
// ---- aggregation multigrid (nle_amg.cpp) ----------------------------------------
// amg_prepare builds what is missing for the current linearization (NLE_OK or
// an error set on c); amg_apply is one V-cycle x = M^-1 b in precision prec
// (x must not alias b);
// amg_invalidate marks the values stale (new linearization); amg_release
// frees everything (new mesh or Dirichlet set, destroy).
nle_status amg_prepare(Ctx *c);
// red_dot (nullable): also write the partials of b . x at red_dot[0 .. vgrid(n));
// first_done: the caller has already taken the finest level's first Chebyshev
// step, x = d = inv_theta D^-1 b, with the arguments amg_first_step gives
// (false when the hierarchy has no such step: one level, or a pressure field)
hipError_t amg_apply(Ctx *c, int prec, const void *b, void *x, double *red_dot = nullptr,
                     bool first_done = false);
bool amg_first_step(Ctx *c, int prec, const void **dinv, void **d, double *inv_theta);
void amg_invalidate(Ctx *c);
void amg_release(Ctx *c);
int amg_levels(const Ctx *c, int64_t *sizes, int cap);

// dashpots act only in an implicit step with a velocity set
inline bool damping_on(const Ctx *c) {
  return c->inr.on && c->inr.cv > 0.0 && c->inr.vt && c->surf.nrf > 0 &&
         (c->surf.cperp != 0.0 || c->surf.cpar != 0.0);
}
// ut = u + dt v + dt^2 (1/2 - beta) a; vt (if not null) = v + dt (1 - gamma) a
hipError_t newmark_predict(Ctx *c, const double *u, const double *v, const double *a, double *ut,
                           double *vt, double dt, double beta, double gamma, int64_t n);
hipError_t newmark_correct(Ctx *c, const double *u, const double *ut, double *v, double *a,
                           double dt, double beta, double gamma, int64_t n);
int vec_wdiff2_partials(Ctx *c, const double *w, const double *x, const double *y, int64_t n,
                        double *red, hipError_t *err);
// y = M^-1 x with pcb = 1 (d: inverse diagonal, identity if null) or
// pcb = 3 (d: nodal block inverses [6][n/3], see block_inverse)
hipError_t pc_apply(Ctx *c, int prec, int pcb, const void *d, const void *x, void *y, int64_t n);
// x_p = -(b_p - t_p) * sinv_p over np entries (lower Schur block)
hipError_t schur_p(Ctx *c, int prec, const void *b, const void *t, const void *sinv, void *x,
                   int64_t np);
// Lower block-triangular preconditioner of a displacement / pressure tangent
// (App. B): x_u = A^-1 b_u (point Jacobi, or the multigrid cycle when amg),
// x_p = S^-1 (b_p - B x_u) with S = -M_p / mu_eff (schur = 1) or minus the
// SIMPLE diagonal (schur = 2, constant pressure).  t1, t2: work vectors of
// the unknown length.  x must not alias b.
hipError_t schur_lower_apply(Ctx *c, int prec, bool amg, int schur, const void *b, void *x,
                             void *t1, void *t2);
// binv64 / binv32 from diag64 and odiag64 (nn nodes)
hipError_t block_inverse(Ctx *c, int64_t nn);
// odiag64 and the block inverses at the current linearization (P1 meshes)
nle_status ensure_block(Ctx *c);

// CG kernels (no per-iteration host arguments: a chunk of iterations can be
// captured as a graph)
struct CgArgs {
  int prec;
  int64_t n;
  void *x, *r, *z, *p, *Ap;
  const void *dinv;   // may be null (no preconditioner)
  int pcb = 1;        // 1: point Jacobi dinv; 3: nodal block inverses in dinv
  double *red_a;      // partials of p.Ap (from the Jacobian-action epilogue)
  int np_a;
  double *red_b;      // partials of (r.z, r.r), 2 x VGRID_MAX
  double *scal;       // device scalars
  int32_t *flag;      // [0] state (1 converged, 2 breakdown, 3 NaN, 5 limit), [1] its
  // with the multigrid: the update also takes the cycle's first Chebyshev
  // step, z = cd = cth D^-1 r (dinv then holds the finest level's D^-1)
  void *cd = nullptr;
  double cth = 0.0;
};
// finish = false leaves out the final reduction (cg_start_finish), so that a
// preconditioner applied outside the kernels can replace z, p and the r.z partials
hipError_t cg_start(Ctx *c, const CgArgs &a, const void *b, double rtol, double atol, int max_it,
                    bool finish = true);
hipError_t cg_start_finish(Ctx *c, const CgArgs &a, double rtol, double atol, int max_it);
hipError_t cg_update(Ctx *c, const CgArgs &a, bool fused = false);
hipError_t cg_direction(Ctx *c, const CgArgs &a);

// MINRES kernels
struct MinresArgs {
  int prec;
  int64_t n;
  void *x, *r1, *r2, *y, *v, *av, *wa, *wb, *za, *zb, *r;
  const void *dinv;
  int pcb = 1;  // as in CgArgs
  double *red_a;  // partials of v.(A v - coef r1) from the Jacobian-action epilogue
  int np_a;
  double *red_b;  // partials of t.(M^-1 t)
  double *red_r;  // partials of r.r
  double *scal;
  int32_t *flag;
};
// finish = false leaves out the scalar set-up (mr_start_finish), so that a
// preconditioner applied outside the kernels can replace y = M^-1 b and the
// partials of b.y (with dinv null the kernels apply the identity)
hipError_t mr_start(Ctx *c, const MinresArgs &a, const void *b, double rtol, double atol,
                    int max_it, bool finish = true);
hipError_t mr_start_finish(Ctx *c, const MinresArgs &a, double rtol, double atol, int max_it);
// pc_outside (nullable): called after the first vector step, it must set
// y = M^-1 r2 and write the partials of r2.y to red_b
hipError_t mr_iterate(Ctx *c, const MinresArgs &a,
                      hipError_t (*pc_outside)(Ctx *, const MinresArgs &) = nullptr);

// GMRES kernels.  The basis grows with the iterations: vectors, Hessenberg
// columns and the partial-sum rows of the multi-dots live in segments that
// are allocated as the cycle needs them, reached through device tables of
// pointers (entry i: basis vector i, Hessenberg column i of length i + 2,
// partial row i) and the host copies of the vector and row pointers.
struct GmresArgs {
  int prec;
  int64_t n;
  int m;             // cycle length (restart, or the iteration limit)
  void **Vp;         // device table [m+1] of basis vectors
  double **Hp;       // device table [m+1] of Hessenberg columns
  double **Rp;       // device table [m+1] of partial rows (VGRID_MAX each)
  void *const *hV;   // host copies of the vector pointers
  double *const *hR; // host copies of the row pointers
  void *w;           // [n] work
  void *z;           // [n] work (preconditioned)
  void *x;           // [n] solution
  const void *dinv;  // may be null
  int pcb = 1;       // as in CgArgs
  double *rot;       // cs[m], sn[m], g[m+1], y[m]
  double *redsq;     // partials of w.w (VGRID_MAX)
  double *scal;
  int32_t *flag;
};
// Fill the device tables for segment [v0, v0 + nv) of the basis pool (entries
// at or beyond `limit` are left alone).
hipError_t gmres_tables(Ctx *c, const GmresArgs &a, int v0, int nv, int limit, void *vbase,
                        size_t vb, double *hbase, double *rbase);
hipError_t gmres_multidot(Ctx *c, const GmresArgs &a, int j);           // h_i = V_i . w, i<=j
hipError_t gmres_subtract(Ctx *c, const GmresArgs &a, int j, int pass, int want_dots);
hipError_t gmres_mgs_step(Ctx *c, const GmresArgs &a, int i, int j);    // fused MGS step
hipError_t gmres_finish_col(Ctx *c, const GmresArgs &a, int j, int mgs);// norm, Givens, test
hipError_t gmres_update_x(Ctx *c, const GmresArgs &a);                  // x += M^-1 V y
hipError_t gmres_start(Ctx *c, const GmresArgs &a, const void *r0, double rtol, double atol,
                       int first);

// L-BFGS two-loop kernels
hipError_t lbfgs_dot(Ctx *c, int prec, const void *s, const void *q, int64_t n, double *red,
                     int *np);
// q -= alpha * y with alpha = rho * sum(red) (stored to alpha_out[0]);
// optionally accumulates partials of s_next . q_new into red_next
hipError_t lbfgs_axpy_dot(Ctx *c, int prec, void *q, const void *y, const double *red, int np,
                          double rho, double *alpha_out, const void *s_next, double *red_next,
                          int64_t n);
// z += (alpha - rho * sum(red)) * s ; optionally partials of y_next . z_new
hipError_t lbfgs_axpy2_dot(Ctx *c, int prec, void *z, const void *s, const double *red, int np,
                           double rho, const double *alpha, const void *y_next, double *red_next,
                           int64_t n);

}  // namespace nle
