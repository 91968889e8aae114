/*
 * nlelast.h -- C ABI of the MI355X (gfx950) nonlinear-elasticity solver library.
 *
 * The library solves the quasi-static hyperelastic balance of the paper
 * (Sec. 2, eq. "momentum strong" without inertia) on P1 tetrahedral meshes,
 * matrix-free, with the nonlinear solvers of Sec. 3: Newton-Krylov (NK),
 * inexact Newton-Krylov with Eisenstat-Walker forcing (iNK) and limited-memory
 * BFGS with an initial inverse Hessian taken from the tangent at the first
 * iterate (BFGS-preonly and inexact BFGS); solver options follow App. A.
 *
 * Conventions (all calls):
 *  - Displacement-like vectors interleave components per node:
 *    dof = 3 * node + component, length 3 * n_nodes.
 *  - The residual is r(u) = f_int(u) - s * f_ext, the gradient of the
 *    potential Pi(u) = sum_e V_e Psi(F_e) - s f_ext . u (Sec. 3, eq.
 *    "minimization"); this is the paper's R = f - div P up to sign (same
 *    root).  r is zero on Dirichlet dofs; the tangent J = dr/du has identity
 *    rows and columns there (strong imposition; u holds the prescribed
 *    values, increments vanish).
 *  - Host pointers are borrowed for the duration of a call and never kept.
 *    Device pointers are caller-owned (e.g. torch tensors on the context's
 *    device) and must stay valid until the work queued on the context's
 *    stream has finished.  The library never frees caller memory.
 *  - Calls are asynchronous on the context's stream unless they return host
 *    scalars (residual norm, solve report), which synchronise that stream.
 *  - A context is bound to one device and one stream and is not thread-safe.
 *  - Return values: 0 = NLE_OK; > 0 a solver outcome (the call ran, the
 *    solve did not converge); < 0 a usage or system error, with a message
 *    from nle_last_error().  No C++ exception crosses this interface.
 *  - Results are deterministic: every sum (element scatter, dot product,
 *    norm) is taken in a fixed order without floating-point atomics, so a
 *    repeated call on the same inputs is bitwise identical.
 */
#ifndef NLELAST_H
#define NLELAST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
typedef int32_t nle_status;
#define NLE_OK 0
#define NLE_DIVERGED_MAXIT 1    /* nonlinear iteration limit reached          */
#define NLE_DIVERGED_NAN 2      /* residual norm became NaN or Inf            */
#define NLE_DIVERGED_INVERTED 3 /* some element has det F <= 0               */
#define NLE_DIVERGED_LINEAR 4   /* Krylov breakdown (e.g. CG p.Ap <= 0)       */
#define NLE_BFGS_BREAKDOWN 5    /* L-BFGS direction unusable                  */
#define NLE_E_INVAL (-1)        /* bad argument                               */
#define NLE_E_BADMESH (-2)      /* index out of range / repeated / V_e <= 0   */
#define NLE_E_STATE (-3)        /* call order violated (e.g. jv before linearize) */
#define NLE_E_OOM (-4)          /* device allocation failed                  */
#define NLE_E_HIP (-5)          /* HIP runtime error                          */
#define NLE_E_UNSUPPORTED (-6)  /* option not implemented                     */

/* ---- enumerations ---------------------------------------------------- */
#define NLE_FP64 0 /* kernel arithmetic / vector storage in double */
#define NLE_FP32 1 /* kernel arithmetic / vector storage in float  */

/* Materials (Sec. 2, Sec. 4 "Cook test"); params in parentheses.
 * M1 compressible neo-Hookean (mu, lambda):
 *      Psi = mu/2 (I1 - 3) - mu ln J + lambda/2 (ln J)^2
 * M2 the paper's Cook law with the isochoric / volumetric split
 *    (mu, lambda, c_vol), kappa = lambda + 2 mu / 3:
 *      Psi = mu/2 (J^(-2/3) I1 - 3) + c_vol kappa (J^2 - 1 - 2 ln J)
 *    The printed law has c_vol = 1; c_vol = 1/4 gives bulk modulus kappa in
 *    the small-strain limit.  n_params = 2 takes c_vol = 1/4. */
#define NLE_MAT_M1 1
#define NLE_MAT_M2 2
#define NLE_MAT_M3 3
#define NLE_MAT_M4 4
/* M5 the twist test's polyconvex law (Sec. 4), on mixed meshes, params
 * (alpha_p, beta_p, alpha_s, beta_s), printed values all 9000:
 *      Psi = alpha_p (F:F - 3) + beta_p (cof F : cof F - 3)
 *            - (4 beta_s + 2 alpha_s) ln J - p (J - 1),   cof F = J F^-T,
 *    the printed "log(F)" read as ln det F (the reading with a stress-free
 *    reference when 2 alpha_p + 4 beta_p = 4 beta_s + 2 alpha_s); small-strain
 *    limit mu = 2 (alpha_p + beta_p), lambda = 4 beta_p. */
#define NLE_MAT_M5 5
/* M6 the heartbeat test's Guccione law (Sec. 4), P1 and quadratic
 * displacement meshes, params
 * (C, b_ff, b_ss, b_nn, b_fs, b_fn, b_sn, B) (the constants are the
 * caller's; the paper refers to Guccione's paper for them):
 *      Psi = C/2 (exp(Q) - 1) + B/2 (J - 1) ln J + gamma sqrt(I4),
 *      Q = b_ff E_ff^2 + b_ss E_ss^2 + b_nn E_nn^2 + b_fs (E_fs^2 + E_sf^2)
 *          + b_fn (E_fn^2 + E_nf^2) + b_sn (E_sn^2 + E_ns^2),
 *    E = (F^T F - I)/2 in the per-element frame {f, s, n = f x s} of
 *    nle_set_fibre_frame; gamma from nle_set_active_tension (the active
 *    stress gamma (F f) (x) f / |F f|).  Nodal block Jacobi is not offered
 *    for it. */
#define NLE_MAT_M6 6

#define NLE_NK 0   /* Newton-Krylov, fixed linear tolerance (App. A)        */
#define NLE_INK 1  /* inexact NK, Eisenstat-Walker forcing (Sec. 3, App. A) */
#define NLE_BFGS 2 /* limited-memory BFGS (Sec. 3, App. A)                  */

#define NLE_KSP_GMRES 0  /* right-preconditioned GMRES(restart)             */
#define NLE_KSP_CG 1     /* preconditioned conjugate gradients (SPD tangent) */
#define NLE_KSP_MINRES 2 /* preconditioned MINRES (symmetric, possibly
                            indefinite tangent; SPD preconditioner)        */

#define NLE_ORTH_MGS 0  /* modified Gram-Schmidt (the paper's choice)       */
#define NLE_ORTH_CGS2 1 /* classical Gram-Schmidt, two passes               */

#define NLE_PC_NONE 0
#define NLE_PC_JACOBI 1 /* point Jacobi: inverse of the tangent diagonal     */
#define NLE_PC_BJACOBI3 2 /* nodal block Jacobi: inverse of each node's 3x3
                             diagonal block of the tangent (P1 meshes; the
                             bs = 3 point-block Jacobi of a PETSc setup)  */
#define NLE_PC_AMG 3 /* aggregation multigrid, one V(1,1)-cycle (the AMG of
                        Sec. 4 and App. A; its construction is this
                        library's, see nle_pc_apply), with GMRES, CG or
                        MINRES (the cycle is symmetric for a symmetric
                        tangent, and positive definite where the tangent
                        is), or as the H0 of BFGS-preonly.  With a pressure
                        field: the block-diagonal field split, GMRES only */

#define NLE_H0_PREONLY 0 /* BFGS-preonly: H0 = one preconditioner application */
#define NLE_H0_KSP 1     /* inexact BFGS: H0 = Krylov solve on J(u0)          */

#define NLE_PREC_FP64 0  /* every vector and kernel in double                */
#define NLE_PREC_MIXED 1 /* FP32 tangent, preconditioner, Krylov and L-BFGS
                            vectors; FP64 residual, norms, state and update */

typedef struct nle_ctx nle_ctx;

/* Optional device allocator (e.g. a framework's caching allocator).  alloc
 * returns device memory on the context's device or NULL; free releases it.
 * With a NULL allocator the library uses hipMalloc / hipFree. */
typedef struct {
  void *(*alloc)(size_t bytes, void *user);
  void (*free)(void *ptr, void *user);
  void *user;
} nle_allocator;

/* Solver options: the PETSc options of App. A as fields. */
typedef struct {
  int32_t precision;  /* NLE_PREC_FP64 / NLE_PREC_MIXED                      */
  int32_t ksp_type;   /* NLE_KSP_GMRES / NLE_KSP_CG / NLE_KSP_MINRES          */
  int32_t orth;       /* GMRES orthogonalisation                              */
  int32_t pc;         /* NLE_PC_JACOBI / NLE_PC_BJACOBI3 / NLE_PC_AMG /
                         NLE_PC_NONE (batched solves: Jacobi only)          */
  int32_t restart;    /* GMRES restart length; <= 0 means ksp_max_it (no
                         restart).  The basis is allocated as the cycle
                         grows (segments of max(64, half the vectors so
                         far), each with its Hessenberg columns), kept by the
                         context for later solves; a failed growth returns
                         NLE_E_OOM.  Up front only O(ksp_max_it) scalars.  */
  int32_t ksp_max_it; /* Krylov iteration limit per linear solve              */
  int32_t snes_max_it;/* nonlinear iteration limit                            */
  int32_t ew_version; /* Eisenstat-Walker variant 1 or 2                      */
  int32_t qn_m;       /* L-BFGS memory (App. A uses 50)                       */
  int32_t h0;         /* NLE_H0_PREONLY / NLE_H0_KSP                          */
  int32_t check_every;/* Krylov iterations queued between host checks        */
  int32_t cg_launches;/* CG launches per iteration besides a multigrid
                         cycle: 4 (a separate direction kernel; also 0,
                         the default) or 3 (the next direction and the
                         stopping test are formed inside the Jacobian
                         action; P1 meshes without surface loads, else 4).
                         Same iterates bit for bit; the copy of r.r that
                         the stagnation test reads lags one iteration in
                         the 3-launch form                               */
  double ksp_rtol, ksp_atol;        /* NK: 1e-6, 1e-10                    */
  double ew_rtol0, ew_rtolmax;      /* iNK: 0.1, 0.1                      */
  double ew_rtolmin;                /* lower clip of eta (0: none); mixed
                                       precision clips at 1e-4 at least   */
  double ew_gamma, ew_alpha, ew_alpha2, ew_threshold; /* 1, phi, phi, 0.1 */
  double ink_ksp_atol;              /* iNK absolute tolerance: 1e-14      */
  double snes_rtol, snes_atol;      /* ||r_k|| <= max(rtol ||r_0||, atol) */
  double h0_rtol, h0_atol;          /* inexact BFGS H0 solve: 1e-2, 1e-14 */
  double curvature_eps;             /* skip pair if s.y <= eps |s||y|     */
  int32_t h0_refresh; /* BFGS: every h0_refresh iterations re-linearize at
                         the current iterate (new tangent, preconditioner
                         and H0) and drop the stored pairs; 0 = once per
                         solve, the single assembly of Sec. 3            */
  int32_t jac_lag;    /* NK / iNK: re-linearize every jac_lag Newton
                         iterations and reuse the last tangent (and
                         preconditioner) in between; 0 or 1 = every
                         iteration.  Jacobian lagging, an extension the
                         conclusions (Sec. 7) name                       */
  int32_t h0_ew;      /* inexact BFGS: nonzero = the H0 solve's relative
                         tolerance follows Eisenstat-Walker choice 2 on
                         the BFGS residual norms, eta_k = gamma (|g_k| /
                         |g_k-1|)^alpha with its safeguard, eta_0 and the
                         upper clip h0_rtol, the lower clip ew_rtolmin
                         (and 1e-4 in mixed precision); 0 = fixed h0_rtol.
                         The adaptive variant Sec. 3 leaves open         */
  int32_t schur;      /* displacement / pressure meshes: NLE_SCHUR_DIAG (the
                         block-diagonal preconditioner, default), or the
                         lower block-triangular form of App. B with GMRES,
                         NLE_SCHUR_LOWER_MASS or NLE_SCHUR_LOWER_SIMPLE; the
                         displacement block takes pc (JACOBI or AMG)      */
} nle_solver_opts;

/* Schur complement preconditioners of a displacement / pressure tangent
 * [[A, B^T], [B, 0]] (App. B, eq. "schur"; Sec. 4 "Twist test"):
 *  NLE_SCHUR_DIAG         diag(A^, S^) with S^ = M_p / mu_eff (positive:
 *                         the lumped pressure mass over the law's
 *                         small-strain shear modulus), symmetric positive
 *                         definite, for MINRES or GMRES;
 *  NLE_SCHUR_LOWER_MASS   the lower factor [[A^, 0], [B, S^]] with
 *                         S^ = -M_p / mu_eff: z_u = A^^-1 r_u,
 *                         z_p = S^^-1 (r_p - B z_u) (one extra Jacobian
 *                         action per application);
 *  NLE_SCHUR_LOWER_SIMPLE the lower factor with SIMPLE, S^ = -diag(B diag(A)^-1
 *                         B^T) (A^-1 approximated by its diagonal, the Schur
 *                         block then by its own diagonal); the constant-
 *                         pressure pair only, where each row of B lives on
 *                         one element.
 * A^ is point Jacobi (pc = NLE_PC_JACOBI) or the multigrid cycle on the
 * displacement block (pc = NLE_PC_AMG). */
#define NLE_SCHUR_DIAG 0
#define NLE_SCHUR_LOWER_MASS 1
#define NLE_SCHUR_LOWER_SIMPLE 2

/* Solve report.  Histories are written to caller buffers of hist_cap
 * entries (any may be NULL); entry k belongs to nonlinear iteration k. */
typedef struct {
  int32_t status;       /* same code as the solve's return value            */
  int32_t nit;          /* nonlinear iterations                             */
  int64_t lit_total;    /* Krylov iterations, summed                        */
  int64_t n_jv;         /* Jacobian actions                                 */
  int64_t n_residual;   /* residual evaluations                             */
  int32_t bfgs_skipped; /* L-BFGS pairs rejected by the curvature test      */
  int32_t hist_cap;
  double rnorm0;        /* ||r|| at the start of the step (after the lift)  */
  double rnorm_final;
  double t_ms;          /* wall time of the solve on the stream (HIP events) */
  double *rnorm_hist;   /* [hist_cap] ||r_k||, k = 0..nit                   */
  double *eta_hist;     /* [hist_cap] linear relative tolerance used        */
  int32_t *lit_hist;    /* [hist_cap] Krylov iterations per step            */
  int32_t cutbacks;     /* batched solves: halved load increments of the
                           instance (0 for single solves, whose load stepping
                           is the caller's)                                 */
  int32_t reserved;
} nle_report;

/* ---- context ---------------------------------------------------------- */
/* Create a context on `device`, queueing work on `hip_stream` (a
 * hipStream_t; NULL = the null stream).  `alloc` may be NULL. */
nle_status nle_create(nle_ctx **out, int32_t device, void *hip_stream, const nle_allocator *alloc);
/* Release every device buffer the library allocated.  NULL is a no-op. */
void nle_destroy(nle_ctx *ctx);
const char *nle_last_error(const nle_ctx *ctx);
const char *nle_version(void);

/* Elements per block of the element partition (fixed-order scatter unit);
 * takes effect at the next nle_upload_mesh.  Range 64..4096, default 512. */
nle_status nle_set_block_size(nle_ctx *ctx, int32_t elems_per_block);

/* ---- problem data ----------------------------------------------------- */
/* Upload a P1 tetrahedral mesh (Sec. 4 geometries; host arrays).
 *   X    [n_nodes][3] reference coordinates (double).
 *   conn [n_elems][4] node indices (int32), positively oriented:
 *        det[X1-X0, X2-X0, X3-X0] > 0.
 * nodes_per_elem = 10 uploads quadratic displacement elements instead (the
 * second-order runs of the Sec. 6 tables): conn [n_elems][10] as in
 * nle_upload_mesh_mixed, no pressure field, laws M1, M2, M4 and M6 at the
 * four points of the degree-2 rule (per-element fibres and sheets in the
 * caller's element order), Dirichlet data, active tension, and on 6-node
 * faces (the vertex triangles passed as for P1 meshes, midpoints found from
 * the elements) dead traction, follower pressure and springs; follower
 * traction, body force, inertia and nodal blocks are NLE_E_UNSUPPORTED
 * there.
 * Validates indices (0 <= i < n_nodes, no repeats within an element) and
 * volumes; on failure returns NLE_E_BADMESH and names the first bad element.
 * Precomputes shape-function gradients and volumes in FP64 (and an FP32
 * copy) and the element partition.  Resets Dirichlet data, loads and the
 * linearization.  n_nodes < 2^28. */
nle_status nle_upload_mesh(nle_ctx *ctx, int64_t n_nodes, const double *X, int64_t n_elems,
                           int32_t nodes_per_elem, const int32_t *conn);
/* Mixed quadratic-displacement / linear-pressure mesh (Sec. 4 "Twist test"
 * with the P2-P1 pair): n_nodes displacement nodes X[n_nodes][3], conn
 * [n_elems][10] (four vertices, positively oriented, then the midpoints of
 * edges (0,1), (1,2), (0,2), (0,3), (1,3), (2,3); straight-sided), and
 * n_pnodes pressure nodes with pconn[n_elems][4] (the pressure at the four
 * vertices).  Host arrays, copied.  The unknown vector then has 3 n_nodes +
 * n_pnodes entries: [u (node-interleaved) | p].  Laws NLE_MAT_M3,
 *   L(u, p) = int mu/2 (I1 - 3) - mu ln J - p (J - 1)   (params = (mu)),
 * and NLE_MAT_M5 apply, integrated by the 4-point degree-2 rule; the tangent
 * is symmetric and indefinite (use MINRES or GMRES).  The Jacobi data
 * (nle_diag) are the displacement-block diagonal and, on pressure rows, the
 * lumped pressure mass over the law's small-strain shear modulus, so
 * NLE_PC_JACOBI is a block-diagonal SPD preconditioner.  Dirichlet
 * dofs index displacement dofs.  Fibres, follower pressure, springs and body
 * forces are NLE_E_UNSUPPORTED on mixed meshes.  NLE_E_BADMESH on bad indices
 * or a non-positive vertex volume. */
nle_status nle_upload_mesh_mixed(nle_ctx *ctx, int64_t n_nodes, const double *X, int64_t n_elems,
                                 const int32_t *conn, int64_t n_pnodes, const int32_t *pconn);
/* The twist test's own pair (Sec. 4): quadratic displacement as in
 * nle_upload_mesh_mixed (conn [n_elems][10]) with one pressure unknown per
 * element (P2-P0; the pressure test function is 1 on its element,
 * R_p[e] = -int_e (J - 1)).  The unknown vector is [u | p], p[e] for user
 * element e, 3 n_nodes + n_elems entries.  Laws M3 and M5 apply; the Jacobi
 * data on pressure rows are the element volume over the law's small-strain
 * shear modulus.  Errors as nle_upload_mesh_mixed. */
nle_status nle_upload_mesh_mixed_p0(nle_ctx *ctx, int64_t n_nodes, const double *X,
                                    int64_t n_elems, const int32_t *conn);
/* Material law and parameters (see NLE_MAT_*).  NLE_MAT_M4 (cardiac-like,
 * Sec. 4 "Heartbeat test" with a stated substitute for its Guccione law):
 *   Psi = a/(2b) (exp(b (J^-2/3 I1 - 3)) - 1)
 *         + a_f/(2 b_f) (exp(b_f (I4 - 1)^2) - 1) [I4 > 1]
 *         + kappa/2 (J - 1)^2 + gamma sqrt(I4),       I4 = |F f|^2,
 * params = (a, b, a_f, b_f, kappa); the last term is the paper's active
 * stress gamma (F f) (x) f / |F f| (gamma from nle_set_active_tension, f per
 * element from nle_set_fibres, both required state for M4). */
nle_status nle_set_material(nle_ctx *ctx, int32_t kind, const double *params, int32_t n_params);
/* Dirichlet dofs and their prescribed displacement (host arrays of n
 * entries; dofs unique, in [0, 3 n_nodes)).  Replaces previous data. */
nle_status nle_set_dirichlet(nle_ctx *ctx, int64_t n, const int64_t *dofs, const double *values);
/* Dead traction t (per unit reference area, 3 doubles) on n_faces
 * triangles tri[n_faces][3]; consistent nodal load t A / 3 per vertex.
 * Replaces the traction part of f_ext. */
nle_status nle_set_traction(nle_ctx *ctx, int64_t n_faces, const int32_t *tri, const double *t);
/* Uniform body force f (3 doubles, per unit reference volume): f V_e / 4 per
 * vertex.  Replaces the body-force part of f_ext. */
nle_status nle_set_body_force(nle_ctx *ctx, const double *f);
/* Load factor s multiplying f_ext and the follower pressure (default 1). */
nle_status nle_set_load_scale(nle_ctx *ctx, double s);
/* Unit fibre direction per element for law M4: fib[n_elems][3] (host, user
 * element order, copied); NLE_E_INVAL unless every |f| = 1 to 1e-6.  P1 and
 * quadratic displacement meshes; NLE_E_UNSUPPORTED with a pressure field. */
nle_status nle_set_fibres(nle_ctx *ctx, const double *fib);
/* Fibre frame per element for law M6: fib and sheet [n_elems][3] (host,
 * user element order, copied), unit vectors to 1e-6 and orthogonal to 1e-6
 * (NLE_E_INVAL otherwise); the third direction is n = f x s.  Also sets the
 * fibres of law M4. */
nle_status nle_set_fibre_frame(nle_ctx *ctx, const double *fib, const double *sheet);
/* Active tension gamma of laws M4 and M6 (Sec. 4, the activation function's
 * value at the current time step; default 0). */
nle_status nle_set_active_tension(nle_ctx *ctx, double gamma);
/* Follower pressure p (times the load scale) on n_faces triangles tri[][3]
 * whose (x1 - x0) x (x2 - x0) points out of the body: it acts on the current
 * surface, against the outward normal (an endocardial cavity pressure, Sec. 4
 * "Heartbeat test").  The residual gains p (x1-x0) x (x2-x0) / 6 per vertex
 * (x = X + u); its Jacobian is not symmetric, so use GMRES.  The Jacobian
 * action uses the pressure at the time of nle_linearize.  Replaces previous
 * pressure faces; n_faces = 0 removes them.  With a pressure set, nle_energy
 * returns NLE_E_UNSUPPORTED (no potential). */
nle_status nle_set_pressure(nle_ctx *ctx, int64_t n_faces, const int32_t *tri, double p);
/* Follower traction on n_faces triangles tri[n][3] (node ids): the
 * traction t[3] has a fixed spatial direction and acts per unit CURRENT area
 * (Sec. 4 applies the Cook load in the deformed configuration; this reads it
 * as a Cauchy traction of fixed direction), scaled by the load scale: each
 * vertex of a face with current area vector a = (x1-x0) x (x2-x0)/2 receives
 * s t |a| / 3.  Its tangent is not symmetric (use GMRES), the diagonal and
 * nodal blocks take its own-node part (blocks: the symmetric part), and
 * nle_energy refuses it.  Replaces any earlier follower traction; P1 meshes
 * only.  Host arrays, copied. */
nle_status nle_set_traction_follower(nle_ctx *ctx, int64_t n_faces, const int32_t *tri,
                                     const double *t);
/* Elastic Robin springs on n_faces triangles (the epicardial condition of
 * Sec. 4 without its damping terms): traction -(k_perp N (x) N + k_par
 * (I - N (x) N)) u with the reference unit normal N, integrated exactly
 * (consistent P1 face mass).  Replaces previous spring faces. */
nle_status nle_set_robin(nle_ctx *ctx, int64_t n_faces, const int32_t *tri, double k_perp,
                         double k_par);
/* Inertia of one implicit time step (Sec. 4 "Heartbeat test" is a dynamic
 * problem; its time integration is not given, this library offers the
 * Newmark average-acceleration step).  With M the row-sum lumped P1 mass of
 * density rho (rho V / 4 per element vertex and direction), the residual
 * gains coef M (u - u_tilde), the tangent coef M, the Jacobi and block
 * diagonals coef M, and nle_energy coef/2 (u - u_tilde)^T M (u - u_tilde)
 * (Dirichlet dofs keep identity rows).  For Newmark, coef = 1/(beta dt^2)
 * and u_tilde comes from nle_newmark_predict.  u_tilde_dev (double, device,
 * 3 n_nodes) is copied.  rho = 0 or coef = 0 switches the term off.  P1
 * meshes only (NLE_E_UNSUPPORTED on a mixed mesh); NLE_E_INVAL for negative
 * or non-finite values or a null u_tilde while on.  Resets linearizations. */
nle_status nle_set_inertia(nle_ctx *ctx, double rho, double coef, const double *u_tilde_dev);
/* Newmark predictor (double, device, 3 n_nodes each):
 * u_tilde = u + dt v + dt^2 (1/2 - beta) a and, if v_tilde_dev is not NULL,
 * v_tilde = v + dt (1 - gamma) a (the part of the new velocity known before
 * the solve; see nle_set_step_velocity).  NLE_E_INVAL for dt <= 0,
 * beta <= 0 or a non-finite gamma. */
nle_status nle_newmark_predict(nle_ctx *ctx, double dt, double beta, double gamma,
                               const double *u_dev, const double *v_dev, const double *a_dev,
                               double *u_tilde_dev, double *v_tilde_dev);
/* Viscous dashpots on the spring faces (the damping terms of the epicardial
 * Robin condition of Sec. 4): traction -(c_perp N (x) N + c_par (I - N (x) N))
 * v with v the velocity, integrated like the springs.  They act only in an
 * implicit step, with inertia on (nle_set_inertia) and the step's velocity
 * set (nle_set_step_velocity): the residual gains M_C (v_tilde + cv (u -
 * u_tilde)), the tangent and its diagonals cv M_C; nle_energy refuses them.
 * Zero coefficients switch them off.  NLE_E_INVAL for negative or
 * non-finite values; P1 meshes only.  Resets linearizations. */
nle_status nle_set_robin_damping(nle_ctx *ctx, double c_perp, double c_par);
/* The implicit step's velocity as an affine function of the unknown u:
 * v(u) = v_tilde + cv (u - u_tilde) (u_tilde from nle_set_inertia).  For
 * Newmark cv = gamma / (beta dt) and v_tilde from nle_newmark_predict.
 * v_tilde_dev (double, device, 3 n_nodes) is copied; cv = 0 switches it off.
 * NLE_E_INVAL for a negative or non-finite cv, or a null v_tilde while on.
 * Resets linearizations. */
nle_status nle_set_step_velocity(nle_ctx *ctx, double cv, const double *v_tilde_dev);
/* Newmark corrector after the step's solve, in place (double, device):
 * a_new = (u - u_tilde) / (beta dt^2), v += dt ((1 - gamma) a + gamma a_new),
 * a = a_new.  Dirichlet dofs are not special-cased: with fixed values there
 * u - u_tilde gives their prescribed motion.  NLE_E_INVAL for a null vector,
 * dt <= 0, beta <= 0 or a non-finite dt, beta or gamma. */
nle_status nle_newmark_correct(nle_ctx *ctx, double dt, double beta, double gamma,
                               const double *u_dev, const double *u_tilde_dev, double *v_dev,
                               double *a_dev);

/* ---- kernels (device vectors of 3 n_nodes entries) ---------------------- */
/* Write the prescribed Dirichlet values into u (double, device). */
nle_status nle_lift(nle_ctx *ctx, double *u_dev);
/* r = f_int(u) - s f_ext with r = 0 on Dirichlet dofs (double, device).
 * If rnorm_host != NULL the stream is synchronised and ||r||_2 stored.
 * Returns NLE_DIVERGED_INVERTED when some element has det F <= 0 (this
 * check synchronises; it is made only when rnorm_host != NULL). */
nle_status nle_residual(nle_ctx *ctx, const double *u_dev, double *r_dev, double *rnorm_host);
/* Fix the linearization point u (double, device): the tangent used by
 * nle_jv is J(u) until the next nle_linearize.  prec = NLE_FP64 prepares the
 * FP64 tangent only; prec = NLE_FP32 prepares the FP64 and the FP32 copies.
 * Each call replaces the previous linearization (both copies). */
nle_status nle_linearize(nle_ctx *ctx, const double *u_dev, int32_t prec);
/* y = J(u_lin) v (Sec. 3, eq. "newton" left-hand side), matrix-free, in
 * precision prec (v and y are double* for NLE_FP64, float* for NLE_FP32).
 * NLE_E_STATE without a linearization in that precision. */
nle_status nle_jv(nle_ctx *ctx, const void *v_dev, void *y_dev, int32_t prec);
/* Allocation-free Jacobian action, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): y = J(u_lin) v exactly as nle_jv (same kernels, same
 * result bit for bit), but the partial sums of nodes shared between element
 * blocks go to a fixed workspace of 64 MiB per device that the library
 * holds from its load until the process ends, instead of to a buffer of the
 * context.  It calls no allocator.  P1 meshes only (NLE_E_UNSUPPORTED on a
 * mixed mesh); NLE_E_STATE without a linearization in prec; NLE_E_INVAL if
 * the mesh's shared-slot partials (3 values of prec per shared block-node
 * slot, nle_partition_info entry 5) exceed 64 MiB.  Every call on a device
 * uses that device's one workspace: calls that overlap in time on one device
 * (several streams or threads) race and give wrong results; serialise them. */
nle_status nle_jv_noalloc(nle_ctx *ctx, const void *v_dev, void *y_dev, int32_t prec);
/* Jacobi data of the current linearization: d = diag J (1 on Dirichlet
 * dofs), double, device. */
nle_status nle_diag(nle_ctx *ctx, double *d_dev);
/* Nodal diagonal blocks of the current linearization (P1 meshes): b[n_nodes]
 * [6] = (K_xx, K_yy, K_zz, K_xy, K_yz, K_xz) of the 3x3 block of node k,
 * double, device.  The blocks are the symmetric parts of the tangent's
 * own-node blocks: the strain energy and the Robin springs give symmetric
 * blocks, a follower pressure only a skew part (which drops out), a follower
 * traction a rank-one part (whose symmetric part enters).  Dirichlet
 * dofs have identity rows and columns.  NLE_E_UNSUPPORTED on a mixed mesh,
 * NLE_E_STATE before nle_linearize. */
nle_status nle_block_diag(nle_ctx *ctx, double *b_dev);
/* y = M^-1 x for the preconditioner pc of the current linearization:
 * NLE_PC_NONE (copy), NLE_PC_JACOBI (y_i = x_i / J_ii), NLE_PC_BJACOBI3
 * (per node, the inverse of its block from nle_block_diag) or NLE_PC_AMG.
 * x and y are device vectors of the unknown length, double for NLE_FP64 and
 * float for NLE_FP32 (which needs a linearization in NLE_FP32); they may
 * not overlap.
 * NLE_PC_AMG: one V(1,1)-
 * cycle of an aggregation multigrid for J.  Candidates: the six rigid-body
 * modes (translations, rotations e_k x X about the origin), zero on
 * Dirichlet dofs.  Each level's graph (level 0: nodes sharing an element,
 * all ten of a quadratic one)
 * is aggregated in two passes over its vertices in order (a vertex whose
 * neighbours are all free forms an aggregate with them; leftovers join the
 * aggregate of their lowest-numbered neighbour aggregated in the first
 * pass); each aggregate's candidate columns are orthonormalised by modified
 * Gram-Schmidt in order (a column is dropped below 1e-8 of its norm) into
 * the prolongator P_l, the projections become the next level's candidates,
 * A_{l+1} = P_l^T A_l P_l; coarsening stops at <= 300 unknowns (solved by a
 * dense inverse) or 10 levels.  Smoothing before and after the coarse
 * correction, with rho_l a 15-step power estimate of the spectral radius of
 * D^-1 A_l from the fixed start vector x_i = frac(i 2654435761 / 2^32) - 1/2:
 * on the finest level the degree-2 Chebyshev smoother on
 * [1.2 rho_0 / 30, 1.2 rho_0], on the coarser levels one Jacobi step of
 * weight 1/rho_l.  The hierarchy's structure is
 * built on first use per mesh and Dirichlet set, its operators once per
 * linearization (synchronising; level 1 by probing with J v), and the
 * cycle runs in precision prec.  NLE_E_UNSUPPORTED if the coarsest level
 * stays above 4000 unknowns, NLE_E_STATE for a zero coarse diagonal or a
 * singular coarsest level.  With a pressure field (mixed meshes) the
 * hierarchy is built for the displacement block (the Jacobian action with
 * zero pressures) and y = (cycle on the displacements, x_p / d_p on the
 * pressures), d_p the pressure entries of nle_diag: the block-diagonal
 * field split. */
nle_status nle_pc_apply(nle_ctx *ctx, int32_t pc, int32_t prec, const void *x_dev, void *y_dev);
/* y = M^-1 x for the lower block-triangular Schur preconditioner `schur`
 * (NLE_SCHUR_LOWER_MASS or NLE_SCHUR_LOWER_SIMPLE, App. B) of the current
 * linearization of a displacement / pressure mesh, with point Jacobi
 * (pc = NLE_PC_JACOBI) or the multigrid cycle (NLE_PC_AMG) on the
 * displacement block: y_u = A^^-1 x_u, y_p = S^^-1 (x_p - B y_u).  Vectors of
 * the unknown length, double (NLE_FP64) or float (NLE_FP32, needs an FP32
 * linearization), not overlapping.  Synchronises (it allocates two work
 * vectors for the call).  NLE_E_UNSUPPORTED without a pressure field, or
 * SIMPLE on the linear-pressure pair; NLE_E_STATE before nle_linearize. */
nle_status nle_schur_apply(nle_ctx *ctx, int32_t pc, int32_t schur, int32_t prec,
                           const void *x_dev, void *y_dev);
/* The SIMPLE diagonal s_e = sum_i B_ei^2 / A_ii (over the element's free
 * displacement dofs) of the constant-pressure pair at the current
 * linearization: s_dev[n_elems] (double, device). */
nle_status nle_simple_diag(nle_ctx *ctx, double *s_dev);
/* Potential Pi(u) = sum_e V_e Psi(F_e) - s f_ext . u + u.R u / 2 with R
 * the spring matrix (synchronises).  NLE_E_UNSUPPORTED with a follower
 * pressure set. */
nle_status nle_energy(nle_ctx *ctx, const double *u_dev, double *pi_host);

/* ---- solvers ------------------------------------------------------------- */
/* Tolerances, iteration limits and Eisenstat-Walker constants of App. A for the
 * method (NK, iNK or BFGS).  The Krylov choice is not App. A's: ksp_type is
 * CG with point Jacobi and orth CGS2, where App. A runs GMRES with modified
 * Gram-Schmidt; set ksp_type = NLE_KSP_GMRES and orth = NLE_ORTH_MGS for
 * that configuration. */
void nle_default_opts(int32_t method, nle_solver_opts *opts);
/* Solve r(u) = 0 at the current load scale, starting from u (double,
 * device, overwritten with the result).  If u does not hold the prescribed
 * Dirichlet values (a new load step of a displacement-driven problem), the
 * change w = g - u is first carried into the interior: u += w + d with
 * K_ff d = -(r(u) + K w)_f at the current u, solved by the configured Krylov
 * method to ksp_rtol / ksp_atol (BFGS: only with h0 = KSP); then the values
 * are lifted.
 * Convergence: ||r_k||_2 <= max(snes_rtol ||r_0||_2, snes_atol) with r_0
 * the residual after the lift, or the imbalance ||(r(u) + K w)_f|| of the
 * step above when that is larger.  `report` may be NULL. */
nle_status nle_solve_nk(nle_ctx *ctx, double *u_dev, const nle_solver_opts *opts, nle_report *report);
nle_status nle_solve_ink(nle_ctx *ctx, double *u_dev, const nle_solver_opts *opts, nle_report *report);
nle_status nle_solve_bfgs(nle_ctx *ctx, double *u_dev, const nle_solver_opts *opts, nle_report *report);

/* ---- batched solves ---------------------------------------------------------
 * Many independent problems (uneven meshes, material parameters, loads and
 * load schedules; the sweeps over size and data magnitude of Sec. 6) solved
 * together: every launch covers all instances, every decision (convergence,
 * Krylov tolerance, step, load-step cutback) is per instance.  Instances of a
 * batch share the material law (kind), not its parameters. */
typedef struct nle_batch nle_batch;
nle_status nle_batch_create(nle_batch **out, int32_t device, void *hip_stream,
                            const nle_allocator *alloc);
void nle_batch_destroy(nle_batch *b);
const char *nle_batch_last_error(const nle_batch *b);
/* Add one instance (host arrays, copied): P1 mesh (as nle_upload_mesh),
 * material (as nle_set_material), Dirichlet dofs / values (instance-local
 * dof numbers), dead traction t on n_faces triangles, and the load scales of
 * its schedule (positive, strictly increasing; solved in order, warm-started).
 * *id receives its index.  NLE_E_INVAL / NLE_E_BADMESH on bad arrays,
 * NLE_E_STATE once the batch is finalized. */
nle_status nle_batch_add(nle_batch *b, int64_t n_nodes, const double *X, int64_t n_elems,
                         const int32_t *conn, int32_t mat_kind, const double *params,
                         int32_t n_params, int64_t n_dir, const int64_t *dofs,
                         const double *values, int64_t n_faces, const int32_t *tri,
                         const double *traction, int32_t n_scales, const double *scales,
                         int32_t *id);
/* Upload the disjoint union of all instances (partition, geometry). */
nle_status nle_batch_finalize(nle_batch *b);
/* Choose the element-block size of the batch's partition for speed: each
 * candidate (128, 256, 512 and 1024 elements per block, those whose LDS need
 * fits the device) re-partitions the union mesh, and the Jacobian action of
 * the whole batch in precision prec (NLE_FP32 for mixed solves) at the lifted
 * zero state is timed with HIP events, within about budget_ms in total.  The
 * fastest partition is kept (the batch stays finalized; the node layout does
 * not change) and *block_size (nullable) receives its size.  NLE_E_STATE
 * before nle_batch_finalize, NLE_E_INVAL on a bad precision or budget. */
nle_status nle_batch_autotune(nle_batch *b, int32_t prec, double budget_ms, int32_t *block_size);
/* node_offsets[n_inst + 1]: instance i owns nodes [off[i], off[i+1]) of the
 * concatenated vector (dof = 3 * node + component). */
nle_status nle_batch_layout(const nle_batch *b, int64_t *node_offsets);
/* Solve every instance over its schedule with NK, iNK (CG + point Jacobi
 * inner solves) or L-BFGS (Sec. 3: inexact BFGS with H0 a CG + Jacobi solve,
 * or BFGS-preonly with pc NLE_PC_JACOBI or NLE_PC_NONE as H0; qn_m 1..64),
 * starting from u (device, concatenated, overwritten).  A load step that
 * diverges is retried from the last converged state with half the increment
 * (at most 8 times per instance).  reports[n_inst] (nullable) receive
 * per-instance outcomes: iterations, histories, bfgs_skipped (pairs rejected
 * by the curvature test) and cutbacks (halved increments); *t_ms the wall
 * time of the whole batch on the stream.  Returns NLE_OK when every instance
 * finished its schedule, else the last failing status.  NLE_E_UNSUPPORTED
 * for another Krylov method or preconditioner, NLE_E_INVAL for a bad method,
 * precision, BFGS memory or iteration limit, NLE_E_STATE before
 * nle_batch_finalize. */
nle_status nle_batch_solve(nle_batch *b, int32_t method, const nle_solver_opts *opts, double *u_dev,
                           nle_report *reports, double *t_ms);
/* Instances that leave the batch rounds (the sweeps of Sec. 6 mix easy and
 * stiff instances, and a round's batched CG lasts as long as its stiffest
 * solve).  An instance leaves when at most max_tail instances are unfinished,
 * or (NK and iNK) when its batched CG solve of a round takes more than max_its
 * iterations; nle_batch_solve then finishes it alone, at once, with the
 * single-problem solver (a context of its own on the batch's device, stream
 * and allocator, the batch's method and options with preconditioner pc, e.g.
 * NLE_PC_AMG), from its last converged state over the rest of its schedule, a
 * failed increment halved as in the batch rounds within the same budget of
 * cutbacks.  Its report then counts the iterations of both parts.  Zero (the
 * default) turns either rule off.  NLE_E_INVAL for a negative count or an
 * unknown pc; errors of the single-problem calls are returned by
 * nle_batch_solve with their message. */
nle_status nle_batch_set_tail(nle_batch *b, int32_t max_tail, int32_t max_its, int32_t pc);

/* Unknowns per level of the multigrid hierarchy built by the last NLE_PC_AMG
 * use (finest first): *n_levels = number of levels (0 if none is built),
 * sizes[0 .. min(n_levels, cap)) filled (host arrays).  NLE_E_INVAL for a
 * null ctx or n_levels, a negative cap, or a null sizes with cap > 0. */
nle_status nle_amg_levels(const nle_ctx *ctx, int32_t *n_levels, int64_t *sizes, int32_t cap);

/* ---- mesh partition inspection (for tests and tuning) --------------------- */
/* info[0..7] = n_blocks, max elems per block, max nodes per block,
 * block-node slots, shared nodes, merge slots, LDS bytes (FP64 Jv),
 * LDS bytes (FP32 Jv). */
nle_status nle_partition_info(const nle_ctx *ctx, int64_t *info);

#ifdef __cplusplus
}
#endif
#endif /* NLELAST_H */
