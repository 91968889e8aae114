"""Set up the workloads on a library context (marshalling only).

Cook test (Sec. 4): clamp on x = 0, dead shear traction (0, tau, 0) per unit
reference area on x = 48, compressible neo-Hookean (M1) or the paper's split
law (M2).  The mesh object needs X, conn, faces['load'] and a
dirichlet_dofs('clamp') method (the synthetic generator's Mesh).
"""

from __future__ import annotations

import numpy as np

from . import nlelast as nl


def setup_cook(ctx: nl.Context, mesh, mu: float, lam: float, tau: float = 1.0,
               material: int = nl.NLE_MAT_M1, c_vol=None, block_size=None,
               follower: bool = False) -> None:
    """Cook's membrane (Sec. 4): clamp x = 0, shear traction (0, tau, 0) on
    x = 48, per unit reference area (dead) or, with follower=True, per unit
    current area with fixed direction."""
    if block_size is not None:
        nl.nle_set_block_size(ctx, block_size)
    nl.nle_upload_mesh(ctx, mesh.X, mesh.conn)
    params = [mu, lam] if material == nl.NLE_MAT_M1 or c_vol is None else [mu, lam, c_vol]
    nl.nle_set_material(ctx, material, params)
    dofs = mesh.dirichlet_dofs("clamp")
    nl.nle_set_dirichlet(ctx, dofs, np.zeros(dofs.size))
    if follower:
        nl.nle_set_traction_follower(ctx, mesh.faces["load"], [0.0, tau, 0.0])
    else:
        nl.nle_set_traction(ctx, mesh.faces["load"], [0.0, tau, 0.0])
    nl.nle_set_load_scale(ctx, 1.0)


SOLVERS = {"nk": nl.nle_solve_nk, "ink": nl.nle_solve_ink, "bfgs": nl.nle_solve_bfgs}
METHOD_IDS = {"nk": nl.NLE_NK, "ink": nl.NLE_INK, "bfgs": nl.NLE_BFGS}


def make_opts(method: str, precision: str = "fp64", **over) -> nl.nle_solver_opts:
    """Options of App. A for `method` ('nk', 'ink', 'bfgs'), plus overrides.

    For 'bfgs', h0='preonly' (BFGS-preonly) or 'ksp' (inexact BFGS).
    """
    o = nl.nle_default_opts(METHOD_IDS[method])
    o.precision = nl.NLE_PREC_MIXED if precision == "mixed" else nl.NLE_PREC_FP64
    h0 = over.pop("h0", None)
    if h0 is not None:
        o.h0 = nl.NLE_H0_KSP if h0 == "ksp" else nl.NLE_H0_PREONLY
    ksp = over.pop("ksp", None)
    if ksp is not None:
        o.ksp_type = {"cg": nl.NLE_KSP_CG, "gmres": nl.NLE_KSP_GMRES,
                      "minres": nl.NLE_KSP_MINRES}[ksp]
    pc = over.pop("pc", None)
    if pc is not None:
        o.pc = {"none": nl.NLE_PC_NONE, "jacobi": nl.NLE_PC_JACOBI,
                "bjacobi3": nl.NLE_PC_BJACOBI3, "amg": nl.NLE_PC_AMG}[pc]
    orth = over.pop("orth", None)
    if orth is not None:
        o.orth = nl.NLE_ORTH_MGS if orth == "mgs" else nl.NLE_ORTH_CGS2
    for k, v in over.items():
        setattr(o, k, v)
    return o


def solve_schedule(ctx: nl.Context, u, method: str, opts, scales, hist_cap: int = 4096,
                   max_cuts: int = 8, start_scale: float = 0.0, progress=None):
    """Solve at each load scale in turn, warm-started from the previous step.

    If a step does not converge (an element inverts, NaN, or the iteration
    limit), the state is restored to the last converged step and the load
    increment is halved (at most `max_cuts` times in total); the failed
    attempts stay in the returned reports (their time is part of the solve).
    Each report carries 'load_scale' and 'accepted'; `progress` (optional) is
    called with each report as it arrives.
    """
    reps = []
    targets = [float(x) for x in scales]
    backup = u.clone()
    s_prev = float(start_scale)
    cuts = 0
    i = 0
    while i < len(targets):
        s = targets[i]
        nl.nle_set_load_scale(ctx, s)
        st, rep = SOLVERS[method](ctx, u, opts, hist_cap)
        rep["load_scale"] = s
        rep["accepted"] = st == nl.NLE_OK
        reps.append(rep)
        if progress is not None:
            progress(rep)
        if st == nl.NLE_OK:
            backup.copy_(u)
            s_prev = s
            i += 1
            continue
        u.copy_(backup)
        if cuts >= max_cuts:
            break
        cuts += 1
        targets.insert(i, 0.5 * (s_prev + s))
    return reps


def schedule_ok(reps, scales) -> bool:
    acc = [r["load_scale"] for r in reps if r["accepted"]]
    return bool(acc) and abs(acc[-1] - float(scales[-1])) == 0.0


def add_cook_instance(batch: nl.Batch, mesh, mu: float, lam: float, tau: float, scales,
                      material: int = nl.NLE_MAT_M1) -> int:
    """One Cook's-membrane instance: traction (0, tau, 0) times each load scale."""
    dofs = mesh.dirichlet_dofs("clamp")
    return nl.nle_batch_add(batch, mesh.X, mesh.conn, material, [mu, lam], dofs,
                            np.zeros(dofs.size), mesh.faces["load"], [0.0, tau, 0.0], scales)


def setup_cardiac(ctx: nl.Context, mesh, consts: dict, dofs, block_size=None) -> None:
    """Cardiac-like shell (Sec. 4, "Heartbeat test", quasi-static): law M4 with
    the mesh's per-element fibres, follower pressure consts['p_max'] on the
    'endo' faces (times the load scale), springs on the 'epi' faces, the given
    constrained dofs held at zero.  Load scale and active tension start at 0."""
    c = consts
    if block_size is not None:
        nl.nle_set_block_size(ctx, block_size)
    nl.nle_upload_mesh(ctx, mesh.X, mesh.conn)
    nl.nle_set_material(ctx, nl.NLE_MAT_M4, [c["a"], c["b"], c["af"], c["bf"], c["kappa"]])
    nl.nle_set_fibres(ctx, mesh.elem_fibre)
    dofs = np.asarray(dofs, dtype=np.int64)
    nl.nle_set_dirichlet(ctx, dofs, np.zeros(dofs.size))
    nl.nle_set_pressure(ctx, mesh.faces["endo"], c["p_max"])
    nl.nle_set_robin(ctx, mesh.faces["epi"], c["k_perp"], c["k_par"])
    nl.nle_set_load_scale(ctx, 0.0)
    nl.nle_set_active_tension(ctx, 0.0)


def setup_guccione(ctx: nl.Context, mesh, consts: dict, law, dofs, block_size=None) -> None:
    """The heartbeat with the paper's Guccione law (Sec. 4; law M6, law =
    (C, b_ff, b_ss, b_nn, b_fs, b_fn, b_sn, B)), the mesh's fibre and sheet
    directions, and the loads and constraints of setup_cardiac."""
    setup_cardiac(ctx, mesh, consts, dofs, block_size=block_size)
    nl.nle_set_material(ctx, nl.NLE_MAT_M6, list(law))
    nl.nle_set_fibre_frame(ctx, mesh.elem_fibre, mesh.elem_sheet)


def setup_shell_p2(ctx: nl.Context, mesh2, consts: dict, law=None, loads: bool = False) -> None:
    """The ventricle shell with quadratic (10-node) displacement elements:
    law M4 with the consts' constants and the mesh's fibres, or with law =
    (C, b_ff, b_ss, b_nn, b_fs, b_fn, b_sn, B) Guccione's law M6 with fibres
    and sheets; base plane held in z (vertices and edge midpoints) plus three
    pins.  loads: the heartbeat's follower pressure consts['p_max'] on the
    'endo' faces and springs on the 'epi' faces (6-node faces).  Load scale
    1, active tension 0."""
    from synthetic import shell_dirichlet

    c = consts
    nl.nle_upload_mesh(ctx, mesh2.X, mesh2.conn)
    if law is None:
        nl.nle_set_material(ctx, nl.NLE_MAT_M4, [c["a"], c["b"], c["af"], c["bf"], c["kappa"]])
        nl.nle_set_fibres(ctx, mesh2.elem_fibre)
    else:
        nl.nle_set_material(ctx, nl.NLE_MAT_M6, list(law))
        nl.nle_set_fibre_frame(ctx, mesh2.elem_fibre, mesh2.elem_sheet)
    dofs = shell_dirichlet(mesh2)
    nl.nle_set_dirichlet(ctx, dofs, np.zeros(dofs.size))
    if loads:
        nl.nle_set_pressure(ctx, mesh2.faces["endo"], c["p_max"])
        nl.nle_set_robin(ctx, mesh2.faces["epi"], c["k_perp"], c["k_par"])
    nl.nle_set_load_scale(ctx, 1.0)
    nl.nle_set_active_tension(ctx, 0.0)


def solve_heartbeat(ctx: nl.Context, u, method: str, opts, schedule, gamma_max: float,
                    hist_cap: int = 4096, max_cuts: int = 8, start=(0.0, 0.0)):
    """Quasi-static heartbeat: for each time step (t, shape) set the active
    tension gamma_max * shape and the pressure load scale shape, then solve,
    warm-started.  A step that fails is retried from the last converged state
    at the midpoint (in t and shape) of the failed increment (at most
    `max_cuts` times in total); `start` is the (t, shape) that u solves.
    Reports carry 't', 'shape' and 'accepted'."""
    reps = []
    targets = [(float(t), float(sh)) for t, sh in schedule]
    backup = u.clone()
    prev = (float(start[0]), float(start[1]))
    cuts = 0
    i = 0
    while i < len(targets):
        t, sh = targets[i]
        nl.nle_set_active_tension(ctx, gamma_max * sh)
        nl.nle_set_load_scale(ctx, sh)
        st, rep = SOLVERS[method](ctx, u, opts, hist_cap)
        rep.update(t=t, shape=sh, accepted=st == nl.NLE_OK)
        reps.append(rep)
        if st == nl.NLE_OK:
            backup.copy_(u)
            prev = (t, sh)
            i += 1
            continue
        u.copy_(backup)
        if cuts >= max_cuts:
            break
        cuts += 1
        targets.insert(i, (0.5 * (prev[0] + t), 0.5 * (prev[1] + sh)))
    return reps


def solve_heartbeat_dynamic(ctx: nl.Context, u, method: str, opts, schedule, gamma_max: float,
                            rho: float, dt: float, beta: float = 0.25, gamma: float = 0.5,
                            v=None, a=None, hist_cap: int = 4096):
    """Heartbeat with inertia: each time step (t, shape) predicts u~ and v~
    with Newmark's rule, sets the inertia c M (u - u~) with c = 1 / (beta
    dt^2) and density rho and the step velocity v~ + gamma / (beta dt)
    (u - u~) (which dashpots set with nle_set_robin_damping act on), the
    active tension gamma_max * shape and the pressure load scale shape,
    solves the implicit step warm-started from u, then corrects v and a in
    place (both start at zero unless given).  Stops at the first step that
    fails (a smaller step would change c).  The inertia and the step
    velocity are switched off on return.  Returns (reports, v, a)."""
    torch = ctx.torch
    v = torch.zeros_like(u) if v is None else v
    a = torch.zeros_like(u) if a is None else a
    ut = torch.empty_like(u)
    vt = torch.empty_like(u)
    c = 1.0 / (beta * dt * dt)
    reps = []
    try:
        for t, sh in schedule:
            nl.nle_newmark_predict(ctx, dt, beta, u, v, a, ut, gamma=gamma, v_tilde=vt)
            nl.nle_set_inertia(ctx, rho, c, ut)
            nl.nle_set_step_velocity(ctx, gamma / (beta * dt), vt)
            nl.nle_set_active_tension(ctx, gamma_max * sh)
            nl.nle_set_load_scale(ctx, sh)
            st, rep = SOLVERS[method](ctx, u, opts, hist_cap)
            rep.update(t=float(t), shape=float(sh), accepted=st == nl.NLE_OK)
            reps.append(rep)
            if st != nl.NLE_OK:
                break
            nl.nle_newmark_correct(ctx, dt, beta, gamma, u, ut, v, a)
    finally:
        nl.nle_set_inertia(ctx, 0.0, 0.0, None)
        nl.nle_set_step_velocity(ctx, 0.0, None)
    return reps, v, a


def heartbeat_ok(reps, schedule) -> bool:
    acc = [r["t"] for r in reps if r["accepted"]]
    return bool(acc) and acc[-1] == float(schedule[-1][0])


def setup_twist(ctx: nl.Context, mesh, mu: float, theta: float = 0.0) -> None:
    """Twist test (Sec. 4): quadratic displacement / linear pressure mesh, law
    M3, bottom clamped, top x/y rotated by theta about x = y = 1/2.  The
    Dirichlet data come from synthetic.twist_dirichlet via set_twist_angle."""
    nl.nle_upload_mesh_mixed(ctx, mesh.X, mesh.conn, mesh.n_pressure, mesh.pconn)
    nl.nle_set_material(ctx, nl.NLE_MAT_M3, [mu])
    nl.nle_set_load_scale(ctx, 1.0)


TWIST_M5 = (9000.0, 9000.0, 9000.0, 9000.0)  # alpha_p, beta_p, alpha_s, beta_s (Sec. 4)


def setup_twist_p0(ctx: nl.Context, mesh, params=TWIST_M5) -> None:
    """The paper's twist statement (Sec. 4): quadratic displacement with one
    pressure per element (P2-P0) and the polyconvex law M5 (default: the
    printed constants, all 9000).  Dirichlet data as for setup_twist."""
    nl.nle_upload_mesh_mixed_p0(ctx, mesh.X, mesh.conn)
    nl.nle_set_material(ctx, nl.NLE_MAT_M5, list(params))
    nl.nle_set_load_scale(ctx, 1.0)


def solve_twist(ctx: nl.Context, x, method: str, opts, angles, dirichlet, hist_cap: int = 4096,
                max_cuts: int = 8, start: float = 0.0, progress=None):
    """Rotate the top face through the given angles in turn (warm-started).
    dirichlet(theta) -> (dofs, values).  A failed step is retried from the last
    converged state at the mid angle (at most max_cuts times in total).
    Reports carry 'theta' and 'accepted'; progress(rep) is called after each
    attempt."""
    reps = []
    targets = [float(a) for a in angles]
    backup = x.clone()
    prev = float(start)
    cuts = 0
    i = 0
    while i < len(targets):
        th = targets[i]
        dofs, vals = dirichlet(th)
        nl.nle_set_dirichlet(ctx, dofs, vals)
        st, rep = SOLVERS[method](ctx, x, opts, hist_cap)
        rep.update(theta=th, accepted=st == nl.NLE_OK)
        reps.append(rep)
        if progress is not None:
            progress(rep)
        if st == nl.NLE_OK:
            backup.copy_(x)
            prev = th
            i += 1
            continue
        x.copy_(backup)
        if cuts >= max_cuts:
            break
        cuts += 1
        targets.insert(i, 0.5 * (prev + th))
    return reps


def twist_ok(reps, angles) -> bool:
    acc = [r["theta"] for r in reps if r["accepted"]]
    return bool(acc) and acc[-1] == float(angles[-1])


def setup_cook_p2(ctx: nl.Context, mesh2, mu: float, lam: float, tau: float = 1.0) -> None:
    """Cook's membrane with quadratic (10-node) displacement tetrahedra, law
    M1, clamped on x = 0 (vertices and edge midpoints), dead shear traction
    (0, tau, 0) on x = 48 (consistent P2 loads)."""
    nl.nle_upload_mesh(ctx, mesh2.X, mesh2.conn)
    nl.nle_set_material(ctx, nl.NLE_MAT_M1, [mu, lam])
    dofs = mesh2.dirichlet_dofs("clamp")
    nl.nle_set_dirichlet(ctx, dofs, np.zeros(dofs.size))
    nl.nle_set_traction(ctx, mesh2.faces["load"], [0.0, tau, 0.0])
    nl.nle_set_load_scale(ctx, 1.0)
