#!/usr/bin/env python
"""Benchmark: time-to-solve on the 64x64x4 Cook's membrane, and the Jacobian
action's HBM roofline on the 256x256x16 Cook mesh (6.29M tetrahedra).

One step = one full solve of the Cook workload over its load schedule with the
chosen method (mesh upload, partition and material setup are done once,
outside the timed region; every load step's linearizations are inside).
Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--method ink_mixed_cg3_amg]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MU = 80.194
RATIO = 5000.0
GRID = (64, 64, 4)
# elements per block of the timed mesh: 98,304 tets in 256 blocks of 384, one
# per compute unit (512 leaves 192 blocks, fewer than the chip's 256 CUs)
HEAD_BLOCK = 384
XL_GRID = (256, 256, 16)
HBM_PEAK_GBS = 8000.0
JV_KERNEL = "nle_jv FP32 (k_elem_block<float,JV> + k_elem_merge<float,JV>)"

# method name -> (solver, precision, option overrides)
# NK keeps the Krylov tolerance of App. A (1e-6): at large load the tangent
# turns indefinite and CG breaks down, so NK uses MINRES; the inexact methods
# stop CG early and use it (MINRES steps truncated at 1e-1 are poor Newton
# directions on this problem).
METHODS = {
    "nk_fp64": ("nk", "fp64", {"ksp": "minres"}),
    "nk_mixed": ("nk", "mixed", {"ksp": "minres"}),
    "nk_fp64_cg": ("nk", "fp64", {"ksp": "cg"}),
    "ink_fp64": ("ink", "fp64", {"ksp": "cg"}),
    "ink_mixed": ("ink", "mixed", {"ksp": "cg"}),
    "ink_mixed_minres": ("ink", "mixed", {"ksp": "minres"}),
    "bfgs_ib_fp64": ("bfgs", "fp64", {"h0": "ksp", "qn_m": 10, "ksp": "cg"}),
    "bfgs_ib_mixed": ("bfgs", "mixed", {"h0": "ksp", "qn_m": 10, "ksp": "cg"}),
    "bfgs_b_mixed": ("bfgs", "mixed", {"h0": "preonly", "qn_m": 10}),
    # BFGS with the Jacobian reassembled every 20 iterations (an extension the
    # paper's conclusions name); MINRES for the H0 solves, since the tangent
    # turns indefinite at large load
    "bfgs_ib_mixed_r20": ("bfgs", "mixed", {"h0": "ksp", "qn_m": 10, "ksp": "minres",
                                            "h0_refresh": 20}),
    "bfgs_ib_mixed_minres": ("bfgs", "mixed", {"h0": "ksp", "qn_m": 10, "ksp": "minres"}),
    # aggregation multigrid (one V-cycle) with GMRES, and BFGS-preonly with
    # the cycle as H0 (the paper's B method)
    "nk_fp64_amg": ("nk", "fp64", {"ksp": "gmres", "pc": "amg"}),
    "ink_mixed_amg": ("ink", "mixed", {"ksp": "gmres", "pc": "amg"}),
    "ink_fp64_amg": ("ink", "fp64", {"ksp": "gmres", "pc": "amg"}),
    "bfgs_b_mixed_amg": ("bfgs", "mixed", {"h0": "preonly", "qn_m": 10, "ksp": "gmres",
                                           "pc": "amg"}),
    "bfgs_ib_mixed_amg": ("bfgs", "mixed", {"h0": "ksp", "qn_m": 10, "ksp": "gmres",
                                            "pc": "amg", "h0_refresh": 20}),
    # the cycle is symmetric for the symmetric dead-load tangent: CG with it
    "ink_mixed_cg_amg": ("ink", "mixed", {"ksp": "cg", "pc": "amg"}),
    # the same iterates with the next direction formed inside the Jacobian
    # action (3 launches per CG iteration besides the cycle)
    "ink_mixed_cg3_amg": ("ink", "mixed", {"ksp": "cg", "pc": "amg", "cg_launches": 3}),
    "ink_fp64_cg_amg": ("ink", "fp64", {"ksp": "cg", "pc": "amg"}),
    # plain FP64 Newton-Krylov with the same multigrid (the like-for-like
    # baseline: App. A tolerances rtol 1e-6 / atol 1e-10)
    "nk_fp64_cg_amg": ("nk", "fp64", {"ksp": "cg", "pc": "amg"}),
    "nk_fp64_gmres30_amg": ("nk", "fp64", {"ksp": "gmres", "restart": 30, "orth": "cgs2",
                                           "pc": "amg"}),
    "nk_fp64_minres_amg": ("nk", "fp64", {"ksp": "minres", "pc": "amg"}),
    "ink_mixed_minres_amg": ("ink", "mixed", {"ksp": "minres", "pc": "amg"}),
    "bfgs_ib_mixed_cg_amg": ("bfgs", "mixed", {"h0": "ksp", "qn_m": 10, "ksp": "cg",
                                               "pc": "amg", "h0_refresh": 20}),
}


def root_error(uh):
    """|u - u*| / |u*| against the oracle's root of the timed schedule, stored
    by tests/golden/make_golden.py (None if that file is absent)."""
    import numpy as np

    path = os.path.join(ROOT, "tests", "golden", "cook64x64x4_l5000_tau16.npy")
    if not os.path.exists(path):
        return None
    ustar = np.load(path)
    if ustar.shape != uh.shape:
        return None
    return float(np.linalg.norm(uh - ustar) / np.linalg.norm(ustar))


def load_schedule():
    from synthetic import fields

    return fields.cook_load_schedule(16.0)


PC = {"pc": "jacobi"}  # preconditioner of every Cook solve (--pc)


def run_solve(ctx, u, method, schedule):
    from paper_2203_05610_amd import problems

    solver, prec, kw = METHODS[method]
    opts = problems.make_opts(solver, prec, **{"pc": PC["pc"], **kw})
    u.zero_()

    def progress(rep):
        print(f"[bench]   {method} tau={rep['load_scale']:g}: {rep['status_name']} "
              f"nit={rep['nit']} lit={rep['lit_total']}", file=sys.stderr, flush=True)

    reps = problems.solve_schedule(ctx, u, solver, opts, schedule, progress=progress)
    return problems.schedule_ok(reps, schedule), reps


def summarize(reps):
    from paper_2203_05610_amd import problems

    return {
        "ok": problems.schedule_ok(reps, load_schedule()),
        "steps": [f"{r['load_scale']:g}:{r['status_name']}" for r in reps],
        "nit": [r["nit"] for r in reps],
        "lit": [int(r["lit_total"]) for r in reps],
        "n_jv": int(sum(r["n_jv"] for r in reps)),
        "t_ms": [round(r["t_ms"], 2) for r in reps],
    }


def jv_roofline(nl, torch, reps: int):
    """FP32 and FP64 Jacobian action on the 6.29M-tet Cook mesh; HIP events
    around `reps` back-to-back calls on the context's stream."""
    import numpy as np

    import synthetic as syn

    mesh = syn.cook_mesh(*XL_GRID, with_faces=False)
    ctx = nl.Context(0)
    nl.nle_upload_mesh(ctx, mesh.X, mesh.conn)
    nl.nle_set_material(ctx, nl.NLE_MAT_M1, [MU, RATIO * MU])
    d = mesh.dirichlet_dofs("clamp")
    nl.nle_set_dirichlet(ctx, d, np.zeros(d.size))
    n = 3 * mesh.n_nodes
    g = torch.Generator(device="cuda").manual_seed(1234)
    u = (torch.tensor(mesh.X, device="cuda") * 1e-3).reshape(-1).contiguous()
    nl.nle_linearize(ctx, u, nl.NLE_FP32)
    out = {}
    n_slots = nl.nle_partition_info(ctx)["block_node_slots"]
    for prec, dt, s in ((nl.NLE_FP32, torch.float32, 4), (nl.NLE_FP64, torch.float64, 8)):
        v = torch.randn(n, dtype=dt, device="cuda", generator=g)
        y = torch.empty_like(v)
        for _ in range(10):
            nl.nle_jv(ctx, v, y, prec)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        ctx.stream.synchronize()
        e0.record(ctx.stream)
        for _ in range(reps):
            nl.nle_jv(ctx, v, y, prec)
        e1.record(ctx.stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        # algorithmic bytes of one Jacobian action (recompute design, each
        # array of the method read or written once): per element 4 node
        # indices (16 B) and 10 scalars (grad N: 9, V: 1); per node u and v
        # read and y written (3 scalars each)
        balg = mesh.n_elems * (16 + 10 * s) + mesh.n_nodes * 3 * 3 * s
        # this library's own layout: per element a 16-byte index record and
        # the one cached tangent coefficient of law M1; per block-node slot its
        # 3 relative coordinates (grad N and V are formed from them); per node
        # u, v, y
        blay = mesh.n_elems * (16 + s) + n_slots * 3 * s + mesh.n_nodes * 9 * s
        out["fp32" if s == 4 else "fp64"] = {
            "ms": ms, "bytes": balg, "gbs": balg / ms / 1e6,
            "layout_bytes": blay, "layout_gbs": blay / ms / 1e6,
            "n_elems": mesh.n_elems, "n_nodes": mesh.n_nodes, "n_slots": n_slots,
        }
    out["partition"] = nl.nle_partition_info(ctx)
    ctx.close()
    return out


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("nle_elem.hip", "nle_kin.hpp", "nle_laws.hpp"):
        with open(os.path.join(ROOT, "paper_2203_05610_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(ms_bytes):
    """HBM bytes per Jv from the committed rocprofv3 counter summary, if it was
    taken on the current element-kernel source; otherwise None."""
    path = os.path.join(ROOT, "profiles", "jv_cookxl_fp32_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return t.get("hbm_bytes_per_jv")


CPU_SNIPPET = r"""
import os, sys, time, json
sys.path.insert(0, {root!r})
import numpy as np
import synthetic as syn
from oracle import fem, newton
m = syn.cook_mesh({nx}, {ny}, {nz})
P = fem.cook_problem(m, mu={mu}, lam={lam}, tau=1.0)
t0 = time.perf_counter()
u, hist = newton.newton_exact(P, np.zeros(P.n_dofs), {scale}, rtol=1e-8)
dt = time.perf_counter() - t0
print(json.dumps(dict(seconds=dt, iterations=len(hist) - 1)))
"""


def _host_cpu():
    """CPU model name and logical core count of the host (from lscpu)."""
    model, cpus = None, os.cpu_count()
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() == "Model name":
                model = v.strip()
            elif k.strip() == "CPU(s)":
                cpus = int(v.strip())
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    return model, cpus


def cpu_baseline(n_load_steps: int):
    """The oracle's exact Newton (assembled complex-step tangent + sparse LU,
    one thread) on the same 64x64x4 mesh, timed on a bounded sample: the first
    load step (tau = 1, from u = 0, to ||r|| <= 1e-8 ||r_0||).  The seconds
    per Newton iteration are scaled by the number of Newton iterations the
    oracle takes over the whole schedule (every attempt, the failed one
    included), which tests/golden/make_golden.py recorded when it wrote the
    stored root; without that record, by the number of load steps."""
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    code = CPU_SNIPPET.format(root=ROOT, nx=GRID[0], ny=GRID[1], nz=GRID[2], mu=MU,
                              lam=RATIO * MU, scale=1.0)
    try:
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                           timeout=300)
    except subprocess.TimeoutExpired:
        return {"error": "oracle sample exceeded 300 s"}
    if r.returncode != 0:
        return {"error": r.stderr[-400:]}
    d = json.loads(r.stdout.strip().splitlines()[-1])
    per_it = d["seconds"] / max(d["iterations"], 1)
    model, cpus = _host_cpu()
    meta_path = os.path.join(ROOT, "tests", "golden", "cook64x64x4_l5000_tau16.json")
    total_its = None
    if os.path.exists(meta_path):
        with open(meta_path) as fh:
            total_its = json.load(fh).get("newton_iterations")
    if total_its:
        value = per_it * total_its
        how = (f"{d['iterations']} Newton iterations of the first load step (tau=1) in "
               f"{d['seconds']:.1f} s = {per_it:.2f} s per iteration, times the {total_its} "
               f"iterations the oracle takes over the schedule 1,2,4,8,16 with its cutback")
    else:
        value = d["seconds"] * n_load_steps
        how = (f"one load step (tau=1): {d['iterations']} iterations in {d['seconds']:.1f} s, "
               f"times the {n_load_steps} load steps")
    return {
        "value": round(value, 2),
        "unit": "s",
        "cores": 1,
        "kind": "oracle",
        "sample": how + " (exact Newton, complex-step tangent, SuperLU, 1 thread, 64x64x4 mesh)",
        "host_cpu": model,
        "host_logical_cpus": cpus,
    }


def batch_c4(nl, torch, count: int, serial_stride: int, steps: int, autotune: bool = True,
             tail: int = 0, tail_its: int = 0):
    """Batched solves: `count` sampled Cook instances (uneven size, lambda/mu and
    traction; doubling load schedules ending at each tau) solved in one batch
    with mixed iNK, against serial FP64 NK solves of every `serial_stride`-th
    instance on the same GPU (the serial time is that sample times the stride).
    tail > 0: the last `tail` unfinished instances, and tail_its > 0: any
    instance whose batched CG solve takes more than tail_its iterations, are
    finished alone with CG and the multigrid."""
    import numpy as np

    import synthetic as syn
    from paper_2203_05610_amd import problems

    recipe = syn.batch_recipe(count)
    t = time.perf_counter()
    B = nl.Batch(0)
    meshes, n_elems = [], 0
    for r in recipe:
        m = syn.cook_mesh(r["nx"], r["ny"], r["nz"])
        problems.add_cook_instance(B, m, r["mu"], r["lam"], 1.0, syn.cook_load_schedule(r["tau"]))
        meshes.append(m)
        n_elems += m.conn.shape[0]
    nl.nle_batch_finalize(B)
    off = nl.nle_batch_layout(B)
    block_size = nl.nle_batch_autotune(B, nl.NLE_FP32, budget_ms=400.0) if autotune else 512
    nl.nle_batch_set_tail(B, tail, tail_its, nl.NLE_PC_AMG)
    u = torch.zeros(int(3 * off[-1]), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t
    print(f"[bench] batch of {count}: {n_elems} tets, {int(off[-1])} nodes, setup {t_setup:.1f}s, "
          f"{block_size} elements per block", file=sys.stderr, flush=True)
    opts = problems.make_opts("ink", "mixed", ksp="cg")
    times, oks = [], []
    for k in range(steps):
        u.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        st, reps, _ = nl.nle_batch_solve(B, nl.NLE_INK, opts, u)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
        oks.append(sum(r["status"] == nl.NLE_OK for r in reps))
        print(f"[bench] batch solve {k}: {times[-1]:.2f}s, {oks[-1]}/{count} solved, "
              f"max nit {max(r['nit'] for r in reps)}, max lit {max(r['lit_total'] for r in reps)}",
              file=sys.stderr, flush=True)
    B.close()
    t_batch = float(np.median(times))
    serial = None
    if serial_stride > 0:
        ctx = nl.Context(0)
        tot, n_ok, ids = 0.0, 0, list(range(0, count, serial_stride))
        for i in ids:
            r, m = recipe[i], meshes[i]
            problems.setup_cook(ctx, m, r["mu"], r["lam"], 1.0)
            v = torch.zeros(3 * m.n_nodes, dtype=torch.float64, device="cuda")
            sched = syn.cook_load_schedule(r["tau"])
            torch.cuda.synchronize()
            t = time.perf_counter()
            reps = problems.solve_schedule(ctx, v, "nk", problems.make_opts("nk", "fp64", ksp="minres"),
                                           sched)
            torch.cuda.synchronize()
            tot += time.perf_counter() - t
            n_ok += problems.schedule_ok(reps, sched)
            print(f"[bench] serial NK fp64 instance {i} ({m.conn.shape[0]} tets): "
                  f"{time.perf_counter() - t:.2f}s", file=sys.stderr, flush=True)
        ctx.close()
        est = tot * count / len(ids)
        serial = {"method": "nk_fp64 (MINRES + Jacobi), one instance at a time",
                  "sample": f"instances {ids[0]}, {ids[0] + serial_stride}, ... ({len(ids)} of {count})",
                  "sample_seconds": round(tot, 3), "solved": f"{n_ok}/{len(ids)}",
                  "estimated_seconds_all": round(est, 2),
                  "instances_per_s": round(count / est, 3)}
    return {
        "workload": f"{count} Cook instances (n x n x nz, n in 8..48, nz in 1..3, "
                    "lambda/mu log-uniform 10..1e4, tau 2^U(0,5)), seed 0",
        "tets": n_elems, "nodes": int(off[-1]), "setup_s": round(t_setup, 2), "elements_per_block": block_size,
        "method": "iNK mixed, CG + Jacobi, all instances per launch" + (
            f"; the last {tail} unfinished instances finished alone with CG + multigrid"
            if tail > 0 else "") + (
            f"; instances whose CG solve takes over {tail_its} iterations finished alone with "
            "CG + multigrid" if tail_its > 0 else ""),
        "seconds": [round(x, 3) for x in times], "solved": f"{min(oks)}/{count}",
        "instances_per_s": round(count / t_batch, 3),
        "serial_fp64_nk": serial,
        "speedup_vs_serial": round(serial["estimated_seconds_all"] / t_batch, 2) if serial else None,
    }


TWIST_METHODS = {
    "nk_fp64": ("nk", "fp64", {"ksp": "minres"}),
    "ink_fp64": ("ink", "fp64", {"ksp": "minres"}),
    "nk_mixed": ("nk", "mixed", {"ksp": "minres"}),
    "ink_mixed": ("ink", "mixed", {"ksp": "minres"}),
    # GMRES with the field split: the multigrid cycle on the displacement block
    "nk_fp64_amg": ("nk", "fp64", {"ksp": "gmres", "pc": "amg"}),
    "ink_fp64_amg": ("ink", "fp64", {"ksp": "gmres", "pc": "amg"}),
    "ink_mixed_amg": ("ink", "mixed", {"ksp": "gmres", "pc": "amg"}),
    # BFGS on the saddle-point system (the paper expects it to fail here):
    # H0 a MINRES solve to rtol 1e-2, or the preconditioner alone
    "bfgs_ib_fp64": ("bfgs", "fp64", {"ksp": "minres", "h0": "ksp", "qn_m": 10}),
    "bfgs_b_fp64": ("bfgs", "fp64", {"ksp": "minres", "h0": "preonly", "qn_m": 10}),
    # the lower block-triangular preconditioner (App. B) with the lumped
    # pressure mass over mu for the Schur complement (schur 1), Jacobi or the
    # multigrid cycle on the displacement block
    "ink_mixed_schur_mass": ("ink", "mixed", {"ksp": "gmres", "schur": 1}),
    "nk_fp64_schur_mass_amg": ("nk", "fp64", {"ksp": "gmres", "schur": 1, "pc": "amg"}),
    "ink_fp64_schur_mass_amg": ("ink", "fp64", {"ksp": "gmres", "schur": 1, "pc": "amg"}),
    "ink_mixed_schur_mass_amg": ("ink", "mixed", {"ksp": "gmres", "schur": 1, "pc": "amg"}),
    # the constant-pressure pair (P2-P0, --twist-p0) also takes the SIMPLE
    # approximation S = B diag(A)^-1 B^T (schur 2)
    "nk_fp64_schur_simple": ("nk", "fp64", {"ksp": "gmres", "schur": 2}),
    "ink_mixed_schur_simple": ("ink", "mixed", {"ksp": "gmres", "schur": 2}),
    "nk_fp64_schur_simple_amg": ("nk", "fp64", {"ksp": "gmres", "schur": 2, "pc": "amg"}),
    "ink_fp64_schur_simple_amg": ("ink", "fp64", {"ksp": "gmres", "schur": 2, "pc": "amg"}),
    "ink_mixed_schur_simple_amg": ("ink", "mixed", {"ksp": "gmres", "schur": 2, "pc": "amg"}),
}


def twist_c3(nl, torch, n: int, methods, p0: bool = False):
    """Twist test: unit cube, n^3 cells -> 6 n^3 quadratic tets, top face
    rotated 10 deg per step to 90 deg (9 steps).  Default pair: linear
    pressure, incompressible neo-Hookean, mu = 1; p0: one pressure per
    element with the polyconvex law and the printed constants (all 9000).
    Setup outside the timed region."""
    import math

    import synthetic as syn
    from paper_2203_05610_amd import problems

    mesh = syn.twist_p2_mesh(n)
    ctx = nl.Context(0)
    if p0:
        problems.setup_twist_p0(ctx, mesh)
    else:
        problems.setup_twist(ctx, mesh, 1.0)
    angles = [math.radians(10 * s) for s in range(1, 10)]
    dirf = lambda th: syn.twist_dirichlet(mesh.X, mesh.sets["bottom"], mesh.sets["top"], th)  # noqa: E731
    pair = ("P0 pressure, polyconvex law, alpha_p=beta_p=alpha_s=beta_s=9000" if p0 else
            "P1 pressure, incompressible neo-Hookean, mu=1")
    out = {"workload": f"twist {n}^3 cells -> {mesh.n_elems} P2 tets + {pair}, "
                       f"{ctx.n_dofs} unknowns, 9 x 10 deg", "methods": {}}
    for m in methods:
        name, prec, kw = TWIST_METHODS[m]
        opts = problems.make_opts(name, prec, **dict(kw))
        x = torch.zeros(ctx.n_dofs, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t = time.perf_counter()
        def progress(rep, m=m):
            print(f"[bench]   twist {m} {math.degrees(rep['theta']):.1f} deg: "
                  f"{rep['status_name']} nit={rep['nit']} lit={rep['lit_total']}",
                  file=sys.stderr, flush=True)

        reps = problems.solve_twist(ctx, x, name, opts, angles, dirf, progress=progress)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        out["methods"][m] = {"seconds": round(dt, 3), "ok": problems.twist_ok(reps, angles),
                             "nit": [r["nit"] for r in reps],
                             "lit": int(sum(r["lit_total"] for r in reps)),
                             "cutbacks": sum(1 for r in reps if not r["accepted"])}
        print(f"[bench] twist {m}: {dt:.2f}s ok={out['methods'][m]['ok']}", file=sys.stderr,
              flush=True)
    ctx.close()
    return out


CARDIAC_METHODS = {
    "ink_fp64": ("ink", "fp64", {"ksp": "minres"}),
    "ink_mixed": ("ink", "mixed", {"ksp": "minres"}),
    "nk_fp64": ("nk", "fp64", {"ksp": "minres"}),
    "bfgs_ib_fp64": ("bfgs", "fp64", {"ksp": "minres", "h0": "ksp", "qn_m": 10}),
    "bfgs_ib_fp64_r20": ("bfgs", "fp64", {"ksp": "minres", "h0": "ksp", "qn_m": 10,
                                          "h0_refresh": 20}),
    "ink_fp64_bj": ("ink", "fp64", {"ksp": "minres", "pc": "bjacobi3"}),
    "bfgs_ib_fp64_r20_bj": ("bfgs", "fp64", {"ksp": "minres", "h0": "ksp", "qn_m": 10,
                                             "h0_refresh": 20, "pc": "bjacobi3"}),
    "bfgs_ib_mixed_r20_bj": ("bfgs", "mixed", {"ksp": "minres", "h0": "ksp", "qn_m": 10,
                                               "h0_refresh": 20, "pc": "bjacobi3"}),
    "ink_fp64_amg": ("ink", "fp64", {"ksp": "gmres", "pc": "amg"}),
    "nk_fp64_amg": ("nk", "fp64", {"ksp": "gmres", "pc": "amg"}),
    "bfgs_b_fp64_amg": ("bfgs", "fp64", {"ksp": "gmres", "h0": "preonly", "qn_m": 10,
                                         "pc": "amg"}),
    "bfgs_ib_fp64_r20_amg": ("bfgs", "fp64", {"ksp": "gmres", "h0": "ksp", "qn_m": 10,
                                              "h0_refresh": 20, "pc": "amg"}),
    "ink_fp64_cg_amg": ("ink", "fp64", {"ksp": "cg", "pc": "amg"}),
    # plain FP64 Newton-Krylov with the same multigrid (the like-for-like
    # baseline: App. A tolerances rtol 1e-6 / atol 1e-10)
    "nk_fp64_cg_amg": ("nk", "fp64", {"ksp": "cg", "pc": "amg"}),
    "nk_fp64_gmres30_amg": ("nk", "fp64", {"ksp": "gmres", "restart": 30, "orth": "cgs2",
                                           "pc": "amg"}),
    "nk_fp64_minres_amg": ("nk", "fp64", {"ksp": "minres", "pc": "amg"}),
    "ink_mixed_minres_amg": ("ink", "mixed", {"ksp": "minres", "pc": "amg"}),
    "ink_fp64_gmres30_amg": ("ink", "fp64", {"ksp": "gmres", "restart": 30, "pc": "amg"}),
    "bfgs_ib_fp64_r20_cg_amg": ("bfgs", "fp64", {"ksp": "cg", "h0": "ksp", "qn_m": 10,
                                                 "h0_refresh": 20, "pc": "amg"}),
}


def cardiac_c5(nl, torch, grid, methods, n_steps: int):
    """Heartbeat (cardiac-like law M4, fibres, active tension, follower
    endocardial pressure, epicardial springs), time steps of the activation
    schedule; MINRES + Jacobi (the follower-pressure asymmetry is ~1e-6 of the
    tangent; MINRES's residual is tracked as b - A x, so its stopping test
    stays exact)."""
    import synthetic as syn
    from paper_2203_05610_amd import problems

    C = syn.CARDIAC
    mesh = syn.shell_mesh(*grid)
    ctx = nl.Context(0)
    problems.setup_cardiac(ctx, mesh, C, syn.shell_dirichlet(mesh))
    steps = syn.heartbeat_schedule()[:n_steps]
    out = {"workload": f"ventricle shell {grid[0]}x{grid[1]}x{grid[2]} -> {mesh.n_elems} P1 tets, "
                       f"{mesh.n_dofs} dofs, {len(steps)} time steps", "methods": {}}
    for m in methods:
        name, prec, kw = CARDIAC_METHODS[m]
        opts = problems.make_opts(name, prec, **dict(kw))
        u = torch.zeros(mesh.n_dofs, dtype=torch.float64, device="cuda")
        prev = (0.0, 0.0)
        t = time.perf_counter()
        reps_all, ok = [], True
        for stp in steps:  # one call per step so progress is printed
            reps = problems.solve_heartbeat(ctx, u, name, opts, [stp], C["gamma_max"], start=prev)
            reps_all += reps
            prev = stp
            print(f"[bench] cardiac {m} t={stp[0]:.2f}: {reps[-1]['status_name']} "
                  f"nit={[r['nit'] for r in reps]}", file=sys.stderr, flush=True)
            if not reps[-1]["accepted"]:
                ok = False
                break
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        out["methods"][m] = {"seconds": round(dt, 3), "ok": ok,
                             "nit": [r["nit"] for r in reps_all],
                             "lit": int(sum(r["lit_total"] for r in reps_all)),
                             "cutbacks": sum(1 for r in reps_all if not r["accepted"])}
    ctx.close()
    return out


FOLLOWER_METHODS = {
    "ink_mixed": ("ink", "mixed", {"ksp": "gmres", "orth": "cgs2", "restart": 300}),
    "nk_fp64": ("nk", "fp64", {"ksp": "gmres", "orth": "cgs2", "restart": 300}),
    "bfgs_ib_mixed_r20": ("bfgs", "mixed", {"h0": "ksp", "qn_m": 10, "ksp": "gmres",
                                            "orth": "cgs2", "restart": 300, "h0_refresh": 20}),
    # restarted GMRES with the multigrid cycle
    "ink_mixed_amg": ("ink", "mixed", {"ksp": "gmres", "orth": "cgs2", "restart": 30,
                                       "pc": "amg"}),
    "nk_fp64_amg": ("nk", "fp64", {"ksp": "gmres", "orth": "cgs2", "restart": 30, "pc": "amg"}),
    "bfgs_ib_mixed_r20_amg": ("bfgs", "mixed", {"h0": "ksp", "qn_m": 10, "ksp": "gmres",
                                                "orth": "cgs2", "restart": 30, "h0_refresh": 20,
                                                "pc": "amg"}),
}


def follower_cook(nl, torch, grid, ratio: float, methods):
    """Cook's membrane with the traction per unit current area (fixed
    direction; the load in the deformed configuration), doubling schedule to
    tau = 16, GMRES(300) + Jacobi (the tangent is not symmetric), at most 5000
    Krylov iterations per linear solve."""
    import synthetic as syn
    from paper_2203_05610_amd import problems

    mesh = syn.cook_mesh(*grid)
    ctx = nl.Context(0)
    problems.setup_cook(ctx, mesh, MU, ratio * MU, 1.0, follower=True)
    sched = load_schedule()
    out = {"workload": f"follower Cook {grid[0]}x{grid[1]}x{grid[2]} -> {mesh.n_elems} P1 tets, "
                       f"{mesh.n_dofs} dofs, lambda/mu={ratio:g}, tau " + ",".join(f"{s:g}" for s in sched),
           "methods": {}}
    u = torch.zeros(mesh.n_dofs, dtype=torch.float64, device="cuda")
    for m in methods:
        name, prec, kw = FOLLOWER_METHODS[m]
        opts = problems.make_opts(name, prec, **dict(kw))
        opts.ksp_max_it = 5000
        u.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        prev, ok, reps_all = 0.0, True, []
        for s in sched:  # one call per load step so progress is printed
            reps = problems.solve_schedule(ctx, u, name, opts, [s], start_scale=prev)
            reps_all += reps
            prev = s
            print(f"[bench] follower {m} tau={s:g}: {reps[-1]['status_name']} "
                  f"nit={[r['nit'] for r in reps]}", file=sys.stderr, flush=True)
            if not problems.schedule_ok(reps, [s]):
                ok = False
                break
        torch.cuda.synchronize()
        out["methods"][m] = {"seconds": round(time.perf_counter() - t, 3), "ok": ok,
                             "nit": [r["nit"] for r in reps_all],
                             "lit": int(sum(r["lit_total"] for r in reps_all)),
                             "cutbacks": sum(1 for r in reps_all if not r["accepted"])}
    ctx.close()
    return out


P2_METHODS = {
    "ink_mixed": ("ink", "mixed", {"ksp": "cg"}),
    "nk_fp64": ("nk", "fp64", {"ksp": "minres"}),
    "bfgs_ib_mixed_r20": ("bfgs", "mixed", {"h0": "ksp", "qn_m": 10, "ksp": "minres",
                                            "h0_refresh": 20}),
    "ink_mixed_cg_amg": ("ink", "mixed", {"ksp": "cg", "pc": "amg"}),
    "nk_fp64_cg_amg": ("nk", "fp64", {"ksp": "cg", "pc": "amg"}),
}


def p2_cook(nl, torch, grid, ratio: float, methods):
    """Cook's membrane with quadratic (10-node) displacement tetrahedra, law
    M1, dead traction, doubling schedule to tau = 16; Jacobi-preconditioned
    unless the method names the multigrid."""
    import synthetic as syn
    from paper_2203_05610_amd import problems

    mesh = syn.cook_p2_mesh(*grid)
    ctx = nl.Context(0)
    problems.setup_cook_p2(ctx, mesh, MU, ratio * MU, 1.0)
    sched = load_schedule()
    out = {"workload": f"P2 Cook {grid[0]}x{grid[1]}x{grid[2]} -> {mesh.n_elems} 10-node tets, "
                       f"{mesh.n_dofs} dofs, lambda/mu={ratio:g}, tau " + ",".join(f"{s:g}" for s in sched),
           "methods": {}}
    u = torch.zeros(mesh.n_dofs, dtype=torch.float64, device="cuda")
    for m in methods:
        name, prec, kw = P2_METHODS[m]
        opts = problems.make_opts(name, prec, **dict(kw))
        u.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        prev, ok, reps_all = 0.0, True, []
        for s in sched:
            reps = problems.solve_schedule(ctx, u, name, opts, [s], start_scale=prev)
            reps_all += reps
            prev = s
            print(f"[bench] p2 {m} tau={s:g}: {reps[-1]['status_name']} "
                  f"nit={[r['nit'] for r in reps]}", file=sys.stderr, flush=True)
            if not problems.schedule_ok(reps, [s]):
                ok = False
                break
        torch.cuda.synchronize()
        out["methods"][m] = {"seconds": round(time.perf_counter() - t, 3), "ok": ok,
                             "nit": [r["nit"] for r in reps_all],
                             "lit": int(sum(r["lit_total"] for r in reps_all)),
                             "cutbacks": sum(1 for r in reps_all if not r["accepted"])}
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--method", default="ink_mixed_cg3_amg", choices=sorted(METHODS))
    ap.add_argument("--baseline", default="nk_fp64_minres_amg", choices=sorted(METHODS))
    ap.add_argument("--compare", default="ink_fp64_cg_amg,ink_mixed,bfgs_ib_mixed_r20",
                    help="comma-separated extra methods, run once each ('' for none)")
    ap.add_argument("--jv-reps", type=int, default=200)
    ap.add_argument("--block-size", type=int, default=HEAD_BLOCK,
                    help="elements per block of the timed Cook mesh")
    ap.add_argument("--pc", default="jacobi", choices=["jacobi", "bjacobi3"],
                    help="preconditioner of the Cook methods that name none (point or nodal "
                         "3x3 block Jacobi)")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-baseline", action="store_true")
    ap.add_argument("--batch", type=int, default=256,
                    help="instances of the batched-solve leg (0 skips it)")
    ap.add_argument("--batch-tail", type=int, default=0,
                    help="finish the last N unfinished instances of the batch alone with CG + "
                         "multigrid (0: all in the batch rounds)")
    ap.add_argument("--batch-tail-its", type=int, default=0,
                    help="finish alone with CG + multigrid any instance whose batched CG solve "
                         "takes more than N iterations (0: never)")
    ap.add_argument("--batch-serial-stride", type=int, default=64,
                    help="serial FP64 NK baseline on every k-th batch instance (0 skips it)")
    ap.add_argument("--batch-only", action="store_true", help="only the batched-solve leg")
    ap.add_argument("--twist", type=int, default=24, help="twist cube cells per edge (0 skips)")
    ap.add_argument("--twist-methods",
                    default="nk_fp64,nk_fp64_schur_mass_amg,ink_mixed_schur_mass_amg")
    ap.add_argument("--twist-p0", type=int, default=12,
                    help="cells per edge of the P2-P0 polyconvex twist leg (0 skips)")
    ap.add_argument("--twist-p0-methods",
                    default="nk_fp64_schur_simple_amg,ink_mixed_schur_simple_amg")
    ap.add_argument("--cardiac", default="8,80,256", help="ventricle shell grid n_t,n_s,n_c "
                    "(empty skips this leg)")
    ap.add_argument("--cardiac-methods", default="ink_fp64_cg_amg")
    ap.add_argument("--cardiac-steps", type=int, default=20)
    ap.add_argument("--follower", default="", help="follower-load Cook grid nx,ny,nz (e.g. "
                    "64,64,4; empty skips)")
    ap.add_argument("--follower-ratio", type=float, default=5.0, help="lambda/mu of that leg")
    ap.add_argument("--follower-methods", default="ink_mixed,nk_fp64,bfgs_ib_mixed_r20")
    ap.add_argument("--p2", default="", help="P2 Cook grid nx,ny,nz (e.g. 32,32,2; empty skips)")
    ap.add_argument("--p2-ratio", type=float, default=5.0, help="lambda/mu of that leg")
    ap.add_argument("--p2-methods", default="ink_mixed,nk_fp64,bfgs_ib_mixed_r20")
    ap.add_argument("--legs-only", action="store_true",
                    help="only the twist and cardiac legs (for their own runs)")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the Jv roofline phase (plus a 256 MB copy kernel used to "
                         "calibrate HBM byte counters); for profiling runs")
    args = ap.parse_args()
    PC["pc"] = args.pc
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); sharding a "
              "solve over several GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synthetic as syn
    from paper_2203_05610_amd import nlelast as nl
    from paper_2203_05610_amd import problems

    if args.roofline_only:
        jv = jv_roofline(nl, torch, args.jv_reps)
        x = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        z = torch.empty_like(x)
        for _ in range(5):
            torch.neg(x, out=z)  # plain copy kernel: 256 MiB read + 256 MiB written
        torch.cuda.synchronize()
        print(json.dumps({"roofline_only": True, "jv": jv}))
        return

    if args.batch_only:
        print(json.dumps({"batch_only": True,
                          "batch": batch_c4(nl, torch, args.batch, args.batch_serial_stride,
                                            max(args.steps, 1), tail=args.batch_tail,
                                            tail_its=args.batch_tail_its)}))
        return

    if args.legs_only:
        res = {"legs_only": True}
        if args.twist > 0:
            res["twist"] = twist_c3(nl, torch, args.twist, args.twist_methods.split(","))
        if args.twist_p0 > 0:
            res["twist_p0"] = twist_c3(nl, torch, args.twist_p0,
                                       args.twist_p0_methods.split(","), p0=True)
        if args.cardiac:
            res["cardiac"] = cardiac_c5(nl, torch, tuple(int(x) for x in args.cardiac.split(",")),
                                        args.cardiac_methods.split(","), args.cardiac_steps)
        if args.follower:
            res["follower"] = follower_cook(nl, torch, tuple(int(x) for x in args.follower.split(",")),
                                            args.follower_ratio, args.follower_methods.split(","))
        if args.p2:
            res["p2"] = p2_cook(nl, torch, tuple(int(x) for x in args.p2.split(",")), args.p2_ratio,
                                args.p2_methods.split(","))
        print(json.dumps(res))
        return

    schedule = load_schedule()
    t_setup = time.perf_counter()
    mesh = syn.cook_mesh(*GRID)
    ctx = nl.Context(0)
    problems.setup_cook(ctx, mesh, MU, RATIO * MU, 1.0, block_size=args.block_size)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    u = torch.zeros(3 * mesh.n_nodes, dtype=torch.float64, device="cuda")

    print(f"[bench] setup {t_setup:.2f}s; warmup {args.warmup} x {args.method}", file=sys.stderr,
          flush=True)
    for _ in range(args.warmup):
        run_solve(ctx, u, args.method, schedule)
    torch.cuda.synchronize()
    runs = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        ok, reps = run_solve(ctx, u, args.method, schedule)
        runs.append(summarize(reps))
        print(f"[bench] step {k}: ok={ok} nit={runs[-1]['nit']}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1000.0 / max(args.steps, 1)
    all_ok = all(r["ok"] for r in runs)
    u_method = u.detach().cpu().numpy().copy()
    accuracy = {"method_vs_oracle_root": root_error(u_method)}

    extra = {}
    base = None
    if not args.no_baseline and args.baseline != args.method:
        torch.cuda.synchronize()
        tb = time.perf_counter()
        ok, reps = run_solve(ctx, u, args.baseline, schedule)
        torch.cuda.synchronize()
        base = {"method": args.baseline, "seconds": time.perf_counter() - tb, **summarize(reps)}
        u_base = u.detach().cpu().numpy()
        accuracy["baseline_vs_oracle_root"] = root_error(u_base)
        accuracy["method_vs_baseline"] = float(np.linalg.norm(u_method - u_base) /
                                               max(np.linalg.norm(u_base), 1e-300))
        print(f"[bench] baseline {args.baseline}: {base['seconds']:.2f}s ok={base['ok']}",
              file=sys.stderr, flush=True)
    for m in [x for x in args.compare.split(",") if x]:
        torch.cuda.synchronize()
        tb = time.perf_counter()
        ok, reps = run_solve(ctx, u, m, schedule)
        torch.cuda.synchronize()
        extra[m] = {"seconds": time.perf_counter() - tb, **summarize(reps),
                    "rel_error_vs_oracle_root": root_error(u.detach().cpu().numpy())}
        print(f"[bench] compare {m}: {extra[m]['seconds']:.2f}s ok={extra[m]['ok']}",
              file=sys.stderr, flush=True)
    ctx.close()

    roof = None
    jv = None
    if not args.no_roofline:
        jv = jv_roofline(nl, torch, args.jv_reps)
        f = jv["fp32"]
        traffic = measured_traffic(f["bytes"])
        roof = {
            "bound": "hbm",
            "achieved": round(f["gbs"], 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(f["gbs"] / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "target_frac": 0.60,
            "target_met": f["gbs"] / HBM_PEAK_GBS >= 0.60,
            "kernel": JV_KERNEL,
            "workload": "Cook 256x256x16, 6,291,456 P1 tets, 1,122,833 nodes, law M1, FP32",
            "bytes_definition": "algorithmic: 56 B per element (4 int32 node ids, grad N and V "
                                "as 10 FP32) + 36 B per node (u, v read, y written)",
            "bytes_per_launch": f["bytes"],
            "ms_per_launch": round(f["ms"], 5),
            "traffic_over_bytes": round(traffic / f["bytes"], 3) if traffic else None,
            "layout": {"definition": "this library's own arrays: 20 B per element, 12 B per "
                                     "block-node slot, 36 B per node",
                       "bytes_per_launch": f["layout_bytes"],
                       "achieved": round(f["layout_gbs"], 1),
                       "traffic_over_bytes": (round(traffic / f["layout_bytes"], 3)
                                              if traffic else None)},
            "fp64": {"achieved": round(jv["fp64"]["gbs"], 1), "ms_per_launch":
                     round(jv["fp64"]["ms"], 5), "bytes_per_launch": jv["fp64"]["bytes"],
                     "frac": round(jv["fp64"]["gbs"] / HBM_PEAK_GBS, 4)},
        }
        print(f"[bench] Jv roofline fp32 {f['gbs']:.0f} GB/s", file=sys.stderr, flush=True)

    batch = None
    if args.batch > 0:
        batch = batch_c4(nl, torch, args.batch, args.batch_serial_stride, 1, tail=args.batch_tail,
                         tail_its=args.batch_tail_its)
    twist = twist_c3(nl, torch, args.twist, args.twist_methods.split(",")) if args.twist > 0 else None
    twist_p0 = (twist_c3(nl, torch, args.twist_p0, args.twist_p0_methods.split(","), p0=True)
                if args.twist_p0 > 0 else None)
    cardiac = None
    if args.cardiac:
        cardiac = cardiac_c5(nl, torch, tuple(int(x) for x in args.cardiac.split(",")),
                             args.cardiac_methods.split(","), args.cardiac_steps)
    follower = None
    if args.follower:
        follower = follower_cook(nl, torch, tuple(int(x) for x in args.follower.split(",")),
                                 args.follower_ratio, args.follower_methods.split(","))
    p2 = None
    if args.p2:
        p2 = p2_cook(nl, torch, tuple(int(x) for x in args.p2.split(",")), args.p2_ratio,
                     args.p2_methods.split(","))

    cpu = None
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle, 1 thread)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(len(schedule))

    value = ms_per_step / 1000.0
    line = {
        "metric": "time-to-solve at rel. residual 1e-8 (NK-FP64 vs iNK/BFGS mixed); Jv HBM GB/s",
        "value": round(value, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64 (mixed)" if METHODS[args.method][1] == "mixed" else "f64",
        "data": "synthetic",
        "config": {
            "workload": "Cook's membrane 64x64x4 hexes -> 98,304 P1 tets, 63,375 dofs, "
                        "lambda/mu=5000, traction schedule " + ",".join(f"{s:g}" for s in schedule),
            "method": args.method,
            "precision": "FP32 inner (tangent, preconditioner, Krylov, L-BFGS vectors), FP64 "
                         "residual/state" if METHODS[args.method][1] == "mixed" else "FP64",
            "preconditioner": {"jacobi": "Jacobi", "bjacobi3": "nodal 3x3 block Jacobi",
                               "amg": "aggregation multigrid, one V(1,1)-cycle"}[
                METHODS[args.method][2].get("pc", PC["pc"])],
            "krylov": METHODS[args.method][2].get("ksp", "cg") + (
                " (next direction formed in the Jacobian action)"
                if METHODS[args.method][2].get("cg_launches") == 3 else ""),
            "elements_per_block": args.block_size,
            "parallelism": "1 GPU",
        },
        "solved": all_ok,
        "runs": runs,
        "setup_s": round(t_setup, 3),
        "gpu_baseline": base,
        "speedup_vs_gpu_baseline": (round(base["seconds"] / value, 3)
                                    if base and base["ok"] and all_ok else None),
        "compare": extra or None,
        "batch": batch,
        "twist": twist,
        "twist_p0": twist_p0,
        "cardiac": cardiac,
        "follower": follower,
        "p2": p2,
        "accuracy": accuracy,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
