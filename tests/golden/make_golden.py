"""Write the stored oracle roots under tests/golden/ (calls only oracle/ and
the seeded input generators in synthetic/; nothing from the GPU path).

  python tests/golden/make_golden.py [case ...]      (default: every case)

Cases:
  cook64   Cook 64x64x4 (98,304 P1 tets), law M1, mu = 80.194, lambda/mu =
           5000, dead traction schedule tau = 1, 2, 4, 8, 16 (doubling, Sec. 4
           load stepping), exact Newton (complex-step tangent + sparse LU) to
           ||r|| <= 1e-13 ||r_0|| per step, halving the increment of a step
           that fails.  Writes cook64x64x4_l5000_tau16.npy (u*) and
           cook64x64x4_l5000_tau16.json (attempts, Newton iterations of all
           attempts, seconds per iteration on one thread).
  batch16  every 16th instance of the 256-instance Cook batch recipe
           (default_rng(0)), each over its doubling schedule ending at its tau:
           batch16_roots.npz (u* per instance, key "i<index>") and
           batch16_roots.json (attempts per instance).
  twist6   the twist cube at 6^3 cells over 9 x 10 deg, P2-P1 (law M3) and
           P2-P0 (law M5): twist6_p1.npy, twist6_p0.npy.
  heart4   the 20-step quasi-static heartbeat on the 4x20x64 shell:
           heart4x20x64_peak.npy (step 10), heart4x20x64.npy (step 20).
"""

from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synthetic as syn  # noqa: E402
from oracle import fem, newton  # noqa: E402

MU = 80.194


def _solve(P, sched):
    log = []
    t0 = time.perf_counter()
    u, hists = newton.solve_schedule(P, sched, max_cuts=8, log=log)
    dt = time.perf_counter() - t0
    its = int(sum(k for _, _, k in log))  # every attempt's Newton steps
    return u, hists, log, dt, its


def cook64():
    mesh = syn.cook_mesh(64, 64, 4)
    P = fem.cook_problem(mesh, mu=MU, lam=5000.0 * MU, tau=1.0)
    sched = syn.cook_load_schedule(16.0)
    u, hists, log, dt, its = _solve(P, sched)
    np.save(os.path.join(HERE, "cook64x64x4_l5000_tau16.npy"), u)
    meta = {
        "workload": "Cook 64x64x4, M1, mu=80.194, lambda/mu=5000, tau 1,2,4,8,16",
        "schedule": sched,
        "attempts": [{"scale": s, "accepted": a, "iterations": k} for s, a, k in log],
        "newton_iterations": its,
        "rnorm_hist": [[float(x) for x in h] for h in hists],
        "seconds": round(dt, 2),
        "seconds_per_iteration": round(dt / max(its, 1), 3),
        "threads": os.environ.get("OMP_NUM_THREADS", "unset"),
    }
    with open(os.path.join(HERE, "cook64x64x4_l5000_tau16.json"), "w") as fh:
        json.dump(meta, fh, indent=1)
    print(f"cook64: {its} Newton iterations in {dt:.1f}s; attempts {log}", flush=True)


def batch16():
    recipe = syn.batch_recipe(256)
    roots, meta = {}, {}
    for i in range(0, 256, 16):
        r = recipe[i]
        mesh = syn.cook_mesh(r["nx"], r["ny"], r["nz"])
        # traction (0, 1, 0) times the load scales of the schedule, the last
        # of which is tau
        P = fem.cook_problem(mesh, mu=r["mu"], lam=r["lam"], tau=1.0)
        sched = syn.cook_load_schedule(r["tau"])
        u, hists, log, dt, its = _solve(P, sched)
        roots[f"i{i}"] = u
        meta[f"i{i}"] = {"recipe": r, "attempts": [[s, a, k] for s, a, k in log],
                         "newton_iterations": its, "seconds": round(dt, 2)}
        print(f"batch16 instance {i}: {mesh.n_elems} tets, {its} its, {dt:.1f}s, {log}",
              flush=True)
    np.savez(os.path.join(HERE, "batch16_roots.npz"), **roots)
    with open(os.path.join(HERE, "batch16_roots.json"), "w") as fh:
        json.dump(meta, fh, indent=1)


def _twist(n, p0):
    import math

    from oracle import mixed

    mesh = syn.twist_p2_mesh(n)
    P = mixed.twist_problem_p0(mesh, 0.0) if p0 else mixed.twist_problem(mesh, 1.0, 0.0)
    xs = np.zeros(P.n_dofs)
    its = []
    t0 = time.perf_counter()
    for s in range(1, 10):
        mixed.set_twist_angle(P, mesh, math.radians(10 * s))
        xs, h = newton.newton_exact(P, xs, 1.0)
        its.append(len(h) - 1)
    return xs, its, time.perf_counter() - t0


def twist6():
    """Twist 6^3 cells, 9 x 10 deg, exact Newton per angle: the P2-P1 form
    with law M3 (mu = 1) and the paper's P2-P0 form with law M5 (all
    constants 9000).  twist6_p1.npy, twist6_p0.npy."""
    for p0, name in ((False, "twist6_p1"), (True, "twist6_p0")):
        xs, its, dt = _twist(6, p0)
        np.save(os.path.join(HERE, name + ".npy"), xs)
        print(f"{name}: Newton iterations per angle {its}, {dt:.1f}s", flush=True)


def heart4():
    """Quasi-static heartbeat on the 4x20x64 ventricle shell (30,720 P1 tets),
    law M4 with the synthetic constants, 20 time steps of the activation
    schedule, exact Newton per step warm-started: heart4x20x64.npy (u at the
    last step) and heart4x20x64_peak.npy (u at the activation peak, step 10)."""
    C = syn.CARDIAC
    mesh = syn.shell_mesh(4, 20, 64)
    P = fem.cardiac_problem(mesh, C)
    steps = syn.heartbeat_schedule()
    t0 = time.perf_counter()
    u_peak, _ = newton.solve_heartbeat(P, steps[:10], C["gamma_max"])
    np.save(os.path.join(HERE, "heart4x20x64_peak.npy"), u_peak)
    u, hists = newton.solve_heartbeat(P, steps[10:], C["gamma_max"], u0=u_peak)
    np.save(os.path.join(HERE, "heart4x20x64.npy"), u)
    print(f"heart4: {time.perf_counter() - t0:.1f}s", flush=True)


CASES = {"cook64": cook64, "batch16": batch16, "twist6": twist6, "heart4": heart4}

if __name__ == "__main__":
    for name in (sys.argv[1:] or list(CASES)):
        CASES[name]()
