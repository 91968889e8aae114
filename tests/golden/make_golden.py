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


CASES = {"cook64": cook64, "batch16": batch16}

if __name__ == "__main__":
    for name in (sys.argv[1:] or list(CASES)):
        CASES[name]()
