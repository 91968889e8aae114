"""GPU parity of the batched solver: several Cook instances of uneven size,
material ratio and load, each with its own doubling load schedule, solved in
one batch; every instance is compared with the oracle's exact-Newton root of
the same schedule (<= 1e-6 mixed, <= 1e-8 FP64 at a tightened stopping rule)
and with a single-problem solve on the GPU."""

import numpy as np
import pytest

import synthetic as syn
from oracle import fem, newton
from tests.gpu_common import MU

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2203_05610_amd import nlelast as nl  # noqa: E402
from paper_2203_05610_amd import problems  # noqa: E402

# (nx, ny, nz, lambda/mu, tau)
INSTANCES = [(8, 8, 1, 5.0, 1.0), (12, 10, 2, 50.0, 3.0), (6, 6, 1, 500.0, 0.7),
             (16, 14, 1, 10.0, 5.0), (9, 9, 3, 2000.0, 1.5)]


def _roots():
    out = []
    for nx, ny, nz, ratio, tau in INSTANCES:
        m = syn.cook_mesh(nx, ny, nz)
        P = fem.cook_problem(m, mu=MU, lam=ratio * MU, tau=1.0)
        sched = syn.cook_load_schedule(tau)
        out.append((m, P, sched, newton.solve_schedule(P, sched)[0]))
    return out


@pytest.mark.parametrize("method,precision", [("ink", "mixed"), ("nk", "mixed"), ("nk", "fp64")])
def test_batch_matches_oracle_per_instance(method, precision):
    data = _roots()
    B = nl.Batch(0)
    for (m, P, sched, _), (nx, ny, nz, ratio, tau) in zip(data, INSTANCES):
        problems.add_cook_instance(B, m, MU, ratio * MU, 1.0, sched)
    nl.nle_batch_finalize(B)
    off = nl.nle_batch_layout(B)
    assert len(off) == len(INSTANCES) + 1
    u = torch.zeros(int(3 * off[-1]), dtype=torch.float64, device="cuda")
    o = problems.make_opts(method, precision, ksp="cg")
    tight = precision == "fp64"
    if tight:
        o.snes_rtol = 1e-11
    st, reps, tms = nl.nle_batch_solve(B, nl.NLE_NK if method == "nk" else nl.NLE_INK, o, u)
    assert st == nl.NLE_OK, reps
    assert tms > 0
    uh = u.cpu().numpy()
    for i, (m, P, sched, ustar) in enumerate(data):
        ui = uh[3 * off[i]: 3 * off[i + 1]]
        err = np.linalg.norm(ui - ustar) / np.linalg.norm(ustar)
        assert err <= (1e-8 if tight else 1e-6), (i, err, reps[i])
        assert reps[i]["nit"] >= len(sched)


def test_batch_instance_equals_single_solve_behaviour():
    # one instance alone in a batch and the single-problem solver reach the same root
    nx, ny, nz, ratio, tau = INSTANCES[1]
    m = syn.cook_mesh(nx, ny, nz)
    sched = syn.cook_load_schedule(tau)
    B = nl.Batch(0)
    problems.add_cook_instance(B, m, MU, ratio * MU, 1.0, sched)
    nl.nle_batch_finalize(B)
    u = torch.zeros(3 * m.n_nodes, dtype=torch.float64, device="cuda")
    st, reps, _ = nl.nle_batch_solve(B, nl.NLE_INK, problems.make_opts("ink", "fp64", ksp="cg"), u)
    assert st == nl.NLE_OK
    ctx = nl.Context(0)
    problems.setup_cook(ctx, m, MU, ratio * MU, 1.0)
    v = torch.zeros_like(u)
    rs = problems.solve_schedule(ctx, v, "ink", problems.make_opts("ink", "fp64", ksp="cg"), sched)
    assert problems.schedule_ok(rs, sched)
    assert torch.allclose(u, v, rtol=0, atol=1e-6 * float(v.abs().max()))


def test_batch_usage_errors():
    B = nl.Batch(0)
    with pytest.raises(nl.NleError):
        nl.nle_batch_finalize(B)  # empty
    m = syn.cook_mesh(4, 4, 1)
    problems.add_cook_instance(B, m, MU, 5 * MU, 1.0, [1.0])
    with pytest.raises(nl.NleError):
        nl.nle_batch_add(B, m.X, m.conn, nl.NLE_MAT_M2, [MU, MU], [], [], m.faces["load"],
                         [0, 1, 0], [1.0])  # mixed laws
    bad = m.conn.copy()
    bad[0, 0] = 10 ** 6
    with pytest.raises(nl.NleError):
        nl.nle_batch_add(B, m.X, bad, nl.NLE_MAT_M1, [MU, MU], [], [], m.faces["load"],
                         [0, 1, 0], [1.0])
    nl.nle_batch_finalize(B)
    u = torch.zeros(3 * m.n_nodes, dtype=torch.float64, device="cuda")
    with pytest.raises(nl.NleError):
        nl.nle_batch_solve(B, nl.NLE_BFGS, problems.make_opts("bfgs"), u)


def test_batch_autotune_keeps_layout_and_results():
    data = _roots()
    B = nl.Batch(0)
    for (m, P, sched, _), (nx, ny, nz, ratio, tau) in zip(data, INSTANCES):
        problems.add_cook_instance(B, m, MU, ratio * MU, 1.0, sched)
    nl.nle_batch_finalize(B)
    off = nl.nle_batch_layout(B).copy()
    with pytest.raises(nl.NleError):
        nl.nle_batch_autotune(B, prec=7)
    be = nl.nle_batch_autotune(B, nl.NLE_FP32, budget_ms=50.0)
    assert be in (128, 256, 512, 1024)
    assert np.array_equal(nl.nle_batch_layout(B), off)
    u = torch.zeros(int(3 * off[-1]), dtype=torch.float64, device="cuda")
    st, reps, tms = nl.nle_batch_solve(B, nl.NLE_INK, problems.make_opts("ink", "mixed", ksp="cg"), u)
    assert st == nl.NLE_OK, reps
    uh = u.cpu().numpy()
    for i, (m, P, sched, ustar) in enumerate(data):
        ui = uh[3 * off[i]: 3 * off[i + 1]]
        assert np.linalg.norm(ui - ustar) <= 1e-6 * np.linalg.norm(ustar), i
