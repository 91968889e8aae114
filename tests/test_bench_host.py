"""Host-side checks of bench.py (no GPU): it refuses more than one GPU with a
message, and every method table it can run builds valid solver options."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2203_05610_amd import nlelast as nl  # noqa: E402
from paper_2203_05610_amd import problems  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.parametrize("table", ["METHODS", "CARDIAC_METHODS", "FOLLOWER_METHODS",
                                   "P2_METHODS", "TWIST_METHODS"])
def test_method_tables_build_options(table):
    pcs = {"jacobi": nl.NLE_PC_JACOBI, "bjacobi3": nl.NLE_PC_BJACOBI3, "amg": nl.NLE_PC_AMG}
    for name, (solver, prec, kw) in getattr(bench, table).items():
        o = problems.make_opts(solver, prec, **{"pc": "jacobi", **kw})
        assert o.pc == pcs[kw.get("pc", "jacobi")], name
        assert o.precision == (nl.NLE_PREC_MIXED if prec == "mixed" else nl.NLE_PREC_FP64)
        if o.pc == nl.NLE_PC_AMG and table == "TWIST_METHODS":  # field split: GMRES only
            assert o.ksp_type == nl.NLE_KSP_GMRES, name
    assert "ink_mixed_cg_amg" in bench.METHODS


def test_timed_mesh_block_size_gives_one_block_per_compute_unit():
    # the timed Cook mesh is cut into element blocks of bench.HEAD_BLOCK: 256
    # equal blocks, one per compute unit of the MI355X
    import synthetic as syn

    m = syn.cook_mesh(*bench.GRID, with_faces=False)
    n_e = len(m.conn)
    assert n_e % bench.HEAD_BLOCK == 0
    assert n_e // bench.HEAD_BLOCK == 256
