"""Host-side checks of the C ABI (no GPU compute): the library loads, exports
every function include/nlelast.h declares, and its pure-host calls behave."""

import ctypes
import os
import re

import pytest

from paper_2203_05610_amd import nlelast as nl

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "nlelast.h")

pytestmark = pytest.mark.skipif(not os.path.exists(nl.LIB_PATH),
                                reason="libnlelast.so not built (run __graft_entry__.build())")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(nle_[a-z_0-9]+)\s*\(", txt)))


def test_header_and_binding_agree():
    assert _declared() == sorted(nl.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = nl.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_version_and_default_options():
    assert "nlelast" in nl.nle_version()
    o = nl.nle_default_opts(nl.NLE_NK)
    assert (o.ksp_rtol, o.ksp_atol) == (1e-6, 1e-10)  # App. A, NK
    assert (o.ew_rtol0, o.ew_rtolmax, o.ink_ksp_atol) == (0.1, 0.1, 1e-14)  # App. A, iNK
    assert abs(o.ew_alpha2 - (1 + 5 ** 0.5) / 2) < 1e-15
    assert o.snes_rtol == 1e-8
    b = nl.nle_default_opts(nl.NLE_BFGS)
    assert (b.h0_rtol, b.h0_atol, b.qn_m) == (1e-2, 1e-14, 50)  # App. A, inexact BFGS
    assert b.snes_max_it == 1000


def test_opts_struct_layout_matches_header():
    # 12 int32 fields then 15 doubles
    assert ctypes.sizeof(nl.nle_solver_opts) == 12 * 4 + 15 * 8
    assert nl.nle_report.rnorm_hist.offset % 8 == 0


def test_null_and_bad_arguments_are_rejected_without_a_device():
    L = nl.lib()
    assert L.nle_create(None, 0, None, None) == nl.NLE_E_INVAL
    assert L.nle_residual(None, None, None, None) == nl.NLE_E_INVAL
    assert L.nle_set_block_size(None, 512) == nl.NLE_E_INVAL
    assert L.nle_last_error(None) == b"null context"
    L.nle_destroy(None)  # no-op
