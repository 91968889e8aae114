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


def test_opts_struct_layout_matches_header(tmp_path):
    # the binding's structs against the C compiler's layout of the header
    import shutil
    import subprocess

    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    fields = [f[0] for f in nl.nle_solver_opts._fields_]
    rfields = [f[0] for f in nl.nle_report._fields_]
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "nlelast.h"', "int main(void) {",
           'printf("%zu\\n", sizeof(nle_solver_opts));']
    src += [f'printf("%zu\\n", offsetof(nle_solver_opts, {f}));' for f in fields]
    src += ['printf("%zu\\n", sizeof(nle_report));']
    src += [f'printf("%zu\\n", offsetof(nle_report, {f}));' for f in rfields]
    src += ["return 0; }"]
    (tmp_path / "layout.c").write_text("\n".join(src) + "\n")
    exe = str(tmp_path / "layout")
    subprocess.run([cc, "-I", inc, str(tmp_path / "layout.c"), "-o", exe], check=True)
    vals = [int(x) for x in subprocess.run([exe], check=True, capture_output=True,
                                           text=True).stdout.split()]
    want = [ctypes.sizeof(nl.nle_solver_opts)]
    want += [getattr(nl.nle_solver_opts, f).offset for f in fields]
    want += [ctypes.sizeof(nl.nle_report)] + [getattr(nl.nle_report, f).offset for f in rfields]
    assert vals == want


def test_null_and_bad_arguments_are_rejected_without_a_device():
    L = nl.lib()
    assert L.nle_create(None, 0, None, None) == nl.NLE_E_INVAL
    assert L.nle_residual(None, None, None, None) == nl.NLE_E_INVAL
    assert L.nle_set_block_size(None, 512) == nl.NLE_E_INVAL
    assert L.nle_last_error(None) == b"null context"
    L.nle_destroy(None)  # no-op


def test_newer_calls_reject_null_arguments_without_a_device():
    import ctypes as ct
    L = nl.lib()
    n = ct.c_int32(-1)
    assert L.nle_amg_levels(None, ct.byref(n), None, 0) == nl.NLE_E_INVAL
    assert n.value == -1  # nothing written on an error
    assert L.nle_newmark_correct(None, 0.1, 0.25, 0.5, None, None, None, None) == nl.NLE_E_INVAL
    assert L.nle_set_inertia(None, 1.0, 1.0, None) == nl.NLE_E_INVAL
    assert L.nle_set_robin_damping(None, 1.0, 1.0) == nl.NLE_E_INVAL
    assert L.nle_set_step_velocity(None, 1.0, None) == nl.NLE_E_INVAL
    assert L.nle_newmark_predict(None, 0.1, 0.25, 0.5, None, None, None, None, None) == nl.NLE_E_INVAL
    assert L.nle_batch_set_tail(None, 4, 0, nl.NLE_PC_AMG) == nl.NLE_E_INVAL
