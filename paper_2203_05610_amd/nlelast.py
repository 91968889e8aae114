"""Thin ctypes binding of libnlelast.so (the C ABI declared in include/nlelast.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Device vectors are torch tensors on the context's device (float64,
or float32 for FP32 Jacobian actions); device memory for the library's own
buffers comes from torch's caching allocator through the nle_allocator
callbacks, and work is queued on torch's current stream.  There is no CPU
fallback: without the built library every call raises.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnlelast.so")

NLE_OK = 0
NLE_DIVERGED_MAXIT, NLE_DIVERGED_NAN, NLE_DIVERGED_INVERTED = 1, 2, 3
NLE_DIVERGED_LINEAR, NLE_BFGS_BREAKDOWN = 4, 5
NLE_E_INVAL, NLE_E_BADMESH, NLE_E_STATE = -1, -2, -3
NLE_E_OOM, NLE_E_HIP, NLE_E_UNSUPPORTED = -4, -5, -6
NLE_FP64, NLE_FP32 = 0, 1
NLE_MAT_M1, NLE_MAT_M2, NLE_MAT_M3, NLE_MAT_M4, NLE_MAT_M5, NLE_MAT_M6 = 1, 2, 3, 4, 5, 6
NLE_NK, NLE_INK, NLE_BFGS = 0, 1, 2
NLE_KSP_GMRES, NLE_KSP_CG, NLE_KSP_MINRES = 0, 1, 2
NLE_ORTH_MGS, NLE_ORTH_CGS2 = 0, 1
NLE_PC_NONE, NLE_PC_JACOBI, NLE_PC_BJACOBI3, NLE_PC_AMG = 0, 1, 2, 3
NLE_H0_PREONLY, NLE_H0_KSP = 0, 1
NLE_PREC_FP64, NLE_PREC_MIXED = 0, 1
NLE_SCHUR_DIAG, NLE_SCHUR_LOWER_MASS, NLE_SCHUR_LOWER_SIMPLE = 0, 1, 2

STATUS_NAMES = {
    0: "OK", 1: "DIVERGED_MAXIT", 2: "DIVERGED_NAN", 3: "DIVERGED_INVERTED",
    4: "DIVERGED_LINEAR", 5: "BFGS_BREAKDOWN", -1: "E_INVAL", -2: "E_BADMESH",
    -3: "E_STATE", -4: "E_OOM", -5: "E_HIP", -6: "E_UNSUPPORTED",
}

# every symbol the header declares (checked by the CPU test suite)
EXPORTS = [
    "nle_create", "nle_destroy", "nle_last_error", "nle_version", "nle_set_block_size",
    "nle_upload_mesh", "nle_set_material", "nle_set_dirichlet", "nle_set_traction",
    "nle_set_body_force", "nle_set_load_scale", "nle_lift", "nle_residual", "nle_linearize",
    "nle_jv", "nle_diag", "nle_energy", "nle_default_opts", "nle_solve_nk", "nle_solve_ink",
    "nle_solve_bfgs", "nle_partition_info", "nle_batch_create", "nle_batch_destroy",
    "nle_batch_last_error", "nle_batch_add", "nle_batch_finalize", "nle_batch_layout",
    "nle_batch_solve", "nle_set_fibres", "nle_set_active_tension", "nle_set_pressure",
    "nle_set_robin", "nle_set_traction_follower", "nle_upload_mesh_mixed", "nle_block_diag", "nle_pc_apply", "nle_batch_autotune",
    "nle_set_inertia", "nle_newmark_predict", "nle_newmark_correct", "nle_amg_levels",
    "nle_set_robin_damping", "nle_set_step_velocity", "nle_jv_noalloc", "nle_upload_mesh_mixed_p0",
    "nle_schur_apply", "nle_simple_diag", "nle_set_fibre_frame", "nle_batch_set_tail",
]


class NleError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class nle_allocator(ctypes.Structure):
    _fields_ = [("alloc", ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)),
                ("free", ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)),
                ("user", ctypes.c_void_p)]


class nle_solver_opts(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in (
        "precision", "ksp_type", "orth", "pc", "restart", "ksp_max_it", "snes_max_it",
        "ew_version", "qn_m", "h0", "check_every", "cg_launches")] + [
        (n, ctypes.c_double) for n in (
            "ksp_rtol", "ksp_atol", "ew_rtol0", "ew_rtolmax", "ew_rtolmin", "ew_gamma",
            "ew_alpha", "ew_alpha2", "ew_threshold", "ink_ksp_atol", "snes_rtol", "snes_atol",
            "h0_rtol", "h0_atol", "curvature_eps")] + [
        ("h0_refresh", ctypes.c_int32), ("jac_lag", ctypes.c_int32),
        ("h0_ew", ctypes.c_int32), ("schur", ctypes.c_int32)]


class nle_report(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("nit", ctypes.c_int32),
                ("lit_total", ctypes.c_int64), ("n_jv", ctypes.c_int64),
                ("n_residual", ctypes.c_int64), ("bfgs_skipped", ctypes.c_int32),
                ("hist_cap", ctypes.c_int32), ("rnorm0", ctypes.c_double),
                ("rnorm_final", ctypes.c_double), ("t_ms", ctypes.c_double),
                ("rnorm_hist", ctypes.POINTER(ctypes.c_double)),
                ("eta_hist", ctypes.POINTER(ctypes.c_double)),
                ("lit_hist", ctypes.POINTER(ctypes.c_int32)),
                ("cutbacks", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libnlelast.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "nle_create": (I32, [ctypes.POINTER(P), I32, P, ctypes.POINTER(nle_allocator)]),
        "nle_destroy": (None, [P]),
        "nle_last_error": (ctypes.c_char_p, [P]),
        "nle_version": (ctypes.c_char_p, []),
        "nle_set_block_size": (I32, [P, I32]),
        "nle_upload_mesh": (I32, [P, I64, P, I64, I32, P]),
        "nle_set_material": (I32, [P, I32, P, I32]),
        "nle_set_dirichlet": (I32, [P, I64, P, P]),
        "nle_set_traction": (I32, [P, I64, P, P]),
        "nle_set_body_force": (I32, [P, P]),
        "nle_set_load_scale": (I32, [P, D]),
        "nle_set_fibres": (I32, [P, P]),
        "nle_upload_mesh_mixed": (I32, [P, I64, P, I64, P, I64, P]),
        "nle_set_active_tension": (I32, [P, D]),
        "nle_set_pressure": (I32, [P, I64, P, D]),
        "nle_set_robin": (I32, [P, I64, P, D, D]),
        "nle_set_traction_follower": (I32, [P, I64, P, P]),
        "nle_set_inertia": (I32, [P, D, D, P]),
        "nle_amg_levels": (I32, [P, P, P, I32]),
        "nle_newmark_predict": (I32, [P, D, D, D, P, P, P, P, P]),
        "nle_set_robin_damping": (I32, [P, D, D]),
        "nle_set_step_velocity": (I32, [P, D, P]),
        "nle_newmark_correct": (I32, [P, D, D, D, P, P, P, P]),
        "nle_lift": (I32, [P, P]),
        "nle_residual": (I32, [P, P, P, ctypes.POINTER(D)]),
        "nle_linearize": (I32, [P, P, I32]),
        "nle_jv": (I32, [P, P, P, I32]),
        "nle_jv_noalloc": (I32, [P, P, P, I32]),
        "nle_upload_mesh_mixed_p0": (I32, [P, I64, P, I64, P]),
        "nle_schur_apply": (I32, [P, I32, I32, I32, P, P]),
        "nle_simple_diag": (I32, [P, P]),
        "nle_set_fibre_frame": (I32, [P, P, P]),
        "nle_diag": (I32, [P, P]),
        "nle_block_diag": (I32, [P, P]),
        "nle_pc_apply": (I32, [P, I32, I32, P, P]),
        "nle_energy": (I32, [P, P, ctypes.POINTER(D)]),
        "nle_default_opts": (None, [I32, ctypes.POINTER(nle_solver_opts)]),
        "nle_solve_nk": (I32, [P, P, ctypes.POINTER(nle_solver_opts), ctypes.POINTER(nle_report)]),
        "nle_solve_ink": (I32, [P, P, ctypes.POINTER(nle_solver_opts), ctypes.POINTER(nle_report)]),
        "nle_solve_bfgs": (I32, [P, P, ctypes.POINTER(nle_solver_opts), ctypes.POINTER(nle_report)]),
        "nle_partition_info": (I32, [P, ctypes.POINTER(I64)]),
        "nle_batch_create": (I32, [ctypes.POINTER(P), I32, P, ctypes.POINTER(nle_allocator)]),
        "nle_batch_destroy": (None, [P]),
        "nle_batch_last_error": (ctypes.c_char_p, [P]),
        "nle_batch_add": (I32, [P, I64, P, I64, P, I32, P, I32, I64, P, P, I64, P, P, I32, P,
                                ctypes.POINTER(I32)]),
        "nle_batch_finalize": (I32, [P]),
        "nle_batch_autotune": (I32, [P, I32, D, P]),
        "nle_batch_set_tail": (I32, [P, I32, I32, I32]),
        "nle_batch_layout": (I32, [P, ctypes.POINTER(I64)]),
        "nle_batch_solve": (I32, [P, I32, ctypes.POINTER(nle_solver_opts), P,
                                  ctypes.POINTER(nle_report), ctypes.POINTER(D)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


class Context:
    """An nle_ctx bound to one device and torch's current stream on it."""

    def __init__(self, device: int = 0, use_torch_allocator: bool = True):
        import torch

        self.torch = torch
        self.device = torch.device("cuda", device)
        L = lib()
        self._keep = []
        alloc_p = None
        if use_torch_allocator:
            dev = device

            @ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
            def _alloc(nbytes, user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), dev)
                except Exception:  # noqa: BLE001 - the C side reports OOM
                    return None

            @ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
            def _free(ptr, user):
                if ptr:
                    torch.cuda.caching_allocator_delete(ptr)

            al = nle_allocator(_alloc, _free, None)
            self._keep += [_alloc, _free, al]
            alloc_p = ctypes.pointer(al)
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        st = L.nle_create(ctypes.byref(h), device, ctypes.c_void_p(self.stream.cuda_stream), alloc_p)
        if st != NLE_OK:
            raise NleError(st, "nle_create failed")
        self.handle = h
        self.n_nodes = 0
        self.n_elems = 0
        self.n_press = 0

    @property
    def n_dofs(self) -> int:
        """Unknowns: 3 per node, plus one per pressure node on mixed meshes."""
        return 3 * self.n_nodes + self.n_press

    def close(self):
        if getattr(self, "handle", None):
            lib().nle_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    def check(self, st: int) -> int:
        if st < 0:
            msg = lib().nle_last_error(self.handle)
            raise NleError(st, msg.decode() if msg else "")
        return st

    def vec(self, t, dtype=None, n=None):
        torch = self.torch
        if not isinstance(t, torch.Tensor) or t.device != self.device or not t.is_contiguous():
            raise ValueError("expected a contiguous tensor on the context's device")
        if dtype is not None and t.dtype != dtype:
            raise ValueError(f"expected dtype {dtype}, got {t.dtype}")
        n = self.n_dofs if n is None else n
        if t.numel() != n:
            raise ValueError(f"expected {n} entries, got {t.numel()}")
        return ctypes.c_void_p(t.data_ptr())


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(ctypes.c_void_p)


# ---- C-ABI mirror (same names) ------------------------------------------------
def nle_version() -> str:
    return lib().nle_version().decode()


def nle_create(device: int = 0, use_torch_allocator: bool = True) -> Context:
    return Context(device, use_torch_allocator)


def nle_destroy(ctx: Context) -> None:
    ctx.close()


def nle_last_error(ctx: Context) -> str:
    return lib().nle_last_error(ctx.handle).decode()


def nle_set_block_size(ctx: Context, elems_per_block: int) -> None:
    ctx.check(lib().nle_set_block_size(ctx.handle, int(elems_per_block)))


def nle_upload_mesh(ctx: Context, X, conn) -> None:
    X, px = _host(X, np.float64)
    conn, pc = _host(conn, np.int32)
    if X.ndim != 2 or X.shape[1] != 3 or conn.ndim != 2:
        raise ValueError("X must be (n, 3) and conn (n_e, k)")
    ctx.check(lib().nle_upload_mesh(ctx.handle, X.shape[0], px, conn.shape[0], conn.shape[1], pc))
    ctx.n_nodes = X.shape[0]
    ctx.n_elems = conn.shape[0]
    ctx.n_press = 0


def nle_upload_mesh_mixed(ctx: Context, X, conn, n_pnodes: int, pconn) -> None:
    X, px = _host(X, np.float64)
    conn, pc = _host(conn, np.int32)
    pconn, ppc = _host(pconn, np.int32)
    if X.ndim != 2 or X.shape[1] != 3 or conn.shape[1:] != (10,) or pconn.shape != (conn.shape[0], 4):
        raise ValueError("X must be (n, 3), conn (n_e, 10) and pconn (n_e, 4)")
    ctx.check(lib().nle_upload_mesh_mixed(ctx.handle, X.shape[0], px, conn.shape[0], pc,
                                          int(n_pnodes), ppc))
    ctx.n_nodes = X.shape[0]
    ctx.n_elems = conn.shape[0]
    ctx.n_press = int(n_pnodes)


def nle_upload_mesh_mixed_p0(ctx: Context, X, conn) -> None:
    """Quadratic displacement, one pressure unknown per element (P2-P0)."""
    X, px = _host(X, np.float64)
    conn, pc = _host(conn, np.int32)
    if X.ndim != 2 or X.shape[1] != 3 or conn.shape[1:] != (10,):
        raise ValueError("X must be (n, 3) and conn (n_e, 10)")
    ctx.check(lib().nle_upload_mesh_mixed_p0(ctx.handle, X.shape[0], px, conn.shape[0], pc))
    ctx.n_nodes = X.shape[0]
    ctx.n_elems = conn.shape[0]
    ctx.n_press = conn.shape[0]


def nle_schur_apply(ctx: Context, pc: int, schur: int, x, y, prec: int = NLE_FP64) -> None:
    T = ctx.torch.float32 if prec == NLE_FP32 else ctx.torch.float64
    ctx.check(lib().nle_schur_apply(ctx.handle, int(pc), int(schur), int(prec), ctx.vec(x, T),
                                    ctx.vec(y, T)))


def nle_simple_diag(ctx: Context, s) -> None:
    """s: float64 device tensor of n_elems entries."""
    ctx.check(lib().nle_simple_diag(ctx.handle, ctx.vec(s, ctx.torch.float64, n=ctx.n_elems)))


def nle_set_material(ctx: Context, kind: int, params) -> None:
    p, pp = _host(params, np.float64)
    ctx.check(lib().nle_set_material(ctx.handle, int(kind), pp, p.size))


def nle_set_dirichlet(ctx: Context, dofs, values) -> None:
    d, pd = _host(dofs, np.int64)
    v, pv = _host(values, np.float64)
    if d.shape != v.shape:
        raise ValueError("dofs and values differ in length")
    ctx.check(lib().nle_set_dirichlet(ctx.handle, d.size, pd, pv))


def nle_set_traction(ctx: Context, tri, t) -> None:
    f, pf = _host(tri, np.int32)
    tt, pt = _host(t, np.float64)
    ctx.check(lib().nle_set_traction(ctx.handle, f.shape[0] if f.size else 0, pf, pt))


def nle_set_fibres(ctx: Context, fib) -> None:
    f, pf = _host(fib, np.float64)
    if f.shape != (ctx.n_elems, 3):
        raise ValueError(f"expected fibres of shape ({ctx.n_elems}, 3)")
    ctx.check(lib().nle_set_fibres(ctx.handle, pf))


def nle_set_fibre_frame(ctx: Context, fib, sheet) -> None:
    f, pf = _host(fib, np.float64)
    sh, ps = _host(sheet, np.float64)
    if f.shape != (ctx.n_elems, 3) or sh.shape != (ctx.n_elems, 3):
        raise ValueError(f"expected fibres and sheets of shape ({ctx.n_elems}, 3)")
    ctx.check(lib().nle_set_fibre_frame(ctx.handle, pf, ps))


def nle_set_active_tension(ctx: Context, gamma: float) -> None:
    ctx.check(lib().nle_set_active_tension(ctx.handle, float(gamma)))


def nle_set_pressure(ctx: Context, tri, p: float) -> None:
    f, pf = _host(tri, np.int32)
    ctx.check(lib().nle_set_pressure(ctx.handle, f.shape[0] if f.size else 0, pf, float(p)))


def nle_set_traction_follower(ctx: Context, tri, t) -> None:
    f, pf = _host(tri, np.int32)
    tt, pt = _host(t, np.float64)
    ctx.check(lib().nle_set_traction_follower(ctx.handle, f.shape[0] if f.size else 0, pf, pt))


def nle_set_robin(ctx: Context, tri, k_perp: float, k_par: float) -> None:
    f, pf = _host(tri, np.int32)
    ctx.check(lib().nle_set_robin(ctx.handle, f.shape[0] if f.size else 0, pf, float(k_perp),
                                  float(k_par)))


def nle_set_inertia(ctx: Context, rho: float, coef: float, u_tilde=None) -> None:
    """Inertia of an implicit step: coef M (u - u_tilde) with the lumped mass of
    density rho (u_tilde: float64 device tensor; rho or coef 0 switches it off)."""
    pu = None if u_tilde is None else ctx.vec(u_tilde, ctx.torch.float64)
    ctx.check(lib().nle_set_inertia(ctx.handle, float(rho), float(coef), pu))


def nle_newmark_predict(ctx: Context, dt: float, beta: float, u, v, a, u_tilde,
                        gamma: float = 0.5, v_tilde=None) -> None:
    """u_tilde = u + dt v + dt^2 (1/2 - beta) a; v_tilde = v + dt (1 - gamma) a if given."""
    T = ctx.torch.float64
    pv = None if v_tilde is None else ctx.vec(v_tilde, T)
    ctx.check(lib().nle_newmark_predict(ctx.handle, float(dt), float(beta), float(gamma),
                                        ctx.vec(u, T), ctx.vec(v, T), ctx.vec(a, T),
                                        ctx.vec(u_tilde, T), pv))


def nle_set_robin_damping(ctx: Context, c_perp: float, c_par: float) -> None:
    """Dashpots on the spring faces, acting on the step velocity (nle_set_step_velocity)."""
    ctx.check(lib().nle_set_robin_damping(ctx.handle, float(c_perp), float(c_par)))


def nle_set_step_velocity(ctx: Context, cv: float, v_tilde=None) -> None:
    """The implicit step's velocity v(u) = v_tilde + cv (u - u_tilde); cv = 0 switches it off."""
    pv = None if v_tilde is None else ctx.vec(v_tilde, ctx.torch.float64)
    ctx.check(lib().nle_set_step_velocity(ctx.handle, float(cv), pv))


def nle_newmark_correct(ctx: Context, dt: float, beta: float, gamma: float, u, u_tilde, v,
                        a) -> None:
    """In place: a' = (u - u_tilde) / (beta dt^2), v += dt ((1 - gamma) a + gamma a'), a = a'."""
    T = ctx.torch.float64
    ctx.check(lib().nle_newmark_correct(ctx.handle, float(dt), float(beta), float(gamma),
                                        ctx.vec(u, T), ctx.vec(u_tilde, T), ctx.vec(v, T),
                                        ctx.vec(a, T)))


def nle_set_body_force(ctx: Context, f) -> None:
    ff, pf = _host(f, np.float64)
    ctx.check(lib().nle_set_body_force(ctx.handle, pf))


def nle_set_load_scale(ctx: Context, s: float) -> None:
    ctx.check(lib().nle_set_load_scale(ctx.handle, float(s)))


def nle_lift(ctx: Context, u) -> None:
    ctx.check(lib().nle_lift(ctx.handle, ctx.vec(u, ctx.torch.float64)))


def nle_residual(ctx: Context, u, r, norm: bool = True) -> Optional[float]:
    """r = f_int(u) - s f_ext; returns ||r|| (synchronising) when norm=True.
    Raises NleError on usage errors; an inverted element raises too."""
    T = ctx.torch.float64
    if norm:
        rn = ctypes.c_double()
        st = lib().nle_residual(ctx.handle, ctx.vec(u, T), ctx.vec(r, T), ctypes.byref(rn))
        if st == NLE_DIVERGED_INVERTED:
            raise NleError(st, nle_last_error(ctx))
        ctx.check(st)
        return rn.value
    ctx.check(lib().nle_residual(ctx.handle, ctx.vec(u, T), ctx.vec(r, T), None))
    return None


def nle_linearize(ctx: Context, u, prec: int = NLE_FP64) -> None:
    ctx.check(lib().nle_linearize(ctx.handle, ctx.vec(u, ctx.torch.float64), int(prec)))


def nle_jv(ctx: Context, v, y, prec: int = NLE_FP64) -> None:
    T = ctx.torch.float32 if prec == NLE_FP32 else ctx.torch.float64
    ctx.check(lib().nle_jv(ctx.handle, ctx.vec(v, T), ctx.vec(y, T), int(prec)))


def nle_jv_noalloc(ctx: Context, v, y, prec: int = NLE_FP64) -> None:
    """y = J v through the allocation-free entry point (fixed per-device
    workspace; same result as nle_jv)."""
    T = ctx.torch.float32 if prec == NLE_FP32 else ctx.torch.float64
    ctx.check(lib().nle_jv_noalloc(ctx.handle, ctx.vec(v, T), ctx.vec(y, T), int(prec)))


def nle_diag(ctx: Context, d) -> None:
    ctx.check(lib().nle_diag(ctx.handle, ctx.vec(d, ctx.torch.float64)))


def nle_block_diag(ctx: Context, b) -> None:
    """b: float64 device tensor of 6 n_nodes entries (xx, yy, zz, xy, yz, xz per node)."""
    if not (b.is_cuda and b.dtype == ctx.torch.float64 and b.is_contiguous()
            and b.numel() == 6 * ctx.n_nodes):
        raise ValueError("expected a contiguous float64 CUDA tensor of 6 n_nodes entries")
    ctx.check(lib().nle_block_diag(ctx.handle, ctypes.c_void_p(b.data_ptr())))


def nle_amg_levels(ctx: Context) -> list:
    """Unknowns per level of the multigrid hierarchy (finest first)."""
    n = ctypes.c_int32()
    sizes = (ctypes.c_int64 * 16)()
    ctx.check(lib().nle_amg_levels(ctx.handle, ctypes.byref(n), sizes, 16))
    return [int(sizes[i]) for i in range(min(n.value, 16))]


def nle_pc_apply(ctx: Context, pc: int, x, y, prec: int = NLE_FP64) -> None:
    T = ctx.torch.float32 if prec == NLE_FP32 else ctx.torch.float64
    ctx.check(lib().nle_pc_apply(ctx.handle, int(pc), int(prec), ctx.vec(x, T), ctx.vec(y, T)))


def nle_energy(ctx: Context, u) -> float:
    out = ctypes.c_double()
    ctx.check(lib().nle_energy(ctx.handle, ctx.vec(u, ctx.torch.float64), ctypes.byref(out)))
    return out.value


def nle_default_opts(method: int) -> nle_solver_opts:
    o = nle_solver_opts()
    lib().nle_default_opts(int(method), ctypes.byref(o))
    return o


def _solve(fn, ctx: Context, u, opts: nle_solver_opts, hist_cap: int):
    rep = nle_report()
    rh = (ctypes.c_double * hist_cap)()
    eh = (ctypes.c_double * hist_cap)()
    lh = (ctypes.c_int32 * hist_cap)()
    rep.hist_cap = hist_cap
    rep.rnorm_hist = rh
    rep.eta_hist = eh
    rep.lit_hist = lh
    st = fn(ctx.handle, ctx.vec(u, ctx.torch.float64), ctypes.byref(opts), ctypes.byref(rep))
    ctx.check(st)
    k = min(rep.nit + 1, hist_cap)
    return st, dict(status=st, status_name=STATUS_NAMES.get(st, str(st)), nit=rep.nit,
                    lit_total=rep.lit_total, n_jv=rep.n_jv, n_residual=rep.n_residual,
                    bfgs_skipped=rep.bfgs_skipped, rnorm0=rep.rnorm0,
                    rnorm_final=rep.rnorm_final, t_ms=rep.t_ms,
                    rnorm_hist=list(rh[:k]), eta_hist=list(eh[:k]), lit_hist=list(lh[:k]))


def nle_solve_nk(ctx: Context, u, opts: nle_solver_opts, hist_cap: int = 2048):
    return _solve(lib().nle_solve_nk, ctx, u, opts, hist_cap)


def nle_solve_ink(ctx: Context, u, opts: nle_solver_opts, hist_cap: int = 2048):
    return _solve(lib().nle_solve_ink, ctx, u, opts, hist_cap)


def nle_solve_bfgs(ctx: Context, u, opts: nle_solver_opts, hist_cap: int = 2048):
    return _solve(lib().nle_solve_bfgs, ctx, u, opts, hist_cap)


def nle_partition_info(ctx: Context) -> dict:
    info = (ctypes.c_int64 * 8)()
    ctx.check(lib().nle_partition_info(ctx.handle, info))
    keys = ["n_blocks", "max_elems_per_block", "max_nodes_per_block", "block_node_slots",
            "shared_nodes", "merge_slots", "lds_bytes_fp64_jv", "lds_bytes_fp32_jv"]
    return dict(zip(keys, list(info)))


# ---- batched solves -------------------------------------------------------------
class Batch:
    """An nle_batch: many independent problems solved together on one device."""

    def __init__(self, device: int = 0, use_torch_allocator: bool = True):
        import torch

        self.torch = torch
        self.device = torch.device("cuda", device)
        L = lib()
        self._keep = []
        alloc_p = None
        if use_torch_allocator:
            dev = device

            @ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
            def _alloc(nbytes, user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), dev)
                except Exception:  # noqa: BLE001 - the C side reports OOM
                    return None

            @ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
            def _free(ptr, user):
                if ptr:
                    torch.cuda.caching_allocator_delete(ptr)

            al = nle_allocator(_alloc, _free, None)
            self._keep += [_alloc, _free, al]
            alloc_p = ctypes.pointer(al)
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        st = L.nle_batch_create(ctypes.byref(h), device, ctypes.c_void_p(self.stream.cuda_stream),
                                alloc_p)
        if st != NLE_OK:
            raise NleError(st, "nle_batch_create failed")
        self.handle = h
        self.n_inst = 0
        self.offsets = None

    def close(self):
        if getattr(self, "handle", None):
            lib().nle_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    def check(self, st: int) -> int:
        if st < 0:
            msg = lib().nle_batch_last_error(self.handle)
            raise NleError(st, msg.decode() if msg else "")
        return st


def nle_batch_create(device: int = 0, use_torch_allocator: bool = True) -> Batch:
    return Batch(device, use_torch_allocator)


def nle_batch_destroy(b: Batch) -> None:
    b.close()


def nle_batch_last_error(b: Batch) -> str:
    return lib().nle_batch_last_error(b.handle).decode()


def nle_batch_add(b: Batch, X, conn, kind: int, params, dofs, values, tri, traction,
                  scales) -> int:
    X, px = _host(X, np.float64)
    conn, pc = _host(conn, np.int32)
    p, pp = _host(params, np.float64)
    d, pd = _host(dofs, np.int64)
    v, pv = _host(values, np.float64)
    f, pf = _host(tri, np.int32)
    t, pt = _host(traction, np.float64)
    s, ps = _host(scales, np.float64)
    out = ctypes.c_int32()
    b.check(lib().nle_batch_add(b.handle, X.shape[0], px, conn.shape[0], pc, int(kind), pp,
                                p.size, d.size, pd, pv, f.shape[0] if f.size else 0, pf, pt,
                                s.size, ps, ctypes.byref(out)))
    b.n_inst = out.value + 1
    return out.value


def nle_batch_finalize(b: Batch) -> None:
    b.check(lib().nle_batch_finalize(b.handle))
    off = (ctypes.c_int64 * (b.n_inst + 1))()
    b.check(lib().nle_batch_layout(b.handle, off))
    b.offsets = np.array(off[:], dtype=np.int64)


def nle_batch_autotune(b: Batch, prec: int = NLE_FP32, budget_ms: float = 200.0) -> int:
    """Pick the element-block size of the batch's partition; returns it."""
    out = ctypes.c_int32()
    b.check(lib().nle_batch_autotune(b.handle, int(prec), float(budget_ms), ctypes.byref(out)))
    return out.value


def nle_batch_set_tail(b: Batch, max_tail: int, max_its: int = 0, pc: int = NLE_PC_AMG) -> None:
    """Finish alone, with preconditioner pc, the last max_tail unfinished
    instances and (NK, iNK) any instance whose batched CG solve takes more
    than max_its iterations in a round (0 turns either rule off)."""
    b.check(lib().nle_batch_set_tail(b.handle, int(max_tail), int(max_its), int(pc)))


def nle_batch_layout(b: Batch):
    return b.offsets


def nle_batch_solve(b: Batch, method: int, opts: nle_solver_opts, u):
    """Solve all instances; u is the concatenated float64 device vector.
    Returns (status, list of per-instance report dicts, t_ms)."""
    torch = b.torch
    n = int(3 * b.offsets[-1])
    if (not isinstance(u, torch.Tensor) or u.device != b.device or u.dtype != torch.float64
            or not u.is_contiguous() or u.numel() != n):
        raise ValueError(f"expected a contiguous float64 tensor of {n} entries on the device")
    reps = (nle_report * b.n_inst)()
    tms = ctypes.c_double()
    st = b.check(lib().nle_batch_solve(b.handle, int(method), ctypes.byref(opts),
                                       ctypes.c_void_p(u.data_ptr()), reps, ctypes.byref(tms)))
    out = [dict(status=r.status, status_name=STATUS_NAMES.get(r.status, str(r.status)),
                nit=r.nit, lit_total=r.lit_total, n_jv=r.n_jv, n_residual=r.n_residual,
                cutbacks=r.cutbacks, bfgs_skipped=r.bfgs_skipped, rnorm0=r.rnorm0,
                rnorm_final=r.rnorm_final)
           for r in reps]
    return st, out, tms.value
