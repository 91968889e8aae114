"""Hyperelastic laws: strain energy Psi(F) and first Piola stress P(F).

All functions are vectorised over leading axes (F has shape (..., 3, 3))
and accept complex input, so complex-step differentiation can be applied
to them (the tangent dP/dF is taken that way in fem.py; Psi is used to
check P).

Paper, Sec. 2: P = dPsi/dF with F = I + grad u, J = det F; the almost
incompressible split Psi = Psi_sol(Fbar) + Psi_vol(J), Fbar = J^(-1/3) F.

M1  compressible neo-Hookean (the Cook workloads' law, with Lame mu, lambda):
      Psi = mu/2 (I1 - 3) - mu ln J + lambda/2 (ln J)^2
      P   = mu (F - F^-T) + lambda ln J F^-T
M2  the paper's Cook law (Sec. 4, "Cook test"), C1 = mu/2, kappa = lambda + 2 mu / 3:
      Psi = C1 (tr(Fbar^T Fbar) - 3) + c_vol kappa (J^2 - 1 - 2 ln J)
      P   = mu J^(-2/3) (F - I1/3 F^-T) + 2 c_vol kappa (J^2 - 1) F^-T
    The printed law has c_vol = 1; we use c_vol = 1/4 by default, the value
    for which the small-strain limit has bulk modulus kappa (Lame lambda
    recovered exactly).  c_vol is the third parameter.
M4  the cardiac-like law: an exponential isotropic term of Holzapfel-Ogden
    type, an exponential fibre term active in fibre tension only, a volumetric
    penalty, and the active stress of Sec. 4 ("Heartbeat test": P_act =
    gamma (F f) (x) f / |F f|), which is the gradient of gamma |F f|:
      Psi = a/(2b) (exp(b (J^(-2/3) I1 - 3)) - 1)
            + af/(2bf) (exp(bf (I4 - 1)^2) - 1) [I4 > 1]
            + kappa/2 (J - 1)^2 + gamma sqrt(I4),        I4 = |F f|^2
    params = (a, b, af, bf, kappa, gamma, fib) with fib the unit fibre
    direction(s), shape (..., 3) broadcasting against F.  The paper's own
    Guccione law needs constants it does not print; this law and its
    constants are a stated substitute.
M6  the paper's heartbeat law (Sec. 4, "Heartbeat test"), Guccione's
    exponential in the fibre frame plus the printed volumetric term and the
    active stress:
      Psi = C/2 (exp(Q) - 1) + B/2 (J - 1) ln J + gamma sqrt(I4),
      Q   = b_ff E_ff^2 + b_ss E_ss^2 + b_nn E_nn^2 + b_fs (E_fs^2 + E_sf^2)
            + b_fn (E_fn^2 + E_nf^2) + b_sn (E_sn^2 + E_ns^2),
    E = (F^T F - I)/2, E_ab = (E a).b in the orthonormal frame {f, s, n}.
    With Eb the frame components and bm the symmetric matrix of the b's,
    S = R (C e^Q bm o Eb) R^T (R = [f s n], o the entrywise product) is
    dPsi/dE, so P = F S + B/2 (J ln J + J - 1) F^-T + gamma (F f)(x)f/|F f|.
    params = (C, b_ff, b_ss, b_nn, b_fs, b_fn, b_sn, B, gamma, fib, sheet):
    the unit fibre f and sheet s per element (n = f x s).  The constants are
    the caller's (the paper refers to Guccione's paper for them).
"""

from __future__ import annotations

import numpy as np

M1 = "M1"
M2 = "M2"
M4 = "M4"
M6 = "M6"


def _det(F):
    return (F[..., 0, 0] * (F[..., 1, 1] * F[..., 2, 2] - F[..., 1, 2] * F[..., 2, 1])
            - F[..., 0, 1] * (F[..., 1, 0] * F[..., 2, 2] - F[..., 1, 2] * F[..., 2, 0])
            + F[..., 0, 2] * (F[..., 1, 0] * F[..., 2, 1] - F[..., 1, 1] * F[..., 2, 0]))


def _cofactor(F):
    """cof F = det(F) F^-T, written out (valid for complex F)."""
    C = np.empty_like(F)
    C[..., 0, 0] = F[..., 1, 1] * F[..., 2, 2] - F[..., 1, 2] * F[..., 2, 1]
    C[..., 0, 1] = F[..., 1, 2] * F[..., 2, 0] - F[..., 1, 0] * F[..., 2, 2]
    C[..., 0, 2] = F[..., 1, 0] * F[..., 2, 1] - F[..., 1, 1] * F[..., 2, 0]
    C[..., 1, 0] = F[..., 0, 2] * F[..., 2, 1] - F[..., 0, 1] * F[..., 2, 2]
    C[..., 1, 1] = F[..., 0, 0] * F[..., 2, 2] - F[..., 0, 2] * F[..., 2, 0]
    C[..., 1, 2] = F[..., 0, 1] * F[..., 2, 0] - F[..., 0, 0] * F[..., 2, 1]
    C[..., 2, 0] = F[..., 0, 1] * F[..., 1, 2] - F[..., 0, 2] * F[..., 1, 1]
    C[..., 2, 1] = F[..., 0, 2] * F[..., 1, 0] - F[..., 0, 0] * F[..., 1, 2]
    C[..., 2, 2] = F[..., 0, 0] * F[..., 1, 1] - F[..., 0, 1] * F[..., 1, 0]
    return C


def det(F):
    return _det(F)


def inv_transpose(F):
    """F^-T = cof F / det F."""
    return _cofactor(F) / _det(F)[..., None, None]


def _fibre_terms(F, params):
    """Ff = F f, I4 = |F f|^2 and the fibre direction (M4)."""
    f = np.asarray(params[6], dtype=np.float64)
    Ff = np.einsum("...ij,...j->...i", F, f)
    I4 = np.einsum("...i,...i->...", Ff, Ff)
    return f, Ff, I4


def _guccione_frame(F, params):
    """R = [f s n] (..., 3, 3), the frame components Eb = R^T E R of
    E = (F^T F - I)/2, and the symmetric coefficient matrix bm."""
    f = np.asarray(params[9], dtype=np.float64)
    sh = np.asarray(params[10], dtype=np.float64)
    n = np.cross(f, sh)
    R = np.stack([f, sh, n], axis=-1)  # columns f, s, n
    C = np.einsum("...ki,...kj->...ij", F, F)
    E = 0.5 * (C - np.eye(3))
    Eb = np.einsum("...ai,...ij,...jb->...ab", np.swapaxes(R, -1, -2), E, R)
    bff, bss, bnn, bfs, bfn, bsn = (float(x) for x in params[1:7])
    bm = np.array([[bff, bfs, bfn], [bfs, bss, bsn], [bfn, bsn, bnn]])
    return R, Eb, bm


def energy(kind: str, F, params):
    """Strain energy density Psi(F)."""
    if kind == M6:
        Cc, B, gamma = float(params[0]), float(params[7]), float(params[8])
        _, Eb, bm = _guccione_frame(F, params)
        Q = np.einsum("ab,...ab->...", bm, Eb * Eb)
        J = _det(F)
        f = np.asarray(params[9], dtype=np.float64)
        Ff = np.einsum("...ij,...j->...i", F, f)
        I4 = np.einsum("...i,...i->...", Ff, Ff)
        return 0.5 * Cc * (np.exp(Q) - 1.0) + 0.5 * B * (J - 1.0) * np.log(J) + gamma * np.sqrt(I4)
    if kind == M4:
        a, b, af, bf, kappa, gamma = (float(x) for x in params[:6])
        J = _det(F)
        I1 = np.einsum("...ij,...ij->...", F, F)
        _, _, I4 = _fibre_terms(F, params)
        iso = a / (2.0 * b) * (np.exp(b * (J ** (-2.0 / 3.0) * I1 - 3.0)) - 1.0)
        fib = np.where(np.real(I4) > 1.0, af / (2.0 * bf) * (np.exp(bf * (I4 - 1.0) ** 2) - 1.0), 0.0)
        return iso + fib + 0.5 * kappa * (J - 1.0) ** 2 + gamma * np.sqrt(I4)
    J = _det(F)
    I1 = np.einsum("...ij,...ij->...", F, F)
    lnJ = np.log(J)
    if kind == M1:
        mu, lam = params[0], params[1]
        return 0.5 * mu * (I1 - 3.0) - mu * lnJ + 0.5 * lam * lnJ ** 2
    if kind == M2:
        mu, lam = params[0], params[1]
        c_vol = params[2] if len(params) > 2 else 0.25
        kappa = lam + 2.0 * mu / 3.0
        return 0.5 * mu * (J ** (-2.0 / 3.0) * I1 - 3.0) + c_vol * kappa * (J ** 2 - 1.0 - 2.0 * lnJ)
    raise ValueError(f"unknown material {kind}")


def piola(kind: str, F, params):
    """First Piola-Kirchhoff stress P(F) = dPsi/dF."""
    J = _det(F)
    FiT = inv_transpose(F)
    if kind == M6:
        # dPsi/dEb = C e^Q (bm o Eb) (Q counts each off-diagonal pair twice),
        # S = R (dPsi/dEb) R^T, P = F S; d[(J - 1) ln J]/dJ = ln J + 1 - 1/J
        Cc, B, gamma = float(params[0]), float(params[7]), float(params[8])
        R, Eb, bm = _guccione_frame(F, params)
        Q = np.einsum("ab,...ab->...", bm, Eb * Eb)
        Sb = (Cc * np.exp(Q))[..., None, None] * (bm * Eb)
        S = np.einsum("...ia,...ab,...jb->...ij", R, Sb, R)
        f = np.asarray(params[9], dtype=np.float64)
        Ff = np.einsum("...ij,...j->...i", F, f)
        I4 = np.einsum("...i,...i->...", Ff, Ff)
        act = (gamma / np.sqrt(I4))[..., None, None] * np.einsum(
            "...i,...j->...ij", Ff, np.broadcast_to(f, Ff.shape))
        vol = (0.5 * B * (J * np.log(J) + J - 1.0))[..., None, None] * FiT
        return np.einsum("...ik,...kj->...ij", F, S) + vol + act
    if kind == M4:
        # d(J^-2/3 I1)/dF = J^-2/3 (2F - 2/3 I1 F^-T), dI4/dF = 2 (Ff) (x) f,
        # dJ/dF = J F^-T, d sqrt(I4)/dF = (Ff) (x) f / sqrt(I4)
        a, b, af, bf, kappa, gamma = (float(x) for x in params[:6])
        I1 = np.einsum("...ij,...ij->...", F, F)
        f, Ff, I4 = _fibre_terms(F, params)
        j23 = J ** (-2.0 / 3.0)
        iso = (a * np.exp(b * (j23 * I1 - 3.0)) * j23)[..., None, None] * (
            F - (I1 / 3.0)[..., None, None] * FiT)
        gf = np.where(np.real(I4) > 1.0, 2.0 * af * (I4 - 1.0) * np.exp(bf * (I4 - 1.0) ** 2), 0.0)
        hf = gf + gamma / np.sqrt(I4)
        fibre = hf[..., None, None] * np.einsum("...i,...j->...ij", Ff, np.broadcast_to(f, Ff.shape))
        vol = (kappa * (J - 1.0) * J)[..., None, None] * FiT
        return iso + fibre + vol
    if kind == M1:
        mu, lam = params[0], params[1]
        lnJ = np.log(J)
        return mu * (F - FiT) + (lam * lnJ)[..., None, None] * FiT
    if kind == M2:
        mu, lam = params[0], params[1]
        c_vol = params[2] if len(params) > 2 else 0.25
        kappa = lam + 2.0 * mu / 3.0
        I1 = np.einsum("...ij,...ij->...", F, F)
        iso = (mu * J ** (-2.0 / 3.0))[..., None, None] * (F - (I1 / 3.0)[..., None, None] * FiT)
        vol = (2.0 * c_vol * kappa * (J ** 2 - 1.0))[..., None, None] * FiT
        return iso + vol
    raise ValueError(f"unknown material {kind}")


def tangent(kind: str, F, params, h: float = 1e-30):
    """A[..., i, J, k, L] = dP_iJ / dF_kL by complex-step differentiation.

    Im P(F + i h E_kL) / h is the exact derivative up to rounding (no
    subtractive cancellation), for any real F where P is analytic.
    """
    F = np.asarray(F, dtype=np.float64)
    out = np.empty(F.shape[:-2] + (3, 3, 3, 3))
    Fc = F.astype(np.complex128)
    for k in range(3):
        for L in range(3):
            Fp = Fc.copy()
            Fp[..., k, L] += 1j * h
            out[..., :, :, k, L] = piola(kind, Fp, params).imag / h
    return out
