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
"""

from __future__ import annotations

import numpy as np

M1 = "M1"
M2 = "M2"


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


def energy(kind: str, F, params):
    """Strain energy density Psi(F)."""
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
