"""Plain FP64 reference implementations of the paper's solver components.

Used on small problems to check the iteration behaviour of the GPU solvers
(and pinned themselves against brute force in the tests).  Operators are
passed as callables so the same code runs on a dense matrix or on the
assembled tangent of fem.Problem.

Paper, Sec. 3 and App. A:
* NK: Newton with a Krylov inner solve, rtol 1e-6, atol 1e-10, full step.
* iNK: the same with the Eisenstat-Walker forcing term as relative
  tolerance (eta_0 = 0.1, eta_max = 0.1), atol 1e-14.
* BFGS: limited-memory inverse update applied by the two-loop recursion,
  H0 = one preconditioner application (BFGS-preonly) or an inexact Krylov
  solve with rtol 1e-2 (inexact BFGS), both built once from the tangent at
  the first iterate; full step.
* GMRES: right preconditioned, modified Gram-Schmidt, restart optional.
"""

from __future__ import annotations

import math
from typing import Callable, List, Optional

import numpy as np

GOLDEN = 0.5 * (1.0 + math.sqrt(5.0))


# ---------------------------------------------------------------- Krylov
def gmres(matvec: Callable, b: np.ndarray, precond: Optional[Callable] = None,
          rtol: float = 1e-6, atol: float = 1e-10, max_it: int = 10000,
          restart: Optional[int] = None, orth: str = "mgs"):
    """Right-preconditioned GMRES from a zero initial guess.

    Solves A x = b through A M^-1 y = b, x = M^-1 y; converged when the
    (unpreconditioned) residual norm is <= max(rtol ||b||, atol).  The
    Arnoldi step orthogonalises with modified Gram-Schmidt (orth='mgs') or
    classical Gram-Schmidt applied twice (orth='cgs2').  Returns
    (x, iterations, residual-norm history, converged flag).
    """
    M = precond if precond is not None else (lambda v: v)
    n = b.size
    m = n if restart is None else int(restart)
    x = np.zeros(n)
    bnorm = float(np.linalg.norm(b))
    ttol = max(rtol * bnorm, atol)
    hist = [bnorm]
    total = 0
    if bnorm <= ttol:
        return x, 0, hist, True
    while True:
        r = b - matvec(x) if total > 0 else b.copy()
        beta = float(np.linalg.norm(r))
        if beta <= ttol:
            return x, total, hist, True
        V = [r / beta]
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        k = 0
        done = False
        for j in range(m):
            w = matvec(M(V[j]))
            if orth == "mgs":
                for i in range(j + 1):
                    H[i, j] = np.dot(w, V[i])
                    w = w - H[i, j] * V[i]
            else:  # cgs2
                Vj = np.array(V)
                h1 = Vj @ w
                w = w - Vj.T @ h1
                h2 = Vj @ w
                w = w - Vj.T @ h2
                H[: j + 1, j] = h1 + h2
            H[j + 1, j] = float(np.linalg.norm(w))
            for i in range(j):  # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = math.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = (1.0, 0.0) if den == 0.0 else (H[j, j] / den, H[j + 1, j] / den)
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            k = j + 1
            hist.append(abs(g[j + 1]))
            if abs(g[j + 1]) <= ttol or total >= max_it:
                done = True
                break
            hn = float(np.linalg.norm(w))
            if hn == 0.0:  # happy breakdown
                done = True
                break
            V.append(w / hn)
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k]) if k > 0 else np.zeros(0)
        x = x + M(np.array(V[:k]).T @ y)
        if done:
            conv = hist[-1] <= ttol
            return x, total, hist, conv
        if total >= max_it:
            return x, total, hist, False


def cg(matvec: Callable, b: np.ndarray, precond: Optional[Callable] = None,
       rtol: float = 1e-6, atol: float = 1e-10, max_it: int = 10000):
    """Preconditioned conjugate gradients from zero; the stopping test is on
    the unpreconditioned residual, ||r|| <= max(rtol ||b||, atol)."""
    M = precond if precond is not None else (lambda v: v)
    x = np.zeros_like(b)
    r = b.copy()
    z = M(r)
    p = z.copy()
    rz = float(np.dot(r, z))
    ttol = max(rtol * float(np.linalg.norm(b)), atol)
    hist = [float(np.linalg.norm(r))]
    k = 0
    while hist[-1] > ttol and k < max_it:
        Ap = matvec(p)
        alpha = rz / float(np.dot(p, Ap))
        x += alpha * p
        r -= alpha * Ap
        z = M(r)
        rz_new = float(np.dot(r, z))
        p = z + (rz_new / rz) * p
        rz = rz_new
        k += 1
        hist.append(float(np.linalg.norm(r)))
    return x, k, hist, hist[-1] <= ttol


def minres(matvec: Callable, b: np.ndarray, precond: Optional[Callable] = None,
           rtol: float = 1e-6, atol: float = 1e-10, max_it: int = 10000):
    """Preconditioned MINRES (Paige & Saunders, SIAM J. Numer. Anal. 12, 1975;
    the Lanczos recurrence with Givens rotations as published) for symmetric, possibly
    indefinite A with an SPD preconditioner M, from a zero initial guess.

    The k-th iterate minimises ||b - A x||_{M^-1} over the Krylov space
    K_k(M^-1 A, M^-1 b).  The stopping test uses the true residual
    ||b - A x||_2 <= max(rtol ||b||, atol), evaluated explicitly here.
    Returns (x, iterations, residual-norm history, converged flag).
    """
    M = precond if precond is not None else (lambda v: v)
    n = b.size
    x = np.zeros(n)
    bnorm = float(np.linalg.norm(b))
    ttol = max(rtol * bnorm, atol)
    hist = [bnorm]
    if bnorm <= ttol:
        return x, 0, hist, True
    r1 = b.copy()
    y = M(r1)
    beta1 = float(np.sqrt(np.dot(r1, y)))
    oldb, beta, dbar, epsln, phibar = 0.0, beta1, 0.0, 0.0, beta1
    cs, sn = -1.0, 0.0
    w = np.zeros(n)
    w2 = np.zeros(n)
    r2 = r1.copy()
    k = 0
    while k < max_it:
        k += 1
        v = y / beta
        y = matvec(v)
        if k >= 2:
            y = y - (beta / oldb) * r1
        alfa = float(np.dot(v, y))
        y = y - (alfa / beta) * r2
        r1, r2 = r2, y
        y = M(r2)
        oldb, beta = beta, float(np.sqrt(np.dot(r2, y)))
        oldeps = epsln
        delta = cs * dbar + sn * alfa
        gbar = sn * dbar - cs * alfa
        epsln = sn * beta
        dbar = -cs * beta
        gamma = max(float(np.hypot(gbar, beta)), 1e-300)
        cs, sn = gbar / gamma, beta / gamma
        phi = cs * phibar
        phibar = sn * phibar
        w1, w2 = w2, w
        w = (v - oldeps * w1 - delta * w2) / gamma
        x = x + phi * w
        hist.append(float(np.linalg.norm(b - matvec(x))))
        if hist[-1] <= ttol or beta == 0.0:
            break
    return x, k, hist, hist[-1] <= ttol


# ---------------------------------------------------------------- EW
def ew_forcing(k: int, rnorm: float, rnorm_prev: float, linres_prev: float, eta_prev: float,
               version: int = 1, rtol0: float = 0.1, rtolmax: float = 0.1,
               gamma: float = 1.0, alpha: float = GOLDEN, alpha2: float = GOLDEN,
               threshold: float = 0.1, rtolmin: float = 0.0) -> float:
    """Eisenstat-Walker relative tolerance eta_k for the k-th Newton step.

    Version 1 (the reading of the paper's garbled formula in Sec. 3):
        eta_k = | ||r_k|| - ||r_{k-1} + J_{k-1} du_{k-1}|| | / ||r_{k-1}||
    safeguarded by eta_k = max(eta_k, eta_{k-1}^alpha2) when
    eta_{k-1}^alpha2 > threshold.  Version 2:
        eta_k = gamma (||r_k|| / ||r_{k-1}||)^alpha,
    safeguarded by gamma eta_{k-1}^alpha.  eta_0 = rtol0; every eta is
    clipped to [rtolmin, rtolmax] (App. A: rtol0 = rtolmax = 0.1).
    """
    if k == 0:
        return min(rtol0, rtolmax)
    if version == 1:
        eta = abs(rnorm - linres_prev) / rnorm_prev
        stol = eta_prev ** alpha2
    else:
        eta = gamma * (rnorm / rnorm_prev) ** alpha
        stol = gamma * eta_prev ** alpha
    if stol > threshold:
        eta = max(eta, stol)
    return max(min(eta, rtolmax), rtolmin)


# ---------------------------------------------------------------- BFGS
def two_loop(g: np.ndarray, pairs: List[tuple], h0: Callable) -> np.ndarray:
    """z = H g by the limited-memory two-loop recursion (pairs oldest first)."""
    q = g.copy()
    alphas = []
    for s, y in reversed(pairs):
        a = np.dot(s, q) / np.dot(y, s)
        q = q - a * y
        alphas.append(a)
    z = h0(q)
    for (s, y), a in zip(pairs, reversed(alphas)):
        b = np.dot(y, z) / np.dot(y, s)
        z = z + (a - b) * s
    return z


def bfgs_inverse_dense(H0: np.ndarray, pairs: List[tuple]) -> np.ndarray:
    """Apply the rank-two inverse update of Sec. 3 once per pair, in order:
    H <- (I - rho s y^T) H (I - rho y s^T) + rho s s^T, rho = 1 / <s, y>."""
    H = np.array(H0, dtype=np.float64, copy=True)
    n = H.shape[0]
    I = np.eye(n)
    for s, y in pairs:
        rho = 1.0 / np.dot(s, y)
        H = (I - rho * np.outer(s, y)) @ H @ (I - rho * np.outer(y, s)) + rho * np.outer(s, s)
    return H


# ---------------------------------------------------------------- outer loops
class Result(dict):
    pass


def newton_krylov(residual: Callable, linearize: Callable, u0: np.ndarray, *,
                  inexact: bool = False, rtol: float = 1e-8, atol: float = 0.0,
                  max_it: int = 50, ksp_rtol: float = 1e-6, ksp_atol: float = 1e-10,
                  ksp: str = "gmres", restart: Optional[int] = None, ksp_max_it: int = 10000,
                  ew_version: int = 1, ew_rtol0: float = 0.1, ew_rtolmax: float = 0.1,
                  lag: int = 1):
    """NK (inexact=False) or iNK (inexact=True) with full steps.

    residual(u) -> r;  linearize(u) -> (matvec, precond) at u.
    Converged when ||r_k|| <= max(rtol ||r_0||, atol).  With lag > 1 the
    tangent is rebuilt only every `lag` iterations and reused in between
    (Jacobian lagging, named as an extension in the conclusions, Sec. 7).
    """
    u = np.array(u0, dtype=np.float64, copy=True)
    r = residual(u)
    rn = [float(np.linalg.norm(r))]
    r0 = rn[0]
    lits, etas = [], []
    eta_prev, linres_prev = 0.0, 0.0
    k = 0
    while rn[-1] > max(rtol * r0, atol) and k < max_it:
        if lag <= 1 or k % lag == 0:
            matvec, prec = linearize(u)
        if inexact:
            eta = ew_forcing(k, rn[-1], rn[-2] if k > 0 else 0.0, linres_prev, eta_prev,
                             version=ew_version, rtol0=ew_rtol0, rtolmax=ew_rtolmax)
            lrtol, latol = eta, 1e-14
        else:
            eta, lrtol, latol = ksp_rtol, ksp_rtol, ksp_atol
        solver = {"gmres": gmres, "cg": cg, "minres": minres}[ksp]
        kw = dict(restart=restart) if ksp == "gmres" else {}
        du, its, _, _ = solver(matvec, -r, prec, rtol=lrtol, atol=latol, max_it=ksp_max_it, **kw)
        linres_prev = float(np.linalg.norm(r + matvec(du)))
        eta_prev = eta
        u = u + du
        r = residual(u)
        rn.append(float(np.linalg.norm(r)))
        lits.append(its)
        etas.append(eta)
        k += 1
    return Result(u=u, rnorm=rn, lits=lits, etas=etas, nit=k,
                  converged=rn[-1] <= max(rtol * r0, atol))


def lbfgs(residual: Callable, h0: Callable, u0: np.ndarray, *, m: int = 10,
          rtol: float = 1e-8, atol: float = 0.0, max_it: int = 1000,
          curvature_eps: float = 1e-12, refresh: int = 0,
          relinearize: Optional[Callable] = None):
    """L-BFGS root finder on g = r(u) with full steps (p = -H g, u += p).

    h0 is the initial inverse-Hessian action (built by the caller once, at
    the first iterate).  A pair (s, y) with s.y <= eps ||s|| ||y|| is skipped.
    With refresh > 0, every `refresh` iterations the initial inverse Hessian
    is rebuilt at the current iterate (h0 = relinearize(u)) and the stored
    pairs are dropped: the occasional Jacobian reassembly for BFGS that the
    paper's conclusions (Sec. 7) name as an extension.
    """
    u = np.array(u0, dtype=np.float64, copy=True)
    g = residual(u)
    rn = [float(np.linalg.norm(g))]
    r0 = rn[0]
    pairs: List[tuple] = []
    skipped = 0
    k = 0
    while rn[-1] > max(rtol * r0, atol) and k < max_it:
        if refresh > 0 and k > 0 and k % refresh == 0:
            h0 = relinearize(u)
            pairs = []
        p = -two_loop(g, pairs, h0)
        u = u + p
        g_new = residual(u)
        y = g_new - g
        if np.dot(p, y) > curvature_eps * np.linalg.norm(p) * np.linalg.norm(y):
            pairs.append((p, y))
            if len(pairs) > m:
                pairs.pop(0)
        else:
            skipped += 1
        g = g_new
        rn.append(float(np.linalg.norm(g)))
        k += 1
    return Result(u=u, rnorm=rn, nit=k, skipped=skipped,
                  converged=rn[-1] <= max(rtol * r0, atol))
