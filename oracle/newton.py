"""Exact Newton on the assembled tangent: the oracle's root u* (FP64).

Paper, Sec. 3, eq. "newton": given u^{n-1}, solve
    dR(u^{n-1}) [du] = -R(u^{n-1}),   u^n = u^{n-1} + du
with full steps.  Here the linear solve is a direct sparse LU
(scipy.sparse.linalg.splu), so every iterate is the exact Newton iterate
and the converged u* is the discrete root to rounding.

Stopping: ||r_k||_2 <= rtol ||r_0||_2 (r_0 is the residual at the start of
the load step, after the Dirichlet lift), or stagnation at the FP64 floor.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla


class NewtonFailure(RuntimeError):
    """Newton failed; `iterations` holds the Newton steps taken before."""

    def __init__(self, msg: str, iterations: int = 0):
        super().__init__(msg)
        self.iterations = iterations


def newton_exact(problem, u0: np.ndarray, load_scale: float = 1.0, rtol: float = 1e-13,
                 max_it: int = 50, floor_rtol: float = 1e-6):
    """Return (u*, history of ||r_k||_2).

    Stops when ||r_k|| <= rtol ||r_0||, or once ||r_k|| <= floor_rtol ||r_0||
    and the next iterate fails to halve the residual: quadratic convergence
    has ended at the rounding floor of the internal forces.
    Raises NewtonFailure on an inverted element or after max_it iterations.
    """
    u = problem.lift(u0)
    r = problem.residual(u, load_scale)
    hist = [float(np.linalg.norm(r))]
    r0 = hist[0]
    if r0 == 0.0:
        return u, hist
    for _ in range(max_it):
        if hist[-1] <= rtol * r0:
            return u, hist
        K = problem.stiffness(u, load_scale=load_scale)
        du = spla.splu(K.tocsc()).solve(-r)
        u_new = u + du
        if problem.min_jacobian(u_new) <= 0.0:
            raise NewtonFailure("inverted element", len(hist))
        r_new = problem.residual(u_new, load_scale)
        n_new = float(np.linalg.norm(r_new))
        if hist[-1] <= floor_rtol * r0 and n_new > 0.5 * hist[-1]:
            return u, hist  # at the rounding floor
        u, r = u_new, r_new
        hist.append(n_new)
    if hist[-1] <= max(rtol, floor_rtol) * r0:
        return u, hist
    raise NewtonFailure(f"no convergence in {max_it} iterations: {hist}", max_it)


def solve_schedule(problem, scales, u0=None, max_cuts: int = 0, start_scale: float = 0.0,
                   log=None, **kw):
    """Exact Newton over a sequence of load scales, warm-started.

    With max_cuts > 0, a load step whose Newton iteration fails (an element
    inverts or the iteration limit is reached) is retried from the last
    converged state at the midpoint of the failed increment, at most
    max_cuts times over the schedule (the load stepping of Sec. 4, read as
    stepping with halving on failure).  Returns (u, Newton histories of the
    accepted steps); with `log` (a list) each attempt appends
    (scale, accepted, Newton iterations taken)."""
    u = np.zeros(problem.n_dofs) if u0 is None else np.array(u0, dtype=np.float64)
    hists = []
    targets = [float(x) for x in scales]
    s_prev = float(start_scale)
    cuts = 0
    i = 0
    while i < len(targets):
        s = targets[i]
        try:
            u_new, h = newton_exact(problem, u, s, **kw)
        except NewtonFailure as exc:
            if log is not None:
                log.append((s, False, exc.iterations))
            if cuts >= max_cuts:
                raise
            cuts += 1
            targets.insert(i, 0.5 * (s_prev + s))
            continue
        if log is not None:
            log.append((s, True, len(h) - 1))
        u = u_new
        hists.append(h)
        s_prev = s
        i += 1
    return u, hists


def newmark_predict(u, v, a, dt: float, beta: float):
    """Newmark predictor u~ = u + dt v + dt^2 (1/2 - beta) a."""
    return u + dt * v + dt * dt * (0.5 - beta) * a


def newmark_correct(u_new, u_tilde, v, a, dt: float, beta: float, gamma: float):
    """Newmark corrector: a' = (u' - u~) / (beta dt^2), v' = v + dt ((1 - gamma) a + gamma a')."""
    a_new = (u_new - u_tilde) / (beta * dt * dt)
    return v + dt * ((1.0 - gamma) * a + gamma * a_new), a_new


def solve_heartbeat_dynamic(problem, schedule, gamma_max: float, rho: float, dt: float,
                            beta: float = 0.25, gamma: float = 0.5, u0=None, **kw):
    """Heartbeat with inertia (Sec. 2, eq. "momentum strong" with the
    acceleration kept): Newmark's average-acceleration rule (beta = 1/4,
    gamma = 1/2) with the lumped mass of density rho; each step sets the
    activation of its time as in solve_heartbeat and solves the implicit step
    c M (u - u~) + r(u) = 0, c = 1 / (beta dt^2), by exact Newton.  With
    dashpots set on the problem (set_robin_damping) the residual also holds
    their force at the step's velocity v~ + gamma / (beta dt) (u - u~),
    v~ = v + dt (1 - gamma) a.  Starts at rest.  Returns (u, v, a, Newton
    histories)."""
    from .fem import set_active_tension

    n = problem.n_dofs
    u = np.zeros(n) if u0 is None else np.array(u0, dtype=np.float64)
    v = np.zeros(n)
    a = np.zeros(n)
    c = 1.0 / (beta * dt * dt)
    hists = []
    for _, shape in schedule:
        ut = newmark_predict(u, v, a, dt, beta)
        problem.set_inertia(rho, c, ut)
        problem.set_step_velocity(gamma / (beta * dt), v + dt * (1.0 - gamma) * a)
        set_active_tension(problem, gamma_max * shape)
        u, h = newton_exact(problem, u, shape, **kw)
        v, a = newmark_correct(u, ut, v, a, dt, beta, gamma)
        hists.append(h)
    problem.set_inertia(0.0, 0.0, u)
    problem.set_step_velocity(0.0, None)
    return u, v, a, hists


def solve_heartbeat(problem, schedule, gamma_max: float, u0=None, **kw):
    """Quasi-static heartbeat (Sec. 4): for each time step (t, shape) set the
    active tension gamma_max * shape and the pressure load scale shape, then
    exact Newton warm-started from the previous step."""
    from .fem import set_active_tension

    u = np.zeros(problem.n_dofs) if u0 is None else np.array(u0, dtype=np.float64)
    hists = []
    for _, shape in schedule:
        set_active_tension(problem, gamma_max * shape)
        u, h = newton_exact(problem, u, shape, **kw)
        hists.append(h)
    return u, hists
