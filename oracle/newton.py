"""Newton's method for the stabilised solid problem (oracle).

Section "Newton's Method": assemble K(v_k), solve K dv = -R(v_k) to a
relative residual eps_1, update v_{k+1} = v_k + dv and stop when
||dv_k||_M <= eps_2 ||dv_0||_M (eq. newstop in the mass-matrix form with
M = diag(M1, M2)).  Loads are applied in increments lambda = k / n_inc,
each starting from the previous converged state.

The relative rule has no meaning when its reference ||dv_0||_M is itself
rounding noise: an increment (or time step) that starts at a solution (a
time step from an equilibrium at rest, for instance) has a first correction
at the fp64 rounding level of the state, and no later correction can be a
further factor eps_2 smaller.  Reading: the increment is converged after its
first correction, taken whole, when ||dv_0||_M <= FLOOR ||v_0||_M, with
FLOOR = 1e-14 (a hundred times the unit roundoff) and v_0 the starting
state.

Adaptive inner tolerance (the inexact-Newton analysis of the same section):
the inner reduction of step k is the square of the outer reduction reached
at step k-1, eps_1,k = eps_2,k-1^2, read here with the relative outer
reduction eps_2,k-1 = ||dv_{k-1}||_M / ||dv_0||_M of the stopping rule;
the first step (no reduction yet) and very small values are clamped to
[eps1_min, eps1_max].

Damped Newton (an option; the paper's Newton method takes full steps): the
update is v + alpha dv with the largest alpha in {1, 1/2, 1/4, ...,
alpha_min} for which every element keeps J > 0 and the Dirichlet-eliminated
residual decreases by the Armijo factor, ||R(v + alpha dv)||_2 <=
(1 - c alpha) ||R(v)||_2; the stopping rule stays eq. newstop on the full
Newton corrections dv_k, met only by a full step (alpha = 1); a correction
that already meets it is taken whole without a search (the residual is then
at its rounding floor).  When no alpha qualifies the increment fails.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import amg, fe, krylov


FLOOR = 1e-14


@dataclasses.dataclass
class NewtonParams:
    eps2: float = 1e-10
    max_iter: int = 25
    lin_tol: float = 1e-8
    restart: int = 50
    lin_maxit: int = 500
    amg: amg.AmgParams = dataclasses.field(default_factory=amg.AmgParams)
    adaptive: bool = False   # eps_1,k = eps_2,k-1^2 instead of lin_tol
    eps1_max: float = 1e-2
    eps1_min: float = 1e-12
    line_search: bool = False  # damped Newton (backtracking on ||R||_2)
    ls_c: float = 1e-4
    ls_alpha_min: float = 2.0 ** -10


def inner_tolerance(prm: NewtonParams, k, dv_prev=None, dv_first=None):
    """Relative residual reduction asked of the linear solve of step k."""
    if not prm.adaptive:
        return prm.lin_tol
    if k == 0 or not dv_first:
        return prm.eps1_max
    return min(prm.eps1_max, max(prm.eps1_min, (dv_prev / dv_first) ** 2))


def linear_system(disc: fe.Discretization, v, load):
    """Dirichlet-eliminated K (CSR), right-hand side -R, blocks A, B2, s."""
    R, val = disc.assemble(v, load)
    R, val = disc.apply_dirichlet(R, val)
    K = disc.csr(val)
    A, B2, s = disc.blocks(val)
    return K, -R, A, B2, s


def newton_direction(disc, v, load, prm: NewtonParams, tol=None):
    """Newton correction dv (K dv = -R), its solve info and ||R(v)||_2."""
    K, b, A, B2, s = linear_system(disc, v.ravel(), load)
    M, _ = krylov.amg_preconditioner(A, B2, s, disc.n, prm.amg)
    dv, info = krylov.fgmres(K, M, b, m=prm.restart, maxit=prm.lin_maxit, tol=prm.lin_tol if tol is None else tol)
    return dv, info, float(np.linalg.norm(b))


def newton_step(disc, v, load, prm: NewtonParams, tol=None):
    """One Newton update; returns (v_new, ||dv||_M, solve info)."""
    dv, info, _ = newton_direction(disc, v, load, prm, tol)
    return v.ravel() + dv, disc.mass_norm(dv), info


def residual_norm(disc, v, load):
    """||R(v)||_2 of the Dirichlet-eliminated residual, or inf when some
    element has J <= 0 (or the residual is not finite)."""
    v = np.asarray(v).reshape(disc.n, 4)
    T = disc.prob.tets
    F = np.eye(3)[None] + np.einsum("mai,maj->mij", v[:, 0:3][T], disc.G)
    if not np.all(np.linalg.det(F) > 0):
        return np.inf
    R = disc.residual(v.ravel(), load)
    R[disc.dirichlet_dofs()] = 0.0
    r = float(np.linalg.norm(R))
    return r if np.isfinite(r) else np.inf


def damped_step(disc, v, dv, load, r0, prm: NewtonParams):
    """Backtracking: the largest alpha = 2^-j >= alpha_min with J > 0 on
    every element and ||R(v + alpha dv)|| <= (1 - c alpha) r0; None if none."""
    alpha = 1.0
    while alpha >= prm.ls_alpha_min:
        if residual_norm(disc, v + alpha * dv, load) <= (1.0 - prm.ls_c * alpha) * r0:
            return alpha
        alpha *= 0.5
    return None


def solve_increment(disc, v, load, prm: NewtonParams, log=None):
    v = v.ravel().copy()
    floor = FLOOR * disc.mass_norm(v)
    n0 = None
    nrm = None
    for k in range(prm.max_iter):
        tol = inner_tolerance(prm, k, nrm, n0)
        dv, info, r0 = newton_direction(disc, v, load, prm, tol)
        nrm = disc.mass_norm(dv)
        alpha = 1.0
        # a correction that already meets the stopping rule is taken whole
        # (near the solution the residual sits at its rounding floor and
        # cannot show the Armijo decrease); so is a first correction at the
        # rounding level of the starting state
        at_floor = n0 is None and nrm <= floor
        small = at_floor or (n0 is not None and nrm <= prm.eps2 * n0)
        if prm.line_search and not small:
            alpha = damped_step(disc, v, dv, load, r0, prm)
            if alpha is None:
                return v, False, k + 1
        v = v + alpha * dv
        if log is not None:
            log.append(dict(load=load, it=k, dv_M=nrm, krylov=info.iterations,
                            rel_res=info.rel_residual, eps1=tol, alpha=alpha))
        if at_floor:
            return v, True, k + 1
        if n0 is None:
            n0 = nrm
        if (nrm <= prm.eps2 * n0 or n0 == 0.0) and alpha == 1.0:
            return v, True, k + 1
    return v, False, prm.max_iter


def load_run(disc, n_inc, prm: NewtonParams, log=None):
    v = np.zeros(4 * disc.n)
    for k in range(1, n_inc + 1):
        v, ok, _ = solve_increment(disc, v, k / n_inc, prm, log)
        if not ok:
            raise RuntimeError(f"Newton did not converge at increment {k}")
    return v
