"""Newmark-beta time stepping of the structure (oracle; test infrastructure).

Section "Temporal discretization for the structure sub-problem": with
displacement d, velocity v and acceleration a at the nodes,
    a^n = (d^n - d^{n-1}) / (beta dt^2) - v^{n-1} / (beta dt) - (1 - 2 beta) / (2 beta) a^{n-1}
    v^n = v^{n-1} + gamma dt a^n + (1 - gamma) dt a^{n-1}
(the paper takes beta = 0.625, gamma = 1).  The step's weak residual (section
"The time semi-discretized structure weak formulation", and its
stabilisation, eq. stelas) carries the inertia coefficient
cm = rho_s / (beta dt^2) and the history field
    r_s = rho_s / (beta dt^2) d^{n-1} + rho_s / (beta dt) v^{n-1} + rho_s (1 - 2 beta) / (2 beta) a^{n-1},
interpolated in P1 from its nodal values; the element terms are in
`fe.element_kernel`.  Each step is solved by Newton's method at a fixed load.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import newton


@dataclasses.dataclass
class NewmarkParams:
    rho: float
    dt: float
    beta: float = 0.625
    gamma: float = 1.0


def coefficient(prm: NewmarkParams):
    """cm = rho_s / (beta dt^2)."""
    return prm.rho / (prm.beta * prm.dt ** 2)


def history(prm: NewmarkParams, d_prev, vel, acc):
    """Nodal r_s of the step that starts from (d_prev, vel, acc), [n,3]."""
    b, dt = prm.beta, prm.dt
    return prm.rho * (d_prev / (b * dt * dt) + vel / (b * dt) + (1.0 - 2.0 * b) / (2.0 * b) * acc)


def update(prm: NewmarkParams, d_new, d_prev, vel, acc):
    """Velocity and acceleration at the end of the step, [n,3] each."""
    b, g, dt = prm.beta, prm.gamma, prm.dt
    acc_new = (d_new - d_prev) / (b * dt * dt) - vel / (b * dt) - (1.0 - 2.0 * b) / (2.0 * b) * acc
    vel_new = vel + g * dt * acc_new + (1.0 - g) * dt * acc
    return vel_new, acc_new


def time_step(disc, v, load, prm: NewmarkParams, nprm: newton.NewtonParams, vel, acc):
    """One time step from state v (node-interleaved [4n]) with velocity and
    acceleration [n,3]; returns (v, vel, acc, Newton iterations)."""
    n = disc.n
    d_prev = np.asarray(v).reshape(n, 4)[:, 0:3].copy()
    disc.set_inertia(coefficient(prm), history(prm, d_prev, vel, acc))
    try:
        v_new, ok, its = newton.solve_increment(disc, v, load, nprm)
    finally:
        disc.set_inertia(0.0, None)
    if not ok:
        raise RuntimeError("Newton did not converge in the time step")
    vel_new, acc_new = update(prm, v_new.reshape(n, 4)[:, 0:3], d_prev, vel, acc)
    return v_new, vel_new, acc_new, its
