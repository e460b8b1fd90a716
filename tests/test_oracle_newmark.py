"""Pins of the oracle's Newmark-beta time stepping.

* the update formulas reproduce a constant-acceleration motion exactly for
  any beta and gamma (closed form);
* with the history field of a step the residual's inertia part is
  rho_s times the Newmark acceleration of the new state, node by node for a
  uniform (rigid) motion;
* a free body (no Dirichlet data, no load) with a uniform initial velocity
  translates rigidly at that velocity through the time steps.
"""
import numpy as np
import pytest

import synth
from oracle import fe, newmark, newton


@pytest.mark.parametrize("beta,gamma", [(0.625, 1.0), (0.25, 0.5), (0.9, 0.7)])
def test_constant_acceleration_is_exact(beta, gamma):
    prm = newmark.NewmarkParams(rho=2.0, dt=0.1, beta=beta, gamma=gamma)
    a0 = np.array([[1.0, -2.0, 0.5]])
    v0 = np.array([[0.3, 0.0, -1.0]])
    d = lambda t: v0 * t + 0.5 * a0 * t * t  # noqa: E731
    vel, acc = v0.copy(), a0.copy()
    for k in range(1, 6):
        vel, acc = newmark.update(prm, d(k * prm.dt), d((k - 1) * prm.dt), vel, acc)
        assert np.allclose(acc, a0, rtol=1e-12, atol=1e-12)
        assert np.allclose(vel, v0 + a0 * k * prm.dt, rtol=1e-12, atol=1e-12)


def test_history_gives_rho_times_the_newmark_acceleration():
    prm = newmark.NewmarkParams(rho=3.0, dt=0.05)
    r = np.random.default_rng(0)
    d_prev, vel, acc, d_new = (r.normal(size=(5, 3)) for _ in range(4))
    cm = newmark.coefficient(prm)
    _, acc_new = newmark.update(prm, d_new, d_prev, vel, acc)
    assert np.allclose(cm * d_new - newmark.history(prm, d_prev, vel, acc), prm.rho * acc_new, rtol=1e-12)


def test_free_body_keeps_a_uniform_velocity():
    """Without supports or loads a body set moving at a uniform velocity v0
    translates rigidly, d(t) = v0 t with p = 0: every term of the step's
    residual vanishes on that state (the stabilisation too, since
    r_s - cm d^n = -rho_s a^n = 0), and Newmark integrates a constant
    velocity exactly."""
    prob = synth.cube_problem(2, jitter=0.1, seed=1)
    prob.dir_mask[:] = 0
    prob.tris = np.zeros((0, 3), np.int32)
    prob.traction = np.zeros((0, 3))
    disc = fe.Discretization(prob)
    prm = newmark.NewmarkParams(rho=2.0, dt=0.02)
    nprm = newton.NewtonParams(eps2=1e-12)
    v0 = np.array([0.4, -0.1, 0.25])
    v = np.zeros(4 * disc.n)
    vel = np.tile(v0, (disc.n, 1))
    acc = np.zeros((disc.n, 3))
    for k in range(1, 4):
        v, vel, acc, its = newmark.time_step(disc, v, 1.0, prm, nprm, vel, acc)
        d = v.reshape(disc.n, 4)
        assert np.allclose(d[:, 0:3], v0 * k * prm.dt, rtol=1e-10, atol=1e-14)
        assert np.abs(d[:, 3]).max() <= 1e-10
        assert np.allclose(vel, v0, rtol=1e-8) and np.abs(acc).max() <= 1e-6
