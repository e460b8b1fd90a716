"""End-to-end pins of the oracle's Newton solve.

A cube on rollers under a dead uniaxial traction sigma has a homogeneous
solution F = diag(l1, l2, l3), p = -kappa (J - 1), which P1 elements
represent exactly.  Its stretches make the potential per unit reference
volume  Pi = Psi_dev(C) + kappa/2 (J-1)^2 - sigma (l1 - 1)  stationary
(the energies of eq. mmreng and eq. areng written in principal stretches);
an independent three-unknown Newton solve of grad Pi = 0 fixes them.
"""
import numpy as np
import pytest

import synth
from oracle import amg, fe, newton


def _pi(l, law, mat, alpha, sigma):
    l1, l2, l3 = l
    J = l1 * l2 * l3
    I1 = l1 ** 2 + l2 ** 2 + l3 ** 2
    I2 = (l1 * l2) ** 2 + (l2 * l3) ** 2 + (l3 * l1) ** 2
    psi = 0.5 * mat["c10"] * (I1 * J ** (-2 / 3) - 3)
    if law == "mr":
        psi += 0.5 * mat["c01"] * (I2 * J ** (-4 / 3) - 3)
    else:
        J4 = J ** (-2 / 3) * (np.cos(alpha) ** 2 * l1 ** 2 + np.sin(alpha) ** 2 * l2 ** 2)
        if J4 > 1:
            psi += 2 * mat["k1"] / (2 * mat["k2"]) * (np.exp(mat["k2"] * (J4 - 1) ** 2) - 1)
    return psi + 0.5 * mat["kappa"] * (J - 1) ** 2 - sigma * (l1 - 1)


def _stretches(law, mat, alpha, sigma):
    l = np.ones(3)
    for s in np.linspace(0.0, sigma, 21)[1:]:   # load continuation
        l = _newton3(l, law, mat, alpha, s)
    return l


def _newton3(l, law, mat, alpha, sigma):
    h = 1e-5
    for _ in range(50):
        g = np.zeros(3)
        H = np.zeros((3, 3))
        for i in range(3):
            e = np.zeros(3); e[i] = h
            g[i] = (_pi(l + e, law, mat, alpha, sigma) - _pi(l - e, law, mat, alpha, sigma)) / (2 * h)
            for j in range(3):
                f = np.zeros(3); f[j] = h
                H[i, j] = (_pi(l + e + f, law, mat, alpha, sigma) - _pi(l + e - f, law, mat, alpha, sigma)
                           - _pi(l - e + f, law, mat, alpha, sigma) + _pi(l - e - f, law, mat, alpha, sigma)) / (4 * h * h)
        dl = np.linalg.solve(H, -g)
        l = l + dl
        if np.abs(dl).max() < 1e-13:
            break
    return l


@pytest.mark.parametrize("law", ["mr", "artery"])
def test_uniaxial_homogeneous_solution(law):
    sigma = 0.4 if law == "mr" else 2.0
    alpha = np.radians(29.0)
    if law == "mr":
        mat = synth.meshes.mooney_rivlin(0.5, 0.1, 1e3)
        prob = synth.uniaxial_problem(2, stress=sigma, materials=[mat])
    else:
        mat = synth.meshes.artery_layer(3.0, 2.3632, 0.8393, 1e3)
        fib = [[np.cos(alpha), np.sin(alpha), 0.0], [np.cos(alpha), -np.sin(alpha), 0.0]]
        prob = synth.uniaxial_problem(2, stress=sigma, materials=[mat], fibres=fib)
    lam = _stretches(law, mat, alpha, sigma)
    d = fe.Discretization(prob)
    prm = newton.NewtonParams(eps2=1e-12, lin_tol=1e-12, amg=amg.AmgParams(max_coarse=50))
    v = np.zeros(4 * d.n)
    for k in range(1, 5):
        v, ok, _ = newton.solve_increment(d, v, k / 4, prm)
        assert ok
    v = v.reshape(-1, 4)
    corner = np.flatnonzero(np.all(prob.lattice == 2, axis=1))[0]
    got = 1.0 + v[corner, 0:3] / prob.X[corner]
    assert np.allclose(got, lam, rtol=0, atol=1e-9)
    J = np.prod(lam)
    assert np.allclose(v[:, 3], -mat["kappa"] * (J - 1), rtol=1e-8, atol=1e-10)
    if law == "artery":
        assert abs(lam[1] - lam[2]) > 1e-4   # the fibres break the transverse symmetry


def test_newton_converges_quadratically():
    prob = synth.cube_problem(4)
    d = fe.Discretization(prob)
    log = []
    prm = newton.NewtonParams(lin_tol=1e-12)
    newton.solve_increment(d, np.zeros(4 * d.n), 1.0, prm, log)
    r = [e["dv_M"] for e in log]
    assert len(r) <= 6
    # log(e_{k+1}) / log(e_k) relative to the first step approaches 2
    ratios = [np.log(r[k + 1] / r[0]) / np.log(r[k] / r[0]) for k in range(1, len(r) - 1) if r[k + 1] > 1e-14 * r[0]]
    assert ratios and min(ratios) > 1.7


def test_adaptive_inner_tolerance_keeps_quadratic_convergence():
    """With eps_1,k = eps_2,k-1^2 the inexact Newton iteration keeps the
    quadratic rate of the exact one (the point of the rule): it reaches the
    same state in at most one more step, every step after the first asks the
    square of the previous relative increment, and it spends fewer Krylov
    iterations than solving every step to 1e-8."""
    prob = synth.cube_problem(4)
    d = fe.Discretization(prob)
    exact, adapt = [], []
    v_exact, ok1, k1 = newton.solve_increment(d, np.zeros(4 * d.n), 1.0, newton.NewtonParams(lin_tol=1e-12), exact)
    prm = newton.NewtonParams(adaptive=True)
    v_adapt, ok2, k2 = newton.solve_increment(d, np.zeros(4 * d.n), 1.0, prm, adapt)
    assert ok1 and ok2 and k2 <= k1 + 1
    assert np.linalg.norm(v_adapt - v_exact) <= 1e-9 * np.linalg.norm(v_exact)
    dv = [e["dv_M"] for e in adapt]
    assert adapt[0]["eps1"] == prm.eps1_max
    for k in range(1, len(adapt)):
        want = min(prm.eps1_max, max(prm.eps1_min, (dv[k - 1] / dv[0]) ** 2))
        assert adapt[k]["eps1"] == want and adapt[k]["rel_res"] <= want
    fixed = []
    newton.solve_increment(d, np.zeros(4 * d.n), 1.0, newton.NewtonParams(), fixed)
    assert sum(e["krylov"] for e in adapt) < sum(e["krylov"] for e in fixed)
    ratios = [np.log(dv[k + 1] / dv[0]) / np.log(dv[k] / dv[0]) for k in range(1, len(dv) - 1)
              if dv[k + 1] > 1e-14 * dv[0]]
    assert ratios and min(ratios) > 1.6


def _tiny_tube():
    return synth.tube_problem(n_theta=8, n_media=1, n_adv=1, n_z=8)


def test_damped_newton_reaches_the_undamped_equilibrium():
    """The artery tube under its full internal pressure in 10 increments:
    plain Newton leaves the admissible states in the first increment (the
    fibres are off in the first tangent), the damped method converges with
    alpha < 1 in its first steps, every accepted step meets the Armijo
    decrease, and its final state is the equilibrium that undamped Newton
    reaches with 40 increments (same state to 1e-8, residual near zero)."""
    prob = _tiny_tube()
    d = fe.Discretization(prob)
    plain = newton.NewtonParams(eps2=1e-10)
    v = np.zeros(prob.n_dofs)
    failed = False
    with np.errstate(all="ignore"):
        try:
            v1, ok, _ = newton.solve_increment(d, v, 0.1, plain)
            failed = not ok or not _converged(d, v1, 0.1)
        except np.linalg.LinAlgError:
            failed = True   # the set-up met non-finite values
    assert failed
    damped = newton.NewtonParams(eps2=1e-10, line_search=True)
    log = []
    v = np.zeros(prob.n_dofs)
    for k in range(1, 11):
        v, ok, _ = newton.solve_increment(d, v, k / 10, damped, log)
        assert ok, k
    alphas = [e["alpha"] for e in log]
    assert min(alphas) < 1.0 and alphas[-1] == 1.0
    ref = np.zeros(prob.n_dofs)
    for k in range(1, 41):
        ref, ok, _ = newton.solve_increment(d, ref, k / 40, plain)
        assert ok, k
    assert np.linalg.norm(v - ref) <= 1e-8 * np.linalg.norm(ref)
    assert newton.residual_norm(d, v, 1.0) <= 1e-9 * newton.residual_norm(d, np.zeros(prob.n_dofs), 1.0)


def _converged(d, v, load):
    r = newton.residual_norm(d, v, load)
    return np.isfinite(r) and r <= 1e-8 * newton.residual_norm(d, np.zeros_like(v), load)


def test_damped_newton_takes_full_steps_where_newton_converges():
    """On the cube (where full steps already decrease the residual) the damped
    method takes alpha = 1 every time and repeats the undamped iterates."""
    prob = synth.cube_problem(3, jitter=0.1, seed=2)
    d = fe.Discretization(prob)
    log_a, log_b = [], []
    va, _, _ = newton.solve_increment(d, np.zeros(prob.n_dofs), 1.0, newton.NewtonParams(), log_a)
    vb, _, _ = newton.solve_increment(d, np.zeros(prob.n_dofs), 1.0, newton.NewtonParams(line_search=True), log_b)
    assert all(e["alpha"] == 1.0 for e in log_b)
    assert np.array_equal(va, vb) and len(log_a) == len(log_b)


def test_residual_norm_rejects_inverted_states():
    prob = synth.cube_problem(2)
    d = fe.Discretization(prob)
    v = np.zeros((prob.n_nodes, 4))
    v[:, 0] = -2.0 * prob.X[:, 0]          # x -> -x: every element inverted
    assert newton.residual_norm(d, v.ravel(), 0.0) == np.inf
    assert np.isfinite(newton.residual_norm(d, np.zeros(prob.n_dofs), 1.0))


def test_time_step_from_equilibrium_is_converged_at_the_floor():
    """A Newmark step from a static equilibrium at rest (zero velocity and
    acceleration) has the equilibrium itself as its solution: the first
    Newton correction is rounding noise (about 1e-16 of the state), and the
    relative rule ||dv_k|| <= eps2 ||dv_0|| could never be met.  The floor
    reading ends the step after that first correction; without it Newton
    runs to its iteration limit (checked by lowering the floor to zero)."""
    from oracle import newmark
    prob = synth.cube_problem(4)
    d = fe.Discretization(prob)
    v, ok, _ = newton.solve_increment(d, np.zeros(prob.n_dofs), 1.0, newton.NewtonParams())
    assert ok
    n = prob.n_nodes
    nm = newmark.NewmarkParams(rho=1.0, dt=0.05)
    zero = np.zeros((n, 3))
    prm = newton.NewtonParams(eps2=1e-10, max_iter=6, lin_tol=1e-12)
    v1, vel, acc, its = newmark.time_step(d, v, 1.0, nm, prm, zero, zero)
    assert its == 1
    assert np.abs(v1 - v).max() <= 1e-13 * np.abs(v).max()
    assert np.abs(vel).max() <= 1e-8 and np.abs(acc).max() <= 1e-6
    saved = newton.FLOOR
    try:
        newton.FLOOR = 0.0
        with pytest.raises(RuntimeError):
            newmark.time_step(d, v, 1.0, nm, prm, zero, zero)
    finally:
        newton.FLOOR = saved
    # a step that moves is not cut short: from rest under the full load the
    # first correction is large and the relative rule decides
    v2, _, _, its2 = newmark.time_step(d, np.zeros(prob.n_dofs), 1.0, nm, prm, zero, zero)
    assert its2 >= 3
