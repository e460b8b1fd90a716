"""GPU parity of the Newmark-beta inertia against the oracle.

* assembly with inertia on (history field from a random previous state,
  velocity and acceleration): R, every stored entry of K and the A block to
  1e-12 relative to the largest entry, as for the quasi-static assembly;
* the update kernel against the oracle's formulas;
* time steps of a cube under a suddenly applied traction (Newton per step,
  then the Newmark update) reproduce the oracle's states, velocities and
  accelerations, also through the one-call hfsi_time_step with the adaptive
  inner tolerance and coarse grids kept across steps.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import torch_dev
from oracle import fe, newmark, newton
from test_gpu_assembly import _blocks_to_csr

pytestmark = pytest.mark.gpu

PRM = newmark.NewmarkParams(rho=1.0, dt=0.05)


def _context(lib, prob):
    ctx = lib.Context(0)
    ctx.set_problem(prob)
    ctx.set_newmark(PRM.rho, dt=PRM.dt, beta=PRM.beta, gamma=PRM.gamma)
    return ctx


@pytest.mark.parametrize("case", ["cube5_jitter", "tube_small"])
def test_inertia_assembly_matches_oracle(lib, case):
    import torch
    print(f"[newmark assembly] case={case}", flush=True)
    prob = (synth.cube_problem(5, jitter=0.1, seed=9) if case == "cube5_jitter"
            else synth.tube_problem(n_theta=16, n_media=2, n_adv=2, n_z=6))
    n = prob.n_nodes
    v = synth.random_state(prob, 21, u_scale=0.05, p_scale=0.2).ravel()
    v_prev = synth.random_state(prob, 22, u_scale=0.05, p_scale=0.2).ravel()
    r = np.random.default_rng(3)
    vel, acc = r.normal(scale=0.5, size=(n, 3)), r.normal(scale=2.0, size=(n, 3))
    ctx = _context(lib, prob)
    ctx.newmark_history(torch_dev(v_prev), torch_dev(vel), torch_dev(acc))
    vt = torch_dev(v)
    R = torch.zeros_like(vt)
    view, _ = ctx.assemble_residual_tangent(vt, 0.6, R)
    out = ctx.export_tangent(view)
    d = fe.Discretization(prob)
    d.set_inertia(newmark.coefficient(PRM), newmark.history(PRM, v_prev.reshape(n, 4)[:, 0:3], vel, acc))
    Ro, val = d.assemble(v, 0.6)
    Ro, val = d.apply_dirichlet(Ro, val)
    K = d.csr(val)
    A, B2, s = d.blocks(val)
    Kg = _blocks_to_csr(out, n)
    assert np.array_equal(Kg.indptr, K.indptr) and np.array_equal(Kg.indices, K.indices)
    assert np.abs(Kg.data - K.data).max() <= 1e-12 * np.abs(K.data).max()
    assert np.abs(R.cpu().numpy() - Ro).max() <= 1e-12 * np.abs(Ro).max()
    assert np.abs(out["a_val"] - A.data).max() <= 1e-12 * np.abs(A.data).max()
    # and the inertia is really in there
    d.set_inertia(0.0, None)
    R0, _ = d.assemble(v, 0.6)
    R0, _ = d.apply_dirichlet(R0, np.zeros(len(d.K_indices)))
    assert np.abs(Ro - R0).max() > 1e-3 * np.abs(Ro).max()


def test_newmark_update_and_order_errors(lib):
    import torch
    prob = synth.cube_problem(3)
    n = prob.n_nodes
    r = np.random.default_rng(4)
    v_new, v_prev = r.normal(size=4 * n), r.normal(size=4 * n)
    vel, acc = r.normal(size=(n, 3)), r.normal(size=(n, 3))
    ctx = _context(lib, prob)
    vel_t, acc_t = torch_dev(vel), torch_dev(acc)
    ctx.newmark_update(torch_dev(v_new), torch_dev(v_prev), vel_t, acc_t)
    vo, ao = newmark.update(PRM, v_new.reshape(n, 4)[:, 0:3], v_prev.reshape(n, 4)[:, 0:3], vel, acc)
    assert np.abs(vel_t.cpu().numpy().reshape(n, 3) - vo).max() <= 1e-13 * np.abs(vo).max()
    assert np.abs(acc_t.cpu().numpy().reshape(n, 3) - ao).max() <= 1e-13 * np.abs(ao).max()
    ctx.set_newmark(0.0)
    with pytest.raises(lib.HfsiError) as e:
        ctx.newmark_update(torch_dev(v_new), torch_dev(v_prev), vel_t, acc_t)
    assert e.value.code == -4
    with pytest.raises(lib.HfsiError) as e:
        ctx.set_newmark(1.0, dt=0.1, beta=0.0)
    assert e.value.code == -1


def test_time_steps_match_oracle(lib):
    """Three steps of the 4^3 cube from rest under the full traction."""
    import torch
    print("[newmark steps] cube4 3 steps", flush=True)
    prob = synth.cube_problem(4)
    n = prob.n_nodes
    ctx = _context(lib, prob)
    v = torch.zeros(4 * n, dtype=torch.float64, device="cuda")
    vel = torch.zeros(3 * n, dtype=torch.float64, device="cuda")
    acc = torch.zeros_like(vel)
    prm = lib.newton_params()
    disc = fe.Discretization(prob)
    vo, velo, acco = np.zeros(4 * n), np.zeros((n, 3)), np.zeros((n, 3))
    for step in range(3):
        v_prev = v.clone()
        ctx.newmark_history(v_prev, vel, acc)
        n0 = None
        for it in range(25):
            info, code = ctx.newton_step(v, 1.0, prm)
            assert code == 0
            n0 = info.dv_mass_norm if n0 is None else n0
            if info.dv_mass_norm <= 1e-10 * n0:
                break
        ctx.newmark_update(v, v_prev, vel, acc)
        vo, velo, acco, _ = newmark.time_step(disc, vo, 1.0, PRM, newton.NewtonParams(), velo, acco)
        assert np.linalg.norm(v.cpu().numpy() - vo) <= 1e-8 * np.linalg.norm(vo)
        assert np.linalg.norm(vel.cpu().numpy().reshape(n, 3) - velo) <= 1e-7 * np.linalg.norm(velo)
        assert np.linalg.norm(acc.cpu().numpy().reshape(n, 3) - acco) <= 1e-7 * np.linalg.norm(acco)
    assert np.linalg.norm(acco) > 0


def test_time_step_entry_with_reuse_matches_oracle(lib):
    """hfsi_time_step (history, Newton solve, update in one call) with the
    adaptive inner tolerance and the coarse grids kept from step to step
    reaches the oracle's time steps (a new hierarchy per Newton iteration,
    fixed inner tolerance) to the Newton tolerance; with inertia off it is
    an order error."""
    import torch
    print("[newmark time_step] cube4 3 steps, adaptive, reused grids", flush=True)
    prob = synth.cube_problem(4)
    n = prob.n_nodes
    ctx = _context(lib, prob)
    v = torch.zeros(4 * n, dtype=torch.float64, device="cuda")
    vel = torch.zeros(3 * n, dtype=torch.float64, device="cuda")
    acc = torch.zeros_like(vel)
    prm = lib.newton_solve_params(step=lib.newton_params(amg_reuse=2), adaptive=1)
    disc = fe.Discretization(prob)
    vo, velo, acco = np.zeros(4 * n), np.zeros((n, 3)), np.zeros((n, 3))
    for step in range(3):
        info, code = ctx.time_step(v, vel, acc, 1.0, prm)
        assert code == 0 and info.converged
        vo, velo, acco, _ = newmark.time_step(disc, vo, 1.0, PRM, newton.NewtonParams(), velo, acco)
        assert np.linalg.norm(v.cpu().numpy() - vo) <= 1e-8 * np.linalg.norm(vo)
        assert np.linalg.norm(vel.cpu().numpy().reshape(n, 3) - velo) <= 1e-7 * np.linalg.norm(velo)
        assert np.linalg.norm(acc.cpu().numpy().reshape(n, 3) - acco) <= 1e-7 * np.linalg.norm(acco)
    ctx.set_newmark(0.0)
    with pytest.raises(lib.HfsiError) as e:
        ctx.time_step(v, vel, acc, 1.0, prm)
    assert e.value.code == -4


def test_time_step_from_equilibrium_ends_at_the_floor(lib):
    """A time step from a static equilibrium at rest: the first Newton
    correction is rounding noise, the step ends after it (both sides), the
    state stays put and velocity and acceleration stay at rounding level."""
    import torch
    print("[newmark floor] cube4 equilibrium at rest", flush=True)
    prob = synth.cube_problem(4)
    n = prob.n_nodes
    ctx = lib.Context(0)
    ctx.set_problem(prob)
    v = torch.zeros(4 * n, dtype=torch.float64, device="cuda")
    info, code = ctx.newton_solve(v, 1.0, lib.newton_solve_params())
    assert code == 0
    v_eq = v.clone()
    ctx.set_newmark(PRM.rho, dt=PRM.dt, beta=PRM.beta, gamma=PRM.gamma)
    vel = torch.zeros(3 * n, dtype=torch.float64, device="cuda")
    acc = torch.zeros_like(vel)
    prm = lib.newton_solve_params(step=lib.newton_params(solve=lib.solve_params(tol=1e-12)), max_newton=6)
    info, code = ctx.time_step(v, vel, acc, 1.0, prm)
    assert code == 0 and info.converged and info.newton_iterations == 1
    assert (v - v_eq).abs().max().item() <= 1e-13 * v_eq.abs().max().item()
    assert vel.abs().max().item() <= 1e-8 and acc.abs().max().item() <= 1e-6
    disc = fe.Discretization(prob)
    vo, _, _ = newton.solve_increment(disc, np.zeros(4 * n), 1.0, newton.NewtonParams())[0], None, None
    _, _, _, its = newmark.time_step(disc, vo, 1.0, PRM, newton.NewtonParams(eps2=1e-10, max_iter=6, lin_tol=1e-12),
                                     np.zeros((n, 3)), np.zeros((n, 3)))
    assert its == 1
