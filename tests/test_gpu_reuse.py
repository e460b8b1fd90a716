"""GPU parity of the AMG re-set-up on kept coarse grids.

After a set-up at one state and an assembly at another, the re-set-up keeps
the splittings and P of the first set-up and rebuilds the Galerkin operators
of the new tangent: level by level they equal the oracle's Galerkin product
of the GPU's own level operator and kept P (pattern exact, values 1e-12
relative), end to end the oracle's re-set-up of the new tangent on the first
hierarchy, and the V-cycle on the rebuilt hierarchy matches the oracle's.
A Newton load run that re-uses the coarse grids converges to the oracle's
states.  A re-set-up may switch the cycle's precision, and keeps learned
level-0 rows bit for bit.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import amg_prm_pair, context_for, export_level_matrix, gpu_hierarchy_to_oracle, oracle_system
from gpu_helpers import torch_dev
from oracle import amg, fe, newton

pytestmark = pytest.mark.gpu


def _assemble(ctx, v, load):
    import torch
    vt = torch_dev(v)
    R = torch.zeros_like(vt)
    ctx.assemble_residual_tangent(vt, load, R)
    return R


@pytest.mark.parametrize("smoother,precision,kind,drop", [(0, 0, "ext+i", 0.0), (1, 0, "ext+i", 0.0),
                                                          (1, 1, "ext+i", 0.0), (1, 0, "classical", 0.0),
                                                          (1, 0, "ext+i", 2e-3)])
def test_resetup_matches_oracle(lib, smoother, precision, kind, drop):
    """ext+i with p_max = 4 takes the narrow value-only product for A P;
    classical interpolation (longer rows of P) the general one; drop > 0:
    sparsified coarse operators, whose patterns the re-set-up keeps."""
    import torch
    print(f"[reuse parity] smoother={smoother} precision={precision} interp={kind} drop={drop}", flush=True)
    prob = synth.cube_problem(6, jitter=0.1, seed=2)
    v0 = synth.random_state(prob, 3, u_scale=0.03, p_scale=0.05).ravel()
    v1 = synth.random_state(prob, 7, u_scale=0.06, p_scale=0.2).ravel()
    gprm, oprm = amg_prm_pair(lib, smoother=smoother, precision=precision, max_coarse=60, schedule="default",
                              kind=kind, drop_tol=drop)
    ctx = context_for(lib, prob)
    _assemble(ctx, v0, 0.4)
    info0 = ctx.amg_setup(gprm)
    assert info0.levels >= 3
    H0 = gpu_hierarchy_to_oracle(ctx, info0, oprm)
    _assemble(ctx, v1, 0.7)
    info1 = ctx.amg_resetup(gprm)
    assert info1.levels == info0.levels and info1.pmis_rounds == 0 and info1.rho == -1.0
    assert [info1.rows[l] for l in range(info1.levels)] == [info0.rows[l] for l in range(info0.levels)]
    _, K1, b1, A1, B2, s = oracle_system(prob, v1, 0.7)
    A1 = A1.tocsr()
    A1.sort_indices()
    G0 = export_level_matrix(ctx, 0, 0)
    assert np.array_equal(G0.indptr, A1.indptr) and np.array_equal(G0.indices, A1.indices)
    assert np.abs(G0.data - A1.data).max() <= 1e-12 * np.abs(A1.data).max()
    Ho = amg.resetup(A1, H0, oprm)
    for l in range(info1.levels - 1):
        P = export_level_matrix(ctx, l, 1)
        Pk = H0.levels[l].P
        assert np.array_equal(P.indptr, Pk.indptr) and np.array_equal(P.indices, Pk.indices)
        assert np.array_equal(P.data, Pk.data), f"P changed on level {l}"
        A = export_level_matrix(ctx, l, 0)
        Ac = export_level_matrix(ctx, l + 1, 0)
        # the Galerkin product on the set-up's (sparsified) pattern
        Aco = amg.on_pattern(amg.galerkin(A, P), H0.levels[l + 1].A)
        assert np.array_equal(Ac.indptr, Aco.indptr) and np.array_equal(Ac.indices, Aco.indices)
        assert np.abs(Ac.data - Aco.data).max() <= 1e-12 * np.abs(Aco.data).max(), f"RAP level {l}"
        Ae = Ho.levels[l + 1].A
        assert np.abs(Ac.data - Ae.data).max() <= 1e-10 * np.abs(Ae.data).max(), f"end-to-end level {l + 1}"
    # the V-cycle on the rebuilt hierarchy
    H1 = gpu_hierarchy_to_oracle(ctx, info1, oprm)
    n3 = 3 * prob.n_nodes
    r = np.random.default_rng(5).normal(size=n3)
    z = torch.zeros(n3, dtype=torch.float64, device="cuda")
    ctx.vcycle(torch_dev(r), z)
    zo = amg.vcycle(H1, r, oprm)
    tol = 1e-12 if precision == 0 else 2e-5
    assert np.linalg.norm(z.cpu().numpy() - zo) <= tol * np.linalg.norm(zo)
    # a second re-set-up at the first state restores the first hierarchy's
    # operators bit for bit (the value-only products add in the order of the
    # full products)
    _assemble(ctx, v0, 0.4)
    ctx.amg_resetup(gprm)
    for l in range(info0.levels):
        A = export_level_matrix(ctx, l, 0)
        assert np.array_equal(A.indptr, H0.levels[l].A.indptr) and np.array_equal(A.indices, H0.levels[l].A.indices)
        assert np.array_equal(A.data, H0.levels[l].A.data), f"level {l} differs from the full set-up"


def test_resetup_order_errors(lib):
    """No hierarchy, one from a caller CSR, a new mesh or a failed set-up:
    nothing to reuse."""
    prob = synth.cube_problem(5)
    ctx = context_for(lib, prob)
    _assemble(ctx, np.zeros(prob.n_dofs), 0.5)
    with pytest.raises(lib.HfsiError) as e:
        ctx.amg_resetup(lib.amg_params())
    assert e.value.code == -4
    ctx.amg_setup(lib.amg_params(max_coarse=40))
    ctx.amg_resetup(lib.amg_params(max_coarse=40))
    ctx.set_problem(prob)
    _assemble(ctx, np.zeros(prob.n_dofs), 0.5)
    with pytest.raises(lib.HfsiError) as e:
        ctx.amg_resetup(lib.amg_params())
    assert e.value.code == -4
    # a set-up that fails (a single level of 6591 rows is over the dense limit)
    big = synth.cube_problem(12)
    ctx12 = context_for(lib, big)
    _assemble(ctx12, np.zeros(big.n_dofs), 0.5)
    ctx12.amg_setup(lib.amg_params())
    with pytest.raises(lib.HfsiError) as e:
        ctx12.amg_setup(lib.amg_params(max_levels=1))
    assert e.value.code == -8
    with pytest.raises(lib.HfsiError) as e:
        ctx12.amg_resetup(lib.amg_params())
    assert e.value.code == -4
    ctx.amg_setup(lib.amg_params(max_coarse=40))
    K_ptr = np.array([0, 1, 2], np.int32)
    ctx.amg_setup_csr(K_ptr, np.array([0, 1], np.int32), np.array([2.0, 3.0]), np.zeros(2, np.int32),
                      lib.amg_params())
    with pytest.raises(lib.HfsiError) as e:
        ctx.amg_resetup(lib.amg_params())
    assert e.value.code == -4


def test_newton_run_with_reused_coarse_grids(lib):
    """The 8^3 cube load run (5 increments, Newton to 1e-10) with the coarse
    grids of each increment's first step kept for its later steps reaches the
    oracle's converged states."""
    import torch
    prob = synth.cube_problem(8)
    print("[newton reuse] cube8 5 increments", flush=True)
    ctx = context_for(lib, prob)
    v = torch.zeros(4 * prob.n_nodes, dtype=torch.float64, device="cuda")
    fresh = lib.newton_params()
    reuse = lib.newton_params(amg_reuse=1)
    reused = []
    for k in range(1, 6):
        n0 = None
        for it in range(25):
            info, code = ctx.newton_step(v, k / 5.0, fresh if it == 0 else reuse)
            assert code == 0
            reused.append(info.amg_reused)
            n0 = info.dv_mass_norm if n0 is None else n0
            if info.dv_mass_norm <= 1e-10 * n0:
                break
    assert reused[0] == 0 and sum(reused) >= 10
    disc = fe.Discretization(prob)
    vo = newton.load_run(disc, 5, newton.NewtonParams())
    assert np.linalg.norm(v.cpu().numpy() - vo) <= 1e-9 * np.linalg.norm(vo)


@pytest.mark.parametrize("p_setup,p_resetup", [(0, 1), (1, 0)])
def test_resetup_changes_cycle_precision(lib, p_setup, p_resetup):
    """A re-set-up may switch the cycle between fp64 and fp32 (the fp32
    copies of P and R are made when the kept grids have none): its V-cycle
    matches the oracle's on the rebuilt operators to the new precision's
    accuracy, and switching back reproduces the first cycle."""
    import torch
    print(f"[reuse precision] {p_setup} -> {p_resetup}", flush=True)
    prob = synth.cube_problem(6, jitter=0.1, seed=2)
    v0 = synth.random_state(prob, 3, u_scale=0.03, p_scale=0.05).ravel()
    v1 = synth.random_state(prob, 7, u_scale=0.06, p_scale=0.2).ravel()
    g0, oprm = amg_prm_pair(lib, smoother=1, precision=p_setup, max_coarse=60, schedule="default")
    g1, _ = amg_prm_pair(lib, smoother=1, precision=p_resetup, max_coarse=60, schedule="default")
    ctx = context_for(lib, prob)
    _assemble(ctx, v0, 0.4)
    ctx.amg_setup(g0)
    n3 = 3 * prob.n_nodes
    r = torch_dev(np.random.default_rng(8).normal(size=n3))
    z0 = torch.zeros(n3, dtype=torch.float64, device="cuda")
    ctx.vcycle(r, z0)
    _assemble(ctx, v1, 0.7)
    info1 = ctx.amg_resetup(g1)
    H1 = gpu_hierarchy_to_oracle(ctx, info1, oprm)
    z = torch.zeros_like(z0)
    ctx.vcycle(r, z)
    zo = amg.vcycle(H1, r.cpu().numpy(), oprm)
    tol = 1e-12 if p_resetup == 0 else 2e-5
    assert np.linalg.norm(z.cpu().numpy() - zo) <= tol * np.linalg.norm(zo)
    _assemble(ctx, v0, 0.4)
    ctx.amg_resetup(g0)
    z2 = torch.zeros_like(z0)
    ctx.vcycle(r, z2)
    assert torch.equal(z0, z2)


def test_resetup_keeps_learned_interpolation(lib):
    """With the trained network the level-0 interpolation carries the learned
    rows; a re-set-up at another state keeps them bit for bit (and reports
    them as kept), and rebuilds the coarse operator as their Galerkin
    product."""
    import os

    from paper_1312_5561_amd import train_mlp
    print("[reuse learned] cube6", flush=True)
    w, _ = train_mlp.load(os.path.join(os.path.dirname(lib.__file__), "weights", "mlp_cube.npz"))
    prob = synth.cube_problem(6, jitter=0.1, seed=3)
    v1 = synth.random_state(prob, 9, u_scale=0.04, p_scale=0.1).ravel()
    prm_c = lib.amg_params(max_coarse=60)
    prm_l = lib.amg_params(max_coarse=60, interp=1, fallback_rho=1.0, judge_classical=0)
    ctx_c = context_for(lib, prob)
    _assemble(ctx_c, np.zeros(prob.n_dofs), 1.0)
    ctx_c.amg_setup(prm_c)
    P_classical = export_level_matrix(ctx_c, 0, 1)
    ctx = context_for(lib, prob)
    ctx.mlp_set_weights(w)
    _assemble(ctx, np.zeros(prob.n_dofs), 1.0)
    info0 = ctx.amg_setup(prm_l)
    assert info0.learned_used == 1
    P0 = export_level_matrix(ctx, 0, 1)
    Ac0 = export_level_matrix(ctx, 1, 0)
    assert (P0 != P_classical).nnz > 0
    _assemble(ctx, v1, 0.8)
    info1 = ctx.amg_resetup(prm_l)
    assert info1.learned_used == 1 and info1.rho == -1.0
    P1 = export_level_matrix(ctx, 0, 1)
    assert np.array_equal(P1.indptr, P0.indptr) and np.array_equal(P1.indices, P0.indices)
    assert np.array_equal(P1.data, P0.data)
    A = export_level_matrix(ctx, 0, 0)
    Ac = export_level_matrix(ctx, 1, 0)
    Aco = amg.on_pattern(amg.galerkin(A, P1), Ac0)
    assert np.array_equal(Ac.indptr, Aco.indptr) and np.array_equal(Ac.indices, Aco.indices)
    assert np.abs(Ac.data - Aco.data).max() <= 1e-12 * np.abs(Aco.data).max()


def test_newton_run_with_kept_preconditioner(lib):
    """amg_reuse = 3: the whole preconditioner of the first set-up serves
    every later Newton iteration of the 8^3 cube load run (FGMRES applies
    each new tangent exactly), and the run still reaches the oracle's
    converged states.  A change of AMG parameters, a set-up through the
    public entry point, a Krylov solve that fails with the kept
    preconditioner and a new inertia term each end the keeping."""
    import torch
    prob = synth.cube_problem(8)
    print("[newton keep] cube8 5 increments", flush=True)
    ctx = context_for(lib, prob)
    v = torch.zeros(4 * prob.n_nodes, dtype=torch.float64, device="cuda")
    keep = lib.newton_params(amg_reuse=3)
    reused = []
    for k in range(1, 6):
        n0 = None
        for it in range(25):
            info, code = ctx.newton_step(v, k / 5.0, keep)
            assert code == 0
            reused.append(info.amg_reused)
            n0 = info.dv_mass_norm if n0 is None else n0
            if info.dv_mass_norm <= 1e-10 * n0:
                break
    print(f"  amg_reused {reused}", flush=True)
    assert reused[0] == 0 and reused.count(2) >= len(reused) // 2
    disc = fe.Discretization(prob)
    vo = newton.load_run(disc, 5, newton.NewtonParams())
    assert np.linalg.norm(v.cpu().numpy() - vo) <= 1e-9 * np.linalg.norm(vo)
    # other AMG parameters: a new set-up, then kept again
    other = lib.newton_params(amg=lib.amg_params(smoother=0), amg_reuse=3)
    assert ctx.newton_step(v, 1.0, other)[0].amg_reused in (0, 1)
    assert ctx.newton_step(v, 1.0, other)[0].amg_reused == 2
    # a public set-up ends it
    R = torch.zeros_like(v)
    ctx.assemble_residual_tangent(v, 1.0, R)
    ctx.amg_setup(lib.amg_params(smoother=0))
    assert ctx.newton_step(v, 1.0, other)[0].amg_reused in (0, 1)
    # a solve that fails with the kept preconditioner ends it
    failing = lib.newton_params(amg=lib.amg_params(smoother=0), amg_reuse=3,
                                solve=lib.solve_params(tol=1e-14, restart=2, max_iter=2))
    v1 = v.clone()
    v1[0::4] += 1e-3
    info, code = ctx.newton_step(v1, 1.0, failing)
    assert info.amg_reused == 2 and code == 1
    assert ctx.newton_step(v1, 1.0, other)[0].amg_reused == 1
    # so does a new inertia term
    assert ctx.newton_step(v1, 1.0, other)[0].amg_reused == 2
    ctx.set_newmark(1.0, 0.05)
    assert ctx.newton_step(v1, 1.0, other)[0].amg_reused in (0, 1)
