"""GPU parity of the AMG set-up against the oracle, level by level.

Every level is checked on identical inputs: the oracle recomputes the
strength pattern, the PMIS splitting, the interpolation and the Galerkin
product from the GPU's own A_l (and P_l), so that rounding in earlier levels
cannot blur the comparison.  Splittings and sparsity patterns must be
bit-exact; values agree to 1e-12 relative.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from gpu_helpers import amg_prm_pair, context_for, export_level_matrix, oracle_system
from oracle import amg

pytestmark = pytest.mark.gpu


def _check_levels(ctx, info, theta, seed, rtol=1e-12, kind="classical", p_max=4, drop_tol=0.0):
    for l in range(info.levels - 1):
        A = export_level_matrix(ctx, l, 0)
        comp = ctx.amg_export(l, 4)
        flags = ctx.amg_export(l, 2)
        st = ctx.amg_export(l, 3)
        S_ptr, S_idx = amg.strength(A, comp, theta)
        rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
        o_flags = np.zeros(A.nnz, np.uint8)
        key_all = rows * A.shape[1] + A.indices
        key_s = np.repeat(np.arange(A.shape[0]), np.diff(S_ptr)) * A.shape[1] + S_idx
        o_flags[np.isin(key_all, key_s)] = 1
        assert np.array_equal(flags, o_flags), f"strength differs on level {l}"
        o_st = amg.pmis(S_ptr, S_idx, A.shape[0], seed, l)
        assert np.array_equal(st, o_st), f"PMIS splitting differs on level {l}"
        P = export_level_matrix(ctx, l, 1)
        Po, _ = amg.interpolation(A, S_ptr, S_idx, o_st, comp, kind, p_max)
        assert np.array_equal(P.indptr, Po.indptr) and np.array_equal(P.indices, Po.indices), f"P pattern level {l}"
        assert np.abs(P.data - Po.data).max() <= rtol * max(1.0, np.abs(Po.data).max())
        Ac = export_level_matrix(ctx, l + 1, 0)
        Aco = amg.coarse_operator(A, P, drop_tol)
        assert np.array_equal(Ac.indptr, Aco.indptr) and np.array_equal(Ac.indices, Aco.indices), f"RAP pattern {l}"
        assert np.abs(Ac.data - Aco.data).max() <= rtol * np.abs(Aco.data).max()


@pytest.mark.parametrize("case,theta,kind,p_max,drop", [
    ("cube8", 0.15, "classical", 4, 0.0), ("cube8", 0.5, "classical", 4, 0.0),
    ("cube5_jitter_state", 0.15, "classical", 4, 0.0), ("tube_small", 0.15, "classical", 4, 0.0),
    ("laplacian3d", 0.15, "classical", 4, 0.0), ("cube8", 0.15, "ext+i", 4, 0.0), ("cube8", 0.15, "ext+i", 0, 0.0),
    ("cube5_jitter_state", 0.15, "ext+i", 4, 0.0), ("tube_small", 0.15, "ext+i", 4, 0.0),
    ("laplacian3d", 0.15, "ext+i", 3, 0.0), ("laplacian3d", 0.25, "ext+i", 0, 0.0),
    ("cube8", 0.15, "ext+i", 4, 2e-3), ("tube_small", 0.15, "ext+i", 4, 1e-3), ("cube5_jitter_state", 0.15,
                                                                               "classical", 4, 5e-3)])
def test_hierarchy_matches_oracle_level_by_level(lib, case, theta, kind, p_max, drop):
    """drop > 0: coarse operators sparsified (drop_tol), patterns bit-exact."""
    print(f"[amg parity] case={case} theta={theta} interp={kind} p_max={p_max} drop={drop}", flush=True)
    if case == "laplacian3d":
        import test_oracle_amg as T
        A = T.laplacian(14, 13, 12)
        comp = np.zeros(A.shape[0], np.int32)
    else:
        if case == "cube8":
            prob = synth.cube_problem(8)
            v = np.zeros(4 * prob.n_nodes)
        elif case == "cube5_jitter_state":
            prob = synth.cube_problem(5, jitter=0.15, seed=4)
            v = synth.random_state(prob, 5, u_scale=0.05, p_scale=0.1).ravel()
        else:
            prob = synth.tube_problem(n_theta=16, n_media=2, n_adv=2, n_z=10)
            v = synth.random_state(prob, 6, u_scale=0.02, p_scale=0.5).ravel()
        _, K, b, A, B2, s = oracle_system(prob, v, 0.3)
        comp = np.tile(np.arange(3, dtype=np.int32), prob.n_nodes)
    gprm, oprm = amg_prm_pair(lib, max_coarse=50, theta=theta, kind=kind, p_max=p_max, drop_tol=drop)
    ctx = lib.Context(0)
    info = ctx.amg_setup_csr(A.indptr, A.indices, A.data, comp, gprm)
    assert info.levels >= 2
    L0 = export_level_matrix(ctx, 0, 0)
    assert np.array_equal(L0.data, A.data)
    _check_levels(ctx, info, oprm.theta, oprm.seed, kind=kind, p_max=p_max, drop_tol=oprm.drop_tol)


def test_full_size_cube48_splitting_and_sampled_rows(lib):
    """48^3 cube at its real size: GPU assembly + set-up; the level-0 splitting
    is bit-exact with the oracle's PMIS on the GPU's A, and sampled rows of P
    match the oracle's interpolation formula row by row."""
    import torch
    prob = synth.cube_problem(48)
    ctx = context_for(lib, prob)
    n = prob.n_nodes
    v = torch.zeros(4 * n, dtype=torch.float64, device="cuda")
    R = torch.zeros_like(v)
    print("[amg full size] cube48 assemble + setup", flush=True)
    ctx.assemble_residual_tangent(v, 1.0, R)
    gprm, oprm = amg_prm_pair(lib)
    info = ctx.amg_setup(gprm)
    A = export_level_matrix(ctx, 0, 0)
    comp = ctx.amg_export(0, 4)
    st = ctx.amg_export(0, 3)
    S_ptr, S_idx = amg.strength(A, comp, oprm.theta)
    o_st = amg.pmis(S_ptr, S_idx, A.shape[0], oprm.seed, 0)
    assert np.array_equal(st, o_st)
    P = export_level_matrix(ctx, 0, 1)
    cidx = np.cumsum(st == 1) - 1
    rng = np.random.default_rng(0)
    for i in rng.choice(A.shape[0], 300, replace=False):
        if st[i] == 1:
            continue
        w = amg.interp_row(A, set(S_idx[S_ptr[i]:S_ptr[i + 1]].tolist()), st, comp, int(i))
        cols = P.indices[P.indptr[i]:P.indptr[i + 1]]
        vals = P.data[P.indptr[i]:P.indptr[i + 1]]
        assert np.array_equal(cols, np.array([cidx[j] for j in sorted(w)], dtype=cols.dtype))
        assert np.allclose(vals, [w[j] for j in sorted(w)], rtol=1e-12, atol=1e-14)
    # Galerkin rows sampled: A_c = R A P row by row
    Ac = export_level_matrix(ctx, 1, 0)
    for I in rng.choice(Ac.shape[0], 50, replace=False):
        ref = (P[:, I].T @ A @ P).toarray().ravel()   # row I of P^T A P
        row = np.zeros(Ac.shape[1])
        row[Ac.indices[Ac.indptr[I]:Ac.indptr[I + 1]]] = Ac.data[Ac.indptr[I]:Ac.indptr[I + 1]]
        assert np.abs(row - ref).max() <= 1e-12 * np.abs(ref).max()
    print(f"[amg full size] levels={info.levels} rows={list(info.rows)[:info.levels]} "
          f"opc={info.op_complexity:.3f} setup={info.seconds*1e3:.1f} ms", flush=True)


def test_capacity_and_order_errors(lib):
    ctx = lib.Context(0)
    with pytest.raises(lib.HfsiError) as e:
        ctx.amg_export(0, 0)
    assert e.value.code == -4
    with pytest.raises(lib.HfsiError):
        ctx.amg_setup_csr(np.array([0, 1]), np.array([5]), np.array([1.0]), np.array([0]))


def test_failed_setup_then_valid_setup(lib):
    """A set-up that fails after work was queued on the second stream (the
    coarsest level exceeds 4096 rows with max_levels = 1) leaves the context
    usable: the next set-up and solve on it succeed."""
    import torch
    prob = synth.cube_problem(12)
    ctx = context_for(lib, prob)
    v = torch.zeros(prob.n_dofs, dtype=torch.float64, device="cuda")
    R = torch.zeros_like(v)
    ctx.assemble_residual_tangent(v, 1.0, R)
    with pytest.raises(lib.HfsiError) as e:
        ctx.amg_setup(lib.amg_params(smoother=1, precision=1, max_levels=1))
    assert e.value.code == -8 and "4096" in str(e.value)
    info = ctx.amg_setup(lib.amg_params(smoother=1, precision=1))
    assert info.levels >= 2
    x = torch.zeros_like(R)
    si, code = ctx.krylov_amg_solve(-R, x, lib.solve_params(tol=1e-8, restart=100, max_iter=500))
    assert code == 0 and si.converged

