"""Run-to-run determinism of the GPU path: the same inputs give the same bits.

The assembly is atomic-free (element colours), the sparse products add in a
fixed order, every reduction sums its partials in a fixed order and the
extended+i weights are accumulated per neighbour group in a fixed order, so
two fresh contexts (and two calls on one context) must produce identical
residuals, tangents, hierarchies, Krylov solutions and Newton updates, in
the fp64 and the fp32 cycle, with the block preconditioner and with the
coupled Vanka cycle (multiplicative and additive).
"""
import numpy as np
import pytest

import synth
from gpu_helpers import context_for, export_level_matrix, torch_dev

pytestmark = pytest.mark.gpu


def _run(lib, prob, v, amg_prm, method=0):
    import torch
    ctx = context_for(lib, prob)
    vt = torch_dev(v)
    R = torch.zeros_like(vt)
    view, _ = ctx.assemble_residual_tangent(vt, 0.7, R)
    K = ctx.export_tangent(view)
    info = ctx.amg_setup(amg_prm)
    levels = []
    if not amg_prm.coupled:
        for lev in range(info.levels):
            A = export_level_matrix(ctx, lev, 0)
            P = export_level_matrix(ctx, lev, 1) if lev + 1 < info.levels else None
            levels.append((A, P))
    else:
        for lev in range(info.levels):
            levels.append(tuple(export_level_matrix(ctx, lev, w) for w in (10, 11, 12, 13)))
    b = -R
    x = torch.zeros_like(b)
    si, code = ctx.krylov_amg_solve(b, x, lib.solve_params(tol=1e-10, restart=100, max_iter=500, method=method))
    assert code == 0
    # a second solve on the same context, same hierarchy
    x2 = torch.zeros_like(b)
    si2, _ = ctx.krylov_amg_solve(b, x2, lib.solve_params(tol=1e-10, restart=100, max_iter=500, method=method))
    return dict(R=R.cpu().numpy(), K=[np.asarray(K[k]).copy() for k in sorted(K)], levels=levels, x=x.cpu().numpy(),
                x2=x2.cpu().numpy(), its=(si.iterations, si2.iterations))


def _same_csr(A, B):
    return (A.shape == B.shape and np.array_equal(A.indptr, B.indptr) and np.array_equal(A.indices, B.indices)
            and np.array_equal(A.data, B.data))


@pytest.mark.parametrize("case", ["fp64", "fp32", "l1jacobi_bicgstab", "coupled", "coupled_additive"])
def test_two_runs_are_bit_identical(lib, case):
    prob = synth.cube_problem(10, jitter=0.1, seed=4)
    v = synth.random_state(prob, 5, u_scale=0.03, p_scale=0.05).ravel()
    method = 0
    if case == "fp64":
        prm = lib.amg_params(precision=0, max_coarse=80)
    elif case == "fp32":
        prm = lib.amg_params(precision=1, max_coarse=80)
    elif case == "l1jacobi_bicgstab":
        prm = lib.amg_params(precision=1, max_coarse=80, smoother=0)
        method = 1
    elif case == "coupled":
        prm = lib.amg_params(max_coarse=80, coupled=1, vanka_steps=2)
    else:
        prm = lib.amg_params(max_coarse=80, coupled=2, vanka_steps=2, vanka_omega=0.8)
    print(f"[determinism] {case}", flush=True)
    a = _run(lib, prob, v, prm, method)
    b = _run(lib, prob, v, prm, method)
    assert np.array_equal(a["R"], b["R"])
    for ka, kb in zip(a["K"], b["K"]):
        assert np.array_equal(ka, kb)
    assert len(a["levels"]) == len(b["levels"]) >= 2
    for la, lb in zip(a["levels"], b["levels"]):
        for ma, mb in zip(la, lb):
            assert (ma is None and mb is None) or _same_csr(ma, mb)
    assert a["its"] == b["its"] and a["its"][0] == a["its"][1]
    assert np.array_equal(a["x"], b["x"])
    assert np.array_equal(a["x"], a["x2"])
