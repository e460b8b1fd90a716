"""GPU parity of residual/tangent assembly against the CPU oracle.

Same seeded mesh and state on both sides; R, every stored entry of the
Dirichlet-eliminated K, the A block (pattern bit-exact) and the Schur
diagonal must agree to 1e-12 relative to the largest entry.
"""
import numpy as np
import pytest

import synth
from oracle import fe

pytestmark = pytest.mark.gpu

CASES = {
    "cube2_jitter": lambda: synth.cube_problem(2, jitter=0.15, seed=3),
    "cube8": lambda: synth.cube_problem(8),
    "cube5_jitter": lambda: synth.cube_problem(5, jitter=0.1, seed=9, kappa=1e5),
    "tube_small": lambda: synth.tube_problem(n_theta=16, n_media=2, n_adv=2, n_z=6),
}


def _gpu_assemble(lib, prob, v, load):
    import torch
    ctx = lib.Context(0)
    ctx.set_problem(prob)
    vt = torch.from_numpy(v.ravel().copy()).cuda()
    R = torch.zeros_like(vt)
    view, info = ctx.assemble_residual_tangent(vt, load, R)
    out = ctx.export_tangent(view)
    out["R"] = R.cpu().numpy()
    out["info"] = info
    return ctx, out


def _oracle(prob, v, load):
    d = fe.Discretization(prob)
    R, val = d.assemble(v.ravel(), load)
    R, val = d.apply_dirichlet(R, val)
    K = d.csr(val)
    A, B2, s = d.blocks(val)
    return d, R, K, A, s


def _blocks_to_csr(out, n):
    import scipy.sparse as sp
    bp, bc, bv = out["block_ptr"], out["block_col"], out["block_val"]
    rows = np.repeat(np.arange(n), np.diff(bp))
    r = (4 * rows[:, None, None] + np.arange(4)[None, :, None]).repeat(4, axis=2)
    c = (4 * bc[:, None, None] + np.arange(4)[None, None, :]).repeat(4, axis=1)
    M = sp.csr_matrix((bv.ravel(), (r.ravel(), c.ravel())), shape=(4 * n, 4 * n))
    M.sum_duplicates()
    M.sort_indices()
    return M


@pytest.mark.parametrize("case", list(CASES))
def test_assembly_matches_oracle(lib, case):
    prob = CASES[case]()
    v = synth.random_state(prob, 21, u_scale=0.05, p_scale=0.2)
    d, R, K, A, s = _oracle(prob, v, 0.6)
    print(f"[assembly parity] case={case} n={prob.n_nodes} m={prob.n_tets}", flush=True)
    _, out = _gpu_assemble(lib, prob, v, 0.6)
    n = prob.n_nodes
    # pattern: node graph identical
    assert np.array_equal(out["block_ptr"], d.node_ptr)
    assert np.array_equal(out["block_col"], d.node_cols)
    Kg = _blocks_to_csr(out, n)
    assert np.array_equal(Kg.indptr, K.indptr) and np.array_equal(Kg.indices, K.indices)
    scale = np.abs(K.data).max()
    assert np.abs(Kg.data - K.data).max() <= 1e-12 * scale
    assert np.abs(out["R"] - R).max() <= 1e-12 * max(np.abs(R).max(), 1e-300)
    assert np.array_equal(out["a_ptr"], A.indptr) and np.array_equal(out["a_col"], A.indices)
    assert np.abs(out["a_val"] - A.data).max() <= 1e-12 * np.abs(A.data).max()
    assert np.allclose(out["schur"], s, rtol=1e-13, atol=0)
    assert out["info"].min_J > 0


def test_inverted_element_is_reported(lib):
    import torch
    prob = synth.cube_problem(2)
    ctx = lib.Context(0)
    ctx.set_problem(prob)
    v = np.zeros((prob.n_nodes, 4))
    v[:, 0] = -2.0 * prob.X[:, 0]   # F_xx = -1: every element inverted
    vt = torch.from_numpy(v.ravel()).cuda()
    R = torch.zeros_like(vt)
    with pytest.raises(lib.HfsiError) as e:
        ctx.assemble_residual_tangent(vt, 0.0, R)
    assert e.value.code == -5
    assert "has J <= 0" in str(e.value)   # the context's own error text


def test_zero_state_zero_residual(lib):
    import torch
    prob = synth.tube_problem(n_theta=8, n_media=1, n_adv=1, n_z=2)
    ctx = lib.Context(0)
    ctx.set_problem(prob)
    vt = torch.zeros(4 * prob.n_nodes, dtype=torch.float64, device="cuda")
    R = torch.ones_like(vt)
    ctx.assemble_residual_tangent(vt, 0.0, R)
    assert float(R.abs().max()) <= 1e-15
