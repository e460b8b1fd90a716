"""Pins of the oracle's learned-interpolation pieces.

* bfloat16 rounding equals torch's float32 -> bfloat16 conversion;
* the hand-written backward pass equals central differences of the loss
  (network evaluated without rounding so that the loss is smooth);
* one Adam step from zero moments moves every weight by lr * g / (|g| + eps')
  (the closed form of the bias-corrected first step);
* with a zero last layer the network output is zero (classical weights);
* where every strong neighbour of an F point is a C point and it has no
  other same-component F neighbour, the local ideal interpolation equals the
  classical weights (closed form -A_FF^{-1} A_FC with a 1x1 A_FF, no weak
  couplings);
* features of the 8^3 cube: centre slot 1, C flags equal the mask, the
  slots of the Kuhn stencil only.
"""
import numpy as np
import pytest

import synth
from oracle import amg, fe, mlp, newton


def test_bf16_rounding_matches_torch():
    import torch
    r = np.random.default_rng(0)
    x = np.concatenate([r.normal(size=5000) * 10.0 ** r.integers(-5, 5, size=5000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 0.0, 65504.0]])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(x), ref)


def _batch(seed, m=40):
    r = np.random.default_rng(seed)
    X = r.normal(size=(m, 64))
    mask = (r.uniform(size=(m, 27)) < 0.4).astype(float)
    wcl = r.normal(size=(m, 27)) * mask * 0.3
    wst = r.normal(size=(m, 27)) * mask * 0.3
    flat = r.normal(size=mlp.NPARAM) * 0.2
    return X, mask, wcl, wst, flat


def test_backward_matches_finite_differences():
    X, mask, wcl, wst, flat = _batch(1)
    loss, g = mlp.loss_and_grad(X, mask, wcl, wst, flat, rounding=False)
    r = np.random.default_rng(2)
    idx = r.choice(mlp.NPARAM, 200, replace=False)
    # only parameters that influence the output (W3/b3 columns < 27 and all hidden ones)
    for k in idx:
        h = 1e-6
        fp = flat.copy(); fp[k] += h
        fm = flat.copy(); fm[k] -= h
        lp, _ = mlp.loss_and_grad(X, mask, wcl, wst, fp, rounding=False)
        lm, _ = mlp.loss_and_grad(X, mask, wcl, wst, fm, rounding=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_first_adam_step_closed_form():
    r = np.random.default_rng(3)
    w = r.normal(size=100)
    g = r.normal(size=100)
    w1, m, v = mlp.adam_step(w, g, np.zeros(100), np.zeros(100), 1, lr=1e-3, eps=1e-8)
    assert np.allclose(w1, w - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_zero_last_layer_gives_zero_correction():
    flat = mlp.init_weights(5)
    X = np.random.default_rng(4).normal(size=(30, 64))
    out, *_ = mlp.forward(X, flat)
    assert np.all(out == 0.0)


def test_ideal_target_reduces_to_classical_when_f_has_no_f_neighbours():
    import scipy.sparse as sp
    # three decoupled components on a chain of 5 lattice nodes C - F - C - F - C:
    # an F point sees only its two C neighbours, so both the ideal and the
    # classical weights are -a_ij / a_ii = 1 / 2.5
    chain = sp.diags([-np.ones(4), 2.5 * np.ones(5), -np.ones(4)], [-1, 0, 1])
    A = sp.kron(chain, sp.identity(3)).tocsr()
    A.sort_indices()
    comp = np.tile(np.arange(3), 5)
    state = np.repeat(np.array([1, -1, 1, -1, 1], np.int8), 3)
    S_ptr, S_idx = amg.strength(A, comp, 0.25)
    P, _ = amg.interpolation(A, S_ptr, S_idx, state, comp)
    lattice = np.stack([np.arange(5), np.zeros(5, int), np.zeros(5, int)], 1)
    for node in (1, 3):
        for c in range(3):
            i = 3 * node + c
            w = mlp.ideal_target(A, comp, state, S_ptr, S_idx, lattice, i)
            assert np.allclose(w[[12, 14]], 0.4, rtol=1e-15)      # slots dx = -1, +1
            assert np.count_nonzero(w) == 2
            assert np.allclose(P.getrow(i).data, 0.4, rtol=1e-15)


def test_cube_features_and_targets():
    prob = synth.cube_problem(6, jitter=0.1, seed=3)
    d = fe.Discretization(prob)
    K, b, A, B2, s = newton.linear_system(d, np.zeros(4 * d.n), 1.0)
    comp = np.tile(np.arange(3), d.n)
    S_ptr, S_idx = amg.strength(A, comp, 0.5)
    st = amg.pmis(S_ptr, S_idx, A.shape[0], 12345, 0)
    P, _ = amg.interpolation(A, S_ptr, S_idx, st, comp)
    rows, X, mask, wcl = mlp.samples(A, comp, st, S_ptr, S_idx, P, prob.lattice,
                                     mlp.material_features(prob.materials))
    assert len(rows) > 0 and np.all(st[rows] == -1)
    assert np.all(X[:, 13] == 1.0)                       # centre slot: a_ii / a_ii
    assert np.array_equal(X[:, 27:54] == 1.0, mask == 1.0)
    nz = (X[:, :27] != 0).sum(1)
    assert nz.max() <= 15                                # Kuhn stencil: 14 neighbours + centre
    # classical rows sum to the P row sums
    assert np.allclose(wcl.sum(1), [P.getrow(i).sum() for i in rows], rtol=1e-6, atol=1e-7)
    # targets exist and live on the mask
    for m in range(0, len(rows), 97):
        t = mlp.ideal_target(A, comp, st, S_ptr, S_idx, prob.lattice, rows[m])
        assert np.all(t[mask[m] == 0] == 0.0)
        assert np.isfinite(t).all()
