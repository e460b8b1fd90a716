"""Further pins of the oracle's AMG pieces, each against a closed form or a
hand-worked case rather than against the oracle itself.

* Chebyshev smoothing of degree k (1..4) on a diagonal D^{-1}A whose
  eigenvalues sit at the k+1 extrema of the shifted Chebyshev polynomial:
  the error components are (-1)^j / T_k(sigma), with T_k from its cosh form;
  a wrong rho update only shows from degree 3 on.
* The V-cycle without smoothing is the Galerkin coarse solve
  Q (Q^T A Q)^{-1} Q^T b with Q the product of the interpolations, on two and
  three levels (a transposed or misplaced transfer fails it).
* The stationary iteration of that cycle is an A-orthogonal projection, so
  the convergence factor is (||E e_0||_A / ||e_0||_A)^(1/k) with E e_0
  computed by a dense solve; a one-level (exact) hierarchy gives at most
  rounding.
* A V-cycle with a symmetric schedule (same sweeps and smoother before and
  after, l1-Jacobi) is a symmetric operator.
* Strength of connection and both interpolations on a hand-worked matrix
  with positive off-diagonal couplings and negative diagonals (the sign
  rules: sgn(a_ii) in the strength test, abar_kl = a_kl only where its sign
  differs from a_kk's); negating the matrix changes neither S nor P.
* Coarse-operator sparsification on a hand-worked matrix (the symmetric
  threshold eps sqrt(|a_ii a_jj|), explicit zeros dropped, diagonal kept),
  and a sparsified hierarchy: coarse values equal the Galerkin product at the
  kept positions, a re-set-up keeps the set-up's pattern.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import amg


def _lap3(n):
    L = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1])
    I = sp.identity(n)
    A = (sp.kron(sp.kron(L, I), I) + sp.kron(sp.kron(I, L), I) + sp.kron(sp.kron(I, I), L)).tocsr()
    A.sort_indices()
    return A


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_chebyshev_equioscillates_at_degree(k):
    lam, ratio = 2.7, 30.0
    a, b = lam / ratio, 1.1 * lam
    theta, delta = 0.5 * (b + a), 0.5 * (b - a)
    sigma = theta / delta
    Tk = math.cosh(k * math.acosh(sigma))
    # eigenvalues of D^{-1}A at the extrema of T_k((theta - x)/delta)
    j = np.arange(k + 1)
    eig = theta - delta * np.cos(j * np.pi / k)
    d = np.linspace(0.5, 3.0, k + 1)           # a non-trivial diagonal D
    A = sp.diags(d * eig).tocsr()
    e0 = np.ones(k + 1)
    x = amg.chebyshev(A, 1.0 / d, lam, np.zeros(k + 1), -e0, degree=k, ratio=ratio)
    # error after smoothing = p(D^{-1}A) e0, with x_true = 0: e = x - 0, e0 = -1
    assert np.allclose(x, -((-1.0) ** j) / Tk, rtol=1e-12, atol=0)
    # and an eigenvalue inside the interval between the extrema is damped more
    mid = theta - delta * np.cos(0.5 * np.pi / k)
    y = amg.chebyshev(sp.diags([mid]).tocsr(), np.ones(1), lam, np.zeros(1), -np.ones(1), degree=k, ratio=ratio)
    assert abs(y[0]) < 1.0 / Tk


def _zero_smoothing(**kw):
    """No smoothing and the exact Galerkin coarse operators."""
    return amg.AmgParams(smoother="l1jacobi", nu_pre=0, nu_post=0, nu_pre_coarse=0, nu_post_coarse=0,
                         drop_tol=0.0, **kw)


@pytest.mark.parametrize("levels", [2, 3])
def test_vcycle_without_smoothing_is_the_galerkin_solve(levels):
    A = _lap3(7)
    n = A.shape[0]
    prm = _zero_smoothing(max_coarse=10, max_levels=levels)
    H = amg.setup(A, np.zeros(n, np.int64), prm)
    assert len(H.levels) == levels
    Q = np.eye(n)
    for L in H.levels[:-1]:
        Q = Q @ L.P.toarray()
    b = np.random.default_rng(4).standard_normal(n)
    Ad = A.toarray()
    ref = Q @ np.linalg.solve(Q.T @ Ad @ Q, Q.T @ b)
    y = amg.vcycle(H, b, prm)
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()


def test_convergence_factor_of_a_projection_cycle():
    A = _lap3(6)
    n = A.shape[0]
    prm = _zero_smoothing(max_coarse=60, max_levels=2)
    H = amg.setup(A, np.zeros(n, np.int64), prm)
    P = H.levels[0].P.toarray()
    Ad = A.toarray()
    from oracle import rng
    e0 = rng.uniform_pm1(777, 0, n)
    e1 = e0 - P @ np.linalg.solve(P.T @ Ad @ P, P.T @ (Ad @ e0))
    ratio = math.sqrt(e1 @ Ad @ e1) / math.sqrt(e0 @ Ad @ e0)
    for cycles in (1, 5, 10):
        rho = amg.convergence_factor(H, prm, cycles=cycles, seed=777)
        assert abs(rho - ratio ** (1.0 / cycles)) <= 1e-9
    # one level: the cycle is the exact solve, the error vanishes to rounding
    H1 = amg.setup(A, np.zeros(n, np.int64), amg.AmgParams(max_coarse=n + 1))
    assert len(H1.levels) == 1
    assert amg.convergence_factor(H1, amg.AmgParams(max_coarse=n + 1), cycles=1) <= 1e-12


def test_symmetric_schedule_gives_a_symmetric_cycle():
    A = _lap3(6)
    n = A.shape[0]
    prm = amg.AmgParams(smoother="l1jacobi", nu_pre=2, nu_post=2, nu_pre_coarse=1, nu_post_coarse=1,
                        cheb_degree_pre=1, cheb_degree=1, cheb_degree_coarse=1, max_coarse=8)
    H = amg.setup(A, np.zeros(n, np.int64), prm)
    assert len(H.levels) >= 3
    B = np.stack([amg.vcycle(H, np.eye(n)[:, j], prm) for j in range(n)], axis=1)
    assert np.abs(B - B.T).max() <= 1e-12 * np.abs(B).max()
    # and positive definite (an SPD smoother on both sides of the correction)
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0


# hand-worked matrix: rows 0 and 3 have positive diagonals, rows 1 and 2
# negative ones; one positive coupling (3, 2) of the same sign as a_33
_HAND = np.array([
    [4.0, -1.0, -1.0, -1.5],
    [-2.0, -4.0, 3.0, 1.0],
    [-1.0, 1.0, -5.0, 0.5],
    [-1.5, -1.0, 0.5, 3.0],
])


def _hand(sign=1.0):
    A = sp.csr_matrix(sign * _HAND)
    A.sort_indices()
    return A


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_strength_sign_rule_by_hand(sign):
    """theta = 0.25.  Row 0 (a_00 > 0): -a_0j = 1, 1, 1.5, m = 1.5 -> all
    strong.  Row 1 (a_11 < 0): -a_1j sgn(a_11) = a_1j = -2, 3, 1 -> m = 3,
    threshold 0.75: {2, 3}.  Row 2: a_2j = -1, 1, 0.5 -> m = 1, threshold
    0.25: {1, 3}.  Row 3: -a_3j = 1.5, 1, -0.5 -> m = 1.5, threshold 0.375:
    {0, 1}.  Negating A changes nothing."""
    ptr, idx = amg.strength(_hand(sign), np.zeros(4, np.int64), theta=0.25)
    S = [sorted(idx[ptr[i]:ptr[i + 1]].tolist()) for i in range(4)]
    assert S == [[1, 2, 3], [2, 3], [1, 3], [0, 1]]


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_classical_interpolation_sign_rule_by_hand(sign):
    """F point 0 with C points 1, 2 and strong F neighbour 3.  abar_31 = -1
    (sign differs from a_33 = 3), abar_32 = 0 (0.5 has a_33's sign), so
    sum_{m in C_0} abar_3m = -1 and
      w_01 = -(-1 + (-1.5)(-1)/(-1)) / 4 = 0.625,
      w_02 = -(-1 + 0) / 4 = 0.25.
    (Without the sign rule: 1.0 and -0.125.)"""
    A = _hand(sign)
    state = np.array([-1, 1, 1, -1], np.int8)
    w = amg.interp_row(A, {1, 2, 3}, state, np.zeros(4, np.int64), 0)
    assert w.keys() == {1, 2}
    assert abs(w[1] - 0.625) <= 1e-15 and abs(w[2] - 0.25) <= 1e-15


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_extpi_sign_rule_by_hand(sign):
    """Extended+i for the same row, with S_3 = {0, 1} (theta 0.25): Chat_0 =
    {1, 2}; s_3 = abar_31 + abar_32 + abar_30 = -1 + 0 - 1.5 = -2.5;
    atilde_00 = 4 + (-1.5)(-1.5)/(-2.5) = 3.1;
    w_01 = -(-1 + (-1.5)(-1)/(-2.5)) / 3.1 = 1.6/3.1, w_02 = 1/3.1."""
    A = _hand(sign)
    ptr, idx = amg.strength(A, np.zeros(4, np.int64), theta=0.25)
    state = np.array([-1, 1, 1, -1], np.int8)
    w = amg.interp_row_extpi(A, ptr, idx, state, np.zeros(4, np.int64), 0)
    assert w.keys() == {1, 2}
    assert abs(w[1] - 1.6 / 3.1) <= 1e-15 and abs(w[2] - 1.0 / 3.1) <= 1e-15


def test_negated_operator_gives_the_same_hierarchy():
    """S, the splitting, P (both interpolations) and -A_c for -A."""
    r = np.random.default_rng(9)
    A = _lap3(6).tolil()
    # some positive couplings (symmetric), diagonal kept dominant
    for _ in range(40):
        i, j = r.integers(0, A.shape[0], 2)
        if i != j:
            A[i, j] = A[j, i] = 0.3
    A = A.tocsr()
    A = (A + sp.diags(np.asarray(abs(A).sum(axis=1)).ravel() * 0.1)).tocsr()
    A.sort_indices()
    for kind in ("classical", "ext+i"):
        prm = amg.AmgParams(interp=kind, max_coarse=20)
        H1 = amg.setup(A, np.zeros(A.shape[0], np.int64), prm)
        H2 = amg.setup((-A).tocsr(), np.zeros(A.shape[0], np.int64), prm)
        assert len(H1.levels) == len(H2.levels) >= 2
        for L1, L2 in zip(H1.levels[:-1], H2.levels[:-1]):
            assert np.array_equal(L1.state, L2.state)
            assert (L1.P != L2.P).nnz == 0
            assert np.abs((L1.A + L2.A).data).max(initial=0.0) == 0.0


def test_drop_small_by_hand():
    """eps = 1e-3 on a hand-made symmetric matrix with diagonal (4, 1, 9, 0.25):
    threshold of (i, j) = 1e-3 sqrt(a_ii a_jj):
      (0,1): 2e-3,  |0.0015| < 2e-3  -> dropped (both sides of the pair);
      (0,2): 6e-3,  |-1|             -> kept;
      (1,2): 3e-3,  |0.0031|         -> kept;
      (2,3): 1.5e-3, |-0.0014|       -> dropped;
      (1,3): 5e-4,  |0.0006|         -> kept (a row-scaled test by a_11 = 1
             would drop it, one scaled by a_33 would keep (3,1) too);
      (0,3): explicit zero           -> dropped.
    The diagonal always stays; eps = 0 changes nothing."""
    A = np.array([[4.0, 0.0015, -1.0, 0.0],
                  [0.0015, 1.0, 0.0031, 0.0006],
                  [-1.0, 0.0031, 9.0, -0.0014],
                  [0.0, 0.0006, -0.0014, 0.25]])
    # every position stored, the zeros of (0,3) and (3,0) explicitly
    rows = [0, 0, 0, 0, 1, 1, 1, 1, 2, 2, 2, 2, 3, 3, 3, 3]
    cols = [0, 1, 2, 3] * 4
    M = sp.csr_matrix((A[rows, cols], (rows, cols)), shape=(4, 4))
    M.sort_indices()
    assert M.nnz == 16
    D = amg.drop_small(M, 1e-3)
    keep = {(0, 0), (0, 2), (1, 1), (1, 2), (1, 3), (2, 0), (2, 1), (2, 2), (3, 1), (3, 3)}
    got = set(zip(np.repeat(np.arange(4), np.diff(D.indptr)).tolist(), D.indices.tolist()))
    assert got == keep
    assert np.array_equal(D.toarray(), np.where([[(i, j) in keep for j in range(4)] for i in range(4)], A, 0.0))
    assert amg.drop_small(M, 0.0) is M


def test_sparsified_hierarchy_and_its_resetup():
    """With drop_tol > 0 every coarse operator is the Galerkin product minus
    the small entries (values equal at the kept positions), symmetric for a
    symmetric A; a re-set-up with a new operator keeps the set-up's pattern
    and takes the new Galerkin values there."""
    r = np.random.default_rng(5)
    A = _lap3(8).tolil()
    for _ in range(60):
        i, j = r.integers(0, A.shape[0], 2)
        if i != j and A[i, j] == 0:
            A[i, j] = A[j, i] = -1e-4 * r.uniform(0.5, 1.5)
    A = A.tocsr()
    A.sort_indices()
    prm = amg.AmgParams(max_coarse=30, drop_tol=2e-3)
    H = amg.setup(A, np.zeros(A.shape[0], np.int64), prm)
    H0 = amg.setup(A, np.zeros(A.shape[0], np.int64), amg.AmgParams(max_coarse=30, drop_tol=0.0))
    assert len(H.levels) >= 3
    assert np.array_equal(H.levels[0].state, H0.levels[0].state)
    G = amg.galerkin(H.levels[0].A, H.levels[0].P)
    Ac = H.levels[1].A
    assert Ac.nnz < G.nnz
    assert np.abs(amg.on_pattern(G, Ac).toarray() - Ac.toarray()).max() == 0.0
    assert np.abs((Ac - Ac.T).toarray()).max() <= 1e-14 * np.abs(Ac.data).max()
    B = (A * 1.5).tocsr()
    HB = amg.resetup(B, H, prm)
    for a, b in zip(H.levels, HB.levels):
        assert np.array_equal(a.A.indptr, b.A.indptr) and np.array_equal(a.A.indices, b.A.indices)
    GB = amg.galerkin(HB.levels[0].A, H.levels[0].P)
    assert np.abs(amg.on_pattern(GB, Ac).toarray() - HB.levels[1].A.toarray()).max() <= 1e-13 * np.abs(GB.data).max()
