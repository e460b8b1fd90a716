"""Pins of the oracle's AMG pieces.

* SplitMix64 reproduces its published test vector;
* vectorised PMIS equals a brute-force replay of the rounds on small graphs,
  and its splitting has the PMIS properties (C independent in the
  symmetrised strength graph, every point decided, every F point with
  lambda > 0 strongly depends on a C point);
* classical interpolation reproduces constants on zero-row-sum matrices
  and is the identity on C rows; so does extended+i, with and without
  truncation (which rescales to the row sum); on the path C-F-F-C it gives
  the linear interpolant (2/3, 1/3) through the distance-two C point, and a
  truncated row keeps the largest weights;
* the Galerkin product equals the dense P^T A P;
* l1-Jacobi never increases the A-norm of the error for SPD A;
* the Chebyshev smoother damps the extreme eigen-components by exactly
  1/T_2((b+a)/(b-a));
* the Lanczos estimate converges to the largest eigenvalue;
* re-set-up on kept coarse grids: with the original operator it rebuilds
  the hierarchy, it is covariant under scaling of the operator, and on two
  levels its coarse correction for a new operator is the energy projection
  onto the kept interpolation's range (which a stale coarse operator fails).
"""
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse as sp

from oracle import amg, rng

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_vector():
    vals = [int(x) for x in open(os.path.join(GOLD, "splitmix64_seed1234567.txt")) if x.strip() and not x.startswith("#")]
    assert [rng.splitmix64_scalar(1234567, k) for k in range(5)] == vals
    assert [int(x) for x in rng.splitmix64(1234567, np.arange(5))] == vals


def laplacian(nx, ny=1, nz=1, neumann=False):
    """7-point (or 5/3-point) finite-difference Laplacian."""
    def lap1(n):
        if n == 1:
            return sp.csr_matrix((1, 1))
        L = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tolil()
        if neumann:
            L[0, 0] = 1
            L[n - 1, n - 1] = 1
        return L.tocsr()
    I = [sp.identity(k) for k in (nx, ny, nz)]
    L = (sp.kron(I[2], sp.kron(I[1], lap1(nx))) + sp.kron(I[2], sp.kron(lap1(ny), I[0]))
         + sp.kron(lap1(nz), sp.kron(I[1], I[0])))
    L = L.tocsr()
    L.sort_indices()
    return L


def _random_strength_graph(r, n):
    S = [sorted(set(int(j) for j in r.choice(n, size=min(int(r.integers(0, 4)), n), replace=False) if j != i)) for i in range(n)]
    ptr = np.zeros(n + 1, np.int64)
    ptr[1:] = np.cumsum([len(s) for s in S])
    idx = np.array([j for s in S for j in s], np.int64)
    return S, ptr, idx


def test_pmis_matches_bruteforce():
    r = np.random.default_rng(0)
    for trial in range(200):
        n = int(r.integers(1, 13))
        S, ptr, idx = _random_strength_graph(r, n)
        a = amg.pmis(ptr, idx, n, seed=trial, level=trial % 3)
        b = amg.pmis_bruteforce(S, n, seed=trial, level=trial % 3)
        assert np.array_equal(a, b), (trial, S)


def _check_pmis(ptr, idx, st):
    n = len(st)
    rows = np.repeat(np.arange(n), np.diff(ptr))
    assert set(np.unique(st)) <= {amg.C_, amg.F_}
    assert not np.any((st[rows] == amg.C_) & (st[idx] == amg.C_))
    lam = np.bincount(idx, minlength=n)
    for i in np.flatnonzero((st == amg.F_) & (lam > 0)):
        assert np.any(st[idx[ptr[i]:ptr[i + 1]]] == amg.C_)


def test_pmis_invariants_on_laplacian():
    A = laplacian(9, 8, 7)
    comp = np.zeros(A.shape[0], np.int64)
    ptr, idx = amg.strength(A, comp, 0.25)
    assert np.array_equal(np.diff(ptr), np.diff(A.indptr) - 1)   # every neighbour is strong
    st = amg.pmis(ptr, idx, A.shape[0], 12345, 0)
    _check_pmis(ptr, idx, st)


def test_interpolation_preserves_constants():
    A = laplacian(10, 9, neumann=True)  # zero row sums
    comp = np.zeros(A.shape[0], np.int64)
    ptr, idx = amg.strength(A, comp, 0.25)
    st = amg.pmis(ptr, idx, A.shape[0], 7, 0)
    P, _ = amg.interpolation(A, ptr, idx, st, comp)
    rs = np.asarray(P.sum(axis=1)).ravel()
    nonempty = np.diff(P.indptr) > 0
    assert np.allclose(rs[nonempty], 1.0, atol=1e-14)
    cidx = np.cumsum(st == amg.C_) - 1
    for i in np.flatnonzero(st == amg.C_):
        row = P.getrow(i)
        assert row.nnz == 1 and row.indices[0] == cidx[i] and row.data[0] == 1.0


@pytest.mark.parametrize("p_max", [0, 4, 2])
def test_extpi_preserves_constants(p_max):
    A = laplacian(10, 9, 4, neumann=True)  # zero row sums
    comp = np.zeros(A.shape[0], np.int64)
    ptr, idx = amg.strength(A, comp, 0.25)
    st = amg.pmis(ptr, idx, A.shape[0], 7, 0)
    P, _ = amg.interpolation(A, ptr, idx, st, comp, "ext+i", p_max)
    Pc, _ = amg.interpolation(A, ptr, idx, st, comp)
    lens = np.diff(P.indptr)
    if p_max:
        assert lens.max() <= p_max
    else:  # distance-two points make the rows longer than classical ones
        assert lens.sum() > np.diff(Pc.indptr).sum()
    rs = np.asarray(P.sum(axis=1)).ravel()
    assert np.allclose(rs[lens > 0], 1.0, atol=1e-13)
    cidx = np.cumsum(st == amg.C_) - 1
    for i in np.flatnonzero(st == amg.C_):
        row = P.getrow(i)
        assert row.nnz == 1 and row.indices[0] == cidx[i] and row.data[0] == 1.0


def test_extpi_is_linear_on_a_path():
    # 1D Laplacian on 0-1-2-3 (Dirichlet-free interior stencil), states C F F C:
    # node 1 sees C point 0 directly and C point 3 through its strong F
    # neighbour 2; the linear interpolant at 1 is 2/3 u_0 + 1/3 u_3
    A = sp.csr_matrix(np.array([[1.0, -1, 0, 0], [-1, 2, -1, 0], [0, -1, 2, -1], [0, 0, -1, 1]]))
    comp = np.zeros(4, np.int64)
    ptr, idx = amg.strength(A, comp, 0.25)
    st = np.array([amg.C_, amg.F_, amg.F_, amg.C_], np.int8)
    w = amg.interp_row_extpi(A, ptr, idx, st, comp, 1)
    assert set(w) == {0, 3}
    assert abs(w[0] - 2.0 / 3.0) < 1e-15 and abs(w[3] - 1.0 / 3.0) < 1e-15
    assert amg.interp_row(A, set(idx[ptr[1]:ptr[2]].tolist()), st, comp, 1) == pytest.approx({0: 1.0})


def test_extpi_truncation_keeps_largest():
    A = laplacian(9, 9, 5)
    comp = np.zeros(A.shape[0], np.int64)
    ptr, idx = amg.strength(A, comp, 0.25)
    st = amg.pmis(ptr, idx, A.shape[0], 11, 0)
    checked = 0
    for i in np.flatnonzero(st == amg.F_):
        full = amg.interp_row_extpi(A, ptr, idx, st, comp, int(i), 0)
        if len(full) <= 3:
            continue
        tr = amg.interp_row_extpi(A, ptr, idx, st, comp, int(i), 3)
        mags = sorted((abs(v) for v in full.values()), reverse=True)
        assert len(tr) == 3 and min(abs(full[j]) for j in tr) >= mags[2] * (1 - 1e-6)
        assert abs(sum(tr.values()) - sum(full.values())) <= 1e-13 * abs(sum(full.values()))
        assert all(np.sign(tr[j]) == np.sign(full[j]) for j in tr)
        checked += 1
    assert checked > 10


def test_interpolation_respects_components():
    A = laplacian(6, 6)
    Ab = sp.kron(A, np.array([[2.0, 0.3], [0.3, 2.0]])).tocsr()
    Ab.sort_indices()
    comp = np.tile([0, 1], A.shape[0])
    ptr, idx = amg.strength(Ab, comp, 0.25)
    assert np.all(comp[idx] == comp[np.repeat(np.arange(len(comp)), np.diff(ptr))])
    st = amg.pmis(ptr, idx, Ab.shape[0], 3, 0)
    P, ccomp = amg.interpolation(Ab, ptr, idx, st, comp)
    r, c = P.nonzero()
    assert np.all(comp[r] == ccomp[c])


def test_galerkin_equals_dense_product():
    r = np.random.default_rng(1)
    A = laplacian(7, 6, 3)
    A = (A + sp.diags(r.uniform(0, 1, A.shape[0]))).tocsr()
    comp = np.zeros(A.shape[0], np.int64)
    ptr, idx = amg.strength(A, comp, 0.25)
    st = amg.pmis(ptr, idx, A.shape[0], 5, 0)
    P, _ = amg.interpolation(A, ptr, idx, st, comp)
    Ac = amg.galerkin(A, P)
    dense = P.toarray().T @ A.toarray() @ P.toarray()
    assert np.abs(Ac.toarray() - dense).max() <= 1e-14 * np.abs(dense).max()
    assert np.abs(Ac.toarray() - Ac.toarray().T).max() <= 1e-14 * np.abs(dense).max()
    # structural pattern: superset of the numerical nonzeros
    assert np.all(Ac.toarray()[np.abs(dense) > 1e-13] != 0)


def test_l1_jacobi_is_monotone_in_energy_norm():
    r = np.random.default_rng(2)
    A = laplacian(8, 7, 6)
    A = (A + sp.diags(r.uniform(0, 0.1, A.shape[0])) + 0.3 * sp.random(A.shape[0], A.shape[0], 0.01, random_state=3)).tocsr()
    A = ((A + A.T) * 0.5 + sp.identity(A.shape[0]) * 2).tocsr()
    L = amg.Level(A, np.zeros(A.shape[0], int))
    L.dinv = 1.0 / amg.l1_diag(A)
    x_true = r.normal(size=A.shape[0])
    b = A @ x_true
    x = np.zeros_like(b)
    e_prev = np.inf
    prm = amg.AmgParams(smoother="l1jacobi")
    for _ in range(10):
        x = amg.smooth(L, b, x, 1, prm, 1)
        e = x - x_true
        en = e @ (A @ e)
        assert en <= e_prev * (1 + 1e-14)
        e_prev = en


def test_chebyshev_closed_form():
    lam = 3.0
    a, b = lam / 30.0, 1.1 * lam
    eig = np.array([a, 0.5 * (a + b), b])
    A = sp.diags(eig).tocsr()
    sigma = (b + a) / (b - a)
    T2 = 2 * sigma ** 2 - 1
    e0 = np.ones(3)
    x = amg.chebyshev(A, np.ones(3), lam, np.zeros(3), -e0)  # solution 0, error -e0
    # the residual polynomial equioscillates: |p| = 1/T_2(sigma) at a, (a+b)/2, b
    assert np.allclose(np.abs(x), 1.0 / T2, rtol=1e-12)


def test_lanczos_largest_eigenvalue():
    A = laplacian(6, 5, 4)
    d = A.diagonal()
    est = amg.lanczos_max(A, d, A.shape[0], 1, 0)
    Dm = np.diag(1 / np.sqrt(d))
    true = np.linalg.eigvalsh(Dm @ A.toarray() @ Dm).max()
    assert abs(est - true) <= 1e-10 * true
    short = amg.lanczos_max(A, d, 10, 1, 0)
    assert 0.8 * true <= short <= true * (1 + 1e-12)


def _reuse_problem(seed=3):
    r = np.random.default_rng(seed)
    A = (laplacian(10, 9, 8) + sp.diags(r.uniform(0.0, 0.5, 720))).tocsr()
    A.sort_indices()
    # a different operator on the same pattern: positive reweighting of the
    # off-diagonal couplings with the diagonal kept dominant
    B = A.copy()
    off = B.indices != np.repeat(np.arange(720), np.diff(B.indptr))
    B.data[off] *= r.uniform(0.5, 1.5, off.sum())
    B = B + sp.diags(r.uniform(0.0, 0.5, 720) + np.asarray(abs(B).sum(axis=1)).ravel() - 2 * B.diagonal())
    B = B.tocsr()
    B.sort_indices()
    return A, B


@pytest.mark.parametrize("smoother", ["l1jacobi", "chebyshev"])
def test_resetup_of_the_same_operator_is_the_setup(smoother):
    """Re-set-up with the operator the hierarchy was built from rebuilds it."""
    A, _ = _reuse_problem()
    prm = amg.AmgParams(max_coarse=40, smoother=smoother, nu_pre=1, nu_post=1)
    H = amg.setup(A, np.zeros(720, np.int64), prm)
    H2 = amg.resetup(A, H, prm)
    assert len(H.levels) >= 3 and len(H2.levels) == len(H.levels)
    for a, b in zip(H.levels, H2.levels):
        assert (a.A != b.A).nnz == 0 and np.array_equal(a.dinv, b.dinv) and a.lam == b.lam
    b = np.random.default_rng(0).standard_normal(720)
    assert np.array_equal(amg.vcycle(H, b, prm), amg.vcycle(H2, b, prm))


@pytest.mark.parametrize("smoother", ["l1jacobi", "chebyshev"])
def test_resetup_is_scale_covariant(smoother):
    """For A' = 4A every coarse operator scales by 4 and the V-cycle of A' on
    4b equals that of A on b (both smoothers are invariant under scaling)."""
    A, _ = _reuse_problem()
    prm = amg.AmgParams(max_coarse=40, smoother=smoother)
    H = amg.setup(A, np.zeros(720, np.int64), prm)
    H4 = amg.resetup((4.0 * A).tocsr(), H, prm)
    for a, b in zip(H.levels, H4.levels):
        assert np.abs((b.A - 4.0 * a.A).data).max(initial=0.0) <= 1e-13 * np.abs(b.A.data).max()
    b = np.random.default_rng(1).standard_normal(720)
    y, y4 = amg.vcycle(H, b, prm), amg.vcycle(H4, 4.0 * b, prm)
    assert np.abs(y4 - y).max() <= 1e-11 * np.abs(y).max()


def test_resetup_coarse_correction_is_an_energy_projection():
    """On two levels the exact coarse correction for the new operator B
    leaves an error B-orthogonal to the kept interpolation's range, and the
    reused hierarchy still preconditions B well."""
    A, B = _reuse_problem()
    prm = amg.AmgParams(max_coarse=400, max_levels=2, drop_tol=0.0)
    H = amg.setup(A, np.zeros(720, np.int64), prm)
    HB = amg.resetup(B, H, prm)
    assert len(HB.levels) == 2
    P = HB.levels[0].P
    e = np.random.default_rng(2).standard_normal(720)
    ec = scipy.linalg.lu_solve(HB.lu, P.T @ (B @ e))
    e_new = e - P @ ec
    g = P.T @ (B @ e_new)
    assert np.abs(g).max() <= 1e-10 * np.abs(P.T @ (B @ e)).max()
    # and the same correction with the stale coarse operator is not
    ec_old = scipy.linalg.lu_solve(H.lu, P.T @ (B @ e))
    assert np.abs(P.T @ (B @ (e - P @ ec_old))).max() > 1e-3 * np.abs(P.T @ (B @ e)).max()
    prm3 = amg.AmgParams(max_coarse=40)
    H3 = amg.resetup(B, amg.setup(A, np.zeros(720, np.int64), prm3), prm3)
    assert amg.convergence_factor(H3, prm3) < 0.5
