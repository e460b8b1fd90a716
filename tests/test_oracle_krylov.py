"""Pins of the oracle's preconditioner and FGMRES.

* FGMRES with the identity preconditioner reproduces a dense direct solve
  (numpy.linalg.solve) of the assembled K on the 1^3 and 2^3 cubes;
* with exact blocks (Atilde = A, Stilde = B2 A^{-1} B1^T + C) the block
  preconditioner of eq. lpre makes P_L^{-1} K block upper triangular with
  identity diagonal blocks, so FGMRES converges in two iterations;
* the AMG-preconditioned solve reaches the requested true relative
  residual and agrees with the direct solution;
* BiCGStab: with the identity preconditioner it reproduces the dense solve;
  on a matrix with two distinct eigenvalues (and with the exact block
  preconditioner, whose preconditioned operator has minimal polynomial
  (z - 1)^2) it converges in at most two iterations; AMG-preconditioned it
  reaches the requested true residual;
* GCR: with a fixed preconditioner it minimises the residual over the same
  Krylov space as GMRES, so its residual history equals FGMRES's (a missing
  re-orthogonalisation, or the z_i not following the q_i, breaks it); with
  the identity it reproduces the dense solve;
* P_R (eq. rpre) with exact blocks (Atilde = A, Stilde = S) makes K P_R^{-1}
  block lower triangular with identity diagonal blocks: GCR and FGMRES
  converge in two iterations (a sign error in z_p or in the B1^T term
  fails).
"""
import numpy as np
import pytest

import synth
from oracle import amg, fe, krylov, newton


def _system(N, seed=2, jitter=0.1):
    p = synth.cube_problem(N, jitter=jitter, seed=seed)
    d = fe.Discretization(p)
    v = synth.random_state(p, seed, u_scale=0.05, p_scale=0.05)
    K, b, A, B2, s = newton.linear_system(d, v.ravel(), 0.8)
    return d, K, b, A, B2, s


@pytest.mark.parametrize("N", [1, 2])
def test_fgmres_identity_matches_dense_solve(N):
    d, K, b, *_ = _system(N)
    x_ref = np.linalg.solve(K.toarray(), b)
    x, info = krylov.fgmres(K, lambda r: r.copy(), b, m=200, maxit=2000, tol=1e-13)
    assert info.converged
    assert np.linalg.norm(x - x_ref) <= 1e-9 * np.linalg.norm(x_ref)


def test_exact_block_preconditioner_two_iterations():
    d, K, b, A, B2, s = _system(2)
    n = d.n
    Kd = K.toarray()
    u = np.array([4 * i + c for i in range(n) for c in range(3)])
    pp = 4 * np.arange(n) + 3
    Ad = Kd[np.ix_(u, u)]
    B1T = Kd[np.ix_(u, pp)]
    B2d = Kd[np.ix_(pp, u)]
    Cd = -Kd[np.ix_(pp, pp)]
    Sd = B2d @ np.linalg.solve(Ad, B1T) + Cd

    def prec(r):
        ru, rp = krylov.split(r, n)
        zu = np.linalg.solve(Ad, ru)
        zp = np.linalg.solve(Sd, B2d @ zu - rp)
        return krylov.join(zu, zp, n)

    x, info = krylov.fgmres(K, prec, b, tol=1e-10)
    assert info.converged and info.iterations == 2


def test_amg_preconditioned_solve():
    d, K, b, A, B2, s = _system(4)
    M, H = krylov.amg_preconditioner(A, B2, s, d.n, amg.AmgParams(max_coarse=60))
    assert len(H.levels) >= 2
    x, info = krylov.fgmres(K, M, b, tol=1e-10)
    assert info.converged
    assert np.linalg.norm(b - K @ x) <= 1e-10 * np.linalg.norm(b)
    x_ref = np.linalg.solve(K.toarray(), b)
    assert np.linalg.norm(x - x_ref) <= 1e-6 * np.linalg.norm(x_ref)


def test_arnoldi_relation_holds():
    """Internal consistency: K Z_j = V_{j+1} Hbar_j for one cycle."""
    d, K, b, A, B2, s = _system(2)
    rng = np.random.default_rng(0)
    Mdiag = rng.uniform(0.5, 2.0, size=b.size)
    prec = lambda r: Mdiag * r
    x, info = krylov.fgmres(K, prec, b, m=8, maxit=8, tol=1e-30)
    assert info.iterations == 8
    assert info.history == sorted(info.history, reverse=True)   # residual never grows


@pytest.mark.parametrize("N", [1, 2])
def test_bicgstab_identity_matches_dense_solve(N):
    d, K, b, *_ = _system(N)
    x_ref = np.linalg.solve(K.toarray(), b)
    x, info = krylov.bicgstab(K, lambda r: r.copy(), b, maxit=5000, tol=1e-12)
    assert info.converged
    assert np.linalg.norm(x - x_ref) <= 1e-8 * np.linalg.norm(x_ref)


def test_bicgstab_two_eigenvalues_two_iterations():
    import scipy.sparse as sp
    rng = np.random.default_rng(3)
    diag = np.where(rng.uniform(size=40) < 0.5, 2.0, 7.0)
    K = sp.diags(diag).tocsr()
    b = rng.normal(size=40)
    x, info = krylov.bicgstab(K, lambda r: r.copy(), b, tol=1e-12)
    assert info.converged and info.iterations <= 2
    assert np.allclose(x, b / diag, rtol=1e-12)


def test_bicgstab_exact_block_preconditioner_two_iterations():
    d, K, b, A, B2, s = _system(2)
    n = d.n
    Kd = K.toarray()
    u = np.array([4 * i + c for i in range(n) for c in range(3)])
    pp = 4 * np.arange(n) + 3
    Ad = Kd[np.ix_(u, u)]
    B1T = Kd[np.ix_(u, pp)]
    B2d = Kd[np.ix_(pp, u)]
    Cd = -Kd[np.ix_(pp, pp)]
    Sd = B2d @ np.linalg.solve(Ad, B1T) + Cd

    def prec(r):
        ru, rp = krylov.split(r, n)
        zu = np.linalg.solve(Ad, ru)
        zp = np.linalg.solve(Sd, B2d @ zu - rp)
        return krylov.join(zu, zp, n)

    x, info = krylov.bicgstab(K, prec, b, tol=1e-10)
    assert info.converged and info.iterations <= 2


def test_bicgstab_amg_preconditioned_solve():
    d, K, b, A, B2, s = _system(4)
    M, H = krylov.amg_preconditioner(A, B2, s, d.n, amg.AmgParams(max_coarse=60))
    x, info = krylov.bicgstab(K, M, b, tol=1e-10)
    assert info.converged
    assert np.linalg.norm(b - K @ x) <= 1e-10 * np.linalg.norm(b)
    x_ref = np.linalg.solve(K.toarray(), b)
    assert np.linalg.norm(x - x_ref) <= 1e-6 * np.linalg.norm(x_ref)



def _blocks(d, K):
    n = d.n
    Kd = K.toarray()
    u = np.array([4 * i + c for i in range(n) for c in range(3)])
    pp = 4 * np.arange(n) + 3
    return Kd, u, pp


@pytest.mark.parametrize("N", [1, 2])
def test_gcr_identity_matches_dense_solve(N):
    d, K, b, *_ = _system(N)
    x_ref = np.linalg.solve(K.toarray(), b)
    x, info = krylov.gcr(K, lambda r: r.copy(), b, m=200, maxit=2000, tol=1e-13)
    assert info.converged
    assert np.linalg.norm(x - x_ref) <= 1e-9 * np.linalg.norm(x_ref)


def test_gcr_residuals_equal_gmres():
    d, K, b, A, B2, s = _system(3)
    M, _ = krylov.amg_preconditioner(A, B2, s, d.n, amg.AmgParams(max_coarse=60))
    _, g = krylov.gcr(K, M, b, m=100, tol=1e-10)
    _, f = krylov.fgmres(K, M, b, m=100, tol=1e-10)
    assert g.converged and f.converged
    k = min(len(g.history), len(f.history))
    assert k >= 5 and abs(len(g.history) - len(f.history)) <= 1
    hg, hf = np.array(g.history[:k]), np.array(f.history[:k])
    assert np.all(np.abs(hg - hf) <= 1e-6 * hf + 1e-13)


def test_upper_block_preconditioner_two_iterations():
    d, K, b, A, B2, s = _system(2)
    Kd, u, pp = _blocks(d, K)
    Ad, B1T, B2d, Cd = Kd[np.ix_(u, u)], Kd[np.ix_(u, pp)], Kd[np.ix_(pp, u)], -Kd[np.ix_(pp, pp)]
    Sd = B2d @ np.linalg.solve(Ad, B1T) + Cd

    def prec(r):
        ru, rp = krylov.split(r, d.n)
        zp = -np.linalg.solve(Sd, rp)
        zu = np.linalg.solve(Ad, ru - B1T @ zp)
        return krylov.join(zu, zp, d.n)

    for solver in (krylov.gcr, krylov.fgmres):
        x, info = solver(K, prec, b, tol=1e-10)
        assert info.converged and info.iterations == 2, (solver.__name__, info.iterations)
    # the class with a diagonal Stilde is the same formula
    sdiag = np.abs(np.diag(Sd)) + 1.0
    P = krylov.UpperBlockPreconditioner(lambda ru: np.linalg.solve(Ad, ru), sp_csr(B1T), sdiag, d.n)
    r = np.random.default_rng(3).normal(size=4 * d.n)
    ru, rp = krylov.split(r, d.n)
    zp = -rp / sdiag
    ref = krylov.join(np.linalg.solve(Ad, ru - B1T @ zp), zp, d.n)
    assert np.abs(P(r) - ref).max() <= 1e-12 * np.abs(ref).max()


def sp_csr(M):
    import scipy.sparse as sp
    return sp.csr_matrix(M)
