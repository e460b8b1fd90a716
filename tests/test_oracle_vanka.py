"""Pins of the coupled-AMG / multiplicative Vanka oracle (section "The
multiplicative Vanka smoother", eq. locsys and eq. vankasmooth).

* the four blocks put back together are the assembled tangent (a wrong
  sign of -C, a transposed B block or a missing Dirichlet zero fails);
* on disjoint patches one sweep is block SOR, written as the textbook
  splitting (D/omega + L) x1 = b - (U + (1 - 1/omega) D) x0 and solved
  densely (a local system from the wrong rows, a residual without the
  earlier updates, or omega applied to the residual instead of the
  correction fails);
* a single patch holding every unknown gives x0 + omega K^-1 (b - K x0);
* the greedy colours are first-fit and valid: no two patches of a colour
  share an unknown or a stored coupling, checked by brute force on the
  dense pattern; a sweep that treats each colour at once (all its local
  residuals from the same iterate) equals the sequential sweep;
* the coarse coupled system is P^T K P with P = diag(P_u, P_p) formed
  densely, and the two-level cycle without smoothing is P K_c^-1 P^T b;
* on the 6^3 Mooney-Rivlin cube the AMG method converges (the paper's
  observation for the solid);
* the additive variant: on disjoint patches one sweep is damped block
  Jacobi; on the identity system with overlapping patches it is exactly
  x0 + omega (b - x0) (the mean of the overlapping corrections, not their
  sum) and leaves an unknown outside every patch alone; on the cube it is
  the dense patch-by-patch formula, and its cycle preconditions FGMRES;
* the fp32 local inverses: on a single patch the sweep is x0 + omega
  fl32(K^-1) (b - K x0) with the inverse from a dense inverse rounded to
  float32 (no rounding, or rounding the correction instead, fails at
  1e-12); on the cube the cycle stays within 1e-5 of the fp64 cycle and
  FGMRES takes at most one more iteration.
"""
import numpy as np
import pytest
import scipy.linalg
import scipy.sparse as sp

import synth
from oracle import amg, fe, krylov, vanka


def _cube_system(N=6, load=1.0, seed_state=None):
    prob = synth.cube_problem(N)
    d = fe.Discretization(prob)
    v = np.zeros(prob.n_dofs) if seed_state is None else synth.random_state(prob, seed_state, 0.05, 0.1).ravel()
    R, val = d.assemble(v, load)
    R, val = d.apply_dirichlet(R, val)
    return prob, d, d.csr(val), -R, val


def _small_prm(steps=2, omega=0.78, max_coarse=150):
    return vanka.VankaParams(omega=omega, steps=steps,
                             amg=amg.AmgParams(smoother="l1jacobi", interp="ext+i", max_coarse=max_coarse))


@pytest.fixture(scope="module")
def cube6():
    prob, d, K, b, val = _cube_system(6, seed_state=3)
    blocks = vanka.tangent_blocks(d, val)
    CH = vanka.setup(*blocks, _small_prm())
    return prob, d, K, b, blocks, CH


def test_blocks_are_the_tangent(cube6):
    prob, d, K, b, blocks, CH = cube6
    n = prob.n_nodes
    Kuu, Kup, Kpu, Kpp = blocks
    perm = np.concatenate([np.arange(4 * n).reshape(n, 4)[:, :3].ravel(), 4 * np.arange(n) + 3])
    Kd = K.toarray()[np.ix_(perm, perm)]
    Kb = sp.bmat([[Kuu, Kup], [Kpu, Kpp]]).toarray()
    assert np.array_equal(Kb, Kd)
    # -C is negative definite on the pressure block
    assert np.linalg.eigvalsh(0.5 * (Kpp + Kpp.T).toarray()).max() < 0
    # vector reordering round trip
    x = np.random.default_rng(0).normal(size=4 * n)
    assert np.array_equal(vanka.to_interleaved(vanka.to_blocked(x, n), n), x)
    assert np.array_equal(vanka.to_blocked(x, n), x[perm])


def _disjoint_system(rng, npr=5, per=3):
    """Saddle system whose patches partition the unknowns: pressure i is
    coupled through B2 to displacement unknowns per*i .. per*i+per-1 only."""
    nu = npr * per
    M = rng.normal(size=(nu, nu))
    Kuu = M @ M.T + nu * np.eye(nu)
    Kpu = np.zeros((npr, nu))
    for i in range(npr):
        Kpu[i, per * i:per * (i + 1)] = rng.normal(size=per)
    Kup = Kpu.T + 0.1 * (Kpu.T != 0) * rng.normal(size=Kpu.T.shape)
    Kpp = -np.diag(rng.uniform(0.5, 1.5, npr))
    Kpp[0, 1] = Kpp[1, 0] = 0.1
    return [sp.csr_matrix(B) for B in (Kuu, Kup, Kpu, Kpp)], nu, npr


def _level_of(blocks, inverse_f32=False):
    L = vanka.CoupledLevel(*[B.tocsr() for B in blocks])
    vanka._vanka_data(L, inverse_f32)
    return L


@pytest.mark.parametrize("omega", [1.0, 0.78, 0.5])
def test_disjoint_patches_give_block_sor(omega):
    rng = np.random.default_rng(4)
    blocks, nu, npr = _disjoint_system(rng)
    L = _level_of(blocks)
    K = L.K().toarray()
    b = rng.normal(size=nu + npr)
    x0 = rng.normal(size=nu + npr)
    x1 = vanka.vanka_sweep(L, b, x0, omega)
    # the patch order, then D, L, U of the block splitting in that order
    order = np.concatenate([np.concatenate([L.patches[i], [nu + i]]) for i in L.order])
    assert sorted(order) == list(range(nu + npr))   # a partition
    Kp = K[np.ix_(order, order)]
    sizes = [len(L.patches[i]) + 1 for i in L.order]
    edges = np.concatenate([[0], np.cumsum(sizes)])
    D = np.zeros_like(Kp)
    for a, e in zip(edges[:-1], edges[1:]):
        D[a:e, a:e] = Kp[a:e, a:e]
    blk = np.zeros(len(order), int)
    for k, (a, e) in enumerate(zip(edges[:-1], edges[1:])):
        blk[a:e] = k
    lower = (blk[:, None] > blk[None, :]) * Kp
    upper = (blk[:, None] < blk[None, :]) * Kp
    y0 = x0[order]
    y1 = np.linalg.solve(D / omega + lower, b[order] - (upper + (1.0 - 1.0 / omega) * D) @ y0)
    assert np.abs(x1[order] - y1).max() <= 1e-12 * np.abs(y1).max()


def test_single_patch_is_the_relaxed_solve():
    rng = np.random.default_rng(5)
    nu = 7
    M = rng.normal(size=(nu, nu))
    Kuu = sp.csr_matrix(M @ M.T + nu * np.eye(nu))
    Kpu = sp.csr_matrix(rng.normal(size=(1, nu)))
    Kup = sp.csr_matrix(rng.normal(size=(nu, 1)))
    Kpp = sp.csr_matrix([[-0.7]])
    L = _level_of([Kuu, Kup, Kpu, Kpp])
    K = L.K().toarray()
    b, x0 = rng.normal(size=nu + 1), rng.normal(size=nu + 1)
    x1 = vanka.vanka_sweep(L, b, x0, 0.6)
    ref = x0 + 0.6 * np.linalg.solve(K, b - K @ x0)
    assert np.abs(x1 - ref).max() <= 1e-12 * np.abs(ref).max()


def _dense_pattern(L):
    K = L.K()
    P = K.copy()
    P.data = np.ones_like(P.data)
    return P.toarray() != 0


def test_colours_are_first_fit_and_valid(cube6):
    *_, CH = cube6
    assert len(CH.levels) >= 3
    for L in CH.levels[:-1]:
        pat = _dense_pattern(L)
        sets = [np.concatenate([L.patches[i], [L.nu + i]]) for i in range(L.np_)]
        col = L.colour
        for c in range(col.max() + 1):
            members = np.flatnonzero(col == c)
            for x in range(len(members)):
                for y in range(x + 1, len(members)):
                    a, b = sets[members[x]], sets[members[y]]
                    assert not np.intersect1d(a, b).size
                    assert not pat[np.ix_(a, b)].any() and not pat[np.ix_(b, a)].any()
        # first fit: a patch of colour c meets every colour below c among
        # the earlier patches it conflicts with
        for i in range(L.np_):
            if col[i] == 0:
                continue
            earlier = [k for k in range(i) if pat[np.ix_(sets[i], sets[k])].any() or pat[np.ix_(sets[k], sets[i])].any()]
            assert set(range(col[i])) <= set(col[earlier].tolist())


def test_colour_at_once_equals_sequential(cube6):
    prob, d, K, b, blocks, CH = cube6
    L = CH.levels[0]
    Kl = L.K()
    rng = np.random.default_rng(6)
    bb, x0 = rng.normal(size=Kl.shape[0]), rng.normal(size=Kl.shape[0])
    seq = vanka.vanka_sweep(L, bb, x0, 0.78, Kl)
    x = x0.copy()
    for c in range(L.colour.max() + 1):
        members = np.flatnonzero(L.colour == c)
        upd = []
        for i in members:
            idx = np.concatenate([L.patches[i], [L.nu + i]])
            r = bb[idx] - Kl[idx] @ x
            upd.append((idx, 0.78 * scipy.linalg.lu_solve(L.lu[i], r)))
        for idx, dx in upd:
            x[idx] += dx
    assert np.abs(x - seq).max() <= 1e-12 * np.abs(seq).max()


def test_coarse_system_and_two_level_cycle(cube6):
    *_, CH = cube6
    L0, L1 = CH.levels[0], CH.levels[1]
    assert L0.Pu is not None and L0.Pp is not None
    P = sp.block_diag([L0.Pu, L0.Pp]).toarray()
    K0 = L0.K().toarray()
    Kc = P.T @ K0 @ P
    K1 = L1.K().toarray()
    assert np.abs(K1 - Kc).max() <= 1e-12 * np.abs(Kc).max()
    # every nonzero of the dense product is stored
    assert not ((Kc != 0) & ~_dense_pattern(L1)).any()
    # two-level cycle without smoothing
    two = vanka.CoupledHierarchy([L0, vanka.CoupledLevel(L1.Kuu, L1.Kup, L1.Kpu, L1.Kpp)],
                                 scipy.linalg.lu_factor(K1), None, None)
    b = np.random.default_rng(7).normal(size=K0.shape[0])
    z = vanka.vcycle(two, b, vanka.VankaParams(steps=0))
    ref = P @ np.linalg.solve(K1, P.T @ b)
    assert np.abs(z - ref).max() <= 1e-10 * np.abs(ref).max()


def test_identity_transfer_below_the_shorter_hierarchy(cube6):
    *_, CH = cube6
    nl = len(CH.levels)
    lu, lp = len(CH.Hu.levels), len(CH.Hp.levels)
    assert nl == max(lu, lp)
    for lev in range(nl - 1):
        L, Lc = CH.levels[lev], CH.levels[lev + 1]
        assert (L.Pu is None) == (lev >= lu - 1)
        assert (L.Pp is None) == (lev >= lp - 1)
        if L.Pu is None:
            assert Lc.nu == L.nu and abs(Lc.Kuu - L.Kuu).max() == 0
        if L.Pp is None:
            assert Lc.np_ == L.np_ and abs(Lc.Kpp - L.Kpp).max() == 0


def test_coupled_amg_solves_the_solid(cube6):
    prob, d, K, b, blocks, CH = cube6
    prm = _small_prm()
    x, hist = vanka.amg_iteration(CH, K, b, prob.n_nodes, prm, tol=1e-8, maxit=40)
    assert hist[-1] <= 1e-8
    rate = hist[-1] ** (1.0 / (len(hist) - 1))
    assert rate < 0.35, hist
    x2, info = krylov.fgmres(K, vanka.preconditioner(CH, prob.n_nodes, prm), b, m=50, tol=1e-8)
    assert info.converged and info.iterations <= 12
    assert np.linalg.norm(b - K @ x2) <= 1e-8 * np.linalg.norm(b)


def test_colours_hand_case():
    """Five patches, each with its own three displacement unknowns and no
    displacement coupling between patches; only C couples pressures 0-1 and
    3-4.  Conflicts: {0,1} and {3,4} alone, so first fit gives colours
    0,1,0,0,1 and a sweep visits patches 0,2,3 then 1,4."""
    rng = np.random.default_rng(8)
    npr, per = 5, 3
    nu = npr * per
    Kuu = np.zeros((nu, nu))
    Kpu = np.zeros((npr, nu))
    for i in range(npr):
        M = rng.normal(size=(per, per))
        Kuu[per * i:per * (i + 1), per * i:per * (i + 1)] = M @ M.T + per * np.eye(per)
        Kpu[i, per * i:per * (i + 1)] = rng.normal(size=per)
    Kpp = -np.eye(npr)
    Kpp[0, 1] = Kpp[1, 0] = Kpp[3, 4] = Kpp[4, 3] = 0.2
    L = _level_of([sp.csr_matrix(B) for B in (Kuu, Kpu.T, Kpu, Kpp)])
    assert L.colour.tolist() == [0, 1, 0, 0, 1]
    assert L.order.tolist() == [0, 2, 3, 1, 4]


@pytest.mark.parametrize("omega", [1.0, 0.5])
def test_additive_on_disjoint_patches_is_block_jacobi(omega):
    """Additive variant, patches that partition the unknowns (every count is
    one): one sweep is damped block Jacobi, x1 = x0 + omega D^-1 (b - K x0),
    D the patch blocks (a residual taken after an update, or a correction
    added twice, fails)."""
    rng = np.random.default_rng(9)
    blocks, nu, npr = _disjoint_system(rng)
    L = _level_of(blocks)
    K = L.K().toarray()
    b, x0 = rng.normal(size=nu + npr), rng.normal(size=nu + npr)
    x1 = vanka.vanka_sweep_additive(L, b, x0, omega)
    D = np.zeros_like(K)
    for i in range(npr):
        idx = np.concatenate([L.patches[i], [nu + i]])
        D[np.ix_(idx, idx)] = K[np.ix_(idx, idx)]
    ref = x0 + omega * np.linalg.solve(D, b - K @ x0)
    assert np.abs(x1 - ref).max() <= 1e-12 * np.abs(ref).max()


def _csr_pattern(rows, cols, pattern, value=0.0):
    """CSR matrix holding `value` at every (row, col) of `pattern`, stored
    explicitly even when it is zero."""
    indptr = np.zeros(rows + 1, np.int64)
    indices = []
    for r in range(rows):
        cs = sorted(c for (rr, c) in pattern if rr == r)
        indices += cs
        indptr[r + 1] = len(indices)
    data = np.full(len(indices), value)
    return sp.csr_matrix((data, np.asarray(indices, np.int64), indptr), shape=(rows, cols))


def test_additive_averages_overlapping_corrections_identity_system():
    """K = I with patches that overlap (explicitly stored zero couplings):
    every local system is the identity, so every patch returns the residual
    on its unknowns and the mean over the patches of an unknown is that
    residual again.  One sweep is x0 + omega (b - x0) exactly on the
    unknowns of some patch, and leaves an unknown in no patch unchanged (the
    plain sum would give the shared unknowns their count times the
    correction)."""
    nu, npr = 6, 3
    # patch 0: u0 u1 u2, patch 1: u1 u2 u3, patch 2: u2 u4; u5 in no patch
    pat = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (1, 3), (2, 2), (2, 4)]
    Kpu = _csr_pattern(npr, nu, pat)
    Kup = _csr_pattern(nu, npr, [(c, r) for (r, c) in pat])
    blocks = [sp.identity(nu, format="csr"), Kup, Kpu, sp.identity(npr, format="csr")]
    L = _level_of(blocks)
    assert [list(p) for p in L.patches] == [[0, 1, 2], [1, 2, 3], [2, 4]]
    rng = np.random.default_rng(11)
    b, x0 = rng.normal(size=nu + npr), rng.normal(size=nu + npr)
    for omega in (1.0, 0.6):
        x1 = vanka.vanka_sweep_additive(L, b, x0, omega)
        ref = x0 + omega * (b - x0)
        ref[5] = x0[5]
        assert np.abs(x1 - ref).max() <= 1e-14 * np.abs(ref).max()


def test_additive_overlapping_patches_average_their_corrections(cube6):
    """With overlapping patches the sweep is x0 + omega M^-1 sum_i P_i K_i^-1
    R_i r (M the patch counts), assembled here densely patch by patch with
    numpy's solver."""
    *_, CH = cube6
    L = CH.levels[0]
    K = L.K().toarray()
    rng = np.random.default_rng(10)
    b, x0 = rng.normal(size=K.shape[0]), rng.normal(size=K.shape[0])
    r = b - K @ x0
    d = np.zeros_like(x0)
    count = np.zeros_like(x0)
    for i in range(L.np_):
        idx = np.concatenate([L.patches[i], [L.nu + i]])
        d[idx] += np.linalg.solve(K[np.ix_(idx, idx)], r[idx])
        count[idx] += 1
    assert count.min() >= 1                # every unknown of the cube is in a patch
    assert count[:L.nu].max() > 1          # and the overlap is real
    ref = x0 + 0.6 * d / count
    got = vanka.vanka_sweep_additive(L, b, x0, 0.6)
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()


def test_additive_cycle_preconditions_the_solid(cube6):
    """The additive V-cycle is a good preconditioner for FGMRES on the solid
    (at most twice the multiplicative cycle's iteration count)."""
    prob, d, K, b, blocks, CH = cube6
    its = {}
    for additive in (False, True):
        prm = vanka.VankaParams(omega=0.8, steps=6, additive=additive,
                                amg=amg.AmgParams(smoother="l1jacobi", interp="ext+i", max_coarse=150))
        x, info = krylov.fgmres(K, vanka.preconditioner(CH, prob.n_nodes, prm), b, m=60, tol=1e-8, maxit=200)
        assert info.converged
        assert np.linalg.norm(b - K @ x) <= 1e-8 * np.linalg.norm(b)
        its[additive] = info.iterations
    assert its[True] <= 2 * its[False]


def test_fp32_inverse_on_a_single_patch():
    rng = np.random.default_rng(15)
    nu = 9
    M = rng.normal(size=(nu, nu))
    Kuu = sp.csr_matrix(M @ M.T + nu * np.eye(nu))
    Kpu = sp.csr_matrix(rng.normal(size=(1, nu)))
    Kup = sp.csr_matrix(rng.normal(size=(nu, 1)))
    Kpp = sp.csr_matrix([[-0.4]])
    L = _level_of([Kuu, Kup, Kpu, Kpp], inverse_f32=True)
    assert L.inv32[0].dtype == np.float32
    K = L.K().toarray()
    b, x0 = rng.normal(size=nu + 1), rng.normal(size=nu + 1)
    Y = np.linalg.inv(K).astype(np.float32).astype(np.float64)
    ref = x0 + 0.7 * (Y @ (b - K @ x0))
    for sweep in (vanka.vanka_sweep, vanka.vanka_sweep_additive):
        got = sweep(L, b, x0, 0.7)
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    exact = x0 + 0.7 * np.linalg.solve(K, b - K @ x0)
    assert np.abs(exact - ref).max() > 1e-10 * np.abs(ref).max()   # the rounding is visible


def test_fp32_inverse_cycle_close_to_fp64(cube6):
    prob, d, K, b, blocks, _ = cube6
    n = prob.n_nodes
    res = {}
    for f32 in (False, True):
        prm = vanka.VankaParams(omega=0.8, steps=2, additive=True, inverse_f32=f32,
                                amg=amg.AmgParams(smoother="l1jacobi", interp="ext+i", max_coarse=150))
        CH = vanka.setup(*blocks, prm)
        r = np.random.default_rng(3).normal(size=4 * n)
        z = vanka.preconditioner(CH, n, prm)(r)
        x, info = krylov.fgmres(K, vanka.preconditioner(CH, n, prm), b, m=60, tol=1e-8, maxit=200)
        assert info.converged
        res[f32] = (z, info.iterations)
    z64, z32 = res[False][0], res[True][0]
    assert 0.0 < np.abs(z32 - z64).max() <= 1e-5 * np.abs(z64).max()
    assert res[True][1] <= res[False][1] + 1
