"""Coupled displacement-pressure AMG with the multiplicative Vanka smoother
(oracle; test infrastructure only).

The paper's own solver for the linearised solid (section "AMG methods for
the mixed problems", subsection "The multiplicative Vanka smoother")
coarsens the whole saddle-point system K = [A B1^T; B2 -C] (eq. globsys),
builds every coarse system by Galerkin projection, and smooths on every
level by sweeping over patches: one patch per pressure unknown i, holding
p_i and the displacement unknowns coupled to it through B2.  On a patch the
local system (eq. locsys) is the restriction of K, solved directly; the
correction is relaxed by omega (eq. vankasmooth) and the patches are
treated one after the other, each with the residual left by the previous
ones (Gauss-Seidel).

The paper leaves the coarsening to its references and does not fix the
order of the patches.  The readings followed here:

* block-diagonal transfer P = diag(P_u, P_p): P_u is the interpolation of
  the displacement hierarchy on A (the same strength, PMIS and
  interpolation as the displacement AMG), P_p that of a hierarchy built by
  the same rules on the pressure block C (one unknown per row); the coupled
  coarse system is P^T K P block by block, on the structural pattern of the
  products.  When one of the two hierarchies has fewer levels, its transfer
  is the identity below its coarsest level.  The coarsest coupled system
  is solved by dense LU with partial pivoting.
* patch order: greedy colouring of the patches, in increasing pressure
  index, with the smallest colour not taken by an earlier patch it
  conflicts with; two patches conflict when K has a stored entry between
  an unknown of one and an unknown of the other (which includes sharing an
  unknown).  A sweep visits the colours in increasing order and the
  patches of a colour in increasing index.  Patches of one colour are
  neither overlapping nor coupled, so the order inside a colour does not
  change the result; this is what lets a GPU treat a colour at once.
* the local systems are those of the stored patterns (a displacement
  unknown is in patch i when B2 stores an entry (i, j), explicit zeros of
  the Dirichlet elimination included).
* the V-cycle uses the same number of sweeps before and after the coarse
  correction on every level, from a zero start.
* the additive variant (the paper points to an additive version of the
  multiplicative Vanka smoother analysed in its references, without fixing
  its weights): every patch's local problem takes the residual of the same
  iterate, and each unknown receives the average of the local corrections
  of the patches holding it, x += omega M^-1 sum_i P_i K_i^-1 R_i (b - K x),
  with P_i the patch's embedding, R_i = P_i^T and M the diagonal of patch
  counts (an unknown in no patch is left as it is).  The plain sum (M = I)
  over-corrects: on the tetrahedral meshes a displacement unknown lies in
  about a dozen patches, and the sum diverges at the relaxation the paper
  uses.  No order is involved, so one sweep is a single parallel step on a
  GPU.
* the fp32 option (inverse_f32, not in the paper: a storage choice of the
  local solves): each local system's exact inverse, rounded entry by entry
  to the nearest float32, is applied to the fp64 residual in fp64
  arithmetic; blocks, transfers and the coarsest solve stay fp64.

Every level's unknowns are ordered [u; p]: the nu displacement unknowns of
the displacement hierarchy, then the np pressure unknowns.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg
import scipy.sparse as sp

from . import amg


# ---------------------------------------------------------------------------
# blocks of the assembled tangent
# ---------------------------------------------------------------------------


def _from_coo_sorted(r, c, v, nr, nc):
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    indptr = np.zeros(nr + 1, np.int64)
    np.add.at(indptr, r + 1, 1)
    return sp.csr_matrix((v, c.astype(np.int32), np.cumsum(indptr)), shape=(nr, nc))


def tangent_blocks(disc, val):
    """Kuu, Kup, Kpu, Kpp of the node-interleaved tangent (values `val` on
    the pattern of `disc`, the Dirichlet elimination already applied).

    Kuu is the displacement block A as the displacement AMG takes it (stored
    entries removed by the elimination dropped); Kup = B1^T, Kpu = B2 and
    Kpp = -C keep every stored entry of their blocks."""
    n = disc.n
    rows = np.repeat(np.arange(4 * n), np.diff(disc.K_indptr))
    cols = disc.K_indices.astype(np.int64)
    rc, cc = rows % 4, cols % 4
    A, _, _ = disc.blocks(val)
    up = (rc < 3) & (cc == 3)
    pu = (rc == 3) & (cc < 3)
    pp = (rc == 3) & (cc == 3)
    Kup = _from_coo_sorted(3 * (rows[up] // 4) + rc[up], cols[up] // 4, val[up], 3 * n, n)
    Kpu = _from_coo_sorted(rows[pu] // 4, 3 * (cols[pu] // 4) + cc[pu], val[pu], n, 3 * n)
    Kpp = _from_coo_sorted(rows[pp] // 4, cols[pp] // 4, val[pp], n, n)
    return A.tocsr(), Kup, Kpu, Kpp


def to_blocked(v, n):
    """Node-interleaved [u0 u1 u2 p] per node -> [u (3n); p (n)]."""
    v = np.asarray(v).reshape(n, 4)
    return np.concatenate([v[:, 0:3].ravel(), v[:, 3]])


def to_interleaved(w, n):
    out = np.empty((n, 4))
    out[:, 0:3] = w[:3 * n].reshape(n, 3)
    out[:, 3] = w[3 * n:]
    return out.ravel()


# ---------------------------------------------------------------------------
# structural products
# ---------------------------------------------------------------------------


def _ones(M):
    Q = M.tocsr().copy()
    Q.data = np.ones_like(Q.data)
    return Q


def triple(L, M, R):
    """L M R with the structural pattern of the product (0/1 patterns, so no
    entry is lost to cancellation); L or R None stands for the identity."""
    vals = M.tocsr()
    pat = _ones(M)
    if L is not None:
        vals = L.tocsr() @ vals
        pat = _ones(L) @ pat
    if R is not None:
        vals = vals @ R.tocsr()
        pat = pat @ _ones(R)
    vals = vals.tocsr()
    pat = pat.tocsr()
    pat.sort_indices()
    rr = np.repeat(np.arange(pat.shape[0]), np.diff(pat.indptr))
    data = np.asarray(vals[rr, pat.indices]).ravel() if pat.nnz else np.zeros(0)
    return sp.csr_matrix((data, pat.indices.copy(), pat.indptr.copy()), shape=pat.shape)


# ---------------------------------------------------------------------------
# patches and their order
# ---------------------------------------------------------------------------


def patches(Kpu):
    """Displacement unknowns of every patch (sorted), from B2's pattern."""
    Kpu = Kpu.tocsr()
    return [Kpu.indices[Kpu.indptr[i]:Kpu.indptr[i + 1]].astype(np.int64) for i in range(Kpu.shape[0])]


def conflict_graph(Kuu, Kup, Kpu, Kpp):
    """Patch conflict pattern: (i, k) stored when K couples an unknown of
    patch i with one of patch k.  With S = [pat(B2) I] the patch incidence it
    is pat(S K S^T), symmetrised."""
    nu = Kuu.shape[0]
    npr = Kpu.shape[0]
    S = sp.hstack([_ones(Kpu), sp.identity(npr, format="csr")]).tocsr()
    K = sp.bmat([[_ones(Kuu), _ones(Kup)], [_ones(Kpu), _ones(Kpp)]]).tocsr()
    assert K.shape == (nu + npr, nu + npr)
    G = (S @ K @ S.T).tocsr()
    G = (_ones(G) + _ones(G).T).tocsr()
    G.sort_indices()
    return G


def greedy_colours(G):
    """First-fit colouring in increasing index: colour(i) is the smallest
    colour not held by a neighbour k < i."""
    n = G.shape[0]
    colour = np.full(n, -1, np.int64)
    for i in range(n):
        nb = G.indices[G.indptr[i]:G.indptr[i + 1]]
        used = set(int(colour[k]) for k in nb if k < i)
        c = 0
        while c in used:
            c += 1
        colour[i] = c
    return colour


def sweep_order(colour):
    """Patches by colour, then by index."""
    return np.lexsort((np.arange(colour.size), colour))


# ---------------------------------------------------------------------------
# the hierarchy
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class VankaParams:
    omega: float = 0.78             # relaxation (eq. vankasmooth): 0.78 Mooney-Rivlin, 0.86 artery
    steps: int = 6                  # sweeps before and after the coarse correction
    additive: bool = False          # the additive variant instead of the multiplicative sweep
    inverse_f32: bool = False       # local solves by the fp32-rounded inverse of each local system
    amg: amg.AmgParams = dataclasses.field(
        default_factory=lambda: amg.AmgParams(smoother="l1jacobi", interp="ext+i"))


@dataclasses.dataclass
class CoupledLevel:
    Kuu: sp.csr_matrix
    Kup: sp.csr_matrix
    Kpu: sp.csr_matrix
    Kpp: sp.csr_matrix
    Pu: sp.csr_matrix | None = None   # None: identity (or the coarsest level)
    Pp: sp.csr_matrix | None = None
    patches: list | None = None
    order: np.ndarray | None = None
    colour: np.ndarray | None = None
    lu: list | None = None
    inv32: list | None = None      # fp32-rounded local inverses (inverse_f32)

    @property
    def nu(self):
        return self.Kuu.shape[0]

    @property
    def np_(self):
        return self.Kpp.shape[0]

    def K(self):
        return sp.bmat([[self.Kuu, self.Kup], [self.Kpu, self.Kpp]]).tocsr()


class CoupledHierarchy:
    def __init__(self, levels, lu, Hu, Hp):
        self.levels, self.lu, self.Hu, self.Hp = levels, lu, Hu, Hp


def _vanka_data(L, inverse_f32=False):
    L.patches = patches(L.Kpu)
    L.colour = greedy_colours(conflict_graph(L.Kuu, L.Kup, L.Kpu, L.Kpp))
    L.order = sweep_order(L.colour)
    K = L.K().toarray() if L.nu + L.np_ <= 4000 else None
    Kc = L.K().tocsr() if K is None else None
    L.lu = []
    for i in range(L.np_):
        idx = np.concatenate([L.patches[i], [L.nu + i]])
        Ki = K[np.ix_(idx, idx)] if K is not None else Kc[idx][:, idx].toarray()
        L.lu.append(scipy.linalg.lu_factor(Ki))
    if inverse_f32:
        L.inv32 = [scipy.linalg.lu_solve(f, np.eye(f[0].shape[0])).astype(np.float32) for f in L.lu]


def _local_solve(L, i, r):
    if L.inv32 is not None:
        return L.inv32[i].astype(np.float64) @ r
    return scipy.linalg.lu_solve(L.lu[i], r)


def setup(Kuu, Kup, Kpu, Kpp, prm: VankaParams = VankaParams()):
    """Coupled hierarchy of K = [Kuu Kup; Kpu Kpp] (block-ordered)."""
    nu, npr = Kuu.shape[0], Kpp.shape[0]
    Hu = amg.setup(Kuu, np.arange(nu) % 3, prm.amg)
    Hp = amg.setup((-Kpp).tocsr(), np.zeros(npr, np.int64), prm.amg)
    nl = max(len(Hu.levels), len(Hp.levels))
    levels = [CoupledLevel(Kuu.tocsr(), Kup.tocsr(), Kpu.tocsr(), Kpp.tocsr())]
    for lev in range(nl - 1):
        L = levels[-1]
        if lev < len(Hu.levels) - 1:
            L.Pu = Hu.levels[lev].P
        if lev < len(Hp.levels) - 1:
            L.Pp = Hp.levels[lev].P
        Kuu_c = Hu.levels[min(lev + 1, len(Hu.levels) - 1)].A
        Kpp_c = (-Hp.levels[min(lev + 1, len(Hp.levels) - 1)].A).tocsr()
        Kup_c = triple(L.Pu.T.tocsr() if L.Pu is not None else None, L.Kup, L.Pp)
        Kpu_c = triple(L.Pp.T.tocsr() if L.Pp is not None else None, L.Kpu, L.Pu)
        levels.append(CoupledLevel(Kuu_c.tocsr(), Kup_c, Kpu_c, Kpp_c))
    for L in levels[:-1]:
        _vanka_data(L, prm.inverse_f32)
    last = levels[-1]
    if last.nu + last.np_ > prm.amg.max_dense:
        raise RuntimeError("coarsest coupled level too large for the dense solve")
    lu = scipy.linalg.lu_factor(last.K().toarray())
    return CoupledHierarchy(levels, lu, Hu, Hp)


# ---------------------------------------------------------------------------
# smoothing and cycling
# ---------------------------------------------------------------------------


def vanka_sweep(L, b, x, omega, K=None):
    """One multiplicative sweep (eq. locsys, eq. vankasmooth) in the patch
    order of L: for each patch, the local residual with every earlier
    update in place, solved directly, added with weight omega."""
    K = L.K() if K is None else K
    x = x.copy()
    for i in L.order:
        idx = np.concatenate([L.patches[i], [L.nu + i]])
        r = b[idx] - K[idx] @ x
        x[idx] += omega * _local_solve(L, i, r)
    return x


def vanka_sweep_additive(L, b, x, omega, K=None):
    """One additive sweep: all local problems from the residual of x, each
    unknown corrected by omega times the mean of its patches' corrections."""
    K = L.K() if K is None else K
    r = b - K @ x
    d = np.zeros_like(x)
    count = np.zeros(x.shape[0], dtype=np.int64)
    for i in range(L.np_):
        idx = np.concatenate([L.patches[i], [L.nu + i]])
        d[idx] += _local_solve(L, i, r[idx])
        count[idx] += 1
    held = count > 0
    x = x.copy()
    x[held] += omega * (d[held] / count[held])
    return x


def _sweep(L, b, x, prm, K):
    if prm.additive:
        return vanka_sweep_additive(L, b, x, prm.omega, K)
    return vanka_sweep(L, b, x, prm.omega, K)


def _restrict(L, r):
    ru, rp = r[:L.nu], r[L.nu:]
    if L.Pu is not None:
        ru = L.Pu.T @ ru
    if L.Pp is not None:
        rp = L.Pp.T @ rp
    return np.concatenate([ru, rp])


def _prolong(L, xc):
    nuc = L.Pu.shape[1] if L.Pu is not None else L.nu
    xu, xp = xc[:nuc], xc[nuc:]
    if L.Pu is not None:
        xu = L.Pu @ xu
    if L.Pp is not None:
        xp = L.Pp @ xp
    return np.concatenate([xu, xp])


def vcycle(CH, b, prm: VankaParams = VankaParams(), lev=0):
    """One V-cycle from a zero start: prm.steps sweeps, the coarse
    correction with R = P^T, prm.steps sweeps."""
    L = CH.levels[lev]
    if lev == len(CH.levels) - 1:
        return scipy.linalg.lu_solve(CH.lu, b)
    K = L.K()
    x = np.zeros_like(b)
    for _ in range(prm.steps):
        x = _sweep(L, b, x, prm, K)
    xc = vcycle(CH, _restrict(L, b - K @ x), prm, lev + 1)
    x = x + _prolong(L, xc)
    for _ in range(prm.steps):
        x = _sweep(L, b, x, prm, K)
    return x


def preconditioner(CH, n, prm: VankaParams = VankaParams()):
    """The V-cycle as a map on node-interleaved vectors."""
    return lambda r: to_interleaved(vcycle(CH, to_blocked(r, n), prm), n)


def amg_iteration(CH, K, b, n, prm: VankaParams = VankaParams(), tol=1e-8, maxit=200):
    """The AMG method as the solver: x <- x + V(b - K x) from x = 0 until
    ||b - K x||_2 <= tol ||b||_2.  Returns x and the residual history."""
    x = np.zeros_like(b)
    bn = np.linalg.norm(b)
    hist = [1.0]
    M = preconditioner(CH, n, prm)
    for _ in range(maxit):
        r = b - K @ x
        hist[-1] = np.linalg.norm(r) / bn
        if hist[-1] <= tol:
            break
        x = x + M(r)
        hist.append(np.inf)
    else:
        hist[-1] = np.linalg.norm(b - K @ x) / bn
    return x, hist
