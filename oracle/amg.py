"""Algebraic multigrid on the displacement block A (oracle).

The paper preconditions the displacement block with AMG cycles (eq. lpre)
and builds coarse operators by Galerkin projection ("AMG methods for the
mixed problems"); it does not fix the coarsening, interpolation or smoother
used here.  The readings followed are:

* unknown-based strength: only entries of the same displacement component
  count; j in S_i iff -a_ij sgn(a_ii) >= theta_s * m_i with
  m_i = max over same-component k != i of -a_ik sgn(a_ii) and m_i > 0;
* PMIS (De Sterck, Yang & Heys 2006) in synchronous rounds with keys
  (lambda_i << 40) | hash40(seed, level, i), ties broken by index;
* modified classical interpolation (Ruge & Stueben 1987, in the form of
  De Sterck et al. 2008) restricted to same-component strong couplings, no
  truncation, C rows the identity;
* Galerkin coarse operators A_c = P^T A P with the structural product
  pattern, then sparsified: off-diagonal entries with
  |a_ij| < drop_tol sqrt(|a_ii a_jj|) are removed (no lumping; drop_tol = 0
  keeps the exact Galerkin operator);
* l1-Jacobi smoothing (Baker, Falgout, Kolev & Yang 2011) or degree-2
  Chebyshev on D^{-1}A, and a dense LU solve on the coarsest level.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg
import scipy.sparse as sp

from . import rng

U_, C_, F_ = 0, 1, -1


def _sgn(x):
    return np.where(x < 0, -1.0, 1.0)


def strength(A: sp.csr_matrix, comp, theta=0.15):
    """Strong-dependence sets S_i as a boolean CSR pattern (indptr, indices)."""
    A = A.tocsr()
    n = A.shape[0]
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    cols = A.indices
    diag = A.diagonal()
    cand = (cols != rows) & (comp[cols] == comp[rows])
    neg = -A.data * _sgn(diag)[rows]
    mi = np.full(n, -np.inf)
    np.maximum.at(mi, rows[cand], neg[cand])
    strong = cand & (mi[rows] > 0) & (neg >= theta * mi[rows])
    r = rows[strong]
    indptr = np.zeros(n + 1, np.int64)
    np.add.at(indptr, r + 1, 1)
    return np.cumsum(indptr), cols[strong].astype(np.int64)


def pmis(S_ptr, S_idx, n, seed, level):
    """C/F splitting by PMIS in synchronous rounds.  Returns state (+1 C, -1 F)."""
    lam = np.bincount(S_idx, minlength=n).astype(np.uint64)   # lambda_i = #{k: i in S_k}
    key = (lam << np.uint64(40)) | rng.pmis_hash40(seed, level, np.arange(n))
    state = np.zeros(n, np.int8)
    state[lam == 0] = F_
    rows = np.repeat(np.arange(n), np.diff(S_ptr))
    cols = S_idx
    while np.any(state == U_):
        U = state == U_
        both = U[rows] & U[cols]
        j_wins = (key[cols] > key[rows]) | ((key[cols] == key[rows]) & (cols > rows))
        notmax = np.zeros(n, bool)
        notmax[rows[both & j_wins]] = True
        notmax[cols[both & ~j_wins]] = True
        state[U & ~notmax] = C_
        U = state == U_
        hasC = np.zeros(n, bool)
        hasC[rows[U[rows] & (state[cols] == C_)]] = True
        state[U & hasC] = F_
    return state


def pmis_bruteforce(S_sets, n, seed, level):
    """The same rounds with Python sets, for tiny graphs (test pin)."""
    lam = [0] * n
    for i in range(n):
        for j in S_sets[i]:
            lam[j] += 1
    keys = [((lam[i] << 40) | int(rng.splitmix64_scalar(seed, (level << 40) | i) >> 24), i) for i in range(n)]
    nb = [set(S_sets[i]) for i in range(n)]
    for i in range(n):
        for j in S_sets[i]:
            nb[j].add(i)
    st = ["F" if lam[i] == 0 else "U" for i in range(n)]
    while "U" in st:
        newc = [i for i in range(n) if st[i] == "U" and all(keys[i] > keys[j] for j in nb[i] if st[j] == "U")]
        for i in newc:
            st[i] = "C"
        for i in range(n):
            if st[i] == "U" and any(st[j] == "C" for j in S_sets[i]):
                st[i] = "F"
    return np.array([1 if s == "C" else -1 for s in st], np.int8)


def interp_row(A, S_set, state, comp, i):
    """Weights {j: w_ij} of one F row (modified classical interpolation).

    w_ij = -(a_ij + sum_{k in F*} a_ik abar_kj / sum_{m in C_i} abar_km)
           / (a_ii + sum_{weak same-component n} a_in + sum_{k in F \\ F*} a_ik)
    where C_i / F_i are the strong C / F neighbours of i, abar_km = a_km when
    its sign differs from that of a_kk (else 0), F* the k with a non-zero
    denominator sum.  Every sum runs over the row in ascending column order.
    """
    lo, hi = A.indptr[i], A.indptr[i + 1]
    cols, vals = A.indices[lo:hi], A.data[lo:hi]
    Ci = [int(j) for j in cols if j in S_set and state[j] == C_]
    if not Ci:
        return {}
    num = {j: 0.0 for j in Ci}
    aii = 0.0
    for j, a in zip(cols, vals):
        if j == i:
            aii = a
    den = aii
    for k, a_ik in zip(cols, vals):
        k = int(k)
        if k == i or comp[k] != comp[i]:
            continue
        if k in S_set and state[k] == C_:
            num[k] += a_ik
        elif k in S_set:  # strong F neighbour: distribute if it sees C_i
            klo, khi = A.indptr[k], A.indptr[k + 1]
            kc, kv = A.indices[klo:khi], A.data[klo:khi]
            akk = kv[kc == k][0]
            sk = -1.0 if akk < 0 else 1.0
            abar = {int(m): (a if a * sk < 0 else 0.0) for m, a in zip(kc, kv) if int(m) in num}
            s = 0.0
            for m in sorted(abar):
                s += abar[m]
            if s != 0.0:
                for j in Ci:
                    num[j] += a_ik * abar.get(j, 0.0) / s
            else:
                den += a_ik
        else:  # weak same-component neighbour: lumped into the diagonal
            den += a_ik
    return {j: -num[j] / den for j in Ci}


def interp_row_extpi(A, S_ptr, S_idx, state, comp, i, p_max=0):
    """Weights {j: w_ij} of one F row by extended+i interpolation (De Sterck,
    Falgout, Nolting, Yang, "Distance-two interpolation for parallel
    algebraic multigrid", 2008), on same-component couplings:

    Chat_i = C_i united with the strong C neighbours of every strong F
    neighbour k of i;
    w_ij = -(a_ij + sum_{k in F_i} a_ik abar_kj / s_k) / atilde_ii,
    atilde_ii = a_ii + sum_{weak n not in Chat_i} a_in
                + sum_{k in F_i} a_ik abar_ki / s_k,
    s_k = sum_{l in Chat_i + {i}} abar_kl (a strong F neighbour with s_k = 0
    is lumped into the diagonal instead), abar_kl = a_kl where its sign
    differs from that of a_kk, else 0.  With p_max > 0 a row with more
    candidates keeps the p_max largest |w| and is rescaled to its full row
    sum; |w| is compared in float32, so that weights equal in exact
    arithmetic (the symmetric stencils of a structured mesh give many) tie
    whatever order their fp64 sums ran in, and ties go to the smaller
    column.  Every sum runs in ascending column order.
    """
    lo, hi = A.indptr[i], A.indptr[i + 1]
    cols, vals = A.indices[lo:hi], A.data[lo:hi]
    S_i = set(S_idx[S_ptr[i]:S_ptr[i + 1]].tolist())
    Fs = [int(k) for k in cols if k in S_i and state[k] == F_]
    chat = {int(j) for j in cols if j in S_i and state[j] == C_}
    for k in Fs:
        S_k = set(S_idx[S_ptr[k]:S_ptr[k + 1]].tolist())
        chat |= {int(m) for m in A.indices[A.indptr[k]:A.indptr[k + 1]] if m in S_k and state[m] == C_}
    if not chat:
        return {}
    num = {j: 0.0 for j in chat}
    den = vals[cols == i][0]
    for j, a in zip(cols, vals):
        j = int(j)
        if j == i or comp[j] != comp[i]:
            continue
        if j in chat:
            num[j] += a
        elif not (j in S_i and state[j] == F_):
            den += a  # weak neighbour outside Chat_i: lumped
    for k in Fs:
        a_ik = vals[cols == k][0]
        kc = A.indices[A.indptr[k]:A.indptr[k + 1]]
        kv = A.data[A.indptr[k]:A.indptr[k + 1]]
        sk = -1.0 if kv[kc == k][0] < 0 else 1.0
        abar = {int(m): (a if a * sk < 0 else 0.0) for m, a in zip(kc, kv)}
        s = 0.0
        for m in sorted(abar):
            if m in chat or m == i:
                s += abar[m]
        if s == 0.0:
            den += a_ik
            continue
        for m in sorted(abar):
            if m in chat:
                num[m] += a_ik * abar[m] / s
        den += a_ik * abar.get(i, 0.0) / s
    w = {j: -num[j] / den for j in chat}
    if p_max and len(w) > p_max:
        keep = sorted(w, key=lambda j: (-float(np.float32(abs(w[j]))), j))[:p_max]
        tot = 0.0
        for j in sorted(w):
            tot += w[j]
        kept = 0.0
        for j in sorted(keep):
            kept += w[j]
        f = tot / kept if kept != 0.0 else 1.0
        w = {j: w[j] * f for j in keep}
    return w


def interpolation(A, S_ptr, S_idx, state, comp, kind="classical", p_max=0):
    """P (n x n_c) and the coarse component array; kind "classical"
    (interp_row) or "ext+i" (interp_row_extpi with truncation p_max)."""
    A = A.tocsr()
    n = A.shape[0]
    cidx = np.cumsum(state == C_) - 1
    nc = int((state == C_).sum())
    rows, cols, vals = [], [], []
    for i in range(n):
        if state[i] == C_:
            rows.append(i); cols.append(cidx[i]); vals.append(1.0)
            continue
        if kind == "ext+i":
            w = interp_row_extpi(A, S_ptr, S_idx, state, comp, i, p_max)
        else:
            S_set = set(S_idx[S_ptr[i]:S_ptr[i + 1]].tolist())
            w = interp_row(A, S_set, state, comp, i)
        for j in sorted(w):
            rows.append(i); cols.append(cidx[j]); vals.append(w[j])
    P = sp.csr_matrix((np.array(vals), (np.array(rows, np.int64), np.array(cols, np.int64))), shape=(n, nc))
    P.sort_indices()
    return P, comp[state == C_]


def _pattern(M):
    Q = M.tocsr().copy()
    Q.data = np.ones_like(Q.data)
    return Q


def galerkin(A, P):
    """A_c = P^T (A P) on the structural pattern of the triple product.

    The values come from the library sparse product; the pattern is the
    product of the 0/1 patterns (all-ones values cannot cancel), so entries
    that happen to sum to zero are kept as explicit zeros.
    """
    R = P.T.tocsr()
    vals = (R @ (A @ P)).tocsr()
    pat = (_pattern(R) @ _pattern(A) @ _pattern(P)).tocsr()
    pat.sort_indices()
    rr = np.repeat(np.arange(pat.shape[0]), np.diff(pat.indptr))
    data = np.asarray(vals[rr, pat.indices]).ravel() if pat.nnz else np.zeros(0)
    return sp.csr_matrix((data, pat.indices.copy(), pat.indptr.copy()), shape=pat.shape)


def drop_small(Ac, eps):
    """Sparsified coarse operator: every off-diagonal entry with
    |a_ij| < eps sqrt(|a_ii a_jj|) is removed, nothing is lumped.  Both
    sides of the comparison are rounded to float32 (the product, square root
    and scaling in fp64 first), so an entry that sits on the threshold in
    exact arithmetic is decided the same way whatever order the sums of the
    Galerkin product ran in.  eps <= 0 returns Ac unchanged."""
    if eps <= 0:
        return Ac
    Ac = Ac.tocsr()
    n = Ac.shape[0]
    rows = np.repeat(np.arange(n), np.diff(Ac.indptr))
    cols = Ac.indices
    d = np.abs(Ac.diagonal())
    thr = (eps * np.sqrt(d[rows] * d[cols])).astype(np.float32)
    keep = (rows == cols) | ~(np.abs(Ac.data).astype(np.float32) < thr)
    indptr = np.zeros(n + 1, np.int64)
    np.add.at(indptr, rows[keep] + 1, 1)
    return sp.csr_matrix((Ac.data[keep], cols[keep], np.cumsum(indptr)), shape=Ac.shape)


def coarse_operator(A, P, drop_tol=0.0):
    """A_c = drop_small(P^T A P, drop_tol)."""
    return drop_small(galerkin(A, P), drop_tol)


def on_pattern(M, pattern):
    """The entries of M at the stored positions of `pattern` (a subset of
    M's pattern), in pattern's layout."""
    M = M.tocsr()
    pattern = pattern.tocsr()
    rr = np.repeat(np.arange(pattern.shape[0]), np.diff(pattern.indptr))
    data = np.asarray(M[rr, pattern.indices]).ravel() if pattern.nnz else np.zeros(0)
    return sp.csr_matrix((data, pattern.indices.copy(), pattern.indptr.copy()), shape=pattern.shape)


# ---------------------------------------------------------------------------
# smoothers
# ---------------------------------------------------------------------------


def l1_diag(A):
    """D1_ii = sum_j |a_ij|."""
    return np.asarray(abs(A).sum(axis=1)).ravel()


def lanczos_max(A, d, steps, seed, level):
    """Largest Ritz value of `steps` Lanczos steps on D^{-1/2} A D^{-1/2}
    (D = diag A) from a SplitMix64 start vector."""
    n = A.shape[0]
    dm = 1.0 / np.sqrt(np.abs(d))
    q = rng.uniform_pm1(seed, 1000 + level, n)
    q /= np.linalg.norm(q)
    alphas, betas = [], []
    q_prev = np.zeros(n)
    beta = 0.0
    for _ in range(min(steps, n)):
        w = dm * (A @ (dm * q)) - beta * q_prev
        alpha = q @ w
        w = w - alpha * q
        alphas.append(alpha)
        beta = np.linalg.norm(w)
        if beta <= 1e-14 * abs(alpha):
            break
        betas.append(beta)
        q_prev, q = q, w / beta
    k = len(alphas)
    T = np.diag(alphas) + np.diag(betas[:k - 1], 1) + np.diag(betas[:k - 1], -1)
    return float(np.linalg.eigvalsh(T).max())


@dataclasses.dataclass
class Level:
    A: sp.csr_matrix
    comp: np.ndarray
    P: sp.csr_matrix | None = None
    R: sp.csr_matrix | None = None
    state: np.ndarray | None = None
    S: tuple | None = None
    dinv: np.ndarray | None = None   # l1 inverse diagonal, or D^{-1} for Chebyshev
    lam: float = 0.0


@dataclasses.dataclass
class AmgParams:
    theta: float = 0.15
    max_coarse: int = 500
    max_levels: int = 25
    seed: int = 12345
    smoother: str = "chebyshev"   # or "l1jacobi"
    nu_pre: int = 1                # level 0: sweeps before the coarse correction
    nu_post: int = 1               # and after it
    cheb_degree: int = 3           # their Chebyshev degree
    cheb_ratio: float = 30.0
    cheb_degree_pre: int = 1       # pre-smoothing degree
    nu_post_coarse: int = 1        # post-smoothing sweeps on levels >= 1
    cheb_degree_coarse: int = 3    # their degree
    nu_pre_coarse: int = 0         # pre-smoothing sweeps on levels >= 1 (degree cheb_degree_pre)
    interp: str = "ext+i"          # or "classical"
    p_max: int = 4                 # ext+i truncation (0: none)
    drop_tol: float = 0.0          # coarse-operator sparsification (0: exact Galerkin)
    lanczos_steps: int = 10
    max_dense: int = 8192


class Hierarchy:
    def __init__(self, levels, lu):
        self.levels = levels
        self.lu = lu


def setup(A, comp, prm: AmgParams = AmgParams()):
    """Build the hierarchy until n_l <= max_coarse, max_levels is reached or
    coarsening stalls (n_{l+1} > 0.9 n_l); the last level is solved by LU."""
    levels = [Level(A.tocsr(), np.asarray(comp))]
    while True:
        L = levels[-1]
        n = L.A.shape[0]
        _smoother_data(L, prm, len(levels) - 1)
        if n <= prm.max_coarse or len(levels) >= prm.max_levels:
            break
        S = strength(L.A, L.comp, prm.theta)
        st = pmis(S[0], S[1], n, prm.seed, len(levels) - 1)
        nc = int((st == C_).sum())
        if nc == 0 or nc > 0.9 * n:
            break
        P, ccomp = interpolation(L.A, S[0], S[1], st, L.comp, prm.interp, prm.p_max)
        L.S, L.state, L.P, L.R = S, st, P, P.T.tocsr()
        levels.append(Level(coarse_operator(L.A, P, prm.drop_tol), ccomp))
    last = levels[-1]
    if last.A.shape[0] > prm.max_dense:
        raise RuntimeError("coarsest level too large for the dense solve")
    lu = scipy.linalg.lu_factor(last.A.toarray())
    return Hierarchy(levels, lu)


def resetup(A, H: Hierarchy, prm: AmgParams = AmgParams()):
    """Hierarchy of a new operator A (same size and component map as the
    level-0 operator of H) on the coarse grids of H: the C/F splittings and
    interpolations P (R = P^T) of H are kept, every coarse operator is the
    Galerkin product of the new level above it restricted to the stored
    pattern of H's operator on that level (the set-up's sparsified pattern),
    and the smoother data and the coarsest LU are recomputed.  With A equal
    to H's own level-0 operator this is H again."""
    old = H.levels
    if A.shape != old[0].A.shape:
        raise ValueError("resetup: operator size differs from the hierarchy's")
    levels = [Level(A.tocsr(), old[0].comp)]
    for lev, o in enumerate(old):
        L = levels[-1]
        _smoother_data(L, prm, lev)
        if o.P is None:
            break
        L.S, L.state, L.P, L.R = o.S, o.state, o.P, o.R
        levels.append(Level(on_pattern(galerkin(L.A, o.P), old[lev + 1].A), old[lev + 1].comp))
    lu = scipy.linalg.lu_factor(levels[-1].A.toarray())
    return Hierarchy(levels, lu)


def _smoother_data(L, prm, lev):
    if prm.smoother == "l1jacobi":
        L.dinv = 1.0 / l1_diag(L.A)
    else:
        d = L.A.diagonal()
        L.dinv = 1.0 / d
        L.lam = lanczos_max(L.A, d, prm.lanczos_steps, prm.seed, lev)


def smooth(L, b, x, nu, prm, degree):
    if prm.smoother == "l1jacobi":
        for _ in range(nu):
            x = x + L.dinv * (b - L.A @ x)
        return x
    for _ in range(nu):
        x = chebyshev(L.A, L.dinv, L.lam, b, x, degree, prm.cheb_ratio)
    return x


def chebyshev(A, dinv, lam, b, x, degree=2, ratio=30.0):
    """Degree-k Chebyshev smoothing of D^{-1}A on [lam/ratio, 1.1 lam]
    (three-term recurrence for the residual polynomial)."""
    hi, lo = 1.1 * lam, lam / ratio
    theta = 0.5 * (hi + lo)
    delta = 0.5 * (hi - lo)
    sigma = theta / delta
    rho = 1.0 / sigma
    r = dinv * (b - A @ x)
    d = r / theta
    x = x + d
    for _ in range(degree - 1):
        r = dinv * (b - A @ x)
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * r
        x = x + d
        rho = rho_new
    return x


def vcycle(H: Hierarchy, b, prm: AmgParams = AmgParams(), lev=0):
    """One V-cycle with zero initial guess on every level: pre-smoothing of
    degree cheb_degree_pre (nu_pre sweeps on level 0, nu_pre_coarse on the
    coarser levels), the coarse correction, then nu_post sweeps of degree
    cheb_degree on level 0 (nu_post_coarse of cheb_degree_coarse on the
    coarser levels)."""
    L = H.levels[lev]
    if lev == len(H.levels) - 1:
        return scipy.linalg.lu_solve(H.lu, b)
    x = smooth(L, b, np.zeros_like(b), prm.nu_pre if lev == 0 else prm.nu_pre_coarse, prm, prm.cheb_degree_pre)
    r = b - L.A @ x
    xc = vcycle(H, L.R @ r, prm, lev + 1)
    x = x + L.P @ xc
    if lev == 0:
        return smooth(L, b, x, prm.nu_post, prm, prm.cheb_degree)
    return smooth(L, b, x, prm.nu_post_coarse, prm, prm.cheb_degree_coarse)


def convergence_factor(H, prm, cycles=10, seed=777):
    """rho = (||e_k||_A / ||e_0||_A)^{1/k} of the stationary V-cycle iteration
    e <- e - V(A e), from a SplitMix64 start vector."""
    A = H.levels[0].A
    e = rng.uniform_pm1(seed, 0, A.shape[0])
    n0 = np.sqrt(e @ (A @ e))
    for _ in range(cycles):
        e = e - vcycle(H, A @ e, prm)
    return float((np.sqrt(abs(e @ (A @ e))) / n0) ** (1.0 / cycles))


def complexity(H):
    nnz = [L.A.nnz for L in H.levels]
    rows = [L.A.shape[0] for L in H.levels]
    return sum(nnz) / nnz[0], sum(rows) / rows[0]
