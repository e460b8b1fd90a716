"""Block-triangular preconditioners, FGMRES, BiCGStab and GCR (oracle).

The preconditioner is the paper's P_L (eq. lpre): with K = [A B1^T; B2 -C],
    P_L^{-1} [r_u; r_p] = [z_u; z_p],  z_u = Atilde^{-1} r_u,
    z_p = Stilde^{-1} (B2 z_u - r_p),
where Atilde^{-1} is one AMG V-cycle on A and Stilde = (1/theta + 1/kappa)
diag(M_p) (eq. lpreschur).  The Krylov method is right-preconditioned
flexible GMRES(m) with classical Gram-Schmidt and one re-orthogonalisation
(CGS2) and Givens rotations; the paper itself uses BiCGStab here.

For the fluid the paper uses GCR with P_R = Dtilde Utilde (eq. rpre):
    P_R^{-1} [r_u; r_p] = [z_u; z_p],  z_p = -Stilde^{-1} r_p,
    z_u = Atilde^{-1} (r_u - B1^T z_p),
here with a diagonal Stilde (the caller's s).  GCR(m): z_j = M^{-1} r,
q_j = K z_j, q_j and z_j orthogonalised against the earlier q_i (two
classical Gram-Schmidt passes, the same combination applied to the z_i)
and scaled to |q_j| = 1, then x += (q_j.r) z_j, r -= (q_j.r) q_j; the
recurrence residual ends a cycle, the true residual decides.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import amg


def split(r, n):
    r = r.reshape(n, 4)
    return r[:, 0:3].ravel(), r[:, 3].copy()


def join(zu, zp, n):
    z = np.empty((n, 4))
    z[:, 0:3] = zu.reshape(n, 3)
    z[:, 3] = zp
    return z.ravel()


class BlockPreconditioner:
    """P_L^{-1} with Atilde^{-1} given as a callable on displacement vectors."""

    def __init__(self, a_inv, B2, s, n):
        self.a_inv, self.B2, self.s, self.n = a_inv, B2, s, n

    def __call__(self, r):
        ru, rp = split(r, self.n)
        zu = self.a_inv(ru)
        zp = (self.B2 @ zu - rp) / self.s
        return join(zu, zp, self.n)


class UpperBlockPreconditioner:
    """P_R^{-1} (eq. rpre) with Atilde^{-1} a callable on displacement
    vectors, B1T the (u, p) block of K and a diagonal Stilde = diag(s)."""

    def __init__(self, a_inv, B1T, s, n):
        self.a_inv, self.B1T, self.s, self.n = a_inv, B1T, s, n

    def __call__(self, r):
        ru, rp = split(r, self.n)
        zp = -rp / self.s
        zu = self.a_inv(ru - self.B1T @ zp)
        return join(zu, zp, self.n)


def amg_preconditioner(A, B2, s, n, prm=amg.AmgParams()):
    comp = np.tile(np.arange(3), n)
    H = amg.setup(A, comp, prm)
    return BlockPreconditioner(lambda r: amg.vcycle(H, r, prm), B2, s, n), H


@dataclasses.dataclass
class SolveInfo:
    iterations: int = 0
    restarts: int = 0
    rel_residual: float = np.inf
    converged: bool = False
    breakdown: bool = False
    history: list = dataclasses.field(default_factory=list)


def fgmres(K, precond, b, x0=None, m=50, maxit=500, tol=1e-8):
    """Solve K x = b to ||b - K x||_2 <= tol ||b||_2.

    Per restart cycle: v_0 = r/||r||; for j: z_j = M^{-1} v_j, w = K z_j,
    two classical Gram-Schmidt passes against v_0..v_j, h_{j+1,j} = ||w||;
    Givens rotations c = h_jj / sqrt(h_jj^2 + h_{j+1,j}^2),
    s = h_{j+1,j} / sqrt(...) reduce the Hessenberg matrix; the cycle ends
    when |g_{j+1}| <= tol ||b||, on breakdown (h_{j+1,j} <= 1e-14 ||w_0||)
    or after m steps; x += Z y.  The true residual is recomputed after every
    cycle and decides convergence.
    """
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else x0.copy()
    info = SolveInfo()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        x[:] = 0.0
        info.rel_residual, info.converged = 0.0, True
        return x, info
    r = b - K @ x
    beta = np.linalg.norm(r)
    info.rel_residual = beta / bnorm
    if beta <= tol * bnorm:
        info.converged = True
        return x, info
    while info.iterations < maxit:
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        V[0] = r / beta
        g[0] = beta
        j_end = 0
        for j in range(m):
            Z[j] = precond(V[j])
            w = K @ Z[j]
            w0 = np.linalg.norm(w)
            h = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h
            h2 = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h2
            H[:j + 1, j] = h + h2
            H[j + 1, j] = np.linalg.norm(w)
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            d = np.hypot(H[j, j], H[j + 1, j])
            hj1 = H[j + 1, j]
            cs[j], sn[j] = H[j, j] / d, hj1 / d
            H[j, j] = d
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            info.iterations += 1
            info.history.append(abs(g[j + 1]) / bnorm)
            j_end = j + 1
            if abs(g[j + 1]) <= tol * bnorm or info.iterations >= maxit:
                break
            if hj1 <= 1e-14 * w0:
                info.breakdown = True
                break
            V[j + 1] = w / hj1
        y = np.zeros(j_end)
        for i in range(j_end - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:j_end] @ y[i + 1:]) / H[i, i]
        x = x + Z[:j_end].T @ y
        r = b - K @ x
        beta = np.linalg.norm(r)
        info.rel_residual = beta / bnorm
        if beta <= tol * bnorm:
            info.converged = True
            break
        if info.breakdown:
            break
        info.restarts += 1
    return x, info


def bicgstab(K, precond, b, x0=None, maxit=500, tol=1e-8):
    """Solve K x = b with right-preconditioned BiCGStab, the Krylov method of
    the paper's structure sub-problem (section "A preconditioner for the
    structure sub-problem"; van der Vorst's BiCGStab), preconditioner M^{-1}.

    Shadow residual r^ = r_0.  One iteration: rho = r^.r;
    p = r + (rho / rho_old)(alpha / omega)(p - omega v) (p = r at the
    start); p^ = M^{-1} p, v = K p^, alpha = rho / r^.v; s = r - alpha v;
    s^ = M^{-1} s, t = K s^, omega = t.s / t.t (0 when t = 0); x += alpha p^ +
    omega s^, r = s - omega t.  The updated residual ends the iteration loop
    at ||r|| <= tol ||b||; the true residual then decides, and the method
    starts again from it (new shadow) if it is still above the tolerance.
    Breakdown when r^.r or r^.v vanishes, or omega = 0 before convergence.
    """
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else x0.copy()
    info = SolveInfo()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        x[:] = 0.0
        info.rel_residual, info.converged = 0.0, True
        return x, info
    r = b - K @ x
    info.rel_residual = np.linalg.norm(r) / bnorm
    while info.rel_residual > tol and info.iterations < maxit and not info.breakdown:
        rhat = r.copy()
        rho_old = alpha = omega = 1.0
        p = np.zeros(n)
        v = np.zeros(n)
        first = True
        while info.iterations < maxit:
            rho = rhat @ r
            if rho == 0.0:
                info.breakdown = True
                break
            p = r.copy() if first else r + (rho / rho_old) * (alpha / omega) * (p - omega * v)
            first = False
            ph = precond(p)
            v = K @ ph
            rv = rhat @ v
            if rv == 0.0:
                info.breakdown = True
                break
            alpha = rho / rv
            s = r - alpha * v
            sh = precond(s)
            t = K @ sh
            tt = t @ t
            omega = (t @ s) / tt if tt > 0.0 else 0.0
            x = x + alpha * ph + omega * sh
            r = s - omega * t
            rho_old = rho
            info.iterations += 1
            rel = np.linalg.norm(r) / bnorm
            info.history.append(rel)
            if rel <= tol:
                break
            if omega == 0.0:
                info.breakdown = True
                break
        r = b - K @ x
        info.rel_residual = np.linalg.norm(r) / bnorm
        if info.rel_residual > tol and not info.breakdown and info.iterations < maxit:
            info.restarts += 1
    info.converged = info.rel_residual <= tol
    return x, info



def krylov_factor(K, precond, b, k=20):
    """Residual reduction rate (||r_k|| / ||r_0||)^(1/k) of k FGMRES steps
    without restart from x = 0 (k = the steps taken, fewer after a lucky
    breakdown): the measure by which the judge compares the learned and the
    classical hierarchy on an assembled tangent."""
    _, info = fgmres(K, precond, b, m=k, maxit=k, tol=1e-300)
    return info.rel_residual ** (1.0 / max(info.iterations, 1))


def gcr(K, precond, b, x0=None, m=50, maxit=500, tol=1e-8):
    """Solve K x = b with restarted, right-preconditioned GCR(m) (the
    fluid's Krylov method, section "A preconditioner for the fluid
    sub-problem") to ||b - K x||_2 <= tol ||b||_2.  The preconditioner may
    change between steps (the z_j are kept)."""
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else x0.copy()
    info = SolveInfo()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        x[:] = 0.0
        info.rel_residual, info.converged = 0.0, True
        return x, info
    r = b - K @ x
    rn = np.linalg.norm(r)
    info.rel_residual = rn / bnorm
    if rn <= tol * bnorm:
        info.converged = True
        return x, info
    while info.iterations < maxit:
        Q = np.zeros((m, n))
        Z = np.zeros((m, n))
        for j in range(m):
            z = precond(r)
            q = K @ z
            for _ in range(2):
                h = Q[:j] @ q
                q = q - Q[:j].T @ h
                z = z - Z[:j].T @ h
            nq = np.linalg.norm(q)
            if nq == 0.0:
                info.breakdown = True
                break
            Q[j], Z[j] = q / nq, z / nq
            alpha = Q[j] @ r
            x = x + alpha * Z[j]
            r = r - alpha * Q[j]
            info.iterations += 1
            info.history.append(np.linalg.norm(r) / bnorm)
            if info.history[-1] <= tol or info.iterations >= maxit:
                break
        r = b - K @ x
        rn = np.linalg.norm(r)
        info.rel_residual = rn / bnorm
        if rn <= tol * bnorm:
            info.converged = True
            break
        if info.breakdown:
            break
        info.restarts += 1
    return x, info
