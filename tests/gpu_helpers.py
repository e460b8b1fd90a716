"""Shared helpers of the GPU parity tests (test infrastructure)."""
import numpy as np
import scipy.linalg
import scipy.sparse as sp

import synth
from oracle import amg, fe, newton


def torch_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, np.float64)).cuda()


def context_for(lib, prob, theta=None):
    ctx = lib.Context(0)
    ctx.set_problem(prob, theta=theta)
    return ctx


def oracle_system(prob, v, load):
    d = fe.Discretization(prob)
    K, b, A, B2, s = newton.linear_system(d, v.ravel(), load)
    return d, K, b, A, B2, s


def export_level_matrix(ctx, level, which):
    ptr, col, val, ncols = ctx.amg_export(level, which)
    return sp.csr_matrix((val, col, ptr), shape=(len(ptr) - 1, ncols))


def gpu_hierarchy_to_oracle(ctx, info, prm: amg.AmgParams):
    """Rebuild an oracle Hierarchy from the GPU's level operators and P."""
    levels = []
    L = info.levels
    for l in range(L):
        A = export_level_matrix(ctx, l, 0)
        comp = ctx.amg_export(l, 4)
        lev = amg.Level(A, comp)
        if l < L - 1:
            lev.P = export_level_matrix(ctx, l, 1)
            lev.R = lev.P.T.tocsr()
        amg._smoother_data(lev, prm, l)
        levels.append(lev)
    lu = scipy.linalg.lu_factor(levels[-1].A.toarray())
    return amg.Hierarchy(levels, lu)


def amg_prm_pair(lib, smoother=0, precision=0, max_coarse=500, theta=0.5, seed=12345, nu=2):
    g = lib.amg_params(theta=theta, max_coarse=max_coarse, seed=seed, smoother=smoother, nu_pre=nu, nu_post=nu,
                       precision=precision)
    o = amg.AmgParams(theta=theta, max_coarse=max_coarse, seed=seed,
                      smoother="l1jacobi" if smoother == 0 else "chebyshev", nu_pre=nu, nu_post=nu)
    return g, o


__all__ = ["torch_dev", "context_for", "oracle_system", "export_level_matrix", "gpu_hierarchy_to_oracle",
           "amg_prm_pair", "synth"]
