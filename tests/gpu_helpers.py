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


def amg_prm_pair(lib, smoother=0, precision=0, max_coarse=500, theta=0.15, seed=12345, nu=2, nu_post=None,
                 cheb=(2, 30.0), kind="classical", p_max=4, schedule=None, drop_tol=None):
    """GPU and oracle AMG parameters with the same settings.  schedule=None:
    the same sweeps (nu, nu_post) and Chebyshev degree cheb[0] on every level;
    schedule="default": the library's default smoothing schedule."""
    if schedule == "default":
        d = lib.amg_params()
        sm = dict(nu_pre=d.nu_pre, nu_post=d.nu_post, cheb_degree=d.cheb_degree, cheb_ratio=d.cheb_ratio,
                  cheb_degree_pre=d.cheb_degree_pre, nu_post_coarse=d.nu_post_coarse,
                  cheb_degree_coarse=d.cheb_degree_coarse, nu_pre_coarse=d.nu_pre_coarse)
    else:
        nu_post = nu if nu_post is None else nu_post
        sm = dict(nu_pre=nu, nu_post=nu_post, cheb_degree=cheb[0], cheb_ratio=cheb[1], cheb_degree_pre=cheb[0],
                  nu_post_coarse=nu_post, cheb_degree_coarse=cheb[0], nu_pre_coarse=nu)
    if drop_tol is None:
        drop_tol = lib.amg_params().drop_tol
    g = lib.amg_params(theta=theta, max_coarse=max_coarse, seed=seed, smoother=smoother,
                       interp_kind=1 if kind == "ext+i" else 0, p_max=p_max, precision=precision,
                       drop_tol=drop_tol, **sm)
    o = amg.AmgParams(theta=theta, max_coarse=max_coarse, seed=seed,
                      smoother="l1jacobi" if smoother == 0 else "chebyshev", interp=kind, p_max=p_max,
                      drop_tol=drop_tol, **sm)
    return g, o


__all__ = ["torch_dev", "context_for", "oracle_system", "export_level_matrix", "gpu_hierarchy_to_oracle",
           "amg_prm_pair", "oracle_sampled_rows", "synth"]


def oracle_sampled_rows(prob, v, load, nodes, inertia=None):
    """Oracle residual entries and Dirichlet-eliminated tangent rows of the
    given nodes, computed on the sub-mesh of the elements incident to them
    (with the loaded boundary triangles that touch them): every contribution
    to those rows comes from such an element or triangle, so the rows are
    those of the full assembly.  inertia = (cm, r_s [n,3]) adds the
    Newmark-beta terms.  Returns {node: (R[4], {global col dof: K row values
    [4]})}."""
    nodes = np.asarray(sorted(set(int(i) for i in nodes)))
    sel = np.isin(prob.tets, nodes).any(axis=1)
    tets = prob.tets[sel]
    sub_nodes = np.unique(tets)
    loc = -np.ones(prob.n_nodes, np.int64)
    loc[sub_nodes] = np.arange(len(sub_nodes))
    tsel = np.isin(prob.tris, nodes).any(axis=1) if len(prob.tris) else np.zeros(0, bool)
    sub = synth.Problem(prob.X[sub_nodes], loc[tets].astype(np.int32), prob.mat_id[sel], prob.materials,
                         prob.dir_mask[sub_nodes], loc[prob.tris[tsel]].astype(np.int32), prob.traction[tsel],
                         prob.lattice[sub_nodes], None if prob.fibres is None else prob.fibres[sel], name="rows")
    d = fe.Discretization(sub)
    if inertia is not None:
        d.set_inertia(inertia[0], np.asarray(inertia[1]).reshape(prob.n_nodes, 3)[sub_nodes])
    vs = np.asarray(v).reshape(prob.n_nodes, 4)[sub_nodes].ravel()
    R, val = d.assemble(vs, load)
    R, val = d.apply_dirichlet(R, val)
    K = d.csr(val)
    out = {}
    for g in nodes:
        li = loc[g]
        rows = {}
        for r in range(4):
            i = 4 * li + r
            for c, a in zip(K.indices[K.indptr[i]:K.indptr[i + 1]], K.data[K.indptr[i]:K.indptr[i + 1]]):
                gc = 4 * sub_nodes[c // 4] + c % 4
                rows.setdefault(int(gc), np.zeros(4))[r] = a
        out[int(g)] = (R[4 * li:4 * li + 4].copy(), rows)
    return out
