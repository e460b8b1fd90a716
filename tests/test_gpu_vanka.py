"""GPU parity of the coupled (u,p) AMG with the multiplicative Vanka smoother
(section "The multiplicative Vanka smoother", eq. locsys, eq. vankasmooth).

The oracle builds its own coupled hierarchy from its own assembly of the
same state; nothing it uses comes from the GPU.  Compared:

* every level's four blocks Kuu, Kup, Kpu, Kpp and the transfers P_u, P_p:
  patterns bit-exact, values to 1e-11 relative;
* the patch colours (first-fit order): bit-exact;
* one V-cycle on a random vector, entry by entry, to 1e-9 relative (a
  sweep is a long chain of dependent local solves);
* the AMG method as the solver (method 2): the same number of V-cycles as
  the oracle, the true residual checked on the host; FGMRES with the coupled
  V-cycle within one iteration of the oracle;
* a Newton step with the coupled hierarchy: the update agrees with the
  oracle's direct solve of the same Newton system;
* at 24^3 (three levels of patches, 15,625 patches on level 0): blocks and
  colours of level 0 bit-exact with the oracle, and the solve's residual
  checked on the host;
* with precision = 1 (patch inverses rounded to fp32), both variants: one
  V-cycle entry by entry to 1e-6 relative of the oracle's cycle with
  rounded inverses, and FGMRES within one iteration of it;
* the additive variant (coupled = 2, corrections averaged over the patches
  of each unknown): the same hierarchy blocks, no colours (export 14 is an
  error), one V-cycle entry by entry to 1e-10 relative, the AMG method with
  the oracle's count of V-cycles and FGMRES within one iteration, and the
  24^3 solve checked on the host.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

import synth
from gpu_helpers import context_for, torch_dev
from oracle import amg, fe, krylov, vanka

pytestmark = pytest.mark.gpu


def _params(lib, omega=0.78, steps=2, max_coarse=150, theta=0.15, seed=12345, additive=False, f32=False):
    g = lib.amg_params(coupled=2 if additive else 1, vanka_omega=omega, vanka_steps=steps, max_coarse=max_coarse,
                       theta=theta, seed=seed, interp_kind=1, p_max=4, precision=1 if f32 else 0)
    o = vanka.VankaParams(omega=omega, steps=steps, additive=additive, inverse_f32=f32,
                          amg=amg.AmgParams(theta=theta, max_coarse=max_coarse, seed=seed, interp="ext+i", p_max=4,
                                            smoother="l1jacobi"))
    return g, o


def _problem(N, law="mr", seed=2):
    if law == "mr":
        return synth.cube_problem(N, jitter=0.1, seed=seed)
    return synth.tube_problem(n_theta=12, n_media=2, n_adv=1, n_z=N)


def _both(lib, prob, v, load, g, o, oracle_hierarchy=True):
    import torch
    ctx = context_for(lib, prob)
    vt = torch_dev(v)
    R = torch.zeros_like(vt)
    ctx.assemble_residual_tangent(vt, load, R)
    info = ctx.amg_setup(g)
    d = fe.Discretization(prob)
    Ro, val = d.assemble(v, load)
    Ro, val = d.apply_dirichlet(Ro, val)
    blocks = vanka.tangent_blocks(d, val)
    CH = vanka.setup(*blocks, o) if oracle_hierarchy else None
    return ctx, info, R, d, d.csr(val), -Ro, blocks, CH


def _export(ctx, lev, which):
    ptr, col, val, ncols = ctx.amg_export(lev, which)
    return sp.csr_matrix((val, col, ptr), shape=(len(ptr) - 1, ncols))


def _same(G, O, what, rtol=1e-11):
    G, O = G.tocsr(), O.tocsr()
    O.sort_indices()
    assert G.shape == O.shape, what
    assert np.array_equal(G.indptr, O.indptr), what
    assert np.array_equal(G.indices, O.indices), what
    scale = max(np.abs(O.data).max(), 1e-300) if O.nnz else 1.0
    assert np.abs(G.data - O.data).max() <= rtol * scale if O.nnz else True, what


@pytest.mark.parametrize("law,N,steps", [("mr", 6, 2), ("mr", 8, 6), ("artery", 4, 2)])
def test_hierarchy_matches_oracle(lib, law, N, steps):
    prob = _problem(N, law)
    v = synth.random_state(prob, 4, u_scale=0.03, p_scale=0.05).ravel()
    print(f"[vanka hierarchy] {law} N={N} steps={steps}", flush=True)
    g, o = _params(lib, omega=0.78 if law == "mr" else 0.86, steps=steps)
    ctx, info, R, d, K, b, blocks, CH = _both(lib, prob, v, 0.4, g, o)
    assert info.levels == len(CH.levels)
    for lev, L in enumerate(CH.levels):
        assert info.rows[lev] == L.nu + L.np_
        for which, M in ((10, L.Kuu), (11, L.Kup), (12, L.Kpu), (13, L.Kpp)):
            _same(_export(ctx, lev, which), M, f"level {lev} block {which}")
        if lev + 1 < len(CH.levels):
            for which, P in ((15, L.Pu), (16, L.Pp)):
                if P is None:
                    with pytest.raises(RuntimeError):
                        ctx.amg_export(lev, which)
                else:
                    _same(_export(ctx, lev, which), P, f"level {lev} transfer {which}")
            colours, ncol = ctx.amg_export(lev, 14)
            assert np.array_equal(colours, L.colour), f"level {lev} colours"
            assert ncol == L.colour.max() + 1


@pytest.mark.parametrize("law,N,steps,omega", [("mr", 6, 2, 0.78), ("mr", 8, 6, 0.78), ("artery", 4, 2, 0.86),
                                               ("mr", 6, 1, 1.0)])
def test_vcycle_matches_oracle(lib, law, N, steps, omega):
    import torch
    prob = _problem(N, law)
    v = synth.random_state(prob, 5, u_scale=0.03, p_scale=0.05).ravel()
    print(f"[vanka cycle] {law} N={N} steps={steps} omega={omega}", flush=True)
    g, o = _params(lib, omega=omega, steps=steps)
    ctx, info, R, d, K, b, blocks, CH = _both(lib, prob, v, 0.4, g, o)
    n = prob.n_nodes
    r = np.random.default_rng(6).normal(size=4 * n)
    z = torch.zeros(4 * n, dtype=torch.float64, device="cuda")
    ctx.apply_preconditioner(torch_dev(r), z)
    zo = vanka.preconditioner(CH, n, o)(r)
    zg = z.cpu().numpy()
    assert np.abs(zg - zo).max() <= 1e-9 * np.abs(zo).max()


@pytest.mark.parametrize("law,N,steps", [("mr", 6, 2), ("artery", 4, 12)])
def test_amg_iteration_and_fgmres_match_oracle(lib, law, N, steps):
    """The artery needs more sweeps: with 2 the stationary iteration
    diverges on this tube, with 12 it contracts by about 0.17 per cycle."""
    import torch
    prob = _problem(N, law)
    v = synth.random_state(prob, 7, u_scale=0.03, p_scale=0.05).ravel()
    print(f"[vanka solve] {law} N={N} steps={steps}", flush=True)
    g, o = _params(lib, omega=0.78 if law == "mr" else 0.86, steps=steps)
    ctx, info, R, d, K, b, blocks, CH = _both(lib, prob, v, 0.4, g, o)
    n = prob.n_nodes
    bt = torch_dev(b)
    x = torch.zeros_like(bt)
    si, code = ctx.krylov_amg_solve(bt, x, lib.solve_params(tol=1e-8, max_iter=60, method=2))
    xo, hist = vanka.amg_iteration(CH, K, b, n, o, tol=1e-8, maxit=60)
    assert code == 0 and si.converged
    assert si.iterations == len(hist) - 1, (si.iterations, len(hist) - 1)
    xg = x.cpu().numpy()
    assert np.linalg.norm(b - K @ xg) <= 1e-8 * np.linalg.norm(b)
    assert np.abs(xg - xo).max() <= 1e-7 * np.abs(xo).max()
    # FGMRES with the coupled V-cycle
    x.zero_()
    si2, code2 = ctx.krylov_amg_solve(bt, x, lib.solve_params(tol=1e-8, restart=50, max_iter=200))
    xo2, oi = krylov.fgmres(K, vanka.preconditioner(CH, n, o), b, m=50, tol=1e-8)
    assert code2 == 0 and oi.converged
    assert abs(si2.iterations - oi.iterations) <= 1, (si2.iterations, oi.iterations)
    assert np.linalg.norm(b - K @ x.cpu().numpy()) <= 1e-8 * np.linalg.norm(b)


def test_newton_step_with_coupled_hierarchy(lib):
    import torch
    prob = _problem(6, "mr", seed=3)
    v0 = synth.random_state(prob, 8, u_scale=0.02, p_scale=0.02).ravel()
    g, _ = _params(lib, steps=2)
    ctx = context_for(lib, prob)
    vt = torch_dev(v0)
    info, code = ctx.newton_step(vt, 0.5, lib.newton_params(amg=g, solve=lib.solve_params(tol=1e-10, max_iter=100)))
    assert code == 0
    d = fe.Discretization(prob)
    Ro, val = d.assemble(v0, 0.5)
    Ro, val = d.apply_dirichlet(Ro, val)
    dv = spl.spsolve(d.csr(val).tocsc(), -Ro)
    got = vt.cpu().numpy() - v0
    assert np.abs(got - dv).max() <= 1e-8 * np.abs(dv).max()
    assert info.amg_levels >= 3


def test_full_size_blocks_colours_and_solve(lib):
    import torch
    N = 24
    prob = synth.cube_problem(N)
    v = np.zeros(prob.n_dofs)
    print(f"[vanka 24^3] {prob.n_dofs} dofs", flush=True)
    g, o = _params(lib, steps=6, max_coarse=500)
    ctx, info, R, d, K, b, blocks, _ = _both(lib, prob, v, 1.0, g, o, oracle_hierarchy=False)
    Kuu, Kup, Kpu, Kpp = blocks
    for which, M in ((10, Kuu), (11, Kup), (12, Kpu), (13, Kpp)):
        _same(_export(ctx, 0, which), M, f"block {which}")
    colours, ncol = ctx.amg_export(0, 14)
    ref = vanka.greedy_colours(vanka.conflict_graph(Kuu, Kup, Kpu, Kpp))
    assert np.array_equal(colours, ref)
    print(f"  levels {info.levels} rows {list(info.rows[:info.levels])} colours(0) {ncol}", flush=True)
    bt = torch_dev(b)
    x = torch.zeros_like(bt)
    si, code = ctx.krylov_amg_solve(bt, x, lib.solve_params(tol=1e-8, max_iter=60, method=2))
    assert code == 0
    assert np.linalg.norm(b - K @ x.cpu().numpy()) <= 1e-8 * np.linalg.norm(b)
    print(f"  AMG iterations {si.iterations} in {si.seconds:.3f} s", flush=True)


@pytest.mark.parametrize("law,N,steps,omega", [("mr", 6, 2, 0.8), ("mr", 8, 6, 0.8), ("artery", 4, 6, 0.86)])
def test_additive_vcycle_matches_oracle(lib, law, N, steps, omega):
    import torch
    prob = _problem(N, law)
    v = synth.random_state(prob, 5, u_scale=0.03, p_scale=0.05).ravel()
    print(f"[vanka additive cycle] {law} N={N} steps={steps} omega={omega}", flush=True)
    g, o = _params(lib, omega=omega, steps=steps, additive=True)
    ctx, info, R, d, K, b, blocks, CH = _both(lib, prob, v, 0.4, g, o)
    assert info.levels == len(CH.levels)
    for lev, L in enumerate(CH.levels):
        for which, M in ((10, L.Kuu), (11, L.Kup), (12, L.Kpu), (13, L.Kpp)):
            _same(_export(ctx, lev, which), M, f"level {lev} block {which}")
    with pytest.raises(RuntimeError):
        ctx.amg_export(0, 14)
    n = prob.n_nodes
    r = np.random.default_rng(6).normal(size=4 * n)
    z = torch.zeros(4 * n, dtype=torch.float64, device="cuda")
    ctx.apply_preconditioner(torch_dev(r), z)
    zo = vanka.preconditioner(CH, n, o)(r)
    zg = z.cpu().numpy()
    assert np.abs(zg - zo).max() <= 1e-10 * np.abs(zo).max()


@pytest.mark.parametrize("law,N,steps,omega", [("mr", 6, 2, 0.8), ("artery", 4, 12, 0.86)])
def test_additive_amg_iteration_and_fgmres_match_oracle(lib, law, N, steps, omega):
    """The additive cycle needs more sweeps than the multiplicative one on
    the artery (with 6 the stationary iteration diverges on this tube)."""
    import torch
    prob = _problem(N, law)
    v = synth.random_state(prob, 7, u_scale=0.03, p_scale=0.05).ravel()
    print(f"[vanka additive solve] {law} N={N} steps={steps}", flush=True)
    g, o = _params(lib, omega=omega, steps=steps, additive=True)
    ctx, info, R, d, K, b, blocks, CH = _both(lib, prob, v, 0.4, g, o)
    n = prob.n_nodes
    bt = torch_dev(b)
    x = torch.zeros_like(bt)
    si, code = ctx.krylov_amg_solve(bt, x, lib.solve_params(tol=1e-8, max_iter=60, method=2))
    xo, hist = vanka.amg_iteration(CH, K, b, n, o, tol=1e-8, maxit=60)
    assert code == 0 and si.converged
    assert si.iterations == len(hist) - 1, (si.iterations, len(hist) - 1)
    xg = x.cpu().numpy()
    assert np.linalg.norm(b - K @ xg) <= 1e-8 * np.linalg.norm(b)
    assert np.abs(xg - xo).max() <= 1e-7 * np.abs(xo).max()
    x.zero_()
    si2, code2 = ctx.krylov_amg_solve(bt, x, lib.solve_params(tol=1e-8, restart=50, max_iter=200))
    xo2, oi = krylov.fgmres(K, vanka.preconditioner(CH, n, o), b, m=50, tol=1e-8)
    assert code2 == 0 and oi.converged
    assert abs(si2.iterations - oi.iterations) <= 1, (si2.iterations, oi.iterations)
    assert np.linalg.norm(b - K @ x.cpu().numpy()) <= 1e-8 * np.linalg.norm(b)


def test_additive_full_size_solve(lib):
    import torch
    N = 24
    prob = synth.cube_problem(N)
    v = np.zeros(prob.n_dofs)
    print(f"[vanka additive 24^3] {prob.n_dofs} dofs", flush=True)
    g, o = _params(lib, omega=0.8, steps=6, max_coarse=500, additive=True)
    ctx, info, R, d, K, b, blocks, _ = _both(lib, prob, v, 1.0, g, o, oracle_hierarchy=False)
    Kuu, Kup, Kpu, Kpp = blocks
    for which, M in ((10, Kuu), (11, Kup), (12, Kpu), (13, Kpp)):
        _same(_export(ctx, 0, which), M, f"block {which}")
    bt = torch_dev(b)
    x = torch.zeros_like(bt)
    si, code = ctx.krylov_amg_solve(bt, x, lib.solve_params(tol=1e-8, restart=100, max_iter=200))
    assert code == 0 and si.converged
    assert np.linalg.norm(b - K @ x.cpu().numpy()) <= 1e-8 * np.linalg.norm(b)
    print(f"  levels {info.levels} FGMRES iterations {si.iterations} in {si.seconds:.3f} s", flush=True)


@pytest.mark.parametrize("additive", [False, True])
def test_fp32_inverse_cycle_matches_oracle(lib, additive):
    """precision = 1: the patch inverses rounded to fp32 on both sides (the
    GPU's LU inverse and the oracle's may round a few entries to
    neighbouring floats, hence 1e-6 rather than rounding level)."""
    import torch
    prob = _problem(6, "mr")
    v = synth.random_state(prob, 5, u_scale=0.03, p_scale=0.05).ravel()
    print(f"[vanka fp32 inverses] additive={additive}", flush=True)
    g, o = _params(lib, omega=0.8, steps=2, additive=additive, f32=True)
    ctx, info, R, d, K, b, blocks, CH = _both(lib, prob, v, 0.4, g, o)
    n = prob.n_nodes
    r = np.random.default_rng(6).normal(size=4 * n)
    z = torch.zeros(4 * n, dtype=torch.float64, device="cuda")
    ctx.apply_preconditioner(torch_dev(r), z)
    zo = vanka.preconditioner(CH, n, o)(r)
    zg = z.cpu().numpy()
    assert np.abs(zg - zo).max() <= 1e-6 * np.abs(zo).max()
    bt = torch_dev(b)
    x = torch.zeros_like(bt)
    si, code = ctx.krylov_amg_solve(bt, x, lib.solve_params(tol=1e-8, restart=50, max_iter=200))
    _, oi = krylov.fgmres(K, vanka.preconditioner(CH, n, o), b, m=50, tol=1e-8)
    print(f"  FGMRES gpu {si.iterations} oracle {oi.iterations}", flush=True)
    assert code == 0 and oi.converged and abs(si.iterations - oi.iterations) <= 1
    assert np.linalg.norm(b - K @ x.cpu().numpy()) <= 1e-8 * np.linalg.norm(b)
