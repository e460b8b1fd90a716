"""GPU parity of the V-cycle, the block preconditioner, FGMRES and Newton.

* V-cycle and P_L^{-1}: the oracle applies the same operators (the GPU's
  hierarchy exported level by level) to the same vector; fp64 results agree
  to 1e-12 relative, the fp32 cycle to fp32 accuracy;
* FGMRES in fp64 solved to 1e-12 agrees with a sparse direct solve to 1e-9;
  at 1e-8 the true fp64 residual is below 1e-8 for both the fp64 and the
  mixed-precision (fp32 V-cycle) preconditioner;
* the 8^3 cube load run (5 increments, Newton to 1e-10) reproduces the
  oracle's converged states to 1e-9 relative.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spl

import synth
from gpu_helpers import amg_prm_pair, context_for, gpu_hierarchy_to_oracle, oracle_system, torch_dev
from oracle import amg, krylov, newton

pytestmark = pytest.mark.gpu


def _setup(lib, prob, v, load, smoother=0, precision=0, max_coarse=500, nu=(2, 2), cheb=(2, 30.0), schedule=None):
    import torch
    ctx = context_for(lib, prob)
    vt = torch_dev(v)
    R = torch.zeros_like(vt)
    ctx.assemble_residual_tangent(vt, load, R)
    gprm, oprm = amg_prm_pair(lib, smoother=smoother, precision=precision, max_coarse=max_coarse, nu=nu[0],
                              nu_post=nu[1], cheb=cheb, schedule=schedule)
    info = ctx.amg_setup(gprm)
    return ctx, R, info, oprm


@pytest.mark.parametrize("smoother,precision,nu,cheb", [(0, 0, (2, 2), (2, 30.0)), (1, 0, (2, 2), (2, 30.0)),
                                                        (0, 1, (2, 2), (2, 30.0)), (1, 1, (2, 2), (2, 30.0)),
                                                        (1, 0, (1, 2), (2, 30.0)), (1, 1, (1, 2), (2, 30.0)),
                                                        (0, 0, (1, 2), (2, 30.0)), (1, 0, (1, 1), (3, 10.0)),
                                                        (1, 1, (1, 2), (4, 20.0)),
                                                        (1, 0, None, None), (1, 1, None, None)])
def test_vcycle_and_preconditioner_match_oracle(lib, smoother, precision, nu, cheb):
    """nu = cheb = None: the default schedule (on level 0 one degree-1 sweep
    before the correction and one degree-3 sweep after it; on the coarser
    levels no pre-smoothing and one degree-3 sweep after)."""
    import torch
    prob = synth.cube_problem(6, jitter=0.1, seed=2)
    v = synth.random_state(prob, 3, u_scale=0.03, p_scale=0.05).ravel()
    print(f"[vcycle parity] smoother={smoother} precision={precision} nu={nu} cheb={cheb}", flush=True)
    if nu is None:
        ctx, R, info, oprm = _setup(lib, prob, v, 0.4, smoother, precision, max_coarse=60, schedule="default")
    else:
        ctx, R, info, oprm = _setup(lib, prob, v, 0.4, smoother, precision, max_coarse=60, nu=nu, cheb=cheb)
    H = gpu_hierarchy_to_oracle(ctx, info, oprm)
    rng = np.random.default_rng(1)
    n3 = H.levels[0].A.shape[0]
    r = rng.normal(size=n3)
    z = torch.zeros(n3, dtype=torch.float64, device="cuda")
    ctx.vcycle(torch_dev(r), z)
    zo = amg.vcycle(H, r, oprm)
    tol = 1e-12 if precision == 0 else 2e-5
    assert np.linalg.norm(z.cpu().numpy() - zo) <= tol * np.linalg.norm(zo)
    # block preconditioner
    d, K, b, A, B2, s = oracle_system(prob, v, 0.4)
    M = krylov.BlockPreconditioner(lambda x: amg.vcycle(H, x, oprm), B2, s, prob.n_nodes)
    rr = rng.normal(size=4 * prob.n_nodes)
    rr[prob.dir_mask.ravel().astype(bool)] = 0.0
    y = torch.zeros(4 * prob.n_nodes, dtype=torch.float64, device="cuda")
    ctx.apply_preconditioner(torch_dev(rr), y)
    yo = M(rr)
    assert np.linalg.norm(y.cpu().numpy() - yo) <= tol * np.linalg.norm(yo)
    # tangent product
    ky = torch.zeros_like(y)
    ctx.apply_tangent(torch_dev(rr), ky)
    ko = K @ rr
    assert np.linalg.norm(ky.cpu().numpy() - ko) <= 1e-13 * np.linalg.norm(ko)


def _lanes_per_row(A):
    """Lanes per row the library's padded-CSR smoother picks for a coarse
    level (3 to 6 four-entry chunks per lane, more lanes on small levels):
    the test asserts which kernel variants a case exercises."""
    chunks = int(np.sum((np.diff(A.indptr) + 3) // 4))
    rows = A.shape[0]
    avg = chunks / rows if rows else 1.0
    G = 2
    while G < 64 and 6.0 * G <= avg:
        G *= 2
    while G < 64 and rows * G < 65536:
        G *= 2
    return G


@pytest.mark.timeout(900)
@pytest.mark.parametrize("N,precision", [(24, 0), (24, 1), (48, 0), (48, 1)])
def test_vcycle_and_preconditioner_entrywise_on_large_levels(lib, N, precision):
    """The default cycle and hierarchy at 24^3 and 48^3, where level 1 has
    more than 8192 rows and its smoother runs with few lanes per row, as on
    the benchmark sizes (the lanes of every level are printed): V-cycle, P_L
    and K x against the oracle applying the same operators, entry by entry
    (|z_i - zo_i| <= tol max|zo|)."""
    import torch
    prob = synth.cube_problem(N, jitter=0.1, seed=2)
    v = synth.random_state(prob, 3, u_scale=0.01, p_scale=0.05).ravel()
    print(f"[vcycle entrywise] N={N} precision={precision}", flush=True)
    ctx, R, info, oprm = _setup(lib, prob, v, 0.4, 1, precision, schedule="default")
    H = gpu_hierarchy_to_oracle(ctx, info, oprm)
    lanes = [_lanes_per_row(L.A) for L in H.levels[1:-1]]
    print(f"[vcycle entrywise] rows={[L.A.shape[0] for L in H.levels]} lanes={lanes}", flush=True)
    assert H.levels[1].A.shape[0] >= 8192 and lanes[0] <= 8
    rng = np.random.default_rng(1)
    n3 = H.levels[0].A.shape[0]
    r = rng.normal(size=n3)
    z = torch.zeros(n3, dtype=torch.float64, device="cuda")
    ctx.vcycle(torch_dev(r), z)
    zo = amg.vcycle(H, r, oprm)
    tol = 1e-12 if precision == 0 else 2e-5
    dz = np.abs(z.cpu().numpy() - zo)
    print(f"[vcycle entrywise] max |z - zo| / max |zo| = {dz.max() / np.abs(zo).max():.2e}", flush=True)
    assert dz.max() <= tol * np.abs(zo).max()
    d, K, b, A, B2, s = oracle_system(prob, v, 0.4)
    M = krylov.BlockPreconditioner(lambda x: amg.vcycle(H, x, oprm), B2, s, prob.n_nodes)
    rr = rng.normal(size=4 * prob.n_nodes)
    rr[prob.dir_mask.ravel().astype(bool)] = 0.0
    y = torch.zeros(4 * prob.n_nodes, dtype=torch.float64, device="cuda")
    ctx.apply_preconditioner(torch_dev(rr), y)
    yo = M(rr)
    dy = np.abs(y.cpu().numpy() - yo)
    print(f"[vcycle entrywise] P_L: max |y - yo| / max |yo| = {dy.max() / np.abs(yo).max():.2e}", flush=True)
    assert dy.max() <= tol * np.abs(yo).max()
    ky = torch.zeros_like(y)
    ctx.apply_tangent(torch_dev(rr), ky)
    ko = K @ rr
    assert np.abs(ky.cpu().numpy() - ko).max() <= 1e-13 * np.abs(ko).max()


@pytest.mark.parametrize("precision", [0, 1])
def test_fgmres_solution(lib, precision):
    import torch
    prob = synth.cube_problem(8)
    v = synth.random_state(prob, 8, u_scale=0.02, p_scale=0.02).ravel()
    print(f"[fgmres parity] precision={precision}", flush=True)
    ctx, R, info, oprm = _setup(lib, prob, v, 0.6, precision=precision)
    d, K, b, A, B2, s = oracle_system(prob, v, 0.6)
    assert np.allclose(-R.cpu().numpy(), b, rtol=0, atol=1e-12 * np.abs(b).max())
    x_ref = spl.spsolve(K.tocsc(), b)
    bt = -R
    x = torch.zeros_like(bt)
    sinfo, code = ctx.krylov_amg_solve(bt, x, lib.solve_params(tol=1e-12, max_iter=2000))
    assert code == 0 and sinfo.converged
    err = np.linalg.norm(x.cpu().numpy() - x_ref) / np.linalg.norm(x_ref)
    assert err <= 1e-9
    x.zero_()
    sinfo, code = ctx.krylov_amg_solve(bt, x, lib.solve_params(tol=1e-8))
    true_res = np.linalg.norm(b - K @ x.cpu().numpy()) / np.linalg.norm(b)
    assert sinfo.converged and true_res <= 1e-8
    assert abs(sinfo.rel_residual - true_res) <= 1e-10
    # the oracle's FGMRES with the GPU's hierarchy needs about as many iterations
    H = gpu_hierarchy_to_oracle(ctx, info, oprm)
    M = krylov.BlockPreconditioner(lambda r: amg.vcycle(H, r, oprm), B2, s, prob.n_nodes)
    _, oinfo = krylov.fgmres(K, M, b, tol=1e-8)
    print(f"[fgmres] gpu its={sinfo.iterations} oracle its={oinfo.iterations} err={err:.2e}", flush=True)
    assert abs(sinfo.iterations - oinfo.iterations) <= (1 if precision == 0 else 3)


@pytest.mark.parametrize("precision", [0, 1])
def test_bicgstab_solution(lib, precision):
    """BiCGStab (method 1) with the same P_L: the direct solution to 1e-9 at
    a 1e-12 tolerance, the true residual at 1e-8, and about as many
    iterations as the oracle's BiCGStab with the GPU's hierarchy: within one
    with the fp64 cycle, within three with the fp32 cycle (its rounding,
    relative 1e-7 per application, is not in the oracle)."""
    import torch
    prob = synth.cube_problem(8)
    v = synth.random_state(prob, 8, u_scale=0.02, p_scale=0.02).ravel()
    print(f"[bicgstab parity] precision={precision}", flush=True)
    ctx, R, info, oprm = _setup(lib, prob, v, 0.6, smoother=1, precision=precision, schedule="default")
    d, K, b, A, B2, s = oracle_system(prob, v, 0.6)
    x_ref = spl.spsolve(K.tocsc(), b)
    bt = -R
    x = torch.zeros_like(bt)
    sinfo, code = ctx.krylov_amg_solve(bt, x, lib.solve_params(tol=1e-12, max_iter=2000, method=1))
    assert code == 0 and sinfo.converged
    err = np.linalg.norm(x.cpu().numpy() - x_ref) / np.linalg.norm(x_ref)
    assert err <= 1e-9
    x.zero_()
    sinfo, code = ctx.krylov_amg_solve(bt, x, lib.solve_params(tol=1e-8, method=1))
    true_res = np.linalg.norm(b - K @ x.cpu().numpy()) / np.linalg.norm(b)
    assert sinfo.converged and true_res <= 1e-8
    assert abs(sinfo.rel_residual - true_res) <= 1e-10
    H = gpu_hierarchy_to_oracle(ctx, info, oprm)
    M = krylov.BlockPreconditioner(lambda r: amg.vcycle(H, r, oprm), B2, s, prob.n_nodes)
    _, oinfo = krylov.bicgstab(K, M, b, tol=1e-8)
    print(f"[bicgstab] gpu its={sinfo.iterations} oracle its={oinfo.iterations} err={err:.2e}", flush=True)
    assert oinfo.converged
    assert abs(sinfo.iterations - oinfo.iterations) <= (1 if precision == 0 else 3)
    with pytest.raises(lib.HfsiError):
        ctx.krylov_amg_solve(bt, x, lib.solve_params(method=4))


def test_tangent_product_any_alignment(lib):
    """K x with x 32-byte aligned (wide loads) and with x at an 8-byte offset
    (the per-entry kernel) both equal the oracle tangent times x."""
    import torch
    prob = synth.cube_problem(5, jitter=0.1, seed=3)
    v = synth.random_state(prob, 5, u_scale=0.03, p_scale=0.05).ravel()
    ctx, R, info, oprm = _setup(lib, prob, v, 0.4, 1, 0, max_coarse=60)
    d, K, b, A, B2, s = oracle_system(prob, v, 0.4)
    n4 = 4 * prob.n_nodes
    xr = np.random.default_rng(6).normal(size=n4)
    ref = K @ xr
    buf = torch.zeros(n4 + 1, dtype=torch.float64, device="cuda")
    for off in (0, 1):
        x = buf[off:off + n4]
        x.copy_(torch_dev(xr))
        assert (x.data_ptr() % 32 == 0) == (off == 0)
        y = torch.zeros(n4, dtype=torch.float64, device="cuda")
        ctx.apply_tangent(x, y)
        assert np.linalg.norm(y.cpu().numpy() - ref) <= 1e-13 * np.linalg.norm(ref), off


@pytest.mark.parametrize("precision", [0, 1])
def test_vcycle_after_nonfinite_cycle(lib, precision):
    """A cycle run after one on a non-finite vector equals the cycle before
    it: no step reads a work vector it has not written in the same cycle
    (levels without pre-smoothing start their post-smoothing with no
    previous Chebyshev direction)."""
    import torch
    prob = synth.cube_problem(6, jitter=0.1, seed=2)
    v = synth.random_state(prob, 3, u_scale=0.03, p_scale=0.05).ravel()
    ctx, R, info, oprm = _setup(lib, prob, v, 0.4, 1, precision, max_coarse=60, schedule="default")
    assert info.levels >= 3
    n3 = 3 * prob.n_nodes
    r = torch_dev(np.random.default_rng(4).normal(size=n3))
    z1 = torch.zeros(n3, dtype=torch.float64, device="cuda")
    ctx.vcycle(r, z1)
    bad = torch.full_like(r, float("nan"))
    zb = torch.zeros_like(z1)
    ctx.vcycle(bad, zb)
    assert not bool(torch.isfinite(zb).any())
    z2 = torch.zeros_like(z1)
    ctx.vcycle(r, z2)
    assert torch.equal(z1, z2)


def test_zero_rhs_and_not_converged(lib):
    import torch
    prob = synth.cube_problem(3)
    ctx, R, info, oprm = _setup(lib, prob, np.zeros(4 * prob.n_nodes), 1.0, max_coarse=20)
    x = torch.ones(4 * prob.n_nodes, dtype=torch.float64, device="cuda")
    sinfo, code = ctx.krylov_amg_solve(torch.zeros_like(x), x, lib.solve_params())
    assert code == 0 and float(x.abs().max()) == 0.0
    x.zero_()
    sinfo, code = ctx.krylov_amg_solve(-R, x, lib.solve_params(max_iter=1))
    assert code == 1 and sinfo.iterations == 1 and not sinfo.converged


def test_newton_load_run_matches_oracle(lib):
    import torch
    prob = synth.cube_problem(8)
    print("[newton parity] cube8 5 increments", flush=True)
    ctx = context_for(lib, prob)
    v = torch.zeros(4 * prob.n_nodes, dtype=torch.float64, device="cuda")
    prm = lib.newton_params()
    its = []
    for k in range(1, 6):
        n0 = None
        for it in range(25):
            info, code = ctx.newton_step(v, k / 5.0, prm)
            assert code == 0
            n0 = info.dv_mass_norm if n0 is None else n0
            if info.dv_mass_norm <= 1e-10 * n0:
                break
        its.append(it + 1)
    d = synth  # noqa: F841
    from oracle import fe
    disc = fe.Discretization(prob)
    vo = newton.load_run(disc, 5, newton.NewtonParams())
    vg = v.cpu().numpy()
    assert np.linalg.norm(vg - vo) <= 1e-9 * np.linalg.norm(vo)
    assert all(3 <= k <= 6 for k in its), its


def test_time_kernel_levels_and_errors(lib):
    """Per-level timing ids: levels >= 1 run on the padded CSR copy (rows
    padded to 4 entries, fp32 values and 16-bit column offsets unless a row
    spans more than 65535 columns), so an fp32 Chebyshev step moves
    (4 + 2) B per padded entry plus 8 B (chunk pointer, column base) and
    24 B of vectors per row, the residual 8 B of vectors per row; rotating
    operator copies leaves the byte count unchanged; unknown levels and
    negative sizes are errors."""
    prob = synth.cube_problem(6)
    print("[time_kernel] cube6", flush=True)
    ctx, R, info, oprm = _setup(lib, prob, np.zeros(prob.n_dofs), 1.0, smoother=1, precision=1, max_coarse=60)
    assert info.levels >= 3
    H = gpu_hierarchy_to_oracle(ctx, info, oprm)
    for lev in range(1, info.levels):
        A = H.levels[lev].A.tocsr()
        lens = np.diff(A.indptr)
        padded = int(np.sum(4 * ((lens + 3) // 4)))
        spans = [A.indices[a:b].max() - A.indices[a:b].min() for a, b in zip(A.indptr[:-1], A.indptr[1:]) if b > a]
        cb = 4 if max(spans) > 65535 else 2
        ms, b = ctx.time_kernel(100 + lev, 3)
        assert ms > 0.0 and b == padded * (4 + cb) + info.rows[lev] * (8 + 24)
        ms, b2 = ctx.time_kernel(200 + lev, 3, 1 << 20)
        assert ms > 0.0 and b2 == padded * (4 + cb) + info.rows[lev] * (8 + 8)
    assert ctx.time_kernel(0, 2)[1] == ctx.time_kernel(100, 2, 1 << 22)[1]
    with pytest.raises(Exception):
        ctx.time_kernel(100 + info.levels, 1)
    with pytest.raises(Exception):
        ctx.time_kernel(2, 1, -1)


def test_fp32_cycle_is_fp32(lib):
    """The mixed-precision hierarchy really cycles in fp32: on the same
    operator and vector its V-cycle differs from the fp64 cycle by fp32
    rounding (well above fp64 rounding, well below the cycle's own size)."""
    import torch
    prob = synth.cube_problem(6)
    print("[precision] cube6 fp32 vs fp64 V-cycle", flush=True)
    ctx, R, info, oprm = _setup(lib, prob, np.zeros(prob.n_dofs), 1.0, smoother=1, precision=1, max_coarse=60)
    r = torch_dev(np.random.default_rng(8).normal(size=3 * prob.n_nodes))
    z32 = torch.zeros_like(r)
    ctx.vcycle(r, z32)
    gprm, _ = amg_prm_pair(lib, smoother=1, precision=0, max_coarse=60)
    ctx.amg_setup(gprm)
    z64 = torch.zeros_like(r)
    ctx.vcycle(r, z64)
    rel = float(torch.linalg.norm(z32 - z64) / torch.linalg.norm(z64))
    print(f"[precision] relative difference {rel:.2e}", flush=True)
    assert 1e-9 < rel < 1e-4


@pytest.mark.parametrize("precision", [0, 1])
def test_vcycle_with_rows_spanning_more_than_16_bits(lib, precision):
    """A caller matrix (hfsi_amg_setup_csr) whose rows partly span more than
    65535 columns: the padded smoother keeps int32 columns for those rows
    and 16-bit offsets for the others; the V-cycle matches the oracle on the
    exported hierarchy entry by entry."""
    import torch
    import scipy.sparse as sp
    import test_oracle_amg as T
    A = T.laplacian(48, 48, 48).tolil()
    n = A.shape[0]
    rng = np.random.default_rng(11)
    for i in rng.choice(n - 70000, 400, replace=False):
        j = int(i) + 70000
        A[i, j] = A[j, i] = -0.05
        A[i, i] += 0.05
        A[j, j] += 0.05
    A = A.tocsr()
    A.sort_indices()
    comp = np.zeros(n, np.int32)
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    span = np.maximum.reduceat(A.indices, A.indptr[:-1]) - np.minimum.reduceat(A.indices, A.indptr[:-1])
    assert (span > 65535).sum() >= 400
    gprm, oprm = amg_prm_pair(lib, smoother=1, precision=precision, max_coarse=200, schedule="default")
    ctx = lib.Context(0)
    print(f"[vcycle wide rows] n={n} precision={precision}", flush=True)
    info = ctx.amg_setup_csr(A.indptr, A.indices, A.data, comp, gprm)
    H = gpu_hierarchy_to_oracle(ctx, info, oprm)
    r = rng.normal(size=n)
    z = torch.zeros(n, dtype=torch.float64, device="cuda")
    ctx.vcycle(torch_dev(r), z)
    zo = amg.vcycle(H, r, oprm)
    tol = 1e-12 if precision == 0 else 2e-5
    dz = np.abs(z.cpu().numpy() - zo)
    print(f"[vcycle wide rows] max |z - zo| / max |zo| = {dz.max() / np.abs(zo).max():.2e}", flush=True)
    assert dz.max() <= tol * np.abs(zo).max()



@pytest.mark.parametrize("form", [0, 1])
def test_gcr_and_upper_block_preconditioner(lib, form):
    """GCR (method 3, the paper's Krylov method for the fluid) with P_L or
    P_R (eq. rpre): the direct solution to 1e-9 at a 1e-12 tolerance, the
    true residual at 1e-8, and within one iteration of the oracle's GCR with
    the GPU's hierarchy and the same block form; FGMRES with P_R within one
    of the oracle's FGMRES."""
    import torch
    prob = synth.cube_problem(8)
    v = synth.random_state(prob, 8, u_scale=0.02, p_scale=0.02).ravel()
    print(f"[gcr parity] form={form}", flush=True)
    ctx, R, info, oprm = _setup(lib, prob, v, 0.6, smoother=1, precision=0, schedule="default")
    d, K, b, A, B2, s = oracle_system(prob, v, 0.6)
    x_ref = spl.spsolve(K.tocsc(), b)
    bt = -R
    x = torch.zeros_like(bt)
    sinfo, code = ctx.krylov_amg_solve(bt, x, lib.solve_params(tol=1e-12, restart=100, max_iter=2000, method=3,
                                                               precond_form=form))
    assert code == 0 and sinfo.converged
    assert np.linalg.norm(x.cpu().numpy() - x_ref) <= 1e-9 * np.linalg.norm(x_ref)
    H = gpu_hierarchy_to_oracle(ctx, info, oprm)
    a_inv = lambda r: amg.vcycle(H, r, oprm)  # noqa: E731
    if form == 0:
        M = krylov.BlockPreconditioner(a_inv, B2, s, prob.n_nodes)
    else:
        n = prob.n_nodes
        Kc = K.tocsr()
        u = np.array([4 * i + c for i in range(n) for c in range(3)])
        B1T = Kc[u][:, 4 * np.arange(n) + 3]
        M = krylov.UpperBlockPreconditioner(a_inv, B1T, s, n)
    for method, oracle_solver in ((3, krylov.gcr), (0, krylov.fgmres)):
        x.zero_()
        sinfo, code = ctx.krylov_amg_solve(bt, x, lib.solve_params(tol=1e-8, restart=100, method=method,
                                                                   precond_form=form))
        true_res = np.linalg.norm(b - K @ x.cpu().numpy()) / np.linalg.norm(b)
        assert code == 0 and sinfo.converged and true_res <= 1e-8
        _, oinfo = oracle_solver(K, M, b, m=100, tol=1e-8)
        print(f"[gcr parity] method {method} form {form}: gpu its={sinfo.iterations} oracle its={oinfo.iterations}",
              flush=True)
        assert oinfo.converged and abs(sinfo.iterations - oinfo.iterations) <= 1
