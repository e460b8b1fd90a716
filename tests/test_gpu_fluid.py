"""GPU parity of the fluid sub-problem and of the partitioned FSI step
(sections "The fluid sub-problem", "Stabilization for the fluid
sub-problem", "A Dirichlet-Neumann FSI iteration", "Aitken relaxation";
eq. nstdis, eq. stabweakfluid, eq. harext, eq. acceit, eq. dnomega).

The oracle assembles and solves with its own numpy code on the same seeded
duct models; nothing it uses comes from the GPU.  Compared:

* the fluid residual and Jacobian on a moved mesh with random velocity,
  pressure, previous velocity and mesh velocity (Dirichlet rows replaced),
  entry by entry to 1e-12 relative, on two ducts (one with several
  hundred elements per colour); the Schur diagonal against
  diag(C) + diag(B2 diag(A)^-1 B1^T) formed from the oracle's Jacobian;
* the harmonic extension of a random interface displacement to 1e-9;
* a fluid Newton solve on a moved mesh: the same iteration count and the
  state to 1e-8; the interface force to 1e-10;
* two DN time steps of the 2 x 1 x 4 duct, and of the 2 x 3 x 4 duct with
  the two-layer artery wall: the DN iteration counts within two of the
  oracle's and the states to 1e-4 of their size (both stop at
  |r| / sqrt(n) < 1e-8, which the DN map's conditioning amplifies);
* three steps of the small artery tube with its round lumen and the Oseen
  fluid: equal DN counts (within one) and states to 1e-4, with the default
  sub-solvers and with the coupled fluid AMG and kept preconditioners;
* one step of the 3 x 2 x 12 duct checked on the host: the kinematic
  condition on the interface and the interface gap below the tolerance.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from gpu_helpers import torch_dev
from oracle import fluid, fsi

pytestmark = pytest.mark.gpu

PRM = dict(rho_f=1.0, mu=0.0035, dt=0.125, rho_s=1.2)


def _model(a=2, t=1, n_z=4, length=4.0):
    return synth.fsi_duct(a=a, t=t, n_z=n_z, length=length)


def _random_fields(model, seed, scale=0.02):
    rng = np.random.default_rng(seed)
    nf = model.nf
    X = model.fluid_X
    ext = X.max(axis=0) - X.min(axis=0)
    dmesh = (X @ (rng.uniform(-1, 1, (3, 3)) * scale / ext.max()).T) * (~model.fluid_boundary)[:, None]
    v = np.zeros((nf, 4))
    v[:, 0:3] = rng.normal(size=(nf, 3)) * 0.1
    v[:, 3] = rng.normal(size=nf) * 0.5
    uo = rng.normal(size=(nf, 3)) * 0.1
    w = rng.normal(size=(nf, 3)) * 0.05
    return dmesh, v, uo, w


def _blocks_to_csr(out, n):
    bp, bc, bv = out["block_ptr"], out["block_col"], out["block_val"]
    rows = np.repeat(np.arange(n), np.diff(bp))
    r = (4 * rows[:, None, None] + np.arange(4)[None, :, None]).repeat(4, axis=2)
    c = (4 * bc[:, None, None] + np.arange(4)[None, None, :]).repeat(4, axis=1)
    M = sp.csr_matrix((bv.ravel(), (r.ravel(), c.ravel())), shape=(4 * n, 4 * n))
    M.sum_duplicates()
    M.sort_indices()
    return M


@pytest.mark.parametrize("case", ["duct_2x1x4", "duct_3x2x12", "tube_oseen"])
def test_fluid_assembly_matches_oracle(lib, case):
    import torch
    oseen = case == "tube_oseen"
    if oseen:
        model = synth.fsi_tube(8, 3, 2, 1, 6, length=1.5)
    else:
        shape = (2, 1, 4) if case == "duct_2x1x4" else (3, 2, 12)
        model = _model(*shape, length=2.0 * shape[2] / 4)
    print(f"[fluid assembly] {case} nf={model.nf} m={len(model.fluid_tets)}", flush=True)
    dmesh, v, uo, w = _random_fields(model, 3)
    g_in = np.array([0.0, 0.0, 0.7])
    fl, me, so = lib.fsi_contexts(model, p_in=0.7, oseen=int(oseen), **PRM)
    fl.set_fluid_fields(torch_dev(dmesh), torch_dev(uo), torch_dev(w))
    vt = torch_dev(v)
    R = torch.zeros_like(vt)
    view, _ = fl.assemble_residual_tangent(vt, 1.0, R)
    out = fl.export_tangent(view)
    d = fluid.FluidDiscretization(model.fluid_X, model.fluid_tets, model.fluid_dir, model.inlet_tris,
                                  fluid.FluidParams(rho=PRM["rho_f"], mu=PRM["mu"], dt=PRM["dt"], oseen=oseen))
    Ro, val = d.assemble(v.ravel(), dmesh, uo, w, g_in)
    Ro, val = d.apply_dirichlet(Ro, val)
    K = d.csr(val)
    K.sort_indices()
    Kg = _blocks_to_csr(out, model.nf)
    assert np.array_equal(Kg.indptr, K.indptr) and np.array_equal(Kg.indices, K.indices)
    assert np.abs(Kg.data - K.data).max() <= 1e-12 * np.abs(K.data).max()
    assert np.abs(R.cpu().numpy().ravel() - Ro).max() <= 1e-12 * np.abs(Ro).max()
    # Schur diagonal: diag(C) + diag(B2 diag(A)^-1 B1^T)
    Kd = K.toarray()
    up = np.arange(4 * model.nf) % 4 == 3
    A = Kd[np.ix_(~up, ~up)]
    s = -np.diag(Kd[np.ix_(up, up)]) + np.einsum("ij,ji->i", Kd[np.ix_(up, ~up)] / np.diag(A)[None, :],
                                                  Kd[np.ix_(~up, up)])
    assert np.abs(out["schur"] - s).max() <= 1e-12 * np.abs(s).max()


def test_harmonic_extension_matches_oracle(lib):
    import torch
    model = _model()
    fl, me, so = lib.fsi_contexts(model, **PRM)
    rng = np.random.default_rng(4)
    nf = model.nf
    vals = np.zeros((nf, 3))
    vals[model.iface_f] = rng.normal(size=(len(model.iface_f), 3)) * 0.01
    z = model.fluid_X[:, 2]
    vals[(z == 0) | (z == z.max())] = 0.0
    vm = np.zeros((nf, 4))
    vm[:, 0:3] = vals * model.fluid_boundary[:, None]
    vt = torch_dev(vm)
    me.newton_step(vt, 0.0, lib.newton_params(solve=lib.solve_params(tol=1e-13, restart=100, max_iter=500)))
    got = vt.cpu().numpy()[:, 0:3]
    fixed = np.flatnonzero(model.fluid_boundary)
    ref = fluid.harmonic_extension(fluid.laplacian(model.fluid_X, model.fluid_tets), fixed, vm[fixed, 0:3])
    assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max()
    assert not np.any(vt.cpu().numpy()[:, 3])


def test_fluid_newton_and_force_match_oracle(lib):
    import torch
    model = _model()
    dmesh, _, uo, w = _random_fields(model, 5, scale=0.01)
    nf = model.nf
    v0 = np.zeros((nf, 4))
    v0[model.iface_f, 0:3] = w[model.iface_f]
    fl, me, so = lib.fsi_contexts(model, p_in=0.4, **PRM)
    fl.set_fluid_fields(torch_dev(dmesh), torch_dev(uo), torch_dev(w))
    vt = torch_dev(v0)
    prm = lib.fsi_params()
    info, code = fl.newton_solve(vt, 1.0, lib.newton_solve_params(step=prm.fluid_step, eps2=1e-10))
    assert code == 0
    d = fluid.FluidDiscretization(model.fluid_X, model.fluid_tets, model.fluid_dir, model.inlet_tris,
                                  fluid.FluidParams(rho=PRM["rho_f"], mu=PRM["mu"], dt=PRM["dt"]))
    g_in = np.array([0.0, 0.0, 0.4])
    vo, its, _ = fluid.newton_solve(d, v0, dmesh, uo, w, g_in)
    vg = vt.cpu().numpy().ravel()
    assert info.newton_iterations == its
    assert np.abs(vg - vo).max() <= 1e-8 * np.abs(vo).max()
    f = torch.zeros((len(model.iface_f), 3), dtype=torch.float64, device="cuda")
    fl.fluid_interface_force(torch_dev(vo), 1.0, model.iface_f, f)
    fo = fluid.interface_force(d, vo, dmesh, uo, w, g_in, model.iface_f)
    assert np.abs(f.cpu().numpy() - fo).max() <= 1e-10 * np.abs(fo).max()


def test_fluid_newton_gcr_upper_block(lib):
    """The paper's fluid solver, GCR with P_R (eq. rpre, here with the
    SIMPLE diagonal), inside the fluid Newton solve: the oracle's state and
    iteration count."""
    import torch
    model = _model()
    dmesh, _, uo, w = _random_fields(model, 5, scale=0.01)
    nf = model.nf
    v0 = np.zeros((nf, 4))
    v0[model.iface_f, 0:3] = w[model.iface_f]
    fl, me, so = lib.fsi_contexts(model, p_in=0.4, **PRM)
    fl.set_fluid_fields(torch_dev(dmesh), torch_dev(uo), torch_dev(w))
    vt = torch_dev(v0)
    step = lib.newton_params(amg=lib.amg_params(smoother=0, nu_pre=2, nu_post=2),
                             solve=lib.solve_params(tol=1e-10, restart=100, max_iter=1000, method=3, precond_form=1))
    info, code = fl.newton_solve(vt, 1.0, lib.newton_solve_params(step=step, eps2=1e-10))
    assert code == 0
    d = fluid.FluidDiscretization(model.fluid_X, model.fluid_tets, model.fluid_dir, model.inlet_tris,
                                  fluid.FluidParams(rho=PRM["rho_f"], mu=PRM["mu"], dt=PRM["dt"]))
    vo, its, _ = fluid.newton_solve(d, v0, dmesh, uo, w, np.array([0.0, 0.0, 0.4]))
    print(f"[fluid gcr+P_R] Newton {info.newton_iterations} (oracle {its}), Krylov {info.krylov_iterations}",
          flush=True)
    assert info.newton_iterations == its
    assert np.abs(vt.cpu().numpy().ravel() - vo).max() <= 1e-8 * np.abs(vo).max()


def _gpu_fsi(lib, model, p_in, steps, omega0=0.05):
    import torch
    fl, me, so = lib.fsi_contexts(model, p_in=p_in, **PRM)
    nf, ns = model.nf, model.solid.n_nodes
    z = lambda k: torch.zeros(k, dtype=torch.float64, device="cuda")  # noqa: E731
    vf, df, vs, vel, acc = z(4 * nf), z(3 * nf), z(4 * ns), z(3 * ns), z(3 * ns)
    infos = []
    for s in range(steps):
        info, code = lib.fsi_time_step(fl, me, so, model.iface_f, model.iface_s, vf, df, vs, vel, acc, 1.0,
                                       lib.fsi_params(omega0=omega0))
        assert code == 0 and info.converged
        infos.append(info)
    return infos, [x.cpu().numpy() for x in (vf, df, vs)]


def test_fsi_steps_match_oracle(lib):
    model = _model()
    print(f"[fsi] duct 2x1x4: nf={model.nf} ns={model.solid.n_nodes} iface={len(model.iface_f)}", flush=True)
    infos, (vf, df, vs) = _gpu_fsi(lib, model, 0.1, 2)
    st = fsi.FsiState(model, fsi.FsiParams(omega0=0.05, p_in=0.1))
    ks = [st.time_step()[0] for _ in range(2)]
    for info, k in zip(infos, ks):
        print(f"  DN iterations gpu {info.dn_iterations} oracle {k}", flush=True)
        assert abs(info.dn_iterations - k) <= 2
    assert np.abs(vs.reshape(-1, 4)[:, 0:3] - st.vs[:, 0:3]).max() <= 1e-4 * np.abs(st.vs[:, 0:3]).max()
    assert np.abs(vf.reshape(-1, 4)[:, 0:3] - st.vf[:, 0:3]).max() <= 1e-4 * np.abs(st.vf[:, 0:3]).max()
    assert np.abs(df.reshape(-1, 3) - st.df).max() <= 1e-4 * np.abs(st.df).max()


def test_fsi_artery_steps_match_oracle(lib):
    """The same with the paper's two-layer artery as the wall (media on the
    two inner wall rings, adventitia outside, fibres at +/-29 and +/-62
    degrees)."""
    model = synth.fsi_duct(a=2, t=3, n_z=4, length=4.0, artery=True)
    print(f"[fsi artery] duct 2x3x4: nf={model.nf} ns={model.solid.n_nodes}", flush=True)
    infos, (vf, df, vs) = _gpu_fsi(lib, model, 0.3, 2)
    st = fsi.FsiState(model, fsi.FsiParams(omega0=0.05, p_in=0.3))
    ks = [st.time_step()[0] for _ in range(2)]
    for info, k in zip(infos, ks):
        print(f"  DN iterations gpu {info.dn_iterations} oracle {k}", flush=True)
        assert abs(info.dn_iterations - k) <= 2
    assert np.abs(vs.reshape(-1, 4)[:, 0:3] - st.vs[:, 0:3]).max() <= 1e-4 * np.abs(st.vs[:, 0:3]).max()
    assert np.abs(vf.reshape(-1, 4)[:, 0:3] - st.vf[:, 0:3]).max() <= 1e-4 * np.abs(st.vf[:, 0:3]).max()


def _tube_solvers(lib, which):
    if which == "default":
        return lib.fsi_params(omega0=0.05)
    # the coupled (u,p) AMG with the additive Vanka smoother for the fluid,
    # and every sub-problem keeping its whole preconditioner across Newton
    # iterations, DN iterations and steps
    sv = lib.solve_params(tol=1e-10, restart=100, max_iter=1000)
    return lib.fsi_params(
        omega0=0.05, adaptive=1,
        fluid_step=lib.newton_params(amg=lib.amg_params(coupled=2, vanka_steps=1, interp_kind=0), solve=sv,
                                     amg_reuse=3),
        solid_step=lib.newton_params(amg=lib.amg_params(smoother=1, precision=1), solve=sv, amg_reuse=3),
        mesh_step=lib.newton_params(solve=lib.solve_params(tol=1e-12, restart=100, max_iter=1000), amg_reuse=3))


@pytest.mark.parametrize("solvers", ["default", "coupled_kept"])
def test_fsi_tube_oseen_steps_match_oracle(lib, solvers):
    """The partitioned FSI sequence's workload in small: the two-layer artery
    tube and its round lumen, the Oseen fluid with a Poiseuille inflow
    (peak 0.3 mm/ms), dt = 1 ms; three steps against the oracle (equal DN
    counts, states to 1e-4 of their size), with the default sub-solvers and
    with the coupled fluid AMG and kept preconditioners (there each step
    starts from the previous step's last Aitken factor, on both sides)."""
    import torch
    model = synth.fsi_tube(8, 2, 2, 1, 4, length=1.0)
    print(f"[fsi tube {solvers}] nf={model.nf} ns={model.solid.n_nodes} iface={len(model.iface_f)}", flush=True)
    prm = dict(rho_f=1.0, mu=0.0035, dt=1.0, rho_s=1.2)
    fl, me, so = lib.fsi_contexts(model, p_in=0.0, oseen=1, **prm)
    nf, ns = model.nf, model.solid.n_nodes
    z = lambda k: torch.zeros(k, dtype=torch.float64, device="cuda")  # noqa: E731
    vf0 = np.zeros((nf, 4))
    vf0[:, 0:3] = model.inflow
    vf, df, vs, vel, acc = torch_dev(vf0.ravel()), z(3 * nf), z(4 * ns), z(3 * ns), z(3 * ns)
    st = fsi.FsiState(model, fsi.FsiParams(fluid=fluid.FluidParams(rho=1.0, mu=0.0035, dt=1.0, oseen=True),
                                           rho_s=1.2, p_in=0.0, omega0=0.05))
    prm = _tube_solvers(lib, solvers)
    for step in range(3):
        info, code = lib.fsi_time_step(fl, me, so, model.iface_f, model.iface_s, vf, df, vs, vel, acc, 1.0, prm)
        k, omegas, _ = st.time_step()
        print(f"  step {step + 1}: DN iterations gpu {info.dn_iterations} oracle {k}", flush=True)
        assert code == 0 and info.converged and abs(info.dn_iterations - k) <= 1
        if solvers == "coupled_kept" and k >= 2 and info.dn_iterations >= 2:
            # both sides start the next step from their last Aitken factor
            print(f"  last Aitken factor gpu {info.omega[info.dn_iterations - 2]:.6f} oracle {omegas[-1]:.6f}",
                  flush=True)
            assert abs(info.omega[info.dn_iterations - 2] - omegas[-1]) <= 2e-2 * abs(omegas[-1])
            prm.omega0 = min(max(info.omega[info.dn_iterations - 2], 0.01), 1.0)
            st.prm.omega0 = min(max(omegas[-1], 0.01), 1.0)
    vs_, vf_ = vs.cpu().numpy().reshape(-1, 4), vf.cpu().numpy().reshape(-1, 4)
    assert np.abs(vs_[:, 0:3] - st.vs[:, 0:3]).max() <= 1e-4 * np.abs(st.vs[:, 0:3]).max()
    assert np.abs(vf_ - st.vf).max() <= 1e-4 * np.abs(st.vf).max()
    assert np.array_equal(vf_[model.inflow[:, 2] > 0, 0:3], model.inflow[model.inflow[:, 2] > 0])


def test_fsi_step_larger_duct_host_checks(lib):
    model = _model(3, 2, 12, length=6.0)
    print(f"[fsi] duct 3x2x12: nf={model.nf} ns={model.solid.n_nodes}", flush=True)
    infos, (vf, df, vs) = _gpu_fsi(lib, model, 0.2, 1)
    info = infos[0]
    print(f"  DN {info.dn_iterations} its, fluid Newton {info.fluid_newton}, structure Newton {info.solid_newton}, "
          f"{info.seconds:.2f} s", flush=True)
    vf, df, vs = vf.reshape(-1, 4), df.reshape(-1, 3), vs.reshape(-1, 4)
    w = df / PRM["dt"]            # from rest: d_f^{n-1} = 0
    assert np.abs(vf[model.iface_f, 0:3] - w[model.iface_f]).max() <= 1e-14 * np.abs(w).max()
    gap = df[model.iface_f] - vs[model.iface_s, 0:3]
    assert np.linalg.norm(gap) / np.sqrt(len(model.iface_f)) < 1e-8
    assert info.residual[info.dn_iterations - 1] < 1e-8


def test_stalled_coarsening_solves_by_l1_jacobi(lib):
    """The fluid operator of the 3 x 2 x 36 duct is mass-dominated: no
    coupling is strong, the coarsening stops on level 0 (5,439 rows, above
    the dense limit), and the V-cycle is then 16 l1-Jacobi sweeps from zero,
    checked against the same sweeps in numpy on the exported operator."""
    import torch
    model = _model(3, 2, 36, length=18.0)
    fl, me, so = lib.fsi_contexts(model, **PRM)
    nf = model.nf
    vt = torch.zeros(4 * nf, dtype=torch.float64, device="cuda")
    R = torch.zeros_like(vt)
    fl.assemble_residual_tangent(vt, 1.0, R)
    info = fl.amg_setup(lib.amg_params(smoother=0, nu_pre=2, nu_post=2))
    print(f"[stalled coarsening] levels {info.levels} rows {info.rows[0]}", flush=True)
    assert info.levels == 1 and info.rows[0] == 3 * nf > 4096
    ptr, col, val, ncols = fl.amg_export(0, 0)
    A = sp.csr_matrix((val, col, ptr), shape=(len(ptr) - 1, ncols))
    r = np.random.default_rng(7).normal(size=A.shape[0])
    z = torch.zeros(A.shape[0], dtype=torch.float64, device="cuda")
    fl.vcycle(torch_dev(r), z)
    dinv = 1.0 / np.asarray(abs(A).sum(axis=1)).ravel()
    x = dinv * r
    for _ in range(15):
        x = x + dinv * (r - A @ x)
    assert np.abs(z.cpu().numpy() - x).max() <= 1e-12 * np.abs(x).max()
