"""Pins of the fluid oracle (section "The fluid sub-problem", eq. nstdis,
eq. weakns, eq. stabweakfluid) and of the harmonic extension (eq. harext).

* Jacobian: central differences of the residual with tau held fixed, with
  and without the stabilisation, and in the Oseen form (a dropped
  derivative of the convective velocity in the SUPG test function, or a
  transposed velocity gradient, fails); the Oseen step is linear: one
  Newton correction leaves a zero residual, and with u_old = u it is the
  Navier-Stokes residual;
* the Galerkin mass and convection terms against the closed form of the P1
  mass matrix, sum_b M_ab (rho/dt (u_b - u_old_b) + rho Gu c_b), and the
  SUPG and PSPG terms against the same closed form with the nodal strong
  residuals (a wrong quadrature point or weight fails);
* the viscous rows 2 mu (eps(u), eps(N_a e_i)) are the gradient of
  mu V eps:eps, half the element's dissipation rate (a missing factor 2 or
  an unsymmetrised gradient fails);
* exact discrete solutions: uniform flow, plane shear flow and a pressure
  gradient balanced by the time derivative give zero residual at every
  interior node (a sign error between the mass and pressure terms fails);
* the pressure block is -C with C symmetric positive semi-definite and
  constants in its kernel, and without stabilisation B2 = B1;
* tau: the closed form, and dt/2 at rest on a large element;
* the interface force of a fluid at rest under a constant pressure is
  p0 times the area-weighted normals of the wall faces (Green's formula);
* the harmonic extension reproduces an affine field exactly (P1 exactness).
"""
import numpy as np
import pytest

import synth
from oracle import fluid


def _batch(rng, m=6, scale=0.3):
    ref = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]])
    x = ref[None] + rng.uniform(-0.15, 0.15, size=(m, 4, 3))
    ue = rng.normal(size=(m, 4, 3)) * scale
    pe = rng.normal(size=(m, 4))
    uo = rng.normal(size=(m, 4, 3)) * scale
    we = rng.normal(size=(m, 4, 3)) * scale
    return x, ue, pe, uo, we


@pytest.mark.parametrize("stabilise,oseen", [(True, False), (False, False), (True, True)])
def test_jacobian_matches_differences(stabilise, oseen):
    rng = np.random.default_rng(1)
    prm = fluid.FluidParams(rho=1.3, mu=0.07, dt=0.2, stabilise=stabilise, oseen=oseen)
    x, ue, pe, uo, we = _batch(rng)
    G, V, h = fluid.geometry(x)
    tau = fluid.tau_of(((uo if oseen else ue) - we).mean(axis=1), h, prm)
    _, K = fluid.element_kernel(x, ue, pe, uo, we, prm, tau=tau)
    v = np.concatenate([ue, pe[:, :, None]], axis=2).reshape(len(x), 16)
    eps = 1e-6
    Kfd = np.zeros_like(K)
    for j in range(16):
        vp, vm = v.copy(), v.copy()
        vp[:, j] += eps
        vm[:, j] -= eps
        Rp, _ = fluid.element_kernel(x, vp.reshape(-1, 4, 4)[:, :, 0:3], vp.reshape(-1, 4, 4)[:, :, 3], uo, we, prm,
                                     want_tangent=False, tau=tau)
        Rm, _ = fluid.element_kernel(x, vm.reshape(-1, 4, 4)[:, :, 0:3], vm.reshape(-1, 4, 4)[:, :, 3], uo, we, prm,
                                     want_tangent=False, tau=tau)
        Kfd[:, :, j] = (Rp - Rm).reshape(len(x), 16) / (2 * eps)
    assert np.abs(K - Kfd).max() <= 1e-7 * np.abs(K).max()


def _mass(V):
    return V[:, None, None] * (1.0 + np.eye(4))[None] / 20.0


def test_galerkin_mass_and_convection_closed_form():
    rng = np.random.default_rng(2)
    prm = fluid.FluidParams(rho=1.7, mu=0.0, dt=0.3, stabilise=False)
    x, ue, pe, uo, we = _batch(rng)
    pe[:] = 0.0
    R, _ = fluid.element_kernel(x, ue, pe, uo, we, prm, want_tangent=False)
    G, V, h = fluid.geometry(x)
    Gu = np.einsum("mbi,mbj->mij", ue, G)
    c = ue - we
    nodal = prm.rho * ((ue - uo) / prm.dt + np.einsum("mij,mbj->mbi", Gu, c))
    ref = np.einsum("mab,mbi->mai", _mass(V), nodal)
    assert np.abs(R[:, :, 0:3] - ref).max() <= 1e-13 * np.abs(ref).max()
    # continuity: -V/4 div u at every node
    assert np.allclose(R[:, :, 3], -(V / 4.0 * np.einsum("mii->m", Gu))[:, None], rtol=1e-13, atol=0)


def test_supg_pspg_closed_form():
    rng = np.random.default_rng(3)
    prm = fluid.FluidParams(rho=1.2, mu=0.05, dt=0.25, stabilise=True)
    x, ue, pe, uo, we = _batch(rng)
    G, V, h = fluid.geometry(x)
    tau = fluid.tau_of((ue - we).mean(axis=1), h, prm)
    Rs, _ = fluid.element_kernel(x, ue, pe, uo, we, prm, want_tangent=False, tau=tau)
    R0, _ = fluid.element_kernel(x, ue, pe, uo, we, prm, want_tangent=False, tau=np.zeros(len(x)))
    Gu = np.einsum("mbi,mbj->mij", ue, G)
    gp = np.einsum("mb,mbj->mj", pe, G)
    c = ue - we
    r = (ue - uo) / prm.dt + np.einsum("mij,mbj->mbi", Gu, c) + gp[:, None, :] / prm.rho   # nodal, linear in x
    cG = np.einsum("mbj,maj->mba", c, G)                  # c_b . G_a
    M = _mass(V)
    supg = prm.rho * tau[:, None, None] * np.einsum("mba,mbd,mdi->mai", cG, M, r)
    pspg = -tau[:, None] * np.einsum("maj,mdj->ma", G, r) * (V / 4.0)[:, None]
    assert np.abs((Rs - R0)[:, :, 0:3] - supg).max() <= 1e-12 * np.abs(supg).max()
    assert np.abs((Rs - R0)[:, :, 3] - pspg).max() <= 1e-12 * np.abs(pspg).max()


def test_viscous_rows_are_the_dissipation_gradient():
    rng = np.random.default_rng(4)
    prm = fluid.FluidParams(rho=1.0, mu=0.3, dt=0.1)
    x, ue, pe, uo, we = _batch(rng)
    pe[:] = 0.0
    # u_old = u and w = u: no time derivative, no convection, zero strong residual
    R, _ = fluid.element_kernel(x, ue, pe, ue, ue, prm, want_tangent=False)
    G, V, h = fluid.geometry(x)

    def dissipation(u):
        Gu = np.einsum("mbi,mbj->mij", u, G)
        e = 0.5 * (Gu + Gu.transpose(0, 2, 1))
        return prm.mu * V * np.einsum("mij,mij->m", e, e)

    g = np.zeros_like(ue)
    eps = 1e-6
    for a in range(4):
        for i in range(3):
            up, um = ue.copy(), ue.copy()
            up[:, a, i] += eps
            um[:, a, i] -= eps
            g[:, a, i] = (dissipation(up) - dissipation(um)) / (2 * eps)
    assert np.abs(R[:, :, 0:3] - g).max() <= 1e-8 * np.abs(g).max()


@pytest.fixture(scope="module")
def duct():
    model = synth.fsi_duct(a=2, t=1, n_z=4, half_width=1.0, wall=0.3, length=2.0)
    prm = fluid.FluidParams(rho=1.0, mu=0.05, dt=0.125)
    d = fluid.FluidDiscretization(model.fluid_X, model.fluid_tets, model.fluid_dir, model.inlet_tris, prm)
    return model, d


def _interior(model):
    return ~model.fluid_boundary


@pytest.mark.parametrize("case", ["uniform", "shear", "pressure"])
def test_exact_discrete_solutions(duct, case):
    model, d = duct
    X = model.fluid_X
    n = d.n
    v = np.zeros((n, 4))
    uo = np.zeros((n, 3))
    w = np.zeros((n, 3))
    if case == "uniform":
        v[:, 0:3] = [0.3, -0.2, 0.5]
        v[:, 3] = 1.7
        uo[:] = v[:, 0:3]
    elif case == "shear":
        v[:, 0] = 0.4 * X[:, 1]
        v[:, 3] = -0.3
        uo[:] = v[:, 0:3]
        w[:, 2] = 0.1               # a mesh moving along the flow's invariant direction
    else:
        g = np.array([0.2, -0.1, 0.35])
        v[:, 3] = X @ g
        uo[:] = d.prm.dt * g / d.prm.rho
    R, _ = d.assemble(v.ravel(), np.zeros((n, 3)), uo, w, np.zeros(3), want_tangent=False)
    R = R.reshape(n, 4)[_interior(model)]
    scale = max(np.abs(v).max(), 1.0) * d.prm.rho / d.prm.dt * 0.1
    assert np.abs(R).max() <= 1e-12 * scale


def test_pressure_block_and_saddle_symmetry(duct):
    model, d = duct
    rng = np.random.default_rng(5)
    n = d.n
    v = rng.normal(size=(n, 4)) * 0.1
    uo = rng.normal(size=(n, 3)) * 0.1
    w = rng.normal(size=(n, 3)) * 0.1
    _, val = d.assemble(v.ravel(), np.zeros((n, 3)), uo, w, np.zeros(3))
    K = d.csr(val).toarray()
    up = np.arange(4 * n) % 4 == 3
    Kpp = K[np.ix_(up, up)]
    assert np.abs(Kpp - Kpp.T).max() <= 1e-14 * np.abs(Kpp).max()
    assert np.linalg.eigvalsh(Kpp).max() <= 1e-12 * np.abs(Kpp).max()
    assert np.abs(Kpp @ np.ones(n)).max() <= 1e-12 * np.abs(Kpp).max()
    d0 = fluid.FluidDiscretization(model.fluid_X, model.fluid_tets, model.fluid_dir, model.inlet_tris,
                                   fluid.FluidParams(stabilise=False))
    _, val0 = d0.assemble(v.ravel(), np.zeros((n, 3)), uo, w, np.zeros(3))
    K0 = d0.csr(val0).toarray()
    B1T = K0[np.ix_(~up, up)]
    B2 = K0[np.ix_(up, ~up)]
    assert np.abs(B2 - B1T.T).max() <= 1e-15 * np.abs(B2).max()
    assert not np.any(K0[np.ix_(up, up)])


def test_tau():
    prm = fluid.FluidParams(rho=2.0, mu=0.4, dt=0.1)
    c = np.array([[0.3, -0.4, 1.2]])
    h = np.array([0.7])
    nu = 0.2
    ref = 1.0 / np.sqrt((2 / 0.1) ** 2 + (2 * 1.3 / 0.7) ** 2 + (4 * nu / 0.49) ** 2)
    assert abs(fluid.tau_of(c, h, prm)[0] - ref) <= 1e-15 * ref
    assert abs(fluid.tau_of(np.zeros((1, 3)), np.array([1e8]), prm)[0] - 0.05) <= 1e-15


def test_interface_force_of_a_fluid_at_rest(duct):
    model, d = duct
    n = d.n
    p0 = 2.5
    v = np.zeros((n, 4))
    v[:, 3] = p0
    zero = np.zeros((n, 3))
    # wall nodes off the inlet and outlet rims: only wall faces touch them
    z = model.fluid_X[:, 2]
    nodes = model.iface_f[(z[model.iface_f] > 0) & (z[model.iface_f] < z.max())]
    f = fluid.interface_force(d, v.ravel(), zero, zero, zero, np.zeros(3), nodes)
    faces = synth.boundary_faces(model.fluid_tets)
    ref = np.zeros((n, 3))
    cen = model.fluid_X.mean(axis=0)
    for tri in faces:
        x = model.fluid_X[tri]
        an = 0.5 * np.cross(x[1] - x[0], x[2] - x[0])
        if np.dot(an, x.mean(axis=0) - cen) < 0 and abs(an[2]) < 1e-14:
            an = -an                      # outward from the fluid
        for a in tri:
            ref[a] += p0 * an / 3.0
    assert np.abs(f - ref[nodes]).max() <= 1e-12 * np.abs(ref[nodes]).max()
    assert np.abs(f).max() > 0


def test_harmonic_extension_is_exact_for_affine_fields(duct):
    model, d = duct
    L = fluid.laplacian(model.fluid_X, model.fluid_tets)
    rng = np.random.default_rng(6)
    A, b = rng.normal(size=(3, 3)), rng.normal(size=3)
    exact = model.fluid_X @ A.T + b
    fixed = np.flatnonzero(model.fluid_boundary)
    got = fluid.harmonic_extension(L, fixed, exact[fixed])
    assert np.abs(got - exact).max() <= 1e-12 * np.abs(exact).max()
    assert np.abs(L @ np.ones(d.n)).max() <= 1e-13 * abs(L).max()


def test_oseen_is_linear_and_agrees_with_navier_stokes_at_u_old(duct):
    model, d = duct
    rng = np.random.default_rng(12)
    n = d.n
    po = fluid.FluidParams(rho=1.0, mu=0.05, dt=0.125, oseen=True)
    do = fluid.FluidDiscretization(model.fluid_X, model.fluid_tets, model.fluid_dir, model.inlet_tris, po)
    v = rng.normal(size=(n, 4)) * 0.1
    uo = rng.normal(size=(n, 3)) * 0.1
    w = rng.normal(size=(n, 3)) * 0.05
    dm = np.zeros((n, 3))
    g = np.array([0.0, 0.0, 0.3])
    R, val = do.assemble(v.ravel(), dm, uo, w, g)
    R, val = do.apply_dirichlet(R, val)
    import scipy.sparse.linalg as spl
    dv = spl.spsolve(do.csr(val).tocsc(), -R)
    R1, _ = do.assemble(v.ravel() + dv, dm, uo, w, g, want_tangent=False)
    R1 = R1.reshape(n, 4)
    R1[model.fluid_dir.astype(bool)] = 0.0
    assert np.abs(R1).max() <= 1e-11 * np.abs(R).max()
    # at u_old = u the Oseen residual is the Navier-Stokes one
    vu = v.copy()
    Ro, _ = do.assemble(vu.ravel(), dm, vu[:, 0:3], w, g, want_tangent=False)
    Rn, _ = d.assemble(vu.ravel(), dm, vu[:, 0:3], w, g, want_tangent=False)
    assert np.abs(Ro - Rn).max() <= 1e-14 * np.abs(Rn).max()
