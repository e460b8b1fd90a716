"""Pins of the oracle's element residual, tangent and assembly.

* the tangent is the derivative of the residual (central differences);
* the Galerkin part of the residual is the gradient of the discrete
  Lagrangian  L = sum_T V_T [Psi'(C_T) - pbar_T (J_T - 1)]
                  - sum_T p^T M_T p / (2 kappa) - f.u
  (the stabilisation term has no potential and is excluded);
* structure stated in eq. globsys: A = A^T, C = C^T, and translations
  are in the kernel of the displacement rows;
* a homogeneous (affine) state with p = -kappa (J-1) is an exact discrete
  solution on interior nodes (patch test).
"""
import numpy as np
import pytest

import synth
from oracle import fe


def _problem(law, jitter=0.15, seed=3):
    if law == "mr":
        return synth.cube_problem(2, jitter=jitter, seed=seed)
    p = synth.tube_problem(n_theta=8, n_media=1, n_adv=1, n_z=2)
    return p


def _fd_jacobian(d, v, load, h=1e-6):
    x = v.ravel().copy()
    J = np.zeros((x.size, x.size))
    for j in range(x.size):
        xp = x.copy(); xp[j] += h
        xm = x.copy(); xm[j] -= h
        J[:, j] = (d.residual(xp, load) - d.residual(xm, load)) / (2 * h)
    return J


@pytest.mark.parametrize("law", ["mr", "artery"])
def test_tangent_matches_finite_differences(law):
    p = _problem(law)
    d = fe.Discretization(p)
    v = synth.random_state(p, 11, u_scale=0.1, p_scale=0.3)
    R, val = d.assemble(v, 0.5)
    K = d.csr(val).toarray()
    Kfd = _fd_jacobian(d, v, 0.5)
    assert np.abs(K - Kfd).max() <= 1e-6 * np.abs(K).max()
    assert np.allclose(R, d.residual(v, 0.5), rtol=0, atol=1e-15 * np.abs(R).max())


def _lagrangian(d, v, load):
    v = v.reshape(d.n, 4)
    T = d.prob.tets
    u = v[:, 0:3]
    p = v[:, 3]
    F = np.eye(3)[None] + np.einsum("mai,maj->mij", u[T], d.G)
    C = np.einsum("mki,mkj->mij", F, F)
    J = np.linalg.det(F)
    psi = fe.deviatoric_energy(C, d.mat, d.fib)
    pe = p[T]
    Mab = (1.0 + np.eye(4)) / 20.0
    pMp = np.einsum("m,ab,ma,mb->m", d.V, Mab, pe, pe)
    return (np.sum(d.V * (psi - pe.mean(1) * (J - 1.0))) - np.sum(pMp / (2 * d.mat["kappa"]))
            - load * np.sum(d.f_ext * u))


@pytest.mark.parametrize("law", ["mr", "artery"])
def test_residual_is_lagrangian_gradient(law):
    p = _problem(law)
    d = fe.Discretization(p)
    v = synth.random_state(p, 12, u_scale=0.1, p_scale=0.3).ravel()
    # the Galerkin residual: drop the stabilisation by taking tau -> 0
    d.h = np.zeros_like(d.h)
    R = d.residual(v, 0.7)
    h = 1e-6
    g = np.zeros_like(v)
    for j in range(v.size):
        vp = v.copy(); vp[j] += h
        vm = v.copy(); vm[j] -= h
        g[j] = (_lagrangian(d, vp, 0.7) - _lagrangian(d, vm, 0.7)) / (2 * h)
    assert np.abs(R - g).max() <= 1e-7 * max(1.0, np.abs(R).max())


@pytest.mark.parametrize("law", ["mr", "artery"])
def test_block_structure(law):
    p = _problem(law)
    d = fe.Discretization(p)
    v = synth.random_state(p, 13, u_scale=0.1, p_scale=0.3)
    _, val = d.assemble(v, 0.3)
    K = d.csr(val).toarray()
    n = d.n
    u = np.array([4 * i + c for i in range(n) for c in range(3)])
    pp = np.arange(n) * 4 + 3
    A = K[np.ix_(u, u)]
    C = -K[np.ix_(pp, pp)]
    assert np.abs(A - A.T).max() <= 1e-12 * np.abs(A).max()
    assert np.abs(C - C.T).max() <= 1e-12 * np.abs(C).max()
    for c in range(3):
        t = np.zeros(4 * n)
        t[4 * np.arange(n) + c] = 1.0
        assert np.abs(K @ t).max() <= 1e-12 * np.abs(K).max()


@pytest.mark.parametrize("law", ["mr", "artery"])
def test_homogeneous_patch(law):
    p = synth.cube_problem(3, jitter=0.2, seed=7)
    if law == "artery":
        p.materials = [synth.meshes.artery_layer(3.0, 2.3632, 0.8393, 1e5)]
        p.fibres = np.tile(np.array([[0.0, 0.87, 0.49], [0.0, 0.87, -0.49]])[None], (p.n_tets, 1, 1))
    d = fe.Discretization(p)
    F0 = np.array([[1.05, 0.02, -0.01], [0.03, 0.97, 0.04], [-0.02, 0.01, 1.08]])
    J0 = np.linalg.det(F0)
    kappa = p.materials[0]["kappa"]
    v = np.zeros((p.n_nodes, 4))
    v[:, 0:3] = p.X @ (F0 - np.eye(3)).T
    v[:, 3] = -kappa * (J0 - 1.0)
    R = d.residual(v, 0.0).reshape(-1, 4)
    interior = np.all((p.lattice > 0) & (p.lattice < 3), axis=1)
    scale = np.abs(R).max()
    assert np.abs(R[interior]).max() <= 1e-12 * scale
    assert np.abs(R[:, 3]).max() <= 1e-12 * max(1.0, kappa * abs(J0 - 1.0))
    assert np.abs(R[~interior, 0:3]).max() > 1e-6 * scale  # boundary traction is not zero


def test_zero_state_zero_residual():
    for p in (synth.cube_problem(2), synth.tube_problem(n_theta=8, n_media=1, n_adv=1, n_z=2)):
        d = fe.Discretization(p)
        R = d.residual(np.zeros(4 * p.n_nodes), 0.0)
        assert np.abs(R).max() <= 1e-15


def test_sizes_of_the_cube_workload():
    p = synth.cube_problem(8)
    d = fe.Discretization(p)
    assert (p.n_nodes, p.n_tets, len(d.K_indices)) == (729, 3072, 145552)
    assert len(p.tris) == 128 and p.dir_mask[:, 0:3].sum() == 3 * 81
    # total load equals traction times loaded area (unit face)
    assert np.allclose(d.f_ext.sum(axis=0), [0.0, 0.0, 0.05], atol=1e-15)


@pytest.mark.parametrize("make", [lambda: synth.cube_problem(4, jitter=0.1, seed=5),
                                  lambda: synth.tube_problem(n_theta=12, n_media=1, n_adv=1, n_z=4)])
def test_sampled_rows_equal_full_assembly(make):
    """The sub-mesh row helper used by the full-size GPU tests reproduces the
    rows of the full assembly (residual and Dirichlet-eliminated tangent)."""
    from gpu_helpers import oracle_sampled_rows
    prob = make()
    v = synth.random_state(prob, 4, u_scale=0.04, p_scale=0.1)
    d = fe.Discretization(prob)
    R, val = d.assemble(v.ravel(), 0.7)
    R, val = d.apply_dirichlet(R, val)
    K = d.csr(val)
    nodes = np.random.default_rng(1).choice(prob.n_nodes, 12, replace=False)
    rows = oracle_sampled_rows(prob, v, 0.7, nodes)
    for g, (Rg, Kg) in rows.items():
        assert np.allclose(Rg, R[4 * g:4 * g + 4], rtol=1e-12, atol=1e-14 * np.abs(R).max())
        for r in range(4):
            i = 4 * g + r
            ref = dict(zip(K.indices[K.indptr[i]:K.indptr[i + 1]].tolist(), K.data[K.indptr[i]:K.indptr[i + 1]]))
            got = {c: vals[r] for c, vals in Kg.items() if c in ref or vals[r] != 0.0}
            assert set(got) == set(ref)
            for c in ref:
                assert abs(got[c] - ref[c]) <= 1e-12 * np.abs(K.data).max()


# ---------------------------------------------------------------- inertia


def _with_inertia(d, seed, cm=37.0):
    r = np.random.default_rng(seed)
    d.set_inertia(cm, r.normal(scale=2.0, size=(d.n, 3)))
    return d


@pytest.mark.parametrize("law", ["mr", "artery"])
def test_inertia_tangent_matches_finite_differences(law):
    """With the Newmark-beta inertia terms (mass and history in R^u, the
    history in the stabilisation of R^p) the tangent is still the derivative
    of the residual."""
    p = _problem(law)
    d = _with_inertia(fe.Discretization(p), 5)
    v = synth.random_state(p, 12, u_scale=0.1, p_scale=0.3)
    R, val = d.assemble(v, 0.5)
    K = d.csr(val).toarray()
    Kfd = _fd_jacobian(d, v, 0.5)
    assert np.abs(K - Kfd).max() <= 1e-6 * np.abs(K).max()
    d0 = fe.Discretization(p)
    R0, val0 = d0.assemble(v, 0.5)
    assert np.abs(K - d0.csr(val0).toarray()).max() > 1e-3 * np.abs(K).max()


def test_inertia_of_a_rigid_translation():
    """A uniform displacement t with p = 0 and a uniform history r0 leaves
    only inertia: the displacement rows sum to |Omega| (cm t - r0) (the
    consistent mass integrates to the volume) and the pressure rows of every
    element sum to zero (sum_a G_a = 0)."""
    p = _problem("mr")
    d = fe.Discretization(p)
    t, r0, cm = np.array([0.3, -0.2, 0.5]), np.array([1.5, 0.7, -2.0]), 11.0
    d.set_inertia(cm, np.tile(r0, (d.n, 1)))
    v = np.zeros((d.n, 4))
    v[:, 0:3] = t
    R = d.residual(v.ravel(), 0.0).reshape(d.n, 4)
    vol = d.V.sum()
    assert np.allclose(R[:, 0:3].sum(axis=0), vol * (cm * t - r0), rtol=1e-12, atol=1e-12)
    assert abs(R[:, 3].sum()) <= 1e-12 * np.abs(R[:, 3]).max()
    assert np.abs(R[:, 3]).max() > 1e-6


def test_inertia_history_matching_the_state_cancels():
    """r_s = cm d at the current (non-uniform) d: the inertia forces cancel
    node by node and the residual is the quasi-static one."""
    p = _problem("artery")
    d = fe.Discretization(p)
    v = synth.random_state(p, 13, u_scale=0.1, p_scale=0.3)
    R0 = d.residual(v.ravel(), 0.4)
    d.set_inertia(25.0, 25.0 * v.reshape(d.n, 4)[:, 0:3])
    R1 = d.residual(v.ravel(), 0.4)
    assert np.abs(R1 - R0).max() <= 1e-12 * np.abs(R0).max()


@pytest.mark.parametrize("law", ["mr", "artery"])
def test_pressure_geometric_part_is_the_derivative_of_the_pressure_force(law):
    """A - A_plus is the derivative with respect to u of the pressure part
    of the displacement residual, -V pbar J F^{-T} G_a, at fixed p: central
    differences of that force alone (written from F with numpy here)."""
    p = _problem(law)
    d = fe.Discretization(p)
    v = synth.random_state(p, 13, u_scale=0.1, p_scale=0.5)
    _, val = d.assemble(v, 0.5)
    _, valp = d.assemble(v, 0.5, pressure_geometric=False)
    D = (d.csr(val) - d.csr(valp)).toarray()
    Duu = D.reshape(p.n_nodes, 4, p.n_nodes, 4)[:, 0:3, :, 0:3].reshape(3 * p.n_nodes, 3 * p.n_nodes)
    # nothing else changes
    mask = np.ones((p.n_nodes, 4, p.n_nodes, 4), bool)
    mask[:, 0:3, :, 0:3] = False
    assert np.abs(D.reshape(p.n_nodes, 4, p.n_nodes, 4)[mask]).max() == 0.0

    def pforce(u):
        T = p.tets
        F = np.eye(3)[None] + np.einsum("mai,maj->mij", u[T], d.G)
        J = np.linalg.det(F)
        g = np.einsum("mji,maj->mai", np.linalg.inv(F), d.G)
        pbar = v[:, 3][T].mean(axis=1)
        f = np.zeros((p.n_nodes, 3))
        fe_ = -(d.V * pbar * J)[:, None, None] * g
        for a in range(4):
            np.add.at(f, T[:, a], fe_[:, a])
        return f.ravel()

    u0 = v[:, 0:3].copy()
    h = 1e-6
    Dfd = np.zeros_like(Duu)
    for j in range(3 * p.n_nodes):
        up = u0.copy().ravel(); up[j] += h
        um = u0.copy().ravel(); um[j] -= h
        Dfd[:, j] = (pforce(up.reshape(-1, 3)) - pforce(um.reshape(-1, 3))) / (2 * h)
    assert np.abs(Duu - Dfd).max() <= 1e-7 * max(1.0, np.abs(Duu).max())
    assert np.abs(Duu).max() > 0
