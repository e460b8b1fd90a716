"""Pins of the oracle's PSPG stabilisation term (eq. stelas) and its mass norm.

The PSPG term of the pressure equation is, per element,
    -tau (J F^{-T} grad p, F^{-T} grad q)_T,  tau = h_T^2 / (4 mu^l),
integrated over the reference element.  With dx = J dX and grad_x = F^{-T}
grad_X it is -tau times the P1 stiffness (Laplacian) matrix of the element
in its deformed position.  These tests compute that matrix by a different
route from the oracle's (barycentric coefficients of the deformed vertices
from a 4x4 solve, volume from the deformed vertices), h_T by brute force over
the six edges, mu^l from the printed formulas and the pressure mass by a
quadrature rule exact for quadratics, and compare:

* the pressure-pressure block of the tangent with -(M/kappa + sum tau K_x),
* the change of the pressure residual when p alone changes,
* the scaling laws: X -> sX scales the PSPG block like the mass (s^3 against
  s^3), c10 and c01 -> k c10, k c01 scales it by 1/k.

A dropped J, F^{-1} in place of F^{-T}, a wrong sign, the shortest edge in
place of the longest, mu^l = c10 + c01 or a missing factor 4 each fails the
first comparison; the scaling checks fail for tau without h^2 or without
1/mu^l.
"""
import itertools

import numpy as np
import pytest

import synth
from oracle import fe

# degree-2 rule on a tetrahedron (Hammer-Stroud, four points, weights V/4):
# barycentric (a, b, b, b) and permutations
_QA, _QB = 0.5854101966249685, 0.1381966011250105


def _quad_mass(xe):
    """Exact P1 mass of one tetrahedron (vertex rows xe [4,3]) by quadrature."""
    V = abs(np.linalg.det(np.stack([xe[1] - xe[0], xe[2] - xe[0], xe[3] - xe[0]], axis=1))) / 6.0
    M = np.zeros((4, 4))
    for q in range(4):
        lam = np.full(4, _QB)
        lam[q] = _QA
        M += (V / 4.0) * np.outer(lam, lam)
    return M


def _deformed_stiffness(xe):
    """P1 stiffness matrix of the tetrahedron with vertices xe [4,3]: the hat
    function phi_a = c_a0 + c_a . x solves [1 x_b] c_a = delta_ab."""
    Mx = np.hstack([np.ones((4, 1)), xe])
    coef = np.linalg.inv(Mx)          # column a: coefficients of phi_a
    grads = coef[1:, :].T             # [4,3]
    vol = abs(np.linalg.det(Mx)) / 6.0
    return vol * grads @ grads.T


def _longest_edge(Xe):
    return max(np.linalg.norm(Xe[a] - Xe[b]) for a, b in itertools.combinations(range(4), 2))


def _mu_l_printed(m):
    if m["model"] == 0:
        return 2.0 * (m["c10"] + m["c01"])
    return 2.0 * (m["c10"] + m["k1"] / (2.0 * m["k2"]))


def _expected_pp(prob, v):
    """-(M/kappa + sum_T tau_T K_x,T) assembled over the mesh (n x n)."""
    n = prob.n_nodes
    v = v.reshape(n, 4)
    x = prob.X + v[:, 0:3]
    out = np.zeros((n, n))
    for e, T in enumerate(prob.tets):
        m = prob.materials[prob.mat_id[e]]
        tau = _longest_edge(prob.X[T]) ** 2 / (4.0 * _mu_l_printed(m))
        blk = _quad_mass(prob.X[T]) / m["kappa"] + tau * _deformed_stiffness(x[T])
        out[np.ix_(T, T)] -= blk
    return out


def _problems():
    cube = synth.cube_problem(2, jitter=0.15, seed=5)
    tube = synth.tube_problem(n_theta=8, n_media=1, n_adv=1, n_z=2)
    return {"mooney-rivlin": cube, "artery": tube}


def _state(prob, seed):
    v = synth.random_state(prob, seed, u_scale=0.1, p_scale=0.5)
    # a pressure with large gradients (the random state's p is nodal noise)
    v[:, 3] += np.random.default_rng(seed).normal(size=prob.n_nodes) * 2.0
    return v


@pytest.mark.parametrize("law", ["mooney-rivlin", "artery"])
def test_pressure_block_is_mass_plus_deformed_laplacian(law):
    prob = _problems()[law]
    d = fe.Discretization(prob)
    v = _state(prob, 21)
    _, val = d.assemble(v, 0.3)
    K = d.csr(val).toarray()
    Kpp = K[3::4, 3::4]
    ref = _expected_pp(prob, v)
    assert np.abs(Kpp - ref).max() <= 1e-12 * np.abs(ref).max()
    # the same at the reference state (F = I, J = 1)
    _, val0 = d.assemble(np.zeros_like(v), 0.0)
    K0 = d.csr(val0).toarray()[3::4, 3::4]
    ref0 = _expected_pp(prob, np.zeros_like(v))
    assert np.abs(K0 - ref0).max() <= 1e-12 * np.abs(ref0).max()


@pytest.mark.parametrize("law", ["mooney-rivlin", "artery"])
def test_pressure_residual_changes_by_the_block(law):
    """R^p(u, p) - R^p(u, 0) = -(M/kappa + sum tau K_x) p: the residual's
    PSPG term, not only its derivative."""
    prob = _problems()[law]
    d = fe.Discretization(prob)
    v = _state(prob, 22)
    v0 = v.copy()
    v0[:, 3] = 0.0
    dR = (d.residual(v, 0.4) - d.residual(v0, 0.4)).reshape(prob.n_nodes, 4)[:, 3]
    ref = _expected_pp(prob, v) @ v[:, 3]
    assert np.abs(dR - ref).max() <= 1e-11 * np.abs(ref).max()


def _pspg_part(prob, v):
    d = fe.Discretization(prob)
    _, val = d.assemble(v, 0.0)
    Kpp = d.csr(val).toarray()[3::4, 3::4]
    Mk = np.zeros_like(Kpp)
    for e, T in enumerate(prob.tets):
        Mk[np.ix_(T, T)] += _quad_mass(prob.X[T]) / prob.materials[prob.mat_id[e]]["kappa"]
    return -Kpp - Mk, Mk


def test_pspg_scales_like_the_mass_under_mesh_scaling():
    """X -> s X (state scaled with it, so F is unchanged): the mass and the
    PSPG block both scale by s^3 (tau ~ h^2, volume ~ s^3, gradients ~ 1/s)."""
    prob = synth.cube_problem(2, jitter=0.15, seed=6)
    v = _state(prob, 23)
    P1, M1 = _pspg_part(prob, v)
    s = 2.5
    ps = synth.Problem(prob.X * s, prob.tets, prob.mat_id, prob.materials, prob.dir_mask, prob.tris,
                       prob.traction, prob.lattice)
    vs = v.copy()
    vs[:, 0:3] *= s
    P2, M2 = _pspg_part(ps, vs)
    assert np.abs(M2 - s ** 3 * M1).max() <= 1e-12 * np.abs(M2).max()
    assert np.abs(P2 - s ** 3 * P1).max() <= 1e-12 * np.abs(P2).max()


def test_pspg_scales_inversely_with_the_shear_moduli():
    prob = synth.cube_problem(2, jitter=0.15, seed=7)
    v = _state(prob, 24)
    P1, _ = _pspg_part(prob, v)
    k = 3.0
    mats = [dict(m, c10=m["c10"] * k, c01=m["c01"] * k) for m in prob.materials]
    pk = synth.Problem(prob.X, prob.tets, prob.mat_id, mats, prob.dir_mask, prob.tris, prob.traction,
                       prob.lattice)
    P2, _ = _pspg_part(pk, v)
    assert np.abs(P2 - P1 / k).max() <= 1e-12 * np.abs(P1).max()
    # and it is positive semi-definite with the constants in its kernel
    w = np.linalg.eigvalsh(0.5 * (P1 + P1.T))
    assert w.min() >= -1e-12 * w.max()
    assert np.abs(P1 @ np.ones(P1.shape[0])).max() <= 1e-12 * np.abs(P1).max()


@pytest.mark.parametrize("jitter", [0.0, 0.2])
def test_mass_norm_of_uniform_and_linear_fields(jitter):
    """||c||_M = |c| sqrt(|Omega|) for a uniform field c; a linear field is its
    own P1 interpolant, so ||x e_0||_M^2 = int_cube x^2 = 1/3 and the same for
    the pressure (M = diag(M1, M2), each the consistent P1 mass)."""
    prob = synth.cube_problem(3, jitter=jitter, seed=8)
    d = fe.Discretization(prob)
    c = np.array([0.3, -1.2, 0.7, 2.0])
    v = np.tile(c, (prob.n_nodes, 1))
    assert abs(d.mass_norm(v.ravel()) - np.linalg.norm(c)) <= 1e-13
    for comp, axis in ((0, 0), (3, 1), (2, 2)):
        v = np.zeros((prob.n_nodes, 4))
        v[:, comp] = prob.X[:, axis]
        assert abs(d.mass_norm(v.ravel()) ** 2 - 1.0 / 3.0) <= 1e-13
    # two components add in squares
    v = np.zeros((prob.n_nodes, 4))
    v[:, 1] = prob.X[:, 0]
    v[:, 3] = 1.0
    assert abs(d.mass_norm(v.ravel()) ** 2 - (1.0 / 3.0 + 1.0)) <= 1e-13


@pytest.mark.parametrize("law", ["mooney-rivlin", "artery"])
def test_schur_diagonal_default_theta(law):
    """s_i = sum_T (1/theta_T + 1/kappa_T) diag(M_T)_i with the default
    theta_T = mu^l_T / 5 (mu^l as printed) and the diagonal of the exact P1
    pressure mass (quadrature)."""
    prob = _problems()[law]
    d = fe.Discretization(prob)
    _, val = d.assemble(np.zeros(prob.n_dofs), 0.0)
    _, _, s = d.blocks(val)
    ref = np.zeros(prob.n_nodes)
    for e, T in enumerate(prob.tets):
        m = prob.materials[prob.mat_id[e]]
        theta = _mu_l_printed(m) / 5.0
        ref[T] += (1.0 / theta + 1.0 / m["kappa"]) * np.diag(_quad_mass(prob.X[T]))
    assert np.abs(s - ref).max() <= 1e-13 * np.abs(ref).max()
    # an explicit theta overrides it
    d2 = fe.Discretization(prob, theta=0.7)
    _, _, s2 = d2.blocks(val)
    ref2 = np.zeros(prob.n_nodes)
    for e, T in enumerate(prob.tets):
        ref2[T] += (1.0 / 0.7 + 1.0 / prob.materials[prob.mat_id[e]]["kappa"]) * np.diag(_quad_mass(prob.X[T]))
    assert np.abs(s2 - ref2).max() <= 1e-13 * np.abs(ref2).max()
