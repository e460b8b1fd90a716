"""Pins of the oracle's material laws against the energies they derive from.

The stresses and tangents in oracle.fe are hand-derived from the energy
functionals (eq. mmreng, eq. areng, S = 2 dPsi/dC); these tests check them
against the energies themselves by finite differences, against the
stress-free reference state and against frame invariance.
"""
import numpy as np
import pytest

from oracle import fe

MR = dict(model=0, c10=0.5, c01=0.1, kappa=1e4, k1=0.0, k2=0.0)
ART = dict(model=1, c10=3.0, c01=0.0, kappa=1e5, k1=2.3632, k2=0.8393)


def _mat(d, m):
    return {k: np.full(m, float(v)) for k, v in d.items()}


def _random_C(rng, m, amp=0.3):
    F = np.eye(3)[None] + amp * rng.uniform(-1, 1, size=(m, 3, 3))
    return np.einsum("mki,mkj->mij", F, F)


def _fibres(m, alpha=np.radians(29.0)):
    a1 = np.array([0.0, np.cos(alpha), np.sin(alpha)])
    a2 = np.array([0.0, np.cos(alpha), -np.sin(alpha)])
    return np.tile(np.stack([a1, a2])[None], (m, 1, 1))


@pytest.mark.parametrize("law", ["mr", "artery"])
def test_reference_state_is_stress_free(law):
    m = 3
    mat = _mat(MR if law == "mr" else ART, m)
    C = np.tile(np.eye(3), (m, 1, 1))
    S, _ = fe.stress_tangent(C, mat, _fibres(m))
    assert np.abs(S).max() <= 1e-15


def _fd_stress(C, mat, fib, h=1e-6):
    """S_IJ = 2 dPsi/dC_IJ, central differences on symmetric perturbations."""
    m = C.shape[0]
    S = np.zeros((m, 3, 3))
    for I in range(3):
        for J in range(3):
            E = np.zeros((3, 3))
            E[I, J] += 0.5
            E[J, I] += 0.5
            pp = fe.deviatoric_energy(C + h * E, mat, fib)
            pm = fe.deviatoric_energy(C - h * E, mat, fib)
            S[:, I, J] = 2.0 * (pp - pm) / (2.0 * h)
    return S


@pytest.mark.parametrize("law", ["mr", "artery"])
def test_stress_is_energy_derivative(law):
    rng = np.random.default_rng(4)
    m = 64
    mat = _mat(MR if law == "mr" else ART, m)
    fib = _fibres(m)
    C = _random_C(rng, m)
    if law == "artery":
        # keep the fibre invariants away from the switch J_i = 1
        A1, A2 = fe.fibre_tensors(fib)
        I3 = np.linalg.det(C)
        for A in (A1, A2):
            Ji = I3 ** (-1 / 3) * np.einsum("mij,mij->m", A, C)
            keep = np.abs(Ji - 1) > 1e-3
            C, fib, I3 = C[keep], fib[keep], I3[keep]
            mat = {k: v[: len(C)] for k, v in mat.items()}
        Jact = [np.linalg.det(C) ** (-1 / 3) * np.einsum("mij,mij->m", A[: len(C)], C) for A in (A1, A2)]
        assert np.any(Jact[0] > 1) and np.any(Jact[0] < 1)
    S, _ = fe.stress_tangent(C, mat, fib)
    Sfd = _fd_stress(C, mat, fib)
    assert np.abs(S - Sfd).max() <= 1e-7 * max(1.0, np.abs(S).max())


@pytest.mark.parametrize("law", ["mr", "artery"])
def test_tangent_is_stress_derivative(law):
    rng = np.random.default_rng(5)
    m = 32
    mat = _mat(MR if law == "mr" else ART, m)
    fib = _fibres(m, np.radians(10.0))
    C = _random_C(rng, m, 0.4)
    S, T = fe.stress_tangent(C, mat, fib)
    h = 1e-6
    for K in range(3):
        for L in range(3):
            E = np.zeros((3, 3))
            E[K, L] += 0.5
            E[L, K] += 0.5
            Sp, _ = fe.stress_tangent(C + h * E, mat, fib)
            Sm, _ = fe.stress_tangent(C - h * E, mat, fib)
            fd = 2.0 * (Sp - Sm) / (2.0 * h)
            ok = np.abs(T[:, :, :, K, L] - fd).max()
            assert ok <= 1e-6 * max(1.0, np.abs(T).max()), (K, L, ok)


def test_mooney_rivlin_uniaxial_incompressible_closed_form():
    """Isochoric uniaxial stretch F = diag(s, s^-1/2, s^-1/2): the textbook
    Cauchy stress difference sigma_11 - sigma_22 of the Mooney-Rivlin
    energy c10/2 (J1-3) + c01/2 (J2-3) is (s^2 - 1/s)(c10 + c01/s)."""
    mat = _mat(MR, 1)
    for s in (0.8, 1.1, 1.5, 2.0):
        F = np.diag([s, s ** -0.5, s ** -0.5])
        C = (F.T @ F)[None]
        S, _ = fe.stress_tangent(C, mat)
        sigma = F @ S[0] @ F.T  # J = 1
        diff = sigma[0, 0] - sigma[1, 1]
        ref = (s * s - 1.0 / s) * (MR["c10"] + MR["c01"] / s)
        assert abs(diff - ref) <= 1e-13 * max(1.0, abs(ref))


@pytest.mark.parametrize("law", ["mr", "artery"])
def test_objectivity(law):
    """Psi(C) is frame invariant, so under F -> QF the first Piola stress
    rotates (P -> QP) and the spatial tangent rotates with Q."""
    rng = np.random.default_rng(9)
    m = 16
    mat = _mat(MR if law == "mr" else ART, m)
    fib = _fibres(m, np.radians(40.0))
    F = np.eye(3)[None] + 0.3 * rng.uniform(-1, 1, size=(m, 3, 3))
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    C1 = np.einsum("mki,mkj->mij", F, F)
    QF = np.einsum("ij,mjk->mik", q, F)
    C2 = np.einsum("mki,mkj->mij", QF, QF)
    S1, T1 = fe.stress_tangent(C1, mat, fib)
    S2, T2 = fe.stress_tangent(C2, mat, fib)
    assert np.abs(S1 - S2).max() <= 1e-12 * np.abs(S1).max()
    assert np.abs(T1 - T2).max() <= 1e-12 * np.abs(T1).max()
    P1 = np.einsum("mij,mjk->mik", F, S1)
    P2 = np.einsum("mij,mjk->mik", QF, S2)
    assert np.abs(np.einsum("ij,mjk->mik", q, P1) - P2).max() <= 1e-12 * np.abs(P1).max()


def test_fibre_switch():
    """Fibres carry no stress in compression (J_i <= 1) and do in extension."""
    mat = _mat(ART, 1)
    fib = _fibres(1, 0.0)  # both fibres along y
    Cc = np.diag([1.0, 0.9, 1.0])[None]
    Ce = np.diag([1.0, 1.2, 1.0])[None]
    iso = dict(ART, k1=0.0)
    Sc, _ = fe.stress_tangent(Cc, mat, fib)
    Sc0, _ = fe.stress_tangent(Cc, _mat(iso, 1), fib)
    Se, _ = fe.stress_tangent(Ce, mat, fib)
    Se0, _ = fe.stress_tangent(Ce, _mat(iso, 1), fib)
    assert np.abs(Sc - Sc0).max() == 0.0
    assert np.abs(Se - Se0).max() > 1e-3
