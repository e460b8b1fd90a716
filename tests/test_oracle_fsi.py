"""Pins of the Dirichlet-Neumann iteration with Aitken relaxation (sections
"A Dirichlet-Neumann FSI iteration" and "Aitken relaxation", eq. acceit,
eq. dnomega, eq. fixepr) and of the coupled time step built on it.

* on an affine scalar map d -> m d + c Aitken's secant step is exact: the
  second factor is 1 / (1 - m) and the third evaluation sits on the fixed
  point (a sign error in eq. dnomega, or the factor applied to the wrong
  residual, fails);
* on an affine map with two eigenvalues the relaxed iteration reaches the
  fixed point (I - M)^-1 c;
* the coupled problem at rest with no inlet traction stays at rest after
  one DN iteration;
* a short pulse on the 2 x 1 x 4 duct: the iteration stops below eps; the
  fluid velocity on the interface is the mesh velocity (d_f - d_f^prev)/dt;
  the mesh displacement is harmonic at the interior fluid nodes and equals
  the structure's interface displacement to within the stopping tolerance;
  and two different first relaxation factors give the same step (the
  relaxation changes the path, not the fixed point).
"""
import numpy as np
import pytest

import synth
from oracle import fluid, fsi


def test_aitken_is_exact_on_an_affine_scalar_map():
    m, c = -3.0, np.array([0.5, -1.0, 2.0])
    evals = []

    def G(d):
        evals.append(d.copy())
        return m * d + c

    k, omegas, norms = fsi.dn_iterate(G, np.zeros(3), 1, 0.3, 1e-12, 10)
    assert k == 3
    assert abs(omegas[1] - 1.0 / (1.0 - m)) <= 1e-14
    assert np.abs(evals[-1] - c / (1.0 - m)).max() <= 1e-14


def test_aitken_reaches_the_fixed_point_of_an_affine_map():
    M = np.diag([-2.0, -2.0, -0.5, 0.3])
    c = np.array([1.0, -2.0, 0.5, 3.0])
    last = {}

    def G(d):
        last["d"] = d.copy()
        return M @ d + c

    k, omegas, norms = fsi.dn_iterate(G, np.zeros(4), 4, 0.2, 1e-13, 50)
    assert np.abs(last["d"] - np.linalg.solve(np.eye(4) - M, c)).max() <= 1e-12
    assert norms[-1] < 1e-13


def test_aitken_factor_closed_form():
    r1 = np.array([1.0, -2.0, 0.5])
    lam = 0.4
    assert abs(fsi.aitken(0.7, r1, lam * r1) - 0.7 / (1.0 - lam)) <= 1e-15


def _state(p_in, omega0=0.05):
    model = synth.fsi_duct(a=2, t=1, n_z=4, length=4.0)
    return fsi.FsiState(model, fsi.FsiParams(omega0=omega0, p_in=p_in, eps=1e-8))


def test_rest_stays_at_rest():
    st = _state(0.0)
    k, omegas, norms = st.time_step()
    assert k == 1 and norms[0] == 0.0
    assert not np.any(st.vs) and not np.any(st.vf) and not np.any(st.df)


@pytest.fixture(scope="module")
def pulse():
    st = _state(0.1)
    df_prev = st.df.copy()
    k, omegas, norms = st.time_step()
    return st, df_prev, k, norms


def test_pulse_step_conditions(pulse):
    st, df_prev, k, norms = pulse
    m = st.model
    assert k > 2 and norms[-1] < 1e-8
    # kinematic condition: fluid velocity = mesh velocity on the interface
    w = (st.df - df_prev) / st.prm.fluid.dt
    assert np.abs(st.vf[m.iface_f, 0:3] - w[m.iface_f]).max() <= 1e-15 * max(np.abs(w).max(), 1.0)
    # harmonic mesh displacement inside, interface values close to the structure's
    interior = ~m.fluid_boundary
    assert np.abs((st.L @ st.df)[interior]).max() <= 1e-12 * np.abs(st.df).max()
    gap = st.df[m.iface_f] - st.vs[m.iface_s, 0:3]
    assert np.linalg.norm(gap) / np.sqrt(len(m.iface_f)) < 1e-8
    assert np.abs(st.vs[:, 0:3]).max() > 1e-4


def test_relaxation_does_not_move_the_fixed_point(pulse):
    st, _, _, _ = pulse
    other = _state(0.1, omega0=0.02)
    other.time_step()
    # both stop at |r| / sqrt(n) < 1e-8 (about 1e-5 of the displacement
    # here); the DN map amplifies that gap by its conditioning, so the states
    # agree to a few parts in 1e5, not to rounding
    scale = np.abs(st.vs[:, 0:3]).max()
    assert np.abs(other.vs[:, 0:3] - st.vs[:, 0:3]).max() <= 2e-5 * scale
    assert np.abs(other.vf[:, 0:3] - st.vf[:, 0:3]).max() <= 2e-5 * np.abs(st.vf[:, 0:3]).max()
