"""Finite-element part of the oracle: materials, element residual/tangent, assembly.

Every function works on batches of tetrahedra with numpy in fp64.  Notation
follows the paper: F = I + grad d, J = det F, C = F^T F, invariants I1, I2, I3,
modified invariants J1 = I1 I3^{-1/3}, J2 = I2 I3^{-2/3}, fibre invariants
J4, J6 (Section "Nonlinear hyperelastic modeling"), S = 2 dPsi/dC.

Readings taken where the paper is silent or garbled:
* the anisotropic stress carries the factor 2 k1 that S = 2 dPsi/dC gives
  (the printed stress formula drops it);
* a fibre contributes stress and tangent only while its invariant J_i > 1;
* quasi-static loading (no inertia, r_s = 0) unless the Newmark-beta
  inertia is set (set_inertia: one density, the exact P1 mass, r_s in P1
  from its nodal values), dead nominal traction;
* one centroid quadrature point per tetrahedron (exact for every term of the
  P1-P1 form except the pressure mass, which uses the exact P1 mass matrix);
* h_T is the longest edge of T in the reference configuration, and the
  stabilisation parameter is tau = h_T^2 / (4 mu^l) with mu^l as printed;
* the Schur parameter theta of eq. lpreschur defaults to mu^l / 5: the paper
  asks for theta = O(c10) adjusted by tests on a coarse mesh and then kept
  fixed, and on the coarse 16^3 cube mu^l / 5 gave the fewest Krylov
  iterations (THETA_OVER_MU_L).
"""
from __future__ import annotations

import numpy as np

CHUNK = 32768
THETA_OVER_MU_L = 0.2   # default Schur parameter theta = mu^l / 5

# ---------------------------------------------------------------------------
# geometry (P1 tetrahedra)
# ---------------------------------------------------------------------------


def tet_geometry(X, tets):
    """Reference gradients of the four hat functions, volume and h_T.

    N_a are the barycentric coordinates; with D = [X1-X0, X2-X0, X3-X0]
    (edge vectors as columns) grad N_a is row a-1 of D^{-1} for a = 1..3 and
    grad N_0 = -(sum of the others).
    Returns G [m,4,3], V [m], h [m].
    """
    x = X[tets]  # (m,4,3)
    D = np.stack([x[:, 1] - x[:, 0], x[:, 2] - x[:, 0], x[:, 3] - x[:, 0]], axis=2)
    V = np.linalg.det(D) / 6.0
    Dinv = np.linalg.inv(D)
    G = np.empty((len(tets), 4, 3))
    G[:, 1:, :] = Dinv
    G[:, 0, :] = -Dinv.sum(axis=1)
    edges = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    h = np.max(np.stack([np.linalg.norm(x[:, a] - x[:, b], axis=1) for a, b in edges], axis=1), axis=1)
    return G, V, h


def material_arrays(materials, mat_id):
    """Per-element material constants: model, c10, c01, kappa, k1, k2."""
    keys = ("model", "c10", "c01", "kappa", "k1", "k2")
    tab = {k: np.array([float(m[k]) for m in materials]) for k in keys}
    return {k: tab[k][mat_id] for k in keys}


def mu_l(mat):
    """Linear shear modulus as printed: 2(c10+c01) (Mooney-Rivlin) and
    2(c10 + k1/(2 k2)) (artery) (stabilisation for the structure)."""
    k2 = np.where(mat["k2"] > 0, mat["k2"], 1.0)
    art = 2.0 * (mat["c10"] + np.where(mat["k2"] > 0, mat["k1"] / (2.0 * k2), 0.0))
    mr = 2.0 * (mat["c10"] + mat["c01"])
    return np.where(mat["model"] == 1, art, mr)


# ---------------------------------------------------------------------------
# tensor helpers on batches: arrays (m,3,3) and (m,3,3,3,3)
# ---------------------------------------------------------------------------
I3x3 = np.eye(3)


def outer(A, B):
    """(A (x) B)_IJKL = A_IJ B_KL."""
    return np.einsum("mij,mkl->mijkl", A, B)


def odot(A, B):
    """(A (.) B)_IJKL = 1/2 (A_IK B_JL + A_IL B_JK)."""
    return 0.5 * (np.einsum("mik,mjl->mijkl", A, B) + np.einsum("mil,mjk->mijkl", A, B))


def sym_identity(m):
    """Fourth-order symmetric identity, 1/2 (d_IK d_JL + d_IL d_JK)."""
    eye = np.broadcast_to(I3x3, (m, 3, 3))
    return odot(eye, eye)


# ---------------------------------------------------------------------------
# energies, stresses S' and material tangents C' = 2 dS'/dC
# ---------------------------------------------------------------------------


def invariants(C):
    I1 = np.trace(C, axis1=1, axis2=2)
    I2 = 0.5 * (I1 ** 2 - np.einsum("mij,mij->m", C, C))
    I3 = np.linalg.det(C)
    return I1, I2, I3


def fibre_tensors(fib):
    """A_i = a_0i (x) a_0i for the two fibre families, fib [m,2,3]."""
    return np.einsum("mi,mj->mij", fib[:, 0], fib[:, 0]), np.einsum("mi,mj->mij", fib[:, 1], fib[:, 1])


def deviatoric_energy(C, mat, fib=None):
    """Psi without the volumetric part (eq. mmreng and eq. areng)."""
    I1, I2, I3 = invariants(C)
    J1 = I1 * I3 ** (-1.0 / 3.0)
    J2 = I2 * I3 ** (-2.0 / 3.0)
    psi = 0.5 * mat["c10"] * (J1 - 3.0)
    mr = mat["model"] == 0
    psi = psi + np.where(mr, 0.5 * mat["c01"] * (J2 - 3.0), 0.0)
    if fib is not None and np.any(~mr):
        A4, A6 = fibre_tensors(fib)
        k2 = np.where(mat["k2"] > 0, mat["k2"], 1.0)
        for A in (A4, A6):
            Ji = I3 ** (-1.0 / 3.0) * np.einsum("mij,mij->m", A, C)
            e = (mat["k1"] / (2.0 * k2)) * (np.exp(k2 * (Ji - 1.0) ** 2) - 1.0)
            psi = psi + np.where((~mr) & (Ji > 1.0), e, 0.0)
    return psi


def stress_tangent(C, mat, fib=None):
    """S' = 2 dPsi'/dC and C' = 2 dS'/dC for a batch of C (m,3,3).

    Mooney-Rivlin (eq. mmrpkt / mmrpktmix):
        S' = c10 dJ1/dC + c01 dJ2/dC,
        dJ1/dC = I3^{-1/3} (I - I1/3 C^{-1}),
        dJ2/dC = I3^{-2/3} (I1 I - C - 2 I2/3 C^{-1}).
    Artery (eq. arpkt / arpktmix, with the factor 2 k1 of S = 2 dPsi/dC):
        S' = c10 dJ1/dC + sum_i [J_i>1] 2 psi'_i dJ_i/dC,
        psi'_i = k1 (J_i-1) exp(k2 (J_i-1)^2),
        dJ_i/dC = I3^{-1/3} (A_i - (A_i:C)/3 C^{-1}).
    """
    m = C.shape[0]
    Ci = np.linalg.inv(C)
    I1, I2, I3 = invariants(C)
    eye = np.broadcast_to(I3x3, (m, 3, 3))
    r13 = I3 ** (-1.0 / 3.0)
    r23 = I3 ** (-2.0 / 3.0)
    CiCi = odot(Ci, Ci)
    c10 = mat["c10"][:, None, None]
    c01 = np.where(mat["model"] == 0, mat["c01"], 0.0)[:, None, None]

    # J1 part
    S = c10 * r13[:, None, None] * (eye - (I1 / 3.0)[:, None, None] * Ci)
    T = (2.0 * c10 * r13[:, None, None])[..., None, None] * (
        -(outer(eye, Ci) + outer(Ci, eye)) / 3.0
        + (I1 / 9.0)[:, None, None, None, None] * outer(Ci, Ci)
        + (I1 / 3.0)[:, None, None, None, None] * CiCi)

    # J2 part (Mooney-Rivlin only; c01 = 0 elsewhere)
    B = I1[:, None, None] * eye - C
    S = S + c01 * r23[:, None, None] * (B - (2.0 * I2 / 3.0)[:, None, None] * Ci)
    T = T + (2.0 * c01 * r23[:, None, None])[..., None, None] * (
        outer(eye, eye) - sym_identity(m)
        - (2.0 / 3.0) * (outer(B, Ci) + outer(Ci, B))
        + (4.0 * I2 / 9.0)[:, None, None, None, None] * outer(Ci, Ci)
        + (2.0 * I2 / 3.0)[:, None, None, None, None] * CiCi)

    # fibre part (artery only, active in extension)
    art = mat["model"] == 1
    if fib is not None and np.any(art):
        A4, A6 = fibre_tensors(fib)
        k1 = mat["k1"]
        k2 = mat["k2"]
        for A in (A4, A6):
            I4 = np.einsum("mij,mij->m", A, C)
            Ji = r13 * I4
            active = art & (Ji > 1.0)
            x = Ji - 1.0
            ex = np.exp(k2 * x * x)
            d1 = np.where(active, k1 * x * ex, 0.0)                       # psi'
            d2 = np.where(active, k1 * ex * (1.0 + 2.0 * k2 * x * x), 0.0)  # psi''
            D = r13[:, None, None] * (A - (I4 / 3.0)[:, None, None] * Ci)
            S = S + (2.0 * d1)[:, None, None] * D
            dD = r13[:, None, None, None, None] * (
                -(outer(A, Ci) + outer(Ci, A)) / 3.0
                + (I4 / 9.0)[:, None, None, None, None] * outer(Ci, Ci)
                + (I4 / 3.0)[:, None, None, None, None] * CiCi)
            T = T + 4.0 * (d2[:, None, None, None, None] * outer(D, D)
                           + d1[:, None, None, None, None] * dD)
    return S, T


# ---------------------------------------------------------------------------
# element residual and consistent tangent
# ---------------------------------------------------------------------------


def element_kernel(G, V, h, mat, ue, pe, fib=None, want_tangent=True, theta=None, cm=0.0, re=None,
                   pressure_geometric=True):
    """Residual R_e [m,4,4] and tangent K_e [m,16,16] of a batch of tetrahedra.

    Dof order inside an element is node-interleaved: 4a + c, c = 0,1,2 the
    displacement components and c = 3 the pressure.

    Residual (eq. weakelas plus the stabilisation term of eq. stelas):
        R^u_a = V (F S' G_a - pbar J F^{-T} G_a) + sum_b M_ab (cm d_b - r_b)
        R^p_a = -V/4 (J-1) - 1/kappa sum_b M_ab p_b - tau V J (F^{-T}G_a).(F^{-T} grad p)
                + tau (F^{-T}G_a) . int_T (r_s - cm d)
    with M_ab = V (1 + delta_ab)/20 the exact P1 mass, pbar the mean of p,
    cm = rho_s/(beta dt^2) the Newmark-beta inertia coefficient and r_b the
    nodal values of the P1 field r_s (re [m,4,3]); cm = 0 and r_s = 0 give
    the quasi-static problem.  int_T (r_s - cm d) = V/4 sum_b (r_b - cm d_b).
    The tangent is the exact derivative of this residual (block structure of
    eq. globsys: K = [A B1^T; B2 -C]).  External loads are added globally.
    pressure_geometric=False leaves the pressure-geometric part
    -pbar V J (g_a g_b^T - g_b g_a^T) out of A (the operator A_plus), and
    the residual unchanged.
    """
    m = len(V)
    F = np.broadcast_to(I3x3, (m, 3, 3)) + np.einsum("mai,maj->mij", ue, G)
    J = np.linalg.det(F)
    Finv = np.linalg.inv(F)
    C = np.einsum("mki,mkj->mij", F, F)
    S, CC = stress_tangent(C, mat, fib)
    g = np.einsum("mji,maj->mai", Finv, G)              # g_a = F^{-T} G_a
    pbar = pe.mean(axis=1)
    gradp = np.einsum("ma,maj->mj", pe, G)
    ghat = np.einsum("mji,mj->mi", Finv, gradp)          # F^{-T} grad p
    kappa = mat["kappa"]
    tau = h * h / (4.0 * mu_l(mat))
    Mab = V[:, None, None] * (1.0 + np.eye(4))[None] / 20.0

    R = np.zeros((m, 4, 4))
    FS = np.einsum("mik,mkj->mij", F, S)
    R[:, :, 0:3] = V[:, None, None] * (np.einsum("mij,maj->mai", FS, G)
                                       - (pbar * J)[:, None, None] * g)
    gdot = np.einsum("mai,mi->ma", g, ghat)
    R[:, :, 3] = (-(V / 4.0 * (J - 1.0))[:, None]
                  - np.einsum("mab,mb->ma", Mab, pe) / kappa[:, None]
                  - (tau * V * J)[:, None] * gdot)
    dynamic = cm != 0.0 or re is not None
    if dynamic:
        r_nodal = np.zeros((m, 4, 3)) if re is None else re
        Mu = (1.0 + np.eye(4)) / 20.0
        R[:, :, 0:3] += V[:, None, None] * np.einsum("ab,mbi->mai", Mu, cm * ue - r_nodal)
        mvec = 0.25 * (r_nodal - cm * ue).sum(axis=1)      # mean of r_s - cm d on T
        R[:, :, 3] += (tau * V)[:, None] * np.einsum("mai,mi->ma", g, mvec)
    if not want_tangent:
        return R, None

    K = np.zeros((m, 4, 4, 4, 4))  # (a, i, b, k)
    # A block: geometric + material - pressure geometric
    geo = np.einsum("maj,mjl,mbl->mab", G, S, G)
    # F_iM G_aJ C'_MJNL F_kN G_bL
    mat_part = np.einsum("zip,zaj,zpjnl,zkn,zbl->zaibk", F, G, CC, F, G, optimize=True)
    pg = np.einsum("mai,mbk->maibk", g, g)
    A = V[:, None, None, None, None] * mat_part
    if pressure_geometric:
        A = A - (pbar * V * J)[:, None, None, None, None] * (pg - pg.transpose(0, 3, 2, 1, 4))
    A = A + (V[:, None, None] * geo)[:, :, None, :, None] * I3x3[None, None, :, None, :]
    K[:, :, 0:3, :, 0:3] = A
    # B1^T: dR^u_a / dp_b = -V/4 J g_a
    K[:, :, 0:3, :, 3] = (-(V * J / 4.0)[:, None, None] * g)[:, :, :, None]
    # B2: dR^p_a / du_b
    gg = np.einsum("mai,mbi->mab", g, g)
    B2 = (-(V * J / 4.0)[:, None, None, None] * np.broadcast_to(g[:, None, :, :], (m, 4, 4, 3))
          - (tau * V * J)[:, None, None, None] * (
              gdot[:, :, None, None] * g[:, None, :, :]
              - gdot[:, None, :, None] * g[:, :, None, :]
              - gg[:, :, :, None] * ghat[:, None, None, :]))
    K[:, :, 3, :, 0:3] = B2
    # -C: dR^p_a / dp_b
    K[:, :, 3, :, 3] = -(Mab / kappa[:, None, None] + (tau * V * J)[:, None, None] * gg)
    if dynamic:
        # inertia: cm M_ab I, and the derivative of tau g_a . int_T (r_s - cm d)
        # through the mean (-cm/4) and through g_a (d g_a = -g_b (g_a . du_b))
        K[:, :, 0:3, :, 0:3] += (cm * V[:, None, None, None, None] * Mu[None, :, None, :, None]
                                 * I3x3[None, None, :, None, :])
        gm = np.einsum("mbi,mi->mb", g, mvec)
        K[:, :, 3, :, 0:3] += ((tau * V)[:, None, None, None] * (-(cm / 4.0) - gm[:, None, :, None])
                               * g[:, :, None, :])
    return R, K.reshape(m, 16, 16)


# ---------------------------------------------------------------------------
# global assembly
# ---------------------------------------------------------------------------


class Discretization:
    """Mesh-dependent data of one solid problem, built once."""

    def __init__(self, prob, theta=None):
        self.prob = prob
        self.n = prob.n_nodes
        self.m = prob.n_tets
        self.G, self.V, self.h = tet_geometry(prob.X, prob.tets)
        if np.any(self.V <= 0):
            raise ValueError("non-positive element volume")
        self.mat = material_arrays(prob.materials, prob.mat_id)
        self.fib = prob.fibres
        mu = mu_l(self.mat)
        self.theta = THETA_OVER_MU_L * mu if theta is None else np.full(self.m, float(theta))
        self._build_pattern()
        self._build_loads()

    # node graph: every pair of nodes that share a tetrahedron (incl. i==i)
    def _build_pattern(self):
        T = self.prob.tets.astype(np.int64)
        rows = np.repeat(T, 4, axis=1).ravel()
        cols = np.tile(T, (1, 4)).ravel()
        key = np.unique(rows * self.n + cols)
        self.node_rows = key // self.n
        self.node_cols = key % self.n
        self.node_ptr = np.searchsorted(self.node_rows, np.arange(self.n + 1))
        # scalar 4n x 4n CSR pattern, node-interleaved dofs 4i+c, sorted columns
        n = self.n
        c4 = np.arange(4)
        r = (4 * self.node_rows[:, None, None] + c4[None, :, None]).repeat(4, axis=2)
        c = (4 * self.node_cols[:, None, None] + c4[None, None, :]).repeat(4, axis=1)
        keys = np.sort((r * (4 * n) + c).ravel())
        self.K_keys = keys
        self.K_indices = keys % (4 * n)
        self.K_indptr = np.searchsorted(keys // (4 * n), np.arange(4 * n + 1))
        # position of element entry (4a+i, 4b+k) in the CSR value array
        er = (4 * T[:, :, None] + c4[None, None]).reshape(self.m, 16)
        ekeys = er[:, :, None] * (4 * n) + er[:, None, :]
        self.elem_pos = np.searchsorted(keys, ekeys)

    def _build_loads(self):
        """Nodal load of a dead nominal traction: f_a = sum_tri t A_tri / 3."""
        p = self.prob
        f = np.zeros((self.n, 3))
        if len(p.tris):
            x = p.X[p.tris]
            area = 0.5 * np.linalg.norm(np.cross(x[:, 1] - x[:, 0], x[:, 2] - x[:, 0]), axis=1)
            contrib = p.traction * (area / 3.0)[:, None]
            for a in range(3):
                np.add.at(f, p.tris[:, a], contrib)
        self.f_ext = f

    def set_inertia(self, cm, rs):
        """Newmark-beta inertia: coefficient cm = rho_s/(beta dt^2) and the
        nodal history field r_s [n,3] (cm = 0, rs = None: quasi-static)."""
        self.cm = float(cm)
        self.rs = None if rs is None else np.asarray(rs, np.float64).reshape(self.n, 3)

    cm = 0.0
    rs = None

    def element_batches(self, v):
        v = np.asarray(v).reshape(self.n, 4)
        for s in range(0, self.m, CHUNK):
            e = slice(s, min(s + CHUNK, self.m))
            T = self.prob.tets[e]
            ve = v[T]
            mat = {k: a[e] for k, a in self.mat.items()}
            fib = None if self.fib is None else self.fib[e]
            yield e, ve, mat, fib

    def _inertia(self, e):
        if self.cm == 0.0 and self.rs is None:
            return {}
        return dict(cm=self.cm, re=None if self.rs is None else self.rs[self.prob.tets[e]])

    def residual(self, v, load):
        """Global residual R (4n, node-interleaved) before Dirichlet handling."""
        R = np.zeros((self.n, 4))
        for e, ve, mat, fib in self.element_batches(v):
            Re, _ = element_kernel(self.G[e], self.V[e], self.h[e], mat, ve[:, :, 0:3], ve[:, :, 3],
                                   fib, want_tangent=False, **self._inertia(e))
            for a in range(4):
                np.add.at(R, self.prob.tets[e, a], Re[:, a])
        R[:, 0:3] -= load * self.f_ext
        return R.ravel()

    def assemble(self, v, load, pressure_geometric=True):
        """Residual and consistent tangent (CSR values on the fixed pattern);
        pressure_geometric=False: the tangent with A_plus in place of A."""
        R = np.zeros((self.n, 4))
        val = np.zeros(len(self.K_indices))
        for e, ve, mat, fib in self.element_batches(v):
            Re, Ke = element_kernel(self.G[e], self.V[e], self.h[e], mat, ve[:, :, 0:3], ve[:, :, 3], fib,
                                    pressure_geometric=pressure_geometric, **self._inertia(e))
            for a in range(4):
                np.add.at(R, self.prob.tets[e, a], Re[:, a])
            np.add.at(val, self.elem_pos[e].ravel(), Ke.ravel())
        R[:, 0:3] -= load * self.f_ext
        return R.ravel(), val

    def csr(self, val):
        import scipy.sparse as sp
        N = 4 * self.n
        return sp.csr_matrix((val, self.K_indices.copy(), self.K_indptr.copy()), shape=(N, N))

    # -- Dirichlet handling and blocks ------------------------------------
    def dirichlet_dofs(self):
        return np.flatnonzero(self.prob.dir_mask.ravel())

    def apply_dirichlet(self, R, val):
        """Rows and columns of fixed dofs zeroed, unit diagonal, R_d = 0."""
        d = np.zeros(4 * self.n, bool)
        d[self.dirichlet_dofs()] = True
        rows = np.repeat(np.arange(4 * self.n), np.diff(self.K_indptr))
        cols = self.K_indices
        val = val.copy()
        hit = d[rows] | d[cols]
        val[hit] = 0.0
        val[hit & (rows == cols)] = 1.0
        R = R.copy()
        R[d] = 0.0
        return R, val

    def blocks(self, val):
        """A (3n x 3n, dof 3i+c), B2 (n x 3n) and the Schur diagonal s.

        A keeps every stored entry of the displacement-displacement block
        except those removed by the Dirichlet elimination (zero off-diagonal
        entries in a fixed row or column); the pattern depends only on the
        mesh and the boundary set.
        s_i = sum_{T contains i} (1/theta_T + 1/kappa_T) V_T / 10
        (eq. lpreschur with the diagonal of the consistent P1 pressure mass).
        """
        import scipy.sparse as sp
        n = self.n
        rows = np.repeat(np.arange(4 * n), np.diff(self.K_indptr))
        cols = self.K_indices
        rc, cc = rows % 4, cols % 4
        d = np.zeros(4 * n, bool)
        d[self.dirichlet_dofs()] = True
        keepA = (rc < 3) & (cc < 3) & ~((d[rows] | d[cols]) & (rows != cols))
        ar = 3 * (rows[keepA] // 4) + rc[keepA]
        ac = 3 * (cols[keepA] // 4) + cc[keepA]
        A = _csr_from_sorted(ar, ac, val[keepA], 3 * n, 3 * n)
        keepB = (rc == 3) & (cc < 3)
        B2 = sp.csr_matrix((val[keepB], (rows[keepB] // 4, 3 * (cols[keepB] // 4) + cc[keepB])),
                           shape=(n, 3 * n))
        w = (1.0 / self.theta + 1.0 / self.mat["kappa"]) * self.V / 10.0
        s = np.zeros(n)
        for a in range(4):
            np.add.at(s, self.prob.tets[:, a], w)
        return A, B2, s

    def mass_norm(self, dv):
        """||dv||_M with M = diag(M1, M2), the consistent P1 mass matrices of
        displacement and pressure (the norm of the Newton stopping rule)."""
        dv = dv.reshape(self.n, 4)
        tot = 0.0
        T = self.prob.tets
        Mab = (1.0 + np.eye(4)) / 20.0
        for s in range(0, self.m, CHUNK):
            e = slice(s, min(s + CHUNK, self.m))
            x = dv[T[e]]  # (m,4,4)
            tot += np.einsum("m,ab,mac,mbc->", self.V[e], Mab, x, x)
        return float(np.sqrt(tot))


def _csr_from_sorted(r, c, v, nr, nc):
    """CSR matrix from (row, col) pairs already sorted by row then column,
    keeping explicit zeros."""
    import scipy.sparse as sp
    indptr = np.zeros(nr + 1, np.int64)
    np.add.at(indptr, r + 1, 1)
    indptr = np.cumsum(indptr)
    M = sp.csr_matrix((np.asarray(v, np.float64), np.asarray(c, np.int64), indptr), shape=(nr, nc))
    return M
