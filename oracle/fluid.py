"""Stabilised P1-P1 fluid sub-problem on a moving mesh, and the harmonic
mesh extension (oracle; test infrastructure only).

Fluid (section "The fluid sub-problem", eq. ns; implicit Euler in time,
eq. nstdis; weak residuals of section "The time semi-discretized fluid weak
formulation", eq. weakns; SUPG/PSPG stabilisation, eq. stabweakfluid).  On
the current mesh x = X + d_f, with velocity u, pressure p, the previous
step's velocity u_old (nodal values: the ALE map carries nodes to nodes, so
u_old composed with the maps of eq. nstdis is u_old at the same node) and
the mesh velocity w (eq. hartdis), the residual rows of node a are

  R^u_a = int rho/dt (u - u_old) N_a + rho ((u - w) . grad) u N_a
          + 2 mu eps(u) : eps(N_a e_i) - p div(N_a e_i)
          + tau rho ((u - w) . grad N_a) r          (SUPG)
          - <g_in, N_a>_inlet
  R^p_a = -int N_a div u - tau grad N_a . r          (PSPG)

with the strong momentum residual per unit mass
r = (u - u_old)/dt + ((u - w) . grad) u + grad p / rho (the viscous term
vanishes for P1).  The paper names SUPG/PSPG but prints no W_f; the
readings taken here:

* one tau per element, tau = ((2/dt)^2 + (2|c|/h)^2 + (4 nu/h^2)^2)^(-1/2)
  with c the mean of u - w over the element's nodes, nu = mu/rho and h the
  longest edge of the current element (the same element size as the
  structure's stabilisation);
* PSPG enters the pressure rows with the sign of the paper's continuity
  residual -(q, div u), so the pressure block of the Jacobian is -C with C
  symmetric positive semi-definite, the block form of eq. globsys;
* integrals by the 4-point degree-2 rule, exact for every term here (the
  integrands are at most quadratic on a tetrahedron);
* the Jacobian is the exact derivative with tau held at its value at the
  current iterate (tau depends on |c| through a non-smooth norm);
* g_in is constant over the inlet, and the inlet does not move (the mesh
  displacement is zero there), so its nodal load is g_in A_tri / 3;
* the Oseen form (an option) takes the previous step's velocity as the
  convective field, c = u_old - w, in the convection term, the SUPG test
  function and tau: the step is then linear in (u, p).

Nodes are node-interleaved (u_x, u_y, u_z, p), the layout and block pattern
of the structure.  The force the fluid exerts on the structure at an
interface node is minus the momentum residual there (before the Dirichlet
rows are replaced): by Green's formula that residual is the boundary
integral of sigma n_f N_a, and the wall feels -sigma n_f.

Harmonic extension (eq. harext): each displacement component solves the P1
Laplace problem on the reference fluid mesh with the interface values given
and zero on the inlet and outlet; the extension's nodal values of every
boundary node are prescribed.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spl

# 4-point rule on a tetrahedron: barycentric (A, B, B, B) and permutations,
# weight V/4 each, exact for polynomials of degree 2
QA = 0.5854101966249685
QB = 0.1381966011250105
QUAD = np.full((4, 4), QB) + np.eye(4) * (QA - QB)   # QUAD[q, a] = N_a at point q


@dataclasses.dataclass
class FluidParams:
    rho: float = 1.0      # mg / mm^3
    mu: float = 0.0035    # kPa ms (0.035 Poise)
    dt: float = 0.125     # ms
    stabilise: bool = True
    oseen: bool = False   # convective velocity u_old - w (Oseen) instead of u - w


def geometry(x):
    """Gradients of the hat functions [m,4,3], volume [m] and longest edge
    [m] of tetrahedra with corner coordinates x [m,4,3]."""
    D = np.stack([x[:, 1] - x[:, 0], x[:, 2] - x[:, 0], x[:, 3] - x[:, 0]], axis=2)
    V = np.linalg.det(D) / 6.0
    Dinv = np.linalg.inv(D)
    G = np.empty(x.shape)
    G[:, 1:, :] = Dinv
    G[:, 0, :] = -Dinv.sum(axis=1)
    edges = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    h = np.max(np.stack([np.linalg.norm(x[:, a] - x[:, b], axis=1) for a, b in edges], axis=1), axis=1)
    return G, V, h


def tau_of(c_mean, h, prm: FluidParams):
    nu = prm.mu / prm.rho
    cn = np.linalg.norm(c_mean, axis=-1)
    return ((2.0 / prm.dt) ** 2 + (2.0 * cn / h) ** 2 + (4.0 * nu / (h * h)) ** 2) ** -0.5


def element_kernel(x, ue, pe, uo, we, prm: FluidParams, want_tangent=True, tau=None):
    """Residual R_e [m,4,4] and Jacobian K_e [m,16,16] (dof 4a + c) of a batch
    of fluid tetrahedra: corners x [m,4,3] (current mesh), velocity ue
    [m,4,3], pressure pe [m,4], previous velocity uo and mesh velocity we
    [m,4,3].  tau [m] overrides the element parameter (the Jacobian treats
    it as a constant either way).  Inlet loads are added globally."""
    rho, mu, dt = prm.rho, prm.mu, prm.dt
    G, V, h = geometry(x)
    m = len(V)
    ce = (uo if prm.oseen else ue) - we                 # nodal convective velocity
    dc = 0.0 if prm.oseen else 1.0                      # d c / d u
    if tau is None:
        tau = tau_of(ce.mean(axis=1), h, prm)
    if not prm.stabilise:
        tau = np.zeros(m)
    Gu = np.einsum("mbi,mbj->mij", ue, G)               # Gu[i, j] = d u_i / d x_j
    gp = np.einsum("mb,mbj->mj", pe, G)
    div = np.einsum("mii->m", Gu)
    uq = np.einsum("qb,mbi->mqi", QUAD, ue)
    uoq = np.einsum("qb,mbi->mqi", QUAD, uo)
    cq = np.einsum("qb,mbi->mqi", QUAD, ce)
    conv = np.einsum("mij,mqj->mqi", Gu, cq)            # ((c . grad) u) at q
    r = (uq - uoq) / dt + conv + gp[:, None, :] / rho   # strong residual per unit mass
    cG = np.einsum("mqj,maj->mqa", cq, G)               # c(q) . grad N_a
    w = V / 4.0                                          # quadrature weight

    R = np.zeros((m, 4, 4))
    # Galerkin momentum
    R[:, :, 0:3] = w[:, None, None] * np.einsum("qa,mqi->mai", QUAD, rho * ((uq - uoq) / dt + conv))
    sym = Gu + Gu.transpose(0, 2, 1)
    R[:, :, 0:3] += (mu * V)[:, None, None] * np.einsum("mij,maj->mai", sym, G)
    R[:, :, 0:3] -= (V * pe.mean(axis=1))[:, None, None] * G
    # SUPG
    R[:, :, 0:3] += (w * rho * tau)[:, None, None] * np.einsum("mqa,mqi->mai", cG, r)
    # continuity and PSPG
    R[:, :, 3] = -(w * div)[:, None] - (w * tau)[:, None] * np.einsum("maj,mqj->ma", G, r)
    if not want_tangent:
        return R, None

    K = np.zeros((m, 4, 4, 4, 4))   # (a, i, b, k)
    I3 = np.eye(3)
    NN = np.einsum("qa,qb->ab", QUAD, QUAD)             # sum_q N_a N_b (times w: the mass)
    cGb = cG                                             # c(q) . grad N_b, [m,q,b]
    # d r_i(q) / d u_bk = delta_ik (N_b(q)/dt + c(q).G_b) + dc Gu_ik N_b(q)
    dr_diag = QUAD[None, :, :] / dt + cGb                # [m,q,b]
    # Galerkin momentum: mass, convection (both factors), viscous
    K[:, :, 0:3, :, 0:3] += ((w * rho / dt)[:, None, None, None, None] * NN[None, :, None, :, None]
                              * I3[None, None, :, None, :])
    K[:, :, 0:3, :, 0:3] += (w * rho)[:, None, None, None, None] * (
        np.einsum("qa,mqb->mab", QUAD, cGb)[:, :, None, :, None] * I3[None, None, :, None, :]
        + dc * NN[None, :, None, :, None] * Gu[:, None, :, None, :])
    GG = np.einsum("maj,mbj->mab", G, G)
    K[:, :, 0:3, :, 0:3] += (mu * V)[:, None, None, None, None] * (
        GG[:, :, None, :, None] * I3[None, None, :, None, :]
        + np.einsum("mak,mbi->maibk", G, G))
    # Galerkin pressure gradient: d/dp_b of -V pbar G_ai
    K[:, :, 0:3, :, 3] += -(V / 4.0)[:, None, None, None] * G[:, :, :, None]
    # SUPG: d/du_bk of w rho tau sum_q (c.G_a) r_i
    s = (w * rho * tau)[:, None, None, None, None]
    K[:, :, 0:3, :, 0:3] += s * (
        dc * np.einsum("qb,mak,mqi->maibk", QUAD, G, r)
        + np.einsum("mqa,mqb->mab", cG, dr_diag)[:, :, None, :, None] * I3[None, None, :, None, :]
        + dc * np.einsum("mqa,qb->mab", cG, QUAD)[:, :, None, :, None] * Gu[:, None, :, None, :])
    K[:, :, 0:3, :, 3] += (w * tau)[:, None, None, None] * np.einsum("mqa,mbi->maib", cG, G)
    # continuity: d/du_bk of -w div u
    K[:, :, 3, :, 0:3] += -w[:, None, None, None] * G[:, None, :, :]
    # PSPG: d/du_bk of -w tau sum_q G_a . r
    K[:, :, 3, :, 0:3] += -(w * tau)[:, None, None, None] * (
        np.einsum("mak,mqb->mabk", G, dr_diag)
        + dc * np.einsum("mai,mik,qb->mabk", G, Gu, QUAD))
    K[:, :, 3, :, 3] += -(V * tau / rho)[:, None, None] * GG
    return R, K.reshape(m, 16, 16)


class FluidDiscretization:
    """Mesh data of one fluid mesh (reference coordinates X0 [n,3], tets)."""

    def __init__(self, X0, tets, dir_mask, inlet_tris, prm: FluidParams = FluidParams()):
        self.X0 = np.asarray(X0, np.float64)
        self.tets = np.asarray(tets, np.int64)
        self.n = len(self.X0)
        self.m = len(self.tets)
        self.dir_mask = np.asarray(dir_mask, np.uint8)
        self.inlet = np.asarray(inlet_tris, np.int64)
        self.prm = prm
        self._pattern()
        x = self.X0[self.inlet]
        self.inlet_area = 0.5 * np.linalg.norm(np.cross(x[:, 1] - x[:, 0], x[:, 2] - x[:, 0]), axis=1)

    def _pattern(self):
        """Scalar 4n x 4n CSR pattern of every node pair sharing a
        tetrahedron (sorted columns) and each element entry's position."""
        n, T = self.n, self.tets
        c4 = np.arange(4)
        er = (4 * T[:, :, None] + c4[None, None]).reshape(self.m, 16)
        keys = np.unique((er[:, :, None] * (4 * n) + er[:, None, :]).ravel())
        self.K_indices = keys % (4 * n)
        self.K_indptr = np.searchsorted(keys // (4 * n), np.arange(4 * n + 1))
        self.elem_pos = np.searchsorted(keys, er[:, :, None] * (4 * n) + er[:, None, :])

    def inlet_load(self, g_in):
        """Nodal load of the constant inlet traction g_in (3,): g_in A / 3."""
        f = np.zeros((self.n, 3))
        for a in range(3):
            np.add.at(f, self.inlet[:, a], np.outer(self.inlet_area / 3.0, g_in))
        return f

    def assemble(self, v, dmesh, u_old, w, g_in, want_tangent=True):
        """Residual R [4n] (inlet load included, no Dirichlet handling) and
        the Jacobian values on the pattern."""
        v = np.asarray(v).reshape(self.n, 4)
        T = self.tets
        x = (self.X0 + np.asarray(dmesh).reshape(self.n, 3))[T]
        Re, Ke = element_kernel(x, v[:, 0:3][T], v[:, 3][T], np.asarray(u_old).reshape(self.n, 3)[T],
                                np.asarray(w).reshape(self.n, 3)[T], self.prm, want_tangent)
        R = np.zeros((self.n, 4))
        for a in range(4):
            np.add.at(R, T[:, a], Re[:, a])
        R[:, 0:3] -= self.inlet_load(np.asarray(g_in, np.float64))
        val = None
        if want_tangent:
            val = np.zeros(len(self.K_indices))
            np.add.at(val, self.elem_pos.ravel(), Ke.ravel())
        return R.ravel(), val

    def csr(self, val):
        N = 4 * self.n
        return sp.csr_matrix((val, self.K_indices.copy(), self.K_indptr.copy()), shape=(N, N))

    def apply_dirichlet(self, R, val):
        d = self.dir_mask.ravel().astype(bool)
        rows = np.repeat(np.arange(4 * self.n), np.diff(self.K_indptr))
        cols = self.K_indices
        val = val.copy()
        hit = d[rows] | d[cols]
        val[hit] = 0.0
        val[hit & (rows == cols)] = 1.0
        R = R.copy()
        R[d] = 0.0
        return R, val

    def mass_norm(self, dv):
        """||dv||_M with the consistent P1 mass on the reference mesh."""
        x = np.asarray(dv).reshape(self.n, 4)[self.tets]
        _, V, _ = geometry(self.X0[self.tets])
        Mab = (1.0 + np.eye(4)) / 20.0
        return float(np.sqrt(np.einsum("m,ab,mac,mbc->", V, Mab, x, x)))


def newton_solve(disc: FluidDiscretization, v, dmesh, u_old, w, g_in, eps2=1e-10, max_iter=25, ref=None):
    """Newton's method for the fluid step (section "Newton's Method" with
    the fluid residual): the prescribed dofs of v keep their values, every
    correction solves K dv = -R directly, stop when ||dv_k||_M <= eps2 ref
    with ref = ||dv_0||_M unless given (a caller that warm-starts the solve
    passes the reference of its first, cold solve), or when the first
    correction is at the rounding level of the state, ||dv_0||_M <= 1e-14
    ||v||_M.  Returns (v, iterations, ||dv_0||_M)."""
    v = np.asarray(v, np.float64).ravel().copy()
    floor = 1e-14 * disc.mass_norm(v)
    n0 = None
    for k in range(max_iter):
        R, val = disc.assemble(v, dmesh, u_old, w, g_in)
        R, val = disc.apply_dirichlet(R, val)
        dv = spl.spsolve(disc.csr(val).tocsc(), -R)
        v += dv
        nrm = disc.mass_norm(dv)
        if n0 is None:
            n0 = nrm
            if nrm <= floor:
                return v, k + 1, n0
        if (k > 0 or ref is not None) and nrm <= eps2 * (n0 if ref is None else ref):
            return v, k + 1, n0
    raise RuntimeError("fluid Newton did not converge")


def interface_force(disc: FluidDiscretization, v, dmesh, u_old, w, g_in, nodes):
    """Force [len(nodes),3] the fluid exerts on the wall at the given nodes:
    minus the momentum residual there."""
    R, _ = disc.assemble(v, dmesh, u_old, w, g_in, want_tangent=False)
    return -R.reshape(disc.n, 4)[nodes, 0:3]


# ---------------------------------------------------------------------------
# harmonic extension
# ---------------------------------------------------------------------------


def laplacian(X0, tets):
    """P1 stiffness matrix of the Laplacian on the reference mesh (CSR n x n)."""
    T = np.asarray(tets, np.int64)
    G, V, _ = geometry(np.asarray(X0)[T])
    Ke = V[:, None, None] * np.einsum("maj,mbj->mab", G, G)
    r = np.repeat(T, 4, axis=1).ravel()
    c = np.tile(T, (1, 4)).ravel()
    n = len(X0)
    return sp.csr_matrix((Ke.ravel(), (r, c)), shape=(n, n))


def harmonic_extension(L, fixed, values):
    """Nodal d [n,3] with -Laplace d = 0 at the free nodes and d = values
    [len(fixed),3] at the fixed nodes (eq. harext), one P1 solve per
    component."""
    n = L.shape[0]
    free = np.setdiff1d(np.arange(n), fixed)
    d = np.zeros((n, 3))
    d[fixed] = values
    Lff = L[free][:, free].tocsc()
    rhs = -(L[free][:, fixed] @ d[fixed])
    for c in range(3):
        d[free, c] = spl.spsolve(Lff, rhs[:, c])
    return d
