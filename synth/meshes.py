"""Structured tetrahedral meshes and boundary data for the solid sub-problem.

The paper meshes its artery with an external mesh generator (Section
"Coarse and fine meshes"); those meshes are not available, so these seeded
lattice meshes stand in for them:

* a unit cube of N^3 hexahedra, each split into the six Kuhn tetrahedra that
  share the hexahedron's main diagonal (conforming across hexahedra);
* a thick-walled two-layer tube (media inside, adventitia outside), periodic
  in the circumferential direction, split the same way in index space.

Every function is deterministic given its arguments (jitter and random
states use ``numpy.random.default_rng(seed)``).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# The six axis permutations; tetrahedron k of a hexahedron walks from corner
# (0,0,0) along axis perm[0], then perm[1], to corner (1,1,1).
KUHN_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


def _kuhn_offsets():
    """Corner offsets (6 tets x 4 corners x 3) of the Kuhn split of a unit hex."""
    out = np.zeros((6, 4, 3), dtype=np.int64)
    for t, perm in enumerate(KUHN_PERMS):
        c = np.zeros(3, dtype=np.int64)
        out[t, 0] = c
        c = c.copy(); c[perm[0]] = 1; out[t, 1] = c
        c = c.copy(); c[perm[1]] = 1; out[t, 2] = c
        out[t, 3] = (1, 1, 1)
    return out


def _signed_volume6(X, tets):
    x0 = X[tets[:, 0]]
    d = np.stack([X[tets[:, 1]] - x0, X[tets[:, 2]] - x0, X[tets[:, 3]] - x0], axis=2)
    return np.linalg.det(d)


def _orient(X, tets):
    """Swap the last two corners of every negatively oriented tetrahedron."""
    vol6 = _signed_volume6(X, tets)
    neg = vol6 < 0
    tets = tets.copy()
    tets[neg, 2], tets[neg, 3] = tets[neg, 3].copy(), tets[neg, 2].copy()
    return tets


def _lattice_tets(shape, node_id, periodic_axis=None):
    """Kuhn tetrahedra of a lattice of hexahedra.

    shape: number of hexahedra per axis (n0, n1, n2).
    node_id(i0, i1, i2) -> node index arrays (with wrap on ``periodic_axis``).
    Elements are ordered hexahedron by hexahedron (axis 0 fastest), six
    tetrahedra per hexahedron in KUHN_PERMS order.
    """
    n0, n1, n2 = shape
    i2, i1, i0 = np.meshgrid(np.arange(n2), np.arange(n1), np.arange(n0), indexing="ij")
    base = np.stack([i0.ravel(), i1.ravel(), i2.ravel()], axis=1)  # (nhex, 3)
    offs = _kuhn_offsets()
    tets = np.empty((base.shape[0], 6, 4), dtype=np.int64)
    for t in range(6):
        for a in range(4):
            c = base + offs[t, a]
            tets[:, t, a] = node_id(c[:, 0], c[:, 1], c[:, 2])
    hex_ijk = base
    return tets.reshape(-1, 4), np.repeat(hex_ijk, 6, axis=0)


def cube_mesh(N: int, jitter: float = 0.0, seed: int = 0, side: float = 1.0):
    """Unit cube [0,side]^3 of N^3 hexahedra split into 6N^3 tetrahedra.

    Node (i,j,k) has index i + (N+1)*(j + (N+1)*k) and reference position
    side*(i,j,k)/N.  ``jitter`` moves every interior node by
    U(-jitter*h, jitter*h)^3, h = side/N (boundary nodes stay on their faces).
    """
    n1 = N + 1
    k, j, i = np.meshgrid(np.arange(n1), np.arange(n1), np.arange(n1), indexing="ij")
    lattice = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.int32)
    h = side / N
    X = lattice.astype(np.float64) * h
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        d = rng.uniform(-jitter * h, jitter * h, size=X.shape)
        interior = np.all((lattice > 0) & (lattice < N), axis=1)
        X[interior] += d[interior]

    def node_id(a, b, c):
        return a + n1 * (b + n1 * c)

    tets, hex_ijk = _lattice_tets((N, N, N), node_id)
    tets = _orient(X, tets)
    return dict(X=X, tets=tets.astype(np.int32), mat_id=np.zeros(len(tets), np.int32),
                lattice=lattice, hex_ijk=hex_ijk.astype(np.int32), h=h)


def tube_radii(r_in=0.71, media=0.26, adventitia=0.13, n_media=5, n_adv=3):
    """Radial node positions: n_media equal media cells then n_adv adventitia cells."""
    rm = r_in + media * np.arange(n_media + 1) / n_media
    ra = r_in + media + adventitia * np.arange(1, n_adv + 1) / n_adv
    return np.concatenate([rm, ra])


def tube_mesh(n_theta=64, n_media=5, n_adv=3, n_z=128, r_in=0.71, media=0.26,
              adventitia=0.13, length=5.0, alpha_media_deg=29.0, alpha_adv_deg=62.0):
    """Two-layer thick-walled tube, periodic in theta, axis = z.

    Lattice index (a, b, c) = (theta, radial, axial); node index
    a + n_theta*(b + (n_r+1)*c).  Material id 0 (media) for radial cells
    b < n_media, 1 (adventitia) otherwise.  The fibre vectors of each element
    are cos(alpha) e_theta +/- sin(alpha) e_z of the local cylindrical basis at
    the element centroid.
    """
    n_r = n_media + n_adv
    radii = tube_radii(r_in, media, adventitia, n_media, n_adv)
    c, b, a = np.meshgrid(np.arange(n_z + 1), np.arange(n_r + 1), np.arange(n_theta), indexing="ij")
    lattice = np.stack([a.ravel(), b.ravel(), c.ravel()], axis=1).astype(np.int32)
    theta = 2.0 * math.pi * lattice[:, 0] / n_theta
    r = radii[lattice[:, 1]]
    z = length * lattice[:, 2] / n_z
    X = np.stack([r * np.cos(theta), r * np.sin(theta), z], axis=1)

    def node_id(ia, ib, ic):
        return (ia % n_theta) + n_theta * (ib + (n_r + 1) * ic)

    tets, hex_ijk = _lattice_tets((n_theta, n_r, n_z), node_id)
    tets = _orient(X, tets)
    mat_id = (hex_ijk[:, 1] >= n_media).astype(np.int32)
    cen = X[tets].mean(axis=1)
    rr = np.hypot(cen[:, 0], cen[:, 1])
    e_t = np.stack([-cen[:, 1] / rr, cen[:, 0] / rr, np.zeros_like(rr)], axis=1)
    e_z = np.tile(np.array([0.0, 0.0, 1.0]), (len(tets), 1))
    alpha = np.where(mat_id == 0, math.radians(alpha_media_deg), math.radians(alpha_adv_deg))[:, None]
    fib = np.stack([np.cos(alpha) * e_t + np.sin(alpha) * e_z,
                    np.cos(alpha) * e_t - np.sin(alpha) * e_z], axis=1)
    return dict(X=X, tets=tets.astype(np.int32), mat_id=mat_id, lattice=lattice,
                hex_ijk=hex_ijk.astype(np.int32), fibres=fib, radii=radii)


def boundary_faces(tets):
    """Triangles (sorted node triples) that belong to exactly one tetrahedron."""
    f = np.concatenate([tets[:, [1, 2, 3]], tets[:, [0, 2, 3]], tets[:, [0, 1, 3]], tets[:, [0, 1, 2]]])
    f = np.sort(f, axis=1).astype(np.int64)
    # one int64 key per sorted triple (lexicographic order = key order) makes
    # the duplicate count a 1-D unique, much faster than unique over rows
    n = int(f.max()) + 1
    assert n < (1 << 21)
    key = (f[:, 0] * n + f[:, 1]) * n + f[:, 2]
    uk, cnt = np.unique(key, return_counts=True)
    uk = uk[cnt == 1]
    return np.stack([uk // (n * n), (uk // n) % n, uk % n], axis=1).astype(np.int32)


@dataclasses.dataclass
class Problem:
    """One solid sub-problem: mesh, materials, Dirichlet mask and dead traction."""
    X: np.ndarray            # f64 [n,3] reference coordinates
    tets: np.ndarray         # i32 [m,4] positively oriented
    mat_id: np.ndarray       # i32 [m]
    materials: list          # list of dicts (model, c10, c01, kappa, k1, k2)
    dir_mask: np.ndarray     # u8 [n,4]: 1 = dof fixed to zero
    tris: np.ndarray         # i32 [k,3] loaded boundary triangles
    traction: np.ndarray     # f64 [k,3] nominal traction at load factor 1
    lattice: np.ndarray      # i32 [n,3] lattice index of each node
    fibres: np.ndarray | None = None   # f64 [m,2,3] (anisotropic model)
    name: str = ""

    @property
    def n_nodes(self):
        return self.X.shape[0]

    @property
    def n_tets(self):
        return self.tets.shape[0]

    @property
    def n_dofs(self):
        return 4 * self.X.shape[0]


def mooney_rivlin(c10=0.5, c01=0.1, kappa=1e4):
    return dict(model=0, c10=float(c10), c01=float(c01), kappa=float(kappa), k1=0.0, k2=0.0)


def artery_layer(c10, k1, k2, kappa=1e5):
    return dict(model=1, c10=float(c10), c01=0.0, kappa=float(kappa), k1=float(k1), k2=float(k2))


def cube_problem(N=8, kappa=1e4, c10=0.5, c01=0.1, traction=(0.0, 0.0, 0.05), jitter=0.0,
                 seed=0, materials=None):
    """Cube clamped (u=0) on x=0, dead traction on the face x=1; p free everywhere."""
    m = cube_mesh(N, jitter=jitter, seed=seed)
    lat = m["lattice"]
    n = len(lat)
    dm = np.zeros((n, 4), np.uint8)
    dm[lat[:, 0] == 0, 0:3] = 1
    bf = boundary_faces(m["tets"])
    on_x1 = np.all(lat[bf][:, :, 0] == N, axis=1)
    tris = bf[on_x1]
    tr = np.tile(np.asarray(traction, np.float64), (len(tris), 1))
    mats = materials if materials is not None else [mooney_rivlin(c10, c01, kappa)]
    return Problem(m["X"], m["tets"], m["mat_id"], mats, dm, tris, tr, lat, None,
                   name=f"cube{N}")


def uniaxial_problem(N=2, kappa=1e4, c10=0.5, c01=0.1, stress=0.05, materials=None,
                     fibres=None):
    """Cube with roller supports (u_x=0 on x=0, u_y=0 on y=0, u_z=0 on z=0) and
    a dead normal traction ``stress`` in +x on x=1: a homogeneous state."""
    m = cube_mesh(N)
    lat = m["lattice"]
    n = len(lat)
    dm = np.zeros((n, 4), np.uint8)
    for c in range(3):
        dm[lat[:, c] == 0, c] = 1
    bf = boundary_faces(m["tets"])
    tris = bf[np.all(lat[bf][:, :, 0] == N, axis=1)]
    tr = np.tile(np.array([stress, 0.0, 0.0]), (len(tris), 1))
    mats = materials if materials is not None else [mooney_rivlin(c10, c01, kappa)]
    fib = None
    if fibres is not None:
        fib = np.tile(np.asarray(fibres, np.float64)[None], (len(m["tets"]), 1, 1))
    return Problem(m["X"], m["tets"], m["mat_id"], mats, dm, tris, tr, lat, fib,
                   name=f"uniaxial{N}")


ARTERY_MEDIA = dict(c10=3.0, k1=2.3632, k2=0.8393)
ARTERY_ADVENTITIA = dict(c10=0.3, k1=0.562, k2=0.7112)


def tube_problem(n_theta=64, n_media=5, n_adv=3, n_z=128, kappa=1e5, p_int=13.3, **kw):
    """Artery tube: u=0 on both ends z=0 and z=length; dead internal pressure
    p_int * e_r(centroid) on the inner surface (per unit reference area)."""
    m = tube_mesh(n_theta, n_media, n_adv, n_z, **kw)
    lat = m["lattice"]
    n = len(lat)
    dm = np.zeros((n, 4), np.uint8)
    ends = (lat[:, 2] == 0) | (lat[:, 2] == n_z)
    dm[ends, 0:3] = 1
    bf = boundary_faces(m["tets"])
    inner = np.all(lat[bf][:, :, 1] == 0, axis=1)
    tris = bf[inner]
    cen = m["X"][tris].mean(axis=1)
    rr = np.hypot(cen[:, 0], cen[:, 1])
    er = np.stack([cen[:, 0] / rr, cen[:, 1] / rr, np.zeros_like(rr)], axis=1)
    tr = p_int * er
    mats = [artery_layer(kappa=kappa, **ARTERY_MEDIA), artery_layer(kappa=kappa, **ARTERY_ADVENTITIA)]
    return Problem(m["X"], m["tets"], m["mat_id"], mats, dm, tris, tr, lat, m["fibres"],
                   name=f"tube{n_theta}x{n_media + n_adv}x{n_z}")


def random_state(prob: Problem, seed: int, u_scale=0.02, p_scale=0.1):
    """Seeded smooth-ish random state v [n,4] that satisfies the Dirichlet mask."""
    rng = np.random.default_rng(seed)
    n = prob.n_nodes
    X = prob.X
    ext = X.max(axis=0) - X.min(axis=0)
    # a random affine field plus small nodal noise keeps every element far from inversion
    Fm = rng.uniform(-1, 1, size=(3, 3)) * u_scale / max(ext.max(), 1e-12)
    v = np.zeros((n, 4))
    v[:, 0:3] = X @ Fm.T + rng.uniform(-1, 1, size=(n, 3)) * u_scale * 0.1
    v[:, 3] = rng.uniform(-1, 1, size=n) * p_scale
    v[prob.dir_mask.astype(bool)] = 0.0
    return v


def config_problem(name: str, kappa=None, N=None):
    """The solid workloads, by name:

    * ``cube8``  : 8^3 cube, Mooney-Rivlin c10=0.5 c01=0.1 kappa=1e4, clamped
      at x=0, dead traction (0,0,0.05) on x=1 (2,916 dofs);
    * ``cube48`` : the same physics on 48^3 hexahedra (470,596 dofs);
    * ``cube96`` : the same on 96^3 hexahedra (3,650,692 dofs);
    * ``tube``   : the two-layer artery tube 64 x 8 x 128 (297,216 dofs),
      kappa=1e5, internal dead pressure 13.3 at load factor 1.
    """
    if name.startswith("cube"):
        n = N if N is not None else int(name[4:])
        return cube_problem(n, kappa=1e4 if kappa is None else kappa)
    if name == "tube":
        return tube_problem(kappa=1e5 if kappa is None else kappa)
    if name.startswith("tube_small"):
        return tube_problem(n_theta=16, n_z=8, kappa=1e5 if kappa is None else kappa)
    raise ValueError(name)


__all__ = ["Problem", "cube_mesh", "tube_mesh", "boundary_faces", "cube_problem",
           "tube_problem", "uniaxial_problem", "random_state", "config_problem",
           "mooney_rivlin", "artery_layer", "KUHN_PERMS"]


# ---------------------------------------------------------------------------
# fluid-structure model: a straight duct with a compliant wall
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class FsiModel:
    """Matching fluid and structure meshes of a straight duct of square
    cross-section (lumen half-width ``half_width``) inside a wall of
    thickness ``wall``, axis z from 0 to ``length``; both meshes are subsets
    of one tensor lattice of hexahedra split into Kuhn tetrahedra, so the
    interface nodes coincide.

    Fluid: nodes ``fluid_X`` [nf,3], tetrahedra ``fluid_tets``; Dirichlet
    velocity on the interface nodes; inlet triangles on z = 0 (traction
    (0, 0, p_in) per unit area), do-nothing outlet on z = length.
    Structure: ``solid`` (a Problem with both ends clamped, no traction).
    Interface: ``iface_f`` / ``iface_s``, the interface nodes in fluid and
    structure numbering (same order).  ``fluid_boundary`` flags every fluid
    boundary node (the harmonic extension prescribes them all).
    """
    fluid_X: np.ndarray
    fluid_tets: np.ndarray
    fluid_dir: np.ndarray        # u8 [nf,4]: 1 = velocity dof prescribed (interface)
    inlet_tris: np.ndarray       # i32 [k,3] fluid inlet triangles
    fluid_boundary: np.ndarray   # bool [nf]
    solid: Problem
    iface_f: np.ndarray
    iface_s: np.ndarray
    fluid_lattice: np.ndarray
    inflow: np.ndarray | None = None   # f64 [nf,3] prescribed inlet velocity (Dirichlet), or None

    @property
    def nf(self):
        return self.fluid_X.shape[0]


def _graded(a, t, half_width, wall):
    """Lattice coordinates -(a+t) .. a+t: a cells of the lumen on each side
    of the axis, then t wall cells."""
    idx = np.arange(-(a + t), a + t + 1)
    s = np.abs(idx)
    x = np.where(s <= a, half_width * s / a, half_width + wall * (s - a) / max(t, 1))
    return idx, np.sign(idx) * x


def fsi_duct(a=3, t=2, n_z=36, half_width=1.43, wall=0.39, length=18.0, c10=3.0, c01=0.3, kappa=1e5,
             artery=False, media_cells=None):
    """FSI model of the paper's experiments (lengths in mm) on a square
    duct: a Mooney-Rivlin wall (c10 = 3 kPa, c01 = 0.3 kPa, kappa = 1e5 kPa),
    or with artery=True the two-layer artery (media on the inner
    media_cells wall rings, default two thirds of them rounded up,
    adventitia outside; the paper's constants and fibre angles, the fibres
    cos(alpha) e_theta +/- sin(alpha) e_z at each element's centroid)."""
    idx, coord = _graded(a, t, half_width, wall)
    nl = len(idx)
    k3, j3, i3 = np.meshgrid(np.arange(n_z + 1), np.arange(nl), np.arange(nl), indexing="ij")
    lat = np.stack([i3.ravel(), j3.ravel(), k3.ravel()], axis=1)
    X = np.stack([coord[lat[:, 0]], coord[lat[:, 1]], length * lat[:, 2] / n_z], axis=1)

    def node_id(i, j, k):
        return i + nl * (j + nl * k)

    tets, hex_ijk = _lattice_tets((nl - 1, nl - 1, n_z), node_id)
    tets = _orient(X, tets)
    hi, hj = hex_ijk[:, 0] - (a + t), hex_ijk[:, 1] - (a + t)   # cell lower corner in signed index
    fluid_cell = (hi >= -a) & (hi < a) & (hj >= -a) & (hj < a)

    def submesh(sel):
        T = tets[sel]
        used = np.unique(T)
        g2l = -np.ones(len(X), np.int64)
        g2l[used] = np.arange(len(used))
        return used, g2l[T].astype(np.int32)

    gf, Tf = submesh(fluid_cell)
    gs, Ts = submesh(~fluid_cell)
    both = np.intersect1d(gf, gs)
    iface_f = np.searchsorted(gf, both).astype(np.int64)
    iface_s = np.searchsorted(gs, both).astype(np.int64)
    # fluid boundary data
    latf = lat[gf]
    nf = len(gf)
    fdir = np.zeros((nf, 4), np.uint8)
    fdir[iface_f, 0:3] = 1
    bf = boundary_faces(Tf)
    inlet = bf[np.all(latf[bf][:, :, 2] == 0, axis=1)]
    fb = np.zeros(nf, bool)
    fb[np.unique(bf)] = True
    # structure: both ends clamped, loaded through the interface only
    lats = lat[gs]
    ns = len(gs)
    dm = np.zeros((ns, 4), np.uint8)
    dm[(lats[:, 2] == 0) | (lats[:, 2] == n_z), 0:3] = 1
    mats = [mooney_rivlin(c10, c01, kappa)]
    mat_id = np.zeros(len(Ts), np.int32)
    fib = None
    if artery:
        ring = np.maximum(np.abs(hi[~fluid_cell] + 0.5), np.abs(hj[~fluid_cell] + 0.5)) - 0.5 - a  # 0 .. t-1
        nm = media_cells if media_cells is not None else -(-2 * t // 3)
        mat_id = (ring >= nm).astype(np.int32)
        mats = [artery_layer(kappa=kappa, **ARTERY_MEDIA), artery_layer(kappa=kappa, **ARTERY_ADVENTITIA)]
        cen = X[gs][Ts].mean(axis=1)
        rr = np.hypot(cen[:, 0], cen[:, 1])
        e_t = np.stack([-cen[:, 1] / rr, cen[:, 0] / rr, np.zeros_like(rr)], axis=1)
        e_z = np.tile(np.array([0.0, 0.0, 1.0]), (len(Ts), 1))
        alpha = np.where(mat_id == 0, math.radians(29.0), math.radians(62.0))[:, None]
        fib = np.stack([np.cos(alpha) * e_t + np.sin(alpha) * e_z, np.cos(alpha) * e_t - np.sin(alpha) * e_z], axis=1)
    solid = Problem(X[gs], Ts, mat_id, mats, dm, np.zeros((0, 3), np.int32), np.zeros((0, 3)),
                    lats.astype(np.int32), fib, name=f"duct_wall{a}x{t}x{n_z}" + ("_artery" if artery else ""))
    return FsiModel(X[gf], Tf, fdir, inlet.astype(np.int32), fb, solid, iface_f, iface_s,
                    latf.astype(np.int32))


def lumen_mesh(n_theta=64, n_r=16, n_z=128, radius=0.71, length=5.0):
    """Structured mesh of the tube's lumen (the disk of the given radius
    times [0, length]): n_r rings of n_theta nodes around an axis node per
    level, the same circumferential and axial positions as the tube's inner
    surface.  Between ring k >= 1 and ring k + 1 the (theta, r, z) lattice
    hexahedra are Kuhn-split as the tube's; the wedges around the axis are
    split into three tetrahedra whose quad-face diagonals match: on the
    outer face the Kuhn diagonal (theta_j, z_c)-(theta_j+1, z_c+1), on the
    radial faces the diagonal from the axis node at z_c to the ring node at
    z_c+1.  Node index: level c holds the axis node c * (1 + n_theta * n_r)
    and then ring k, angle j at c * (1 + n_theta n_r) + 1 + (k - 1) n_theta + j.
    Returns X, tets (positively oriented), and the lattice (j, k, c) of each
    node (j = 0 on the axis)."""
    per = 1 + n_theta * n_r
    c, k, j = np.meshgrid(np.arange(n_z + 1), np.arange(1, n_r + 1), np.arange(n_theta), indexing="ij")
    n = per * (n_z + 1)
    X = np.zeros((n, 3))
    lat = np.zeros((n, 3), np.int32)
    axis = np.arange(n_z + 1) * per
    X[axis, 2] = length * np.arange(n_z + 1) / n_z
    lat[axis, 2] = np.arange(n_z + 1)
    ring = (c * per + 1 + (k - 1) * n_theta + j).ravel()
    th = 2.0 * math.pi * j.ravel() / n_theta
    r = radius * k.ravel() / n_r
    X[ring] = np.stack([r * np.cos(th), r * np.sin(th), length * c.ravel() / n_z], axis=1)
    lat[ring] = np.stack([j.ravel(), k.ravel(), c.ravel()], axis=1)

    def node_id(ia, ib, ic):
        # (theta, ring, level) with ring >= 1, theta periodic
        return ic * per + 1 + (ib - 1) * n_theta + (ia % n_theta)

    # rings 1..n_r: hexahedra between ring b and b + 1 (b = 1 .. n_r - 1)
    tets_h = np.zeros((0, 4), np.int64)
    if n_r > 1:
        th_, _ = _lattice_tets((n_theta, n_r - 1, n_z), lambda a, b, cc: node_id(a, b + 1, cc))
        tets_h = th_
    # wedges around the axis: (C0, A0, B0, B1), (C0, A0, A1, B1), (C0, A1, B1, C1)
    cc, aa = np.meshgrid(np.arange(n_z), np.arange(n_theta), indexing="ij")
    cc, aa = cc.ravel(), aa.ravel()
    C0, C1 = cc * per, (cc + 1) * per
    A0, A1 = node_id(aa, 1, cc), node_id(aa, 1, cc + 1)
    B0, B1 = node_id(aa + 1, 1, cc), node_id(aa + 1, 1, cc + 1)
    tets_w = np.concatenate([np.stack([C0, A0, B0, B1], 1), np.stack([C0, A0, A1, B1], 1),
                             np.stack([C0, A1, B1, C1], 1)])
    tets = np.concatenate([tets_w, tets_h]).astype(np.int64)
    tets = _orient(X, tets)
    return X, tets.astype(np.int32), lat


def fsi_tube(n_theta=64, n_r=16, n_media=5, n_adv=3, n_z=128, r_in=0.71, length=5.0, v_peak=0.3, kappa=1e5):
    """The artery tube with its lumen as a partitioned FSI model: the
    structure is the two-layer tube (both ends clamped, no traction), the
    fluid the lumen mesh whose outer ring is the tube's inner surface; a
    Poiseuille inflow u = v_peak (1 - r^2 / r_in^2) e_z is prescribed on the
    inlet z = 0, the outlet z = length is free (do nothing).  Lengths in mm,
    velocities in mm/ms (v_peak = 0.3 is 30 cm/s)."""
    tm = tube_mesh(n_theta, n_media, n_adv, n_z, r_in=r_in, length=length)
    Xf, Tf, latf = lumen_mesh(n_theta, n_r, n_z, r_in, length)
    nf = len(Xf)
    # interface: fluid ring n_r <-> tube radial index 0, same (theta, level)
    jj, cc = np.meshgrid(np.arange(n_theta), np.arange(n_z + 1), indexing="ij")
    jj, cc = jj.ravel(), cc.ravel()
    per = 1 + n_theta * n_r
    iface_f = (cc * per + 1 + (n_r - 1) * n_theta + jj).astype(np.int64)
    n_rad = n_media + n_adv + 1
    iface_s = (jj + n_theta * (0 + n_rad * cc)).astype(np.int64)
    order = np.argsort(iface_f)
    iface_f, iface_s = iface_f[order], iface_s[order]
    assert np.abs(Xf[iface_f] - tm["X"][iface_s]).max() < 1e-12
    fdir = np.zeros((nf, 4), np.uint8)
    fdir[iface_f, 0:3] = 1
    inlet_nodes = np.flatnonzero(latf[:, 2] == 0)
    fdir[inlet_nodes, 0:3] = 1
    inflow = np.zeros((nf, 3))
    rr2 = Xf[inlet_nodes, 0] ** 2 + Xf[inlet_nodes, 1] ** 2
    inflow[inlet_nodes, 2] = v_peak * np.maximum(0.0, 1.0 - rr2 / (r_in * r_in))
    inflow[iface_f] = 0.0
    bf = boundary_faces(Tf)
    fb = np.zeros(nf, bool)
    fb[np.unique(bf)] = True
    lat_s = tm["lattice"]
    ns = len(lat_s)
    dm = np.zeros((ns, 4), np.uint8)
    dm[(lat_s[:, 2] == 0) | (lat_s[:, 2] == n_z), 0:3] = 1
    mats = [artery_layer(kappa=kappa, **ARTERY_MEDIA), artery_layer(kappa=kappa, **ARTERY_ADVENTITIA)]
    solid = Problem(tm["X"], tm["tets"], tm["mat_id"], mats, dm, np.zeros((0, 3), np.int32), np.zeros((0, 3)),
                    lat_s, tm["fibres"], name=f"tube{n_theta}x{n_media + n_adv}x{n_z}")
    return FsiModel(Xf, Tf, fdir, np.zeros((0, 3), np.int32), fb, solid, iface_f, iface_s, latf, inflow)
