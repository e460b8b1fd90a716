"""Partitioned fluid-structure time step: the Dirichlet-Neumann iteration with
Aitken relaxation (oracle; test infrastructure only).

Section "A Dirichlet-Neumann FSI iteration": each DN iteration
  1. extends the interface displacement d_G harmonically into the fluid
     mesh (eq. harext), giving the current fluid mesh and the mesh velocity
     w = (d_f - d_f^{n-1}) / dt (eq. hartdis);
  2. solves the fluid step (eq. stabweakfluid) by Newton's method with the
     velocity w prescribed on the interface;
  3. takes the fluid's force on the interface and solves the structure step
     (eq. stabweakelas with the Newmark-beta inertia) by Newton's method.
The interface residual r_k = d~_G,k - d_G,k-1 (the new structure
displacement on the interface minus the one the fluid step used) stops the
iteration when |r_k| / sqrt(n_G) < eps (n_G interface vertices, |.| the
Euclidean norm of the 3 n_G components).  Section "Aitken relaxation":
d_G,k = omega_{k-1} d~_G,k + (1 - omega_{k-1}) d_G,k-1 (eq. acceit), with
omega_k = -omega_{k-1} r_k . (r_{k+1} - r_k) / |r_{k+1} - r_k|^2
(eq. dnomega).

Readings (the paper leaves them to its reference):
* the first relaxation factor of every time step is a parameter omega0;
* the first DN iteration of a time step starts from the interface
  displacement extrapolated to the new time level with the structure's
  velocity, d_G^(0) = d^{n-1} + dt v^{n-1} on the interface (the paper
  extrapolates the fluid domain from the previous iterates; a constant
  start lets the fluid see a wall stopped at once, whose added-mass force
  inverts the wall on the duct after a few steps of the pulse);
* the nested Newton solves start from the latest iterate of their own
  sub-problem and use the stopping rule of eq. newstop (eps_2 = 1e-10),
  each linear system solved directly here; the reference of the rule is
  the first correction of the sub-problem's solve in the first DN
  iteration of the time step (the later, warm-started solves have small
  first corrections whose relative reduction would sink below rounding);
* when the iteration stops, the step keeps the fluid and mesh states of its
  last fluid solve and the structure state of its last structure solve.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse.linalg as spl

from . import fe, fluid, newmark, newton


@dataclasses.dataclass
class FsiParams:
    fluid: fluid.FluidParams = dataclasses.field(default_factory=fluid.FluidParams)
    rho_s: float = 1.2            # mg / mm^3
    beta: float = 0.625
    gamma: float = 1.0
    p_in: float = 1.332           # kPa, inlet traction (0, 0, p_in)
    t_pulse: float = 1.0          # ms: the inlet traction acts while t <= t_pulse
    omega0: float = 0.5
    eps: float = 1e-8
    max_dn: int = 100
    eps2: float = 1e-10


def aitken(omega_prev, r_prev, r):
    """Next relaxation factor (eq. dnomega) from the last two interface
    residuals."""
    dr = r - r_prev
    return -omega_prev * float(np.dot(r_prev, dr)) / float(np.dot(dr, dr))


def dn_iterate(evaluate, d0, n_vertices, omega0, eps, max_it, log=None):
    """Fixed-point iteration d = evaluate(d) with Aitken relaxation
    (eq. fixepr, eq. acceit, eq. dnomega): r_k = evaluate(d_{k-1}) -
    d_{k-1}, stop when |r_k| / sqrt(n_vertices) < eps, else d_k = d_{k-1} +
    omega_{k-1} r_k.  Returns (iterations, omegas, norms)."""
    d = np.asarray(d0, np.float64).copy()
    omegas, norms = [], []
    r_prev = omega = None
    for k in range(1, max_it + 1):
        r = evaluate(d) - d
        norms.append(float(np.linalg.norm(r)) / np.sqrt(n_vertices))
        if log is not None:
            log(f"DN {k}: |r|/sqrt(n) = {norms[-1]:.3e}")
        if norms[-1] < eps:
            return k, omegas, norms
        omega = omega0 if r_prev is None else aitken(omega, r_prev, r)
        omegas.append(omega)
        d = d + omega * r
        r_prev = r
    raise RuntimeError("DN iteration did not converge")


def solid_newton(disc: fe.Discretization, v, eps2=1e-10, max_iter=25, ref=None):
    """Newton's method for the structure at load factor 1 (the loads in
    disc.f_ext), direct linear solves, the stopping rule of eq. newstop with
    the reference ref (default: this solve's first correction) and the
    rounding floor of the first correction.  Returns (v, iterations,
    ||dv_0||_M)."""
    v = np.asarray(v, np.float64).ravel().copy()
    floor = newton.FLOOR * disc.mass_norm(v)
    n0 = None
    for k in range(max_iter):
        R, val = disc.assemble(v, 1.0)
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
    raise RuntimeError("structure Newton did not converge")


class FsiState:
    """The coupled problem of an FsiModel and its state at the last time
    level: structure v_s [ns,4] with nodal velocity and acceleration, fluid
    v_f [nf,4], fluid mesh displacement d_f [nf,3]."""

    def __init__(self, model, prm: FsiParams | None = None):
        prm = FsiParams() if prm is None else prm   # a state owns its parameters (omega0 may change per step)
        self.model, self.prm = model, prm
        self.fd = fluid.FluidDiscretization(model.fluid_X, model.fluid_tets, model.fluid_dir, model.inlet_tris,
                                            prm.fluid)
        self.sd = fe.Discretization(model.solid)
        self.L = fluid.laplacian(model.fluid_X, model.fluid_tets)
        self.fixed = np.flatnonzero(model.fluid_boundary)
        ns, nf = model.solid.n_nodes, model.nf
        self.vs = np.zeros((ns, 4))
        self.vel = np.zeros((ns, 3))
        self.acc = np.zeros((ns, 3))
        self.vf = np.zeros((nf, 4))
        if getattr(model, "inflow", None) is not None:   # prescribed inlet velocity (kept by every step)
            self.vf[:, 0:3] = model.inflow
        self.df = np.zeros((nf, 3))
        self.t = 0.0
        self.nm = newmark.NewmarkParams(rho=prm.rho_s, dt=prm.fluid.dt, beta=prm.beta, gamma=prm.gamma)
        # position of each interface node among the extension's fixed nodes
        self._fix_pos = np.searchsorted(self.fixed, model.iface_f)

    def extension(self, dG):
        vals = np.zeros((len(self.fixed), 3))
        vals[self._fix_pos] = dG
        return fluid.harmonic_extension(self.L, self.fixed, vals)

    def time_step(self, log=None):
        """Advance one time step; returns (DN iterations, omegas, residual
        norms |r_k| / sqrt(n_G))."""
        prm, m = self.prm, self.model
        dt = prm.fluid.dt
        t = self.t + dt
        g_in = np.array([0.0, 0.0, prm.p_in if t <= prm.t_pulse + 1e-12 else 0.0])
        d_prev = self.vs[:, 0:3].copy()
        self.sd.set_inertia(newmark.coefficient(self.nm), newmark.history(self.nm, d_prev, self.vel, self.acc))
        u_old = self.vf[:, 0:3].copy()
        nG = len(m.iface_f)
        cur = dict(vf=self.vf.copy(), vs=self.vs.copy(), df=None, ref_f=None, ref_s=None)

        def evaluate(dG):
            df = self.extension(dG.reshape(nG, 3))
            w = (df - self.df) / dt
            vf = cur["vf"].reshape(-1, 4).copy()
            vf[m.iface_f, 0:3] = w[m.iface_f]
            vf, _, n0 = fluid.newton_solve(self.fd, vf, df, u_old, w, g_in, eps2=prm.eps2, ref=cur["ref_f"])
            cur["ref_f"] = n0 if cur["ref_f"] is None else cur["ref_f"]
            f = fluid.interface_force(self.fd, vf, df, u_old, w, g_in, m.iface_f)
            self.sd.f_ext = np.zeros((m.solid.n_nodes, 3))
            self.sd.f_ext[m.iface_s] = f
            vs, _, n0 = solid_newton(self.sd, cur["vs"], prm.eps2, ref=cur["ref_s"])
            cur["ref_s"] = n0 if cur["ref_s"] is None else cur["ref_s"]
            cur.update(vf=vf, vs=vs, df=df)
            return vs.reshape(-1, 4)[m.iface_s, 0:3].ravel()

        d0 = self.vs[m.iface_s, 0:3] + dt * self.vel[m.iface_s]
        k, omegas, norms = dn_iterate(evaluate, d0.ravel(), nG, prm.omega0, prm.eps,
                                      prm.max_dn, None if log is None else (lambda s: log(f"t={t:.4f} " + s)))
        vf, vs, df = cur["vf"], cur["vs"], cur["df"]
        vs = vs.reshape(-1, 4)
        vel, acc = newmark.update(self.nm, vs[:, 0:3], d_prev, self.vel, self.acc)
        self.vs, self.vel, self.acc = vs, vel, acc
        self.vf, self.df, self.t = vf.reshape(-1, 4), df, t
        return k, omegas, norms
