"""Compressible Navier-Stokes right-hand side with the viscous and heat fluxes
through aRDG, FP64.  TEST INFRASTRUCTURE ONLY.

Follows the subsection "Navier-Stokes equations": Q = (rho, rho u, rho v, E),
the inviscid fluxes F_i and the viscous fluxes G_i of eq. aRDG_Navier_Stokes,
the viscous stress of eq. NS_viscosity, the heat flux of eq. NS_heatflux,
Sutherland's law for mu, kappa = Cp mu / Pr, and a Lax-Friedrichs flux for
the hyperbolic terms.  The equation is d Q/dt + div(F + G) = 0, written in
the weak form of the nodal DG method (as the scalar oracle).

Readings of places the paper leaves open:

* Ideal gas: p = (gamma - 1) (E - rho |u|^2 / 2), T = p / (rho R),
  Cp = gamma R / (gamma - 1); Sutherland: mu = mu_ref (T / T_ref)^(3/2)
  (T_ref + S) / (T + S).
* Lax-Friedrichs at each face node: F* . n = (F(Q-) + F(Q+)) . n / 2 -
  lambda (Q+ - Q-) / 2 with lambda = max(|u- . n| + c-, |u+ . n| + c+).
* How aRDG enters the viscous terms (the paper names the method, not the
  variables): the primitive fields u, v and T are formed at every element's
  nodes and reconstructed, each with the same least-squares operator as a
  scalar (Algorithm aRDG), on the enclosed parallelogram of each edge; at
  the diagonal nodes mu and kappa are evaluated from the reconstructed T
  (as the reconstructed coefficient of the alternative form) and the
  interface viscous flux is G . n1 of the reconstructed velocity and
  temperature gradients and values.  In the volume term G is formed at the
  nodes from each element's own nodal primitives and their nodal gradients.
* Boundary faces carry a prescribed exterior state Q_ext(x, y, t): its
  primitives on the ghost sub-triangle enter the reconstruction, and Q_ext
  at the face nodes is the Lax-Friedrichs outer state.
"""
from __future__ import annotations

import numpy as np

from . import ardg
from .mesh import Geometry
from .reference_element import RefOps


class Gas:
    """Ideal gas with Sutherland viscosity."""

    def __init__(self, gamma=1.4, R=1.0, Pr=0.7, mu_ref=1e-2, T_ref=1.0, S=0.4,
                 law: str = "sutherland"):
        if law not in ("sutherland", "constant"):
            raise ValueError("law is 'sutherland' or 'constant'")
        self.gamma, self.R, self.Pr = gamma, R, Pr
        self.mu_ref, self.T_ref, self.S = mu_ref, T_ref, S
        self.law = law
        self.cp = gamma * R / (gamma - 1.0)

    def primitives(self, Q):
        """(rho, u, v, p, T) from Q [4, ...]."""
        rho = Q[0]
        u, v = Q[1] / rho, Q[2] / rho
        p = (self.gamma - 1.0) * (Q[3] - 0.5 * rho * (u * u + v * v))
        return rho, u, v, p, p / (rho * self.R)

    def mu(self, T):
        if self.law == "constant":
            return self.mu_ref + 0.0 * T
        return self.mu_ref * (T / self.T_ref) ** 1.5 * (self.T_ref + self.S) / (T + self.S)

    def kappa(self, T):
        return self.cp * self.mu(T) / self.Pr

    def inviscid(self, Q):
        """(F_x, F_y), each [4, ...] (eq. aRDG_Navier_Stokes)."""
        rho, u, v, p, _ = self.primitives(Q)
        Fx = np.stack([rho * u, rho * u * u + p, rho * u * v, (Q[3] + p) * u])
        Fy = np.stack([rho * v, rho * u * v, rho * v * v + p, (Q[3] + p) * v])
        return Fx, Fy

    def viscous(self, u, v, T, ux, uy, vx, vy, Tx, Ty):
        """(G_x, G_y), each [4, ...], from the primitive values and gradients
        (eqs. aRDG_Navier_Stokes, NS_viscosity, NS_heatflux)."""
        mu, kap = self.mu(T), self.kappa(T)
        div = ux + vy
        Pxx = mu * (2.0 * ux - 2.0 / 3.0 * div)
        Pyy = mu * (2.0 * vy - 2.0 / 3.0 * div)
        Pxy = mu * (uy + vx)
        qx, qy = -kap * Tx, -kap * Ty
        z = 0.0 * u
        Gx = np.stack([z, -Pxx, -Pxy, -(u * Pxx + v * Pxy) + qx])
        Gy = np.stack([z, -Pxy, -Pyy, -(u * Pxy + v * Pyy) + qy])
        return Gx, Gy

    def sound_speed(self, Q):
        rho, _, _, p, _ = self.primitives(Q)
        return np.sqrt(self.gamma * p / rho)


class NavierStokes:
    """The semi-discrete compressible Navier-Stokes system on a triangle mesh.

    exterior: callable (x, y, t) -> Q [4, ...], the prescribed state outside
    the domain (used at boundary faces).  build_edges=False skips the
    per-edge geometry of the whole mesh (rhs_elements builds what it needs
    edge by edge), for sampled checks on large meshes.
    """

    def __init__(self, vxy, etov, N: int, gas: Gas, exterior, build_edges: bool = True):
        self.geom = Geometry(vxy, etov)
        self.ops = RefOps(N)
        self.N = N
        self.gas = gas
        self.exterior = exterior
        g = self.geom
        self.int_geom = self.bdy_geom = None
        if build_edges:
            self.int_geom = [ardg.interior_edge_geometry(g, k1, f1, k2, f2) for (k1, f1, k2, f2) in g.interior]
            self.bdy_geom = [ardg.boundary_edge_geometry(g, k1, f1) for (k1, f1) in g.boundary]

    def nodal_xy(self):
        return self.geom.physical(self.ops.rs)

    # -- reconstruction of one primitive field on one edge -------------------
    def _recon(self, eg, m1, m2):
        """Values and physical gradient of u~ = RDG at the diagonal nodes from
        modal data m_k on Omega'_k."""
        N, Np = self.N, self.ops.Np
        R = ardg.recon_pinv(N)
        c = R[:, :Np] @ m1 + R[:, Np:] @ m2
        E0, ER, ES = ardg.diagonal_eval(N)
        val = E0 @ c
        dR, dS = ER @ c, ES @ c
        return val, eg.Rx * dR + eg.Sx * dS, eg.Ry * dR + eg.Sy * dS

    def _viscous_normal_flux(self, eg, m_sides):
        """G . n1 at the diagonal nodes [4, Nfp] from the modal data on the
        sub-triangles of (u, v, T): m_sides = [(m1, m2) for u, v, T]."""
        (u, ux, uy), (v, vx, vy), (T, Tx, Ty) = (self._recon(eg, a, b) for (a, b) in m_sides)
        Gx, Gy = self.gas.viscous(u, v, T, ux, uy, vx, vy, Tx, Ty)
        return eg.n1[0] * Gx + eg.n1[1] * Gy

    def _lf(self, QL, QR, n):
        """Lax-Friedrichs F* . n [4, Nfp] from the two states at the face
        nodes (n the outward normal of the left state)."""
        FxL, FyL = self.gas.inviscid(QL)
        FxR, FyR = self.gas.inviscid(QR)
        _, uL, vL, _, _ = self.gas.primitives(QL)
        _, uR, vR, _, _ = self.gas.primitives(QR)
        lam = np.maximum(np.abs(uL * n[0] + vL * n[1]) + self.gas.sound_speed(QL),
                         np.abs(uR * n[0] + vR * n[1]) + self.gas.sound_speed(QR))
        return 0.5 * (n[0] * (FxL + FxR) + n[1] * (FyL + FyR)) - 0.5 * lam * (QR - QL)

    # -- face fluxes -----------------------------------------------------------
    def _interior_H(self, Q, P, k1, f1, k2, f2, eg):
        """(F + G)* . n1 [4, Nfp] of one interior edge, side-1 node order."""
        ops = self.ops
        T1 = ardg.total_projection(ops, eg.pi1, f1)
        T2 = ardg.total_projection(ops, eg.pi2, f2)
        Gn = self._viscous_normal_flux(eg, [(T1 @ p[k1], T2 @ p[k2]) for p in P])
        QL = Q[:, k1][:, ops.fmask[f1]]
        QR = Q[:, k2][:, ops.fmask[f2]][:, ::-1]
        return self._lf(QL, QR, eg.n1) + Gn

    def _boundary_H(self, Q, P, k1, f1, eg, t):
        """(F + G)* . n1 [4, Nfp] of one boundary face with the prescribed
        exterior state on the ghost sub-triangle and at the face nodes."""
        ops = self.ops
        T1 = ardg.total_projection(ops, eg.pi1, f1)
        Xg = ardg.ghost_nodes(self.N, eg)
        Qg = np.asarray(self.exterior(Xg[:, 0], Xg[:, 1], t))
        _, ug, vg, _, Tg = self.gas.primitives(Qg)
        Gn = self._viscous_normal_flux(eg, [(T1 @ p[k1], ops.Vinv @ pg)
                                            for p, pg in zip(P, (ug, vg, Tg))])
        Xf = self.geom.physical(ops.rs)[k1, ops.fmask[f1]]
        QL = Q[:, k1][:, ops.fmask[f1]]
        QR = np.asarray(self.exterior(Xf[:, 0], Xf[:, 1], t))
        return self._lf(QL, QR, eg.n1) + Gn

    def _primitive_fields(self, Q):
        _, u, v, _, T = self.gas.primitives(Q)
        return [u, v, T]

    def face_fluxes(self, Q, t):
        """[K, 3, 4, Nfp] numerical flux (F + G)* . n of every element face in
        its own counter-clockwise order and outward normal: side 1 reads the
        edge's flux as is, side 2 negated and in reverse order."""
        g = self.geom
        if self.int_geom is None:
            raise RuntimeError("face_fluxes needs the edge geometry (build_edges=True)")
        P = self._primitive_fields(Q)
        out = np.zeros((g.K, 3, 4, self.ops.Nfp))
        for e, (k1, f1, k2, f2) in enumerate(g.interior):
            H = self._interior_H(Q, P, k1, f1, k2, f2, self.int_geom[e])
            out[k1, f1] = H
            out[k2, f2] = -H[:, ::-1]
        for e, (k1, f1) in enumerate(g.boundary):
            out[k1, f1] = self._boundary_H(Q, P, k1, f1, self.bdy_geom[e], t)
        return out

    def face_flux_one(self, Q, k, f, t, P=None):
        """The flux seen by face f of element k alone (same steps, one edge);
        P: the primitive fields of Q if already formed."""
        g = self.geom
        P = self._primitive_fields(Q) if P is None else P
        k2 = int(g.EToE[k, f])
        if k2 < 0:
            return self._boundary_H(Q, P, k, f, ardg.boundary_edge_geometry(g, k, f), t)
        f2 = int(g.EToF[k, f])
        if k < k2:
            return self._interior_H(Q, P, k, f, k2, f2, ardg.interior_edge_geometry(g, k, f, k2, f2))
        H = self._interior_H(Q, P, k2, f2, k, f, ardg.interior_edge_geometry(g, k2, f2, k, f))
        return -H[:, ::-1]

    # -- right-hand side -------------------------------------------------------
    def _volume(self, Q, els):
        """(r_x Drw + s_x Dsw) H_x + (r_y Drw + s_y Dsw) H_y [4, len(els), Np]
        with H = F + G formed at the nodes from each element's own data."""
        ops, g, gas = self.ops, self.geom, self.gas
        rx, ry, sx, sy = (a[els][:, None] for a in (g.rx, g.ry, g.sx, g.sy))
        Qe = Q[:, els]
        _, u, v, _, T = gas.primitives(Qe)

        def grad(f):
            fr, fs = f @ ops.Dr.T, f @ ops.Ds.T
            return rx * fr + sx * fs, ry * fr + sy * fs
        ux, uy = grad(u)
        vx, vy = grad(v)
        Tx, Ty = grad(T)
        Fx, Fy = gas.inviscid(Qe)
        Gx, Gy = gas.viscous(u, v, T, ux, uy, vx, vy, Tx, Ty)
        Hx, Hy = Fx + Gx, Fy + Gy
        return (rx[None] * (Hx @ ops.Drw.T) + sx[None] * (Hx @ ops.Dsw.T)
                + ry[None] * (Hy @ ops.Drw.T) + sy[None] * (Hy @ ops.Dsw.T))

    def _lift(self, Hs, els):
        """sum_f (sJ_f / J) LIFT_f H*_f from face fluxes [len(els), 3, 4, Nfp]."""
        ops, g = self.ops, self.geom
        surf = 0.0
        for f in range(3):
            scale = (g.sJ[els, f] / g.J[els])[None, :, None]
            Lf = ops.LIFT[:, f * ops.Nfp:(f + 1) * ops.Nfp]
            surf = surf + scale * np.einsum("kcj,ij->cki", Hs[:, f], Lf)
        return surf

    def rhs(self, Q, t: float = 0.0):
        """dQ/dt [4, K, Np]: the weak form of dQ/dt = -div(F + G),
        volume term minus the lifted face fluxes."""
        els = np.arange(self.geom.K)
        return self._volume(Q, els) - self._lift(self.face_fluxes(Q, t), els)

    def rhs_elements(self, Q, elements, t: float = 0.0):
        """dQ/dt on the listed elements only [4, len(elements), Np], each face
        flux computed for its edge alone (sampled checks on large meshes)."""
        els = np.asarray(elements, dtype=np.int64)
        P = self._primitive_fields(Q)
        Hs = np.array([[self.face_flux_one(Q, int(k), f, t, P) for f in range(3)] for k in els])
        return self._volume(Q, els) - self._lift(Hs, els)
