"""Semi-discrete right-hand side, time stepping and error norms, FP64.

TEST INFRASTRUCTURE ONLY.

* Diffusion: the fully reference form (eq.
  NDG_diffusion_once_matrixForm_Fullyreference), in weak form,
      du/dt = -D [ (r_x Drw + s_x Dsw) q_x + (r_y Drw + s_y Dsw) q_y ]
              + sum_f (J_f / J) LIFT_f F_f ,
  q = (r_x Dr + s_x Ds, r_y Dr + s_y Ds) u, Drw = M^{-1} Dr^T M, with F_f the
  reconstructed flux (D included) and J_f = |edge| / 2 with LIFT built from the
  1D mass matrix on [-1, 1] (reading of "ratio between the lengths").  The
  element's own geometric factors are kept in the volume term (eq. for S^k).
  With an element-wise D the volume term carries D_k and the flux comes from
  Algorithm 1 (eq. NDG_diffusion_once_matrixForm_reference_general) or, with
  alg=2, from Algorithm 2 (eq.
  NDG_diffusion_once_matrixForm_reference_general_alternative).
* Convection (the v.grad part of eq. convection_diffusion): nodal collocation
  of v u, weak form, upwind numerical flux f* = max(n.v,0) u- + min(n.v,0) u+,
  with u+ = 0 outside the domain.  The velocity is affine, v(x) = v0 + W x.
* Boundary faces: zero Dirichlet data through the mirror ghost, or, when a
  ghost state g(x, y, t, field) is given, the prescribed exterior state on
  the ghost sub-triangle (the flux then has a part linear in g; the upwind
  flux takes u+ = g at the face nodes).
* Time stepping: classic four-stage RK4 and the five-stage fourth-order
  low-storage RK of Carpenter and Kennedy (the paper's integrator), with the
  stage times c_s where the right-hand side depends on time (through the
  boundary data).
* Norms: cell-normalised L2 and L_inf (eqs. L2_norm_cellUnit,
  Linf_norm_cellUnit) by collapsed Gauss quadrature.
"""
from __future__ import annotations

import numpy as np

from . import ardg
from .mesh import Geometry
from .reference_element import RefOps, vandermonde


class Problem:
    """A mesh, an order N, diffusion coefficients and an optional velocity.

    D_mode: "const" (D is a float, or a list with one value per field),
    "element" (D is an array [K]; flux by Algorithm 1, or Algorithm 2 when
    alg=2), "nodal" (D is an array [K, Np, 3] of the symmetric tensor
    (Dxx, Dxy, Dyy) at each element's nodes; Algorithm 1 with nodal products)
    or "solution" (D is (D0xx, D0xy, D0yy) and the coefficient is u D0).
    ghost: None (zero Dirichlet, mirror ghost) or a callable g(x, y, t,
    field) giving the prescribed exterior state.
    """

    def __init__(self, vxy, etov, N: int, D, D_mode: str = "const",
                 velocity=None, nfields: int = 1, build_edges: bool = True, alg: int = 1,
                 ghost=None):
        self.geom = Geometry(vxy, etov)
        self.ops = RefOps(N)
        self.N = N
        self.nfields = nfields
        self.D_mode = D_mode
        if alg not in (1, 2):
            raise ValueError("alg must be 1 or 2")
        self.alg = alg
        if D_mode == "const":
            Dv = np.atleast_1d(np.asarray(D, dtype=np.float64))
            if Dv.size == 1:
                Dv = np.repeat(Dv, nfields)
            self.Dfield = Dv
        elif D_mode == "element":
            if nfields != 1:
                raise ValueError("element-wise D is for one field")
            self.Delem = np.asarray(D, dtype=np.float64)
        elif D_mode == "nodal":
            if nfields != 1:
                raise ValueError("nodal D is for one field")
            self.Dnodal = np.asarray(D, dtype=np.float64)
        elif D_mode == "solution":
            if nfields != 1:
                raise ValueError("solution-dependent D is for one field")
            self.D0 = np.asarray(D, dtype=np.float64).reshape(3)
        else:
            raise ValueError(D_mode)
        self.velocity = velocity   # None or (v0x, v0y, W11, W12, W21, W22)
        self.ghost = ghost
        if build_edges:
            self._build_edges()

    # -- per-edge operators (literal Algorithm aRDG / Algorithm 1) -----------
    def _build_edges(self):
        g, ops = self.geom, self.ops
        self.int_edges = g.interior
        self.bdy_edges = g.boundary
        E1, E2 = [], []
        self.edge_geom = []
        tensor = self.D_mode in ("nodal", "solution")
        for (k1, f1, k2, f2) in self.int_edges:
            eg = ardg.interior_edge_geometry(g, k1, f1, k2, f2)
            self.edge_geom.append(eg)
            if tensor:
                continue       # the flux is formed from the data on each call
            if self.D_mode == "element":
                W1, W2 = self._element_edge_operator(eg, f1, f2, k1, k2)
            else:
                W1, W2 = ardg.edge_operator(ops, eg, f1, f2)
            E1.append(W1)
            E2.append(W2)
        self.W1 = np.array(E1).reshape(-1, ops.Nfp, ops.Np)
        self.W2 = np.array(E2).reshape(-1, ops.Nfp, ops.Np)
        B, G, GX = [], [], []
        self.bdy_geom = []
        for (k1, f1) in self.bdy_edges:
            eg = ardg.boundary_edge_geometry(g, k1, f1)
            self.bdy_geom.append(eg)
            if tensor:
                GX.append(ardg.ghost_nodes(ops.N, eg))
                continue
            if self.ghost is not None:
                W1, WG = self._prescribed_operators(k1, f1, eg)
                B.append(W1)
                G.append(WG)
                GX.append(ardg.ghost_nodes(ops.N, eg))
            elif self.D_mode == "element":
                B.append(self._element_boundary_operator(k1, f1, eg))
            else:
                B.append(ardg.boundary_edge_operator(ops, g, k1, f1, eg))
        self.WB = np.array(B).reshape(-1, ops.Nfp, ops.Np)
        self.WG = np.array(G).reshape(-1, ops.Nfp, ops.Np)
        self.GX = np.array(GX).reshape(-1, ops.Np, 2)

    def _element_edge_operator(self, eg, f1, f2, k1, k2):
        alg = ardg.edge_operator_alg2 if self.alg == 2 else ardg.edge_operator_alg1
        return alg(self.ops, eg, f1, f2, self.Delem[k1], self.Delem[k2])

    def _element_boundary_operator(self, k1, f1, eg):
        alg = ardg.boundary_edge_operator_alg2 if self.alg == 2 else ardg.boundary_edge_operator_alg1
        return alg(self.ops, self.geom, k1, f1, eg, self.Delem[k1])

    def _prescribed_operators(self, k1, f1, eg):
        if self.D_mode != "element":
            return ardg.prescribed_boundary_operators(self.ops, eg, f1)
        alg = ardg.prescribed_boundary_operators_alg2 if self.alg == 2 else ardg.prescribed_boundary_operators_alg1
        return alg(self.ops, eg, f1, self.Delem[k1])

    def ghost_values(self, X, t, field):
        """The prescribed exterior state at physical points X [..., 2]."""
        return np.asarray(self.ghost(X[..., 0], X[..., 1], t, field), dtype=np.float64)

    # -- nodal tensor coefficient (Algorithm 1 with nodal products) ----------
    def element_tensor(self, u, k):
        """[3, Np] (Dxx, Dxy, Dyy) at element k's nodes."""
        if self.D_mode == "nodal":
            return self.Dnodal[k].T
        return self.D0[:, None] * u[k][None, :]

    def _tensor_edge_flux(self, u, k1, f1, k2, f2, eg, t, field):
        """Flux of one interior edge (k2 >= 0) or boundary face (k2 < 0) with
        the nodal tensor coefficient."""
        ops = self.ops
        m1 = ardg.total_projection(ops, eg.pi1, f1) @ u[k1]
        Dp1 = ardg.nodal_on_subtriangle(ops, eg.pi1, f1, self.element_tensor(u, k1))
        if k2 >= 0:
            m2 = ardg.total_projection(ops, eg.pi2, f2) @ u[k2]
            Dp2 = ardg.nodal_on_subtriangle(ops, eg.pi2, f2, self.element_tensor(u, k2))
        else:
            if self.ghost is not None:
                u2n = self.ghost_values(ardg.ghost_nodes(ops.N, eg), t, field)
            else:
                u2n = -ardg.mirrored_on_ghost(ops, self.geom, k1, eg, u[k1])
            m2 = ops.Vinv @ u2n
            if self.D_mode == "nodal":
                Dp2 = ardg.mirrored_on_ghost(ops, self.geom, k1, eg, self.Dnodal[k1].T)
            else:
                Dp2 = self.D0[:, None] * u2n[None, :]
        return ardg.alg1_tensor_flux(ops, eg, m1, m2, Dp1, Dp2)

    # -- fluxes -----------------------------------------------------------------
    def diffusive_flux(self, u: np.ndarray, field: int = 0, t: float = 0.0):
        """Fluxes F in element-1 (CCW) order: [E_int, Nfp] and [E_bdy, Nfp]."""
        if self.D_mode in ("nodal", "solution"):
            Fi = np.array([self._tensor_edge_flux(u, k1, f1, k2, f2, self.edge_geom[e], t, field)
                           for e, (k1, f1, k2, f2) in enumerate(self.int_edges)]).reshape(-1, self.ops.Nfp)
            Fb = np.array([self._tensor_edge_flux(u, k1, f1, -1, -1, self.bdy_geom[e], t, field)
                           for e, (k1, f1) in enumerate(self.bdy_edges)]).reshape(-1, self.ops.Nfp)
            return Fi, Fb
        k1 = np.array([e[0] for e in self.int_edges], dtype=np.int64)
        k2 = np.array([e[2] for e in self.int_edges], dtype=np.int64)
        kb = np.array([e[0] for e in self.bdy_edges], dtype=np.int64)
        Fi = (np.einsum("eij,ej->ei", self.W1, u[k1]) if len(k1) else np.zeros((0, self.ops.Nfp)))
        if len(k2):
            Fi = Fi + np.einsum("eij,ej->ei", self.W2, u[k2])
        Fb = np.einsum("eij,ej->ei", self.WB, u[kb]) if len(kb) else np.zeros((0, self.ops.Nfp))
        if self.ghost is not None and len(kb):
            Fb = Fb + np.einsum("eij,ej->ei", self.WG, self.ghost_values(self.GX, t, field))
        if self.D_mode == "const":
            Fi = Fi * self.Dfield[field]
            Fb = Fb * self.Dfield[field]
        return Fi, Fb

    def face_fluxes(self, Fi, Fb):
        """[K, 3, Nfp] flux seen by each element face, in its own CCW order.

        Side 1 reads the edge flux as is; side 2 (outward normal reversed, face
        traversed B -> A) reads it negated and in reverse order.
        """
        ops = self.ops
        out = np.zeros((self.geom.K, 3, ops.Nfp))
        if len(self.int_edges):
            ie = np.array(self.int_edges, dtype=np.int64)
            out[ie[:, 0], ie[:, 1]] = Fi
            out[ie[:, 2], ie[:, 3]] = -Fi[:, ::-1]
        if len(self.bdy_edges):
            be = np.array(self.bdy_edges, dtype=np.int64)
            out[be[:, 0], be[:, 1]] = Fb
        return out

    # -- velocity ------------------------------------------------------------
    def velocity_at(self, xy):
        v0x, v0y, a, b, c, d = self.velocity
        return v0x + a * xy[..., 0] + b * xy[..., 1], v0y + c * xy[..., 0] + d * xy[..., 1]

    def upwind_face_flux(self, u, t: float = 0.0, field: int = 0):
        """[K, 3, Nfp] upwind flux f* per element face (CCW order); outside
        the domain u+ is 0, or the prescribed exterior state."""
        ops, g = self.ops, self.geom
        xyn = g.physical(ops.rs)
        vx, vy = self.velocity_at(xyn)
        out = np.zeros((g.K, 3, ops.Nfp))
        for k in range(g.K):
            for f in range(3):
                idx = ops.fmask[f]
                vn = g.nx[k, f] * vx[k, idx] + g.ny[k, f] * vy[k, idx]
                um = u[k, idx]
                k2 = g.EToE[k, f]
                if k2 < 0:
                    up = (np.zeros_like(um) if self.ghost is None
                          else self.ghost_values(xyn[k, idx], t, field))
                else:
                    f2 = g.EToF[k, f]
                    up = u[k2, ops.fmask[f2]][::-1]
                out[k, f] = np.maximum(vn, 0.0) * um + np.minimum(vn, 0.0) * up
        return out

    # -- right-hand side ------------------------------------------------------
    def rhs(self, u: np.ndarray, t: float = 0.0) -> np.ndarray:
        """du/dt at time t for state u [F, K, Np] (or [K, Np] for one field)."""
        single = (u.ndim == 2)
        U = u[None] if single else u
        out = np.stack([self._rhs_field(U[f], f, t) for f in range(U.shape[0])])
        return out[0] if single else out

    def _rhs_field(self, u, field, t=0.0):
        ops, g = self.ops, self.geom
        rx, ry, sx, sy = (a[:, None] for a in (g.rx, g.ry, g.sx, g.sy))
        ur = u @ ops.Dr.T
        us = u @ ops.Ds.T
        qx = rx * ur + sx * us
        qy = ry * ur + sy * us
        if self.D_mode in ("nodal", "solution"):
            # q = D grad u as the nodal tensor-vector product
            Dt = (self.Dnodal.transpose(2, 0, 1) if self.D_mode == "nodal"
                  else self.D0[:, None, None] * u[None])
            qx, qy = Dt[0] * qx + Dt[1] * qy, Dt[1] * qx + Dt[2] * qy
            Dk = 1.0
        else:
            Dk = self.Delem[:, None] if self.D_mode == "element" else self.Dfield[field]
        vol = (rx * (qx @ ops.Drw.T) + sx * (qx @ ops.Dsw.T)
               + ry * (qy @ ops.Drw.T) + sy * (qy @ ops.Dsw.T))
        rhs = -Dk * vol
        Fi, Fb = self.diffusive_flux(u, field, t)
        Ff = self.face_fluxes(Fi, Fb)
        surf = np.zeros_like(u)
        for f in range(3):
            scale = (g.sJ[:, f] / g.J)[:, None]
            surf += scale * (Ff[:, f, :] @ ops.LIFT[:, f * ops.Nfp:(f + 1) * ops.Nfp].T)
        rhs = rhs + surf
        if self.velocity is not None:
            rhs = rhs + self._convection_weak(u, t, field)
        return rhs

    def _convection_weak(self, u, t=0.0, field=0):
        """-div(v u) in weak form: Dxw (vx u) + Dyw (vy u) - sum_f LIFT_f f*."""
        ops, g = self.ops, self.geom
        xyn = g.physical(ops.rs)
        vx, vy = self.velocity_at(xyn)
        fx, fy = vx * u, vy * u
        rx, ry, sx, sy = (a[:, None] for a in (g.rx, g.ry, g.sx, g.sy))
        vol = (rx * (fx @ ops.Drw.T) + sx * (fx @ ops.Dsw.T)
               + ry * (fy @ ops.Drw.T) + sy * (fy @ ops.Dsw.T))
        fs = self.upwind_face_flux(u, t, field)
        surf = np.zeros_like(u)
        for f in range(3):
            scale = (g.sJ[:, f] / g.J)[:, None]
            surf += scale * (fs[:, f, :] @ ops.LIFT[:, f * ops.Nfp:(f + 1) * ops.Nfp].T)
        return vol - surf

    # -- RHS of a few elements only (sampled checks on large meshes) ---------
    def _face_flux_one(self, u, k, f, field, t=0.0):
        """Flux seen by face f of element k (CCW order), computed for that one
        edge with the same steps as the full assembly."""
        g, ops = self.geom, self.ops
        k2 = int(g.EToE[k, f])
        if self.D_mode in ("nodal", "solution"):
            if k2 < 0:
                return self._tensor_edge_flux(u, k, f, -1, -1, ardg.boundary_edge_geometry(g, k, f), t, field)
            f2 = int(g.EToF[k, f])
            k1, fa, kb, fb = (k, f, k2, f2) if k < k2 else (k2, f2, k, f)
            F = self._tensor_edge_flux(u, k1, fa, kb, fb, ardg.interior_edge_geometry(g, k1, fa, kb, fb), t, field)
            return F if k == k1 else -F[::-1]
        if k2 < 0:
            eg = ardg.boundary_edge_geometry(g, k, f)
            if self.ghost is not None:
                W1, WG = self._prescribed_operators(k, f, eg)
                F = W1 @ u[k] + WG @ self.ghost_values(ardg.ghost_nodes(ops.N, eg), t, field)
                return F if self.D_mode == "element" else self.Dfield[field] * F
            if self.D_mode == "element":
                F = self._element_boundary_operator(k, f, eg) @ u[k]
            else:
                F = self.Dfield[field] * (ardg.boundary_edge_operator(ops, g, k, f, eg) @ u[k])
            return F
        f2 = int(g.EToF[k, f])
        k1, fa, kb, fb = (k, f, k2, f2) if k < k2 else (k2, f2, k, f)
        eg = ardg.interior_edge_geometry(g, k1, fa, kb, fb)
        if self.D_mode == "element":
            W1, W2 = self._element_edge_operator(eg, fa, fb, k1, kb)
            F = W1 @ u[k1] + W2 @ u[kb]
        else:
            W1, W2 = ardg.edge_operator(ops, eg, fa, fb)
            F = self.Dfield[field] * (W1 @ u[k1] + W2 @ u[kb])
        return F if k == k1 else -F[::-1]

    def rhs_elements(self, u, elements, field: int = 0, t: float = 0.0):
        """du/dt at time t on the listed elements only, [len(elements), Np];
        u [K, Np] needs valid values on the listed elements and their face
        neighbours."""
        ops, g = self.ops, self.geom
        out = np.zeros((len(elements), ops.Np))
        xyn = g.physical(ops.rs) if self.velocity is not None else None
        for n, k in enumerate(elements):
            rx, ry, sx, sy = g.rx[k], g.ry[k], g.sx[k], g.sy[k]
            uk = u[k]
            qx = rx * (ops.Dr @ uk) + sx * (ops.Ds @ uk)
            qy = ry * (ops.Dr @ uk) + sy * (ops.Ds @ uk)
            if self.D_mode in ("nodal", "solution"):
                Dt = self.element_tensor(u, k)
                qx, qy = Dt[0] * qx + Dt[1] * qy, Dt[1] * qx + Dt[2] * qy
                Dk = 1.0
            else:
                Dk = self.Delem[k] if self.D_mode == "element" else self.Dfield[field]
            r = -Dk * (rx * (ops.Drw @ qx) + sx * (ops.Dsw @ qx) + ry * (ops.Drw @ qy) + sy * (ops.Dsw @ qy))
            for f in range(3):
                F = self._face_flux_one(u, k, f, field, t)
                Lf = ops.LIFT[:, f * ops.Nfp:(f + 1) * ops.Nfp]
                r = r + g.sJ[k, f] / g.J[k] * (Lf @ F)
            if self.velocity is not None:
                vx, vy = self.velocity_at(xyn[k])
                fx, fy = vx * uk, vy * uk
                r = r + rx * (ops.Drw @ fx) + sx * (ops.Dsw @ fx) + ry * (ops.Drw @ fy) + sy * (ops.Dsw @ fy)
                for f in range(3):
                    idx = ops.fmask[f]
                    vn = g.nx[k, f] * vx[idx] + g.ny[k, f] * vy[idx]
                    k2 = g.EToE[k, f]
                    if k2 >= 0:
                        up = u[k2, ops.fmask[g.EToF[k, f]]][::-1]
                    elif self.ghost is not None:
                        up = self.ghost_values(xyn[k, idx], t, field)
                    else:
                        up = np.zeros(ops.Nfp)
                    fs = np.maximum(vn, 0.0) * uk[idx] + np.minimum(vn, 0.0) * up
                    Lf = ops.LIFT[:, f * ops.Nfp:(f + 1) * ops.Nfp]
                    r = r - g.sJ[k, f] / g.J[k] * (Lf @ fs)
            out[n] = r
        return out

    def neighbourhood(self, elements, layers: int):
        """Elements within `layers` face-neighbour hops of the given ones."""
        cur = set(int(k) for k in elements)
        for _ in range(layers):
            nxt = set(cur)
            for k in cur:
                for k2 in self.geom.EToE[k]:
                    if k2 >= 0:
                        nxt.add(int(k2))
            cur = nxt
        return sorted(cur)

    def rk4_step_elements(self, u, dt, elements, field: int = 0):
        """One classic RK4 step evaluated on the listed elements only, using
        the patches of neighbours each stage needs.  Returns [len, Np]."""
        P = [sorted(set(int(k) for k in elements))]
        for _ in range(4):
            P.append(self.neighbourhood(P[-1], 1))
        K, Np = u.shape
        stage_in = u
        acc = {}
        ks = []
        for s in range(4):
            patch = P[3 - s]
            r = self.rhs_elements(stage_in, patch, field)
            ks.append(dict(zip(patch, r)))
            if s < 3:
                c = 0.5 if s < 2 else 1.0
                nxt = np.full((K, Np), np.nan)
                for k, rk in zip(patch, r):
                    nxt[k] = u[k] + c * dt * rk
                stage_in = nxt
        out = np.zeros((len(elements), Np))
        for n, k in enumerate(elements):
            out[n] = u[k] + dt / 6.0 * (ks[0][k] + 2 * ks[1][k] + 2 * ks[2][k] + ks[3][k])
        return out

    # -- nodal coordinates ------------------------------------------------------
    def nodal_xy(self):
        return self.geom.physical(self.ops.rs)


# ----------------------------------------------------------------------------
# Time integration
# ----------------------------------------------------------------------------

def rk4_step(rhs, u, dt, t=None):
    """One classic RK4 step; with t given, rhs(u, t) is evaluated at the
    stage times t, t + dt/2, t + dt/2, t + dt."""
    if t is None:
        k1 = rhs(u)
        k2 = rhs(u + 0.5 * dt * k1)
        k3 = rhs(u + 0.5 * dt * k2)
        k4 = rhs(u + dt * k3)
    else:
        k1 = rhs(u, t)
        k2 = rhs(u + 0.5 * dt * k1, t + 0.5 * dt)
        k3 = rhs(u + 0.5 * dt * k2, t + 0.5 * dt)
        k4 = rhs(u + dt * k3, t + dt)
    return u + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


# Carpenter & Kennedy (1994), five-stage fourth-order 2N-storage scheme
LSERK_A = np.array([0.0,
                    -567301805773.0 / 1357537059087.0,
                    -2404267990393.0 / 2016746695238.0,
                    -3550918686646.0 / 2091501179385.0,
                    -1275806237668.0 / 842570457699.0])
LSERK_B = np.array([1432997174477.0 / 9575080441755.0,
                    5161836677717.0 / 13612068292357.0,
                    1720146321549.0 / 2090206949498.0,
                    3134564353537.0 / 4481467310338.0,
                    2277821191437.0 / 14882151754819.0])


def lserk_stage_times():
    """Stage times c_s of the 2N-storage scheme: the stage values of
    du/dt = 1 (u = t, integrated exactly), c_0 = 0, c_s = sum of B_j r_j with
    r_j = A_j r_{j-1} + 1."""
    c, r, out = 0.0, 0.0, []
    for s in range(5):
        out.append(c)
        r = LSERK_A[s] * r + 1.0
        c = c + LSERK_B[s] * r
    return np.array(out)


LSERK_C = lserk_stage_times()


def lserk_step(rhs, u, dt, t=None):
    """One step of the five-stage low-storage RK; with t given, rhs(u, t) is
    evaluated at the stage times t + c_s dt."""
    res = np.zeros_like(u)
    for s in range(5):
        r = rhs(u) if t is None else rhs(u, t + LSERK_C[s] * dt)
        res = LSERK_A[s] * res + dt * r
        u = u + LSERK_B[s] * res
    return u


# ----------------------------------------------------------------------------
# Norms
# ----------------------------------------------------------------------------

def mass_norm(prob: Problem, e: np.ndarray) -> float:
    """sqrt(sum_k J_k e_k^T M e_k / sum_k |Omega_k|) for nodal e [K, Np]."""
    ops, g = prob.ops, prob.geom
    num = float(np.sum(g.J * np.einsum("ki,ij,kj->k", e, ops.M, e)))
    area = float(np.sum(2.0 * g.J))
    return np.sqrt(num / area)


def error_norms(prob: Problem, u: np.ndarray, exact, nq: int = None):
    """Cell-normalised L2 and L_inf errors against exact(x, y)."""
    ops, g = prob.ops, prob.geom
    N = ops.N
    nq = nq or (N + 4)
    r, s, w = ardg.triangle_quadrature(nq)
    Vq = vandermonde(N, r, s) @ ops.Vinv                     # nodal -> quadrature
    uq = u @ Vq.T                                            # [K, Q]
    xy = g.physical(np.column_stack([r, s]))                 # [K, Q, 2]
    ue = exact(xy[..., 0], xy[..., 1])
    err = uq - ue
    area = 2.0 * g.J
    l2 = np.sqrt(np.sum(g.J * (err ** 2 @ w)) / np.sum(area))
    linf = np.max(g.J * (np.abs(err) @ w) / area)
    return l2, linf
