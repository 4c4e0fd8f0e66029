"""The affine reconstruction (aRDG) and the diffusive flux on an edge, FP64.

TEST INFRASTRUCTURE ONLY.

Follows the section "Affine reconstructed algorithm": the enclosed
parallelogram, the projection Vandermonde V_p (eq. NodalToModalProjection),
the node reordering in I (eq. changeOfHypotenuseProjection), the total
projection V^{-1} V_p V_rf^{-1} u (eq. totalProjection), the least-squares
reconstruction on the parallelogram (subsection "Reconstruction", Algorithm
aRDG) and the reconstructed gradient on the diagonal with the constant
parallelogram factors (eq. lift_physicalDomain_ardg and the gradient formula
after it).  Algorithm 1 (element-wise diffusion coefficients) is
``edge_operator_alg1``; the alternative form with a reconstructed
coefficient (eq. NDG_diffusion_once_matrixForm_reference_general_alternative,
Algorithm nonconstDiff2) is ``edge_operator_alg2``.

Readings of places the paper leaves open:

* Which enclosed parallelogram: the one of maximum area whose diagonal is the
  shared edge AB and whose two halves lie in the two elements.  P1 = m + w and
  P2 = m - w (m the midpoint of AB) with P1 in element 1 and P2 in element 2;
  the height of P1 above AB is maximised.
* Frame of the second sub-triangle: the point reflection (r,s) -> (-r,-s) of
  the square frame, i.e. Omega'_2 with vertex order (P2, B, A).
* Least squares: unweighted, over the 2Np equations written with orthonormal
  test functions on each sub-triangle; the unknowns are the (N+1)^2
  coefficients of a tensor-product Legendre expansion on the square.
* Face node order: counter-clockwise along each element; element 1's edge
  runs A -> B, the diagonal nodes are d_j = (t_j, -t_j) with t_j the LGL points
  from +1 down to -1.
* Boundary faces (the paper gives no boundary treatment): zero Dirichlet data
  through a mirror ghost.  The ghost element is the mirror image of the
  element across the boundary edge and carries -u evaluated at mirrored
  points; the reconstruction then proceeds exactly as for an interior edge.
* Algorithm 1 with element-wise constant D: "Separation" evaluates the
  reconstruction at the nodes of each sub-triangle; "project D" is the
  constant D of each element; Grad uses each sub-triangle's own affine
  factors; the second RDG takes the nodal products D_k grad(u~_k) already on
  the sub-triangles (so no second V_p) and the flux is n1 . (result on the
  diagonal).  At a boundary face the ghost carries the element's own D.
* Prescribed exterior data at a boundary face (inhomogeneous Dirichlet data,
  needed for the paper's Gaussian tests, whose solution is not zero on the
  boundary; the paper does not say how it imposes it): the ghost
  sub-triangle Omega'_2 = (P2, B, A) of the mirror rhombus carries the
  prescribed exterior state g itself, sampled at its nodes, so that
  u~ = RDG(u1, g).  With Algorithms 1 and 2 the ghost carries the element's
  own D.  The default (no data given) stays the zero-Dirichlet mirror ghost.
* Algorithm 1 with a nodal coefficient (eq.
  NDG_diffusion_once_matrixForm_reference_general with D a function of space,
  anisotropic, or of the solution): D is a symmetric tensor field
  [[Dxx, Dxy], [Dxy, Dyy]] given by its nodal values on each element;
  "project D" evaluates each element's D polynomial at the nodes of its
  sub-triangle (the total projection of eq. totalProjection applied to D),
  the product is the nodal tensor-vector product D_p^k grad(u~_k), and the
  rest is as for element-wise D.  A solution-dependent coefficient D = u D0
  (the D0 C of eq. advection_diffusion_nonlinear and of the shear equation
  eq. diffusion_shear, whose cross term is the off-diagonal entry) takes the
  nodal values of u itself.  A ghost carries the coefficient the same way as
  its data: the element's nodal D at the mirrored points, or D0 times the
  ghost's state.
* Algorithm 2 (the alternative form): D~ = RDG(D^1, D^2) is the same
  least-squares reconstruction applied to the coefficient's nodal data of the
  two elements (projected onto the sub-triangles like u), Grad(u~) is the
  gradient of the reconstruction u~ on the parallelogram, and "Product" is
  the pointwise product at the diagonal nodes, so the flux is
  D~(d_j) n1 . grad u~(d_j).  At a boundary face the ghost's coefficient is
  the element's own D at the mirrored points (a coefficient is reflected
  evenly, the solution oddly).
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np
from scipy.special import roots_jacobi, roots_legendre

from .reference_element import (RefOps, jacobi_normalised, jacobi_normalised_deriv,
                                lgl_nodes, nodes, vandermonde)

A2 = np.array([1.0, -1.0])
A3 = np.array([-1.0, 1.0])

# rotated vertex labels (w1, w2, w3) for each face, as element vertex indices:
# face (v1,v2) -> (v3, v1, v2); face (v2,v3) -> (v1, v2, v3); face (v3,v1) -> (v2, v3, v1)
ROTATED_VERTICES = ((2, 0, 1), (0, 1, 2), (1, 2, 0))
_REF_VERTS = np.array([[-1.0, -1.0], [1.0, -1.0], [-1.0, 1.0]])


# ----------------------------------------------------------------------------
# Node reordering in I (three orderings, one per face)
# ----------------------------------------------------------------------------

@lru_cache(maxsize=None)
def rotation_perm(N: int, f: int) -> np.ndarray:
    """Pi_f with (Pi_f u)_i = u at the element node that sits where rotated
    node i sits, the rotated frame mapping face f onto the hypotenuse of I."""
    rs = nodes(N)
    r, s = rs[:, 0], rs[:, 1]
    lam = np.column_stack([-(r + s) / 2.0, (r + 1) / 2.0, (s + 1) / 2.0])
    w = ROTATED_VERTICES[f]
    pts = lam @ _REF_VERTS[list(w)]   # rotated node i in the element's own frame
    perm = np.empty(len(r), dtype=np.int64)
    for i in range(len(r)):
        d = np.hypot(rs[:, 0] - pts[i, 0], rs[:, 1] - pts[i, 1])
        j = int(np.argmin(d))
        if d[j] > 1e-10:
            raise RuntimeError("node set is not rotation symmetric")
        perm[i] = j
    return perm


def rotation_matrix(N: int, f: int) -> np.ndarray:
    p = rotation_perm(N, f)
    P = np.zeros((len(p), len(p)))
    P[np.arange(len(p)), p] = 1.0
    return P


# ----------------------------------------------------------------------------
# Enclosed parallelogram (maximum area), as a small linear program
# ----------------------------------------------------------------------------

def _cross(a, b):
    return a[0] * b[1] - a[1] * b[0]


def _in_triangle(p, a, b, c, tol):
    d1 = _cross(b - a, p - a)
    d2 = _cross(c - b, p - b)
    d3 = _cross(a - c, p - c)
    return d1 >= -tol and d2 >= -tol and d3 >= -tol


def _line_intersection(p1, p2, q1, q2):
    d1, d2 = p2 - p1, q2 - q1
    den = _cross(d1, d2)
    if abs(den) < 1e-300:
        return None
    t = _cross(q1 - p1, d2) / den
    return p1 + t * d1


def parallelogram_apex(A, B, C1, C2) -> np.ndarray:
    """P1 maximising the height above AB subject to P1 in (A,B,C1) and
    A+B-P1 in (B,A,C2).

    The second condition says P1 lies in the triangle (A, B, A+B-C2), so the
    feasible set is the intersection of two triangles on the same side of AB.
    A linear objective over a convex polygon peaks at a vertex: the vertices
    are among C1, C2' = A+B-C2, the pairwise crossings of the lines A-C1,
    B-C1, A-C2', B-C2', and A, B.  The feasible candidate of largest height is
    returned.
    """
    A, B, C1, C2 = (np.asarray(p, dtype=np.float64) for p in (A, B, C1, C2))
    C2p = A + B - C2
    scale = max(np.max(np.abs(np.array([A, B, C1, C2]))), 1.0)
    L2 = float(np.dot(B - A, B - A))
    tol = 1e-12 * L2 * scale
    cands = [C1, C2p, A, B]
    for (p, q) in ((A, C1), (B, C1)):
        for (u, v) in ((A, C2p), (B, C2p)):
            x = _line_intersection(p, q, u, v)
            if x is not None:
                cands.append(x)
    nrm = np.array([-(B - A)[1], (B - A)[0]])     # left normal of A->B (towards C1)
    best, best_h = None, -np.inf
    for p in cands:
        if _in_triangle(p, A, B, C1, tol) and _in_triangle(p, A, B, C2p, tol):
            h = float(np.dot(p - A, nrm))
            if h > best_h:
                best, best_h = p, h
    return best


def ref_coords(w1, w2, w3, P) -> np.ndarray:
    """(r, s) with -(r+s)/2 w1 + (r+1)/2 w2 + (s+1)/2 w3 = P (eq. mapping_tri)."""
    w1, w2, w3, P = (np.asarray(p, dtype=np.float64) for p in (w1, w2, w3, P))
    Jm = 0.5 * np.column_stack([w2 - w1, w3 - w1])
    rhs = P - 0.5 * (w2 + w3)
    return np.linalg.solve(Jm, rhs)


def affine_factors(v1, v2, v3):
    """(r_x, r_y, s_x, s_y, J) of the affine map with vertices (v1, v2, v3)."""
    xr, yr = 0.5 * (v2[0] - v1[0]), 0.5 * (v2[1] - v1[1])
    xs, ys = 0.5 * (v3[0] - v1[0]), 0.5 * (v3[1] - v1[1])
    J = xr * ys - xs * yr
    return ys / J, -xs / J, -yr / J, xr / J, J


# ----------------------------------------------------------------------------
# Projection Vandermonde onto a sub-triangle sharing the hypotenuse
# ----------------------------------------------------------------------------

def subtriangle_points(N: int, pi) -> np.ndarray:
    """Reference points T(rho_i) of the sub-triangle (pi, a2, a3) inside I."""
    rs = nodes(N)
    r, s = rs[:, 0], rs[:, 1]
    pi = np.asarray(pi, dtype=np.float64)
    return (-(r + s)[:, None] / 2.0 * pi[None, :] + (r + 1)[:, None] / 2.0 * A2[None, :]
            + (s + 1)[:, None] / 2.0 * A3[None, :])


def projection_vandermonde(N: int, pi) -> np.ndarray:
    """V_p[i, j] = psi_j(T(rho_i)): modal coefficients on I -> nodal values on
    the sub-triangle."""
    pts = subtriangle_points(N, pi)
    return vandermonde(N, pts[:, 0], pts[:, 1])


def total_projection(ops: RefOps, pi, f: int) -> np.ndarray:
    """V^{-1} V_p V_rf^{-1} as a matrix on the element's native nodal values
    (eq. totalProjection), with V_rf^{-1} u = V^{-1} Pi_f u."""
    return ops.Vinv @ projection_vandermonde(ops.N, pi) @ ops.Vinv @ rotation_matrix(ops.N, f)


# ----------------------------------------------------------------------------
# Least-squares reconstruction on the parallelogram
# ----------------------------------------------------------------------------

def legendre_n(x, n):
    return jacobi_normalised(x, n, 0.0, 0.0)


def legendre_n_deriv(x, n):
    return jacobi_normalised_deriv(x, n, 0.0, 0.0)


def q_modes(N: int):
    return [(a, b) for a in range(N + 1) for b in range(N + 1)]


def phi(R, S, N):
    """[.., Mp] tensor Legendre basis of Q_N on the square [-1,1]^2."""
    return np.stack([legendre_n(R, a) * legendre_n(S, b) for (a, b) in q_modes(N)], axis=-1)


def phi_grad(R, S, N):
    dR = np.stack([legendre_n_deriv(R, a) * legendre_n(S, b) for (a, b) in q_modes(N)], axis=-1)
    dS = np.stack([legendre_n(R, a) * legendre_n_deriv(S, b) for (a, b) in q_modes(N)], axis=-1)
    return dR, dS


def triangle_quadrature(n: int):
    """Collapsed Gauss rule on I, exact for total degree <= 2n-2 (plus margin)."""
    a, wa = roots_legendre(n)
    b, wb = roots_jacobi(n, 1.0, 0.0)
    A_, B_ = np.meshgrid(a, b, indexing="ij")
    W = np.outer(wa, wb) * 0.5
    r = 0.5 * (1.0 + A_) * (1.0 - B_) - 1.0
    return r.ravel(), B_.ravel(), W.ravel()


@lru_cache(maxsize=None)
def recon_system(N: int) -> np.ndarray:
    """A [2Np, Mp]: rows m of sub-triangle 1 hold int_I psi_m(r,s) phi_q(r,s),
    rows Np+m of sub-triangle 2 hold int_I psi_m(r,s) phi_q(-r,-s) (its own
    frame is the point-reflected square frame)."""
    r, s, w = triangle_quadrature(3 * N + 3)
    Vq = vandermonde(N, r, s)             # [Q, Np]
    P1 = phi(r, s, N)                     # [Q, Mp]
    P2 = phi(-r, -s, N)
    top = (Vq * w[:, None]).T @ P1
    bot = (Vq * w[:, None]).T @ P2
    return np.vstack([top, bot])


@lru_cache(maxsize=None)
def recon_pinv(N: int) -> np.ndarray:
    """R = A^+ (least-squares solve via numpy's SVD pseudo-inverse)."""
    return np.linalg.pinv(recon_system(N))


@lru_cache(maxsize=None)
def diagonal_points(N: int) -> np.ndarray:
    """d_j = (t_j, -t_j), t_j the LGL points from +1 down to -1 (A -> B)."""
    t = lgl_nodes(N)[::-1]
    return np.column_stack([t, -t])


def diagonal_eval(N: int):
    """Values and (R, S) derivatives of the Q_N basis at the diagonal nodes."""
    d = diagonal_points(N)
    E0 = phi(d[:, 0], d[:, 1], N)
    ER, ES = phi_grad(d[:, 0], d[:, 1], N)
    return E0, ER, ES


# ----------------------------------------------------------------------------
# Edge geometry
# ----------------------------------------------------------------------------

class EdgeGeometry:
    """Everything about one reconstructed element (one edge)."""

    def __init__(self, A, B, C1, C2, n1):
        self.A, self.B, self.C1, self.C2 = (np.asarray(p, dtype=np.float64) for p in (A, B, C1, C2))
        self.P1 = parallelogram_apex(self.A, self.B, self.C1, self.C2)
        self.P2 = self.A + self.B - self.P1
        self.pi1 = ref_coords(self.C1, self.A, self.B, self.P1)
        self.pi2 = ref_coords(self.C2, self.B, self.A, self.P2)
        # constant factors of the parallelogram (square frame = Omega'_1 frame)
        self.Rx, self.Ry, self.Sx, self.Sy, self.Jp = affine_factors(self.P1, self.A, self.B)
        # Omega'_2 in its own frame (P2, B, A)
        self.Rx2, self.Ry2, self.Sx2, self.Sy2, self.Jp2 = affine_factors(self.P2, self.B, self.A)
        self.n1 = np.asarray(n1, dtype=np.float64)


def interior_edge_geometry(geom, k1, f1, k2, f2) -> EdgeGeometry:
    w = ROTATED_VERTICES[f1]
    C1, A, B = geom.v[k1, w[0]], geom.v[k1, w[1]], geom.v[k1, w[2]]
    w2 = ROTATED_VERTICES[f2]
    C2 = geom.v[k2, w2[0]]
    if not (np.allclose(geom.v[k2, w2[1]], B) and np.allclose(geom.v[k2, w2[2]], A)):
        raise RuntimeError("neighbour face does not run B -> A")
    n1 = np.array([geom.nx[k1, f1], geom.ny[k1, f1]])
    return EdgeGeometry(A, B, C1, C2, n1)


def mirror_point(p, A, B):
    d = B - A
    t = np.dot(p - A, d) / np.dot(d, d)
    foot = A + t * d
    return 2.0 * foot - p


def boundary_edge_geometry(geom, k1, f1) -> EdgeGeometry:
    w = ROTATED_VERTICES[f1]
    C1, A, B = geom.v[k1, w[0]], geom.v[k1, w[1]], geom.v[k1, w[2]]
    C2 = mirror_point(C1, A, B)
    n1 = np.array([geom.nx[k1, f1], geom.ny[k1, f1]])
    return EdgeGeometry(A, B, C1, C2, n1)


# ----------------------------------------------------------------------------
# Flux operators (linear in the nodal data of the two sides)
# ----------------------------------------------------------------------------

def _gradient_on_diagonal(N, c, eg: EdgeGeometry):
    """grad u~ at d_j from Q_N coefficients c [Mp, ...]: G_p^T (dR, dS)."""
    _, ER, ES = diagonal_eval(N)
    uR = ER @ c
    uS = ES @ c
    gx = eg.Rx * uR + eg.Sx * uS
    gy = eg.Ry * uR + eg.Sy * uS
    return gx, gy


def edge_operator(ops: RefOps, eg: EdgeGeometry, f1: int, f2: int):
    """Algorithm aRDG plus the flux n1 . grad u~ at the diagonal nodes.

    Returns (W1, W2), each [Nfp, Np], with flux = W1 u1 + W2 u2 for element 1's
    face f1 in counter-clockwise order (D not included).
    """
    N = ops.N
    P1 = total_projection(ops, eg.pi1, f1)     # u_hat'^1 = V^-1 V_p1 V_r1^-1 u1
    P2 = total_projection(ops, eg.pi2, f2)
    R = recon_pinv(N)
    Np = ops.Np
    c1 = R[:, :Np] @ P1                        # reconstruction from side 1 data
    c2 = R[:, Np:] @ P2
    gx1, gy1 = _gradient_on_diagonal(N, c1, eg)
    gx2, gy2 = _gradient_on_diagonal(N, c2, eg)
    W1 = eg.n1[0] * gx1 + eg.n1[1] * gy1
    W2 = eg.n1[0] * gx2 + eg.n1[1] * gy2
    return W1, W2


def _boundary_ghost_data_operator(ops: RefOps, geom, k1, eg: EdgeGeometry) -> np.ndarray:
    """[Np, Np] map from element data u1 to the ghost's nodal values on
    Omega'_2 (frame (P2, B, A)): u'^2(y_i) = -u1(mirror(y_i))."""
    N = ops.N
    rs = nodes(N)
    r, s = rs[:, 0], rs[:, 1]
    y = (-(r + s)[:, None] / 2.0 * eg.P2[None, :] + (r + 1)[:, None] / 2.0 * eg.B[None, :]
         + (s + 1)[:, None] / 2.0 * eg.A[None, :])
    ym = np.array([mirror_point(p, eg.A, eg.B) for p in y])
    v = geom.v[k1]
    ref = np.array([ref_coords(v[0], v[1], v[2], p) for p in ym])
    Vm = vandermonde(N, ref[:, 0], ref[:, 1])
    return -Vm @ ops.Vinv


def boundary_edge_operator(ops: RefOps, geom, k1, f1, eg: EdgeGeometry) -> np.ndarray:
    """Flux operator [Nfp, Np] of a boundary face (mirror ghost, zero Dirichlet)."""
    N = ops.N
    P1 = total_projection(ops, eg.pi1, f1)
    G = _boundary_ghost_data_operator(ops, geom, k1, eg)
    P2 = ops.Vinv @ G                           # ghost data is already on Omega'_2
    R = recon_pinv(N)
    Np = ops.Np
    c = R[:, :Np] @ P1 + R[:, Np:] @ P2
    gx, gy = _gradient_on_diagonal(N, c, eg)
    return eg.n1[0] * gx + eg.n1[1] * gy


def _alg1_from_subtriangle_modal(ops: RefOps, eg: EdgeGeometry, Q1, Q2, D1, D2):
    """Algorithm 1 given maps Q_k (-> modal data on Omega'_k).  Returns the
    flux operator acting on whatever Q_k act on."""
    N = ops.N
    Np = ops.Np
    R = recon_pinv(N)
    c = R[:, :Np] @ Q1 + R[:, Np:] @ Q2              # u~ = RDG(u1, u2)
    rs = nodes(N)
    # Separation: u~ at the nodes of each sub-triangle (each in its own frame)
    u1n = phi(rs[:, 0], rs[:, 1], N) @ c
    u2n = phi(-rs[:, 0], -rs[:, 1], N) @ c
    # Grad on each sub-triangle with its own affine factors
    g1x = eg.Rx * (ops.Dr @ u1n) + eg.Sx * (ops.Ds @ u1n)
    g1y = eg.Ry * (ops.Dr @ u1n) + eg.Sy * (ops.Ds @ u1n)
    g2x = eg.Rx2 * (ops.Dr @ u2n) + eg.Sx2 * (ops.Ds @ u2n)
    g2y = eg.Ry2 * (ops.Dr @ u2n) + eg.Sy2 * (ops.Ds @ u2n)
    # D_p^k = V_p D^k: an element-wise constant D is constant on Omega'_k
    f1x, f1y = D1 * g1x, D1 * g1y
    f2x, f2y = D2 * g2x, D2 * g2y
    # second RDG on each component (data already on the sub-triangles)
    cx = R[:, :Np] @ (ops.Vinv @ f1x) + R[:, Np:] @ (ops.Vinv @ f2x)
    cy = R[:, :Np] @ (ops.Vinv @ f1y) + R[:, Np:] @ (ops.Vinv @ f2y)
    E0, _, _ = diagonal_eval(N)
    return eg.n1[0] * (E0 @ cx) + eg.n1[1] * (E0 @ cy)


def edge_operator_alg1(ops: RefOps, eg: EdgeGeometry, f1: int, f2: int, D1: float, D2: float):
    """Algorithm 1 (reconstruction of D grad u~) for element-wise constant D.
    Returns (W1, W2), [Nfp, Np] each; the flux includes D."""
    Np = ops.Np
    P1 = total_projection(ops, eg.pi1, f1)
    P2 = total_projection(ops, eg.pi2, f2)
    Z = np.zeros((Np, Np))
    W1 = _alg1_from_subtriangle_modal(ops, eg, P1, Z, D1, D2)
    W2 = _alg1_from_subtriangle_modal(ops, eg, Z, P2, D1, D2)
    return W1, W2


def boundary_edge_operator_alg1(ops: RefOps, geom, k1, f1, eg: EdgeGeometry, D1: float):
    P1 = total_projection(ops, eg.pi1, f1)
    P2 = ops.Vinv @ _boundary_ghost_data_operator(ops, geom, k1, eg)
    return _alg1_from_subtriangle_modal(ops, eg, P1, P2, D1, D1)


# ----------------------------------------------------------------------------
# Algorithm 2: reconstructed coefficient times the reconstructed gradient
# ----------------------------------------------------------------------------

def coefficient_on_diagonal(ops: RefOps, eg: EdgeGeometry, f1: int, f2: int, D1n, D2n) -> np.ndarray:
    """D~ = RDG(D^1, D^2) at the diagonal nodes d_j [Nfp], from the nodal
    coefficient values D^k [Np] of the two elements (Algorithm nonconstDiff2:
    the reconstruction of the coefficient, exactly as for u)."""
    N, Np = ops.N, ops.Np
    P1 = total_projection(ops, eg.pi1, f1)
    P2 = total_projection(ops, eg.pi2, f2)
    R = recon_pinv(N)
    c = R[:, :Np] @ (P1 @ np.asarray(D1n, dtype=np.float64)) + R[:, Np:] @ (P2 @ np.asarray(D2n, dtype=np.float64))
    E0, _, _ = diagonal_eval(N)
    return E0 @ c


def edge_operator_alg2(ops: RefOps, eg: EdgeGeometry, f1: int, f2: int, D1: float, D2: float):
    """Algorithm 2 for element-wise constant D: the flux D~(d_j) n1 . grad u~(d_j).
    Returns (W1, W2), [Nfp, Np] each; the flux includes D~."""
    W1, W2 = edge_operator(ops, eg, f1, f2)
    one = np.ones(ops.Np)
    Dt = coefficient_on_diagonal(ops, eg, f1, f2, D1 * one, D2 * one)
    return Dt[:, None] * W1, Dt[:, None] * W2


def boundary_coefficient_on_diagonal(ops: RefOps, eg: EdgeGeometry, f1: int, D1n) -> np.ndarray:
    """D~ at the diagonal nodes of a boundary face: side 1 projected as usual,
    the mirror ghost's coefficient on Omega'_2 is the element's D at the
    mirrored points (constant D: the constant itself)."""
    N, Np = ops.N, ops.Np
    D1n = np.asarray(D1n, dtype=np.float64)
    if np.ptp(D1n) != 0.0:
        raise ValueError("boundary coefficient: only element-wise constant D")
    P1 = total_projection(ops, eg.pi1, f1)
    R = recon_pinv(N)
    c = R[:, :Np] @ (P1 @ D1n) + R[:, Np:] @ (ops.Vinv @ D1n)
    E0, _, _ = diagonal_eval(N)
    return E0 @ c


def boundary_edge_operator_alg2(ops: RefOps, geom, k1, f1, eg: EdgeGeometry, D1: float):
    W = boundary_edge_operator(ops, geom, k1, f1, eg)
    Dt = boundary_coefficient_on_diagonal(ops, eg, f1, D1 * np.ones(ops.Np))
    return Dt[:, None] * W


# ----------------------------------------------------------------------------
# Boundary faces with prescribed exterior data on the ghost sub-triangle
# ----------------------------------------------------------------------------

def ghost_nodes(N: int, eg: EdgeGeometry) -> np.ndarray:
    """[Np, 2] physical points of the nodes of Omega'_2 = (P2, B, A), in the
    node order of the reference triangle mapped with those vertices."""
    rs = nodes(N)
    r, s = rs[:, 0], rs[:, 1]
    return (-(r + s)[:, None] / 2.0 * eg.P2[None, :] + (r + 1)[:, None] / 2.0 * eg.B[None, :]
            + (s + 1)[:, None] / 2.0 * eg.A[None, :])


def prescribed_boundary_operators(ops: RefOps, eg: EdgeGeometry, f1: int):
    """(W1, WG), [Nfp, Np] each: the flux n1 . grad u~ of a boundary face with
    u~ = RDG(u1, g), W1 acting on the element's nodal data and WG on the
    exterior state at ghost_nodes (already on Omega'_2: no projection)."""
    N, Np = ops.N, ops.Np
    R = recon_pinv(N)
    c1 = R[:, :Np] @ total_projection(ops, eg.pi1, f1)
    cg = R[:, Np:] @ ops.Vinv
    g1x, g1y = _gradient_on_diagonal(N, c1, eg)
    ggx, ggy = _gradient_on_diagonal(N, cg, eg)
    return eg.n1[0] * g1x + eg.n1[1] * g1y, eg.n1[0] * ggx + eg.n1[1] * ggy


def prescribed_boundary_operators_alg1(ops: RefOps, eg: EdgeGeometry, f1: int, D1: float):
    """Algorithm 1 at a boundary face with prescribed exterior data; the ghost
    carries the element's D."""
    Np = ops.Np
    P1 = total_projection(ops, eg.pi1, f1)
    Z = np.zeros((Np, Np))
    W1 = _alg1_from_subtriangle_modal(ops, eg, P1, Z, D1, D1)
    WG = _alg1_from_subtriangle_modal(ops, eg, Z, ops.Vinv, D1, D1)
    return W1, WG


def prescribed_boundary_operators_alg2(ops: RefOps, eg: EdgeGeometry, f1: int, D1: float):
    """Algorithm 2 at a boundary face with prescribed exterior data: the
    coefficient reconstructed from the element's D on both halves."""
    W1, WG = prescribed_boundary_operators(ops, eg, f1)
    Dt = boundary_coefficient_on_diagonal(ops, eg, f1, D1 * np.ones(ops.Np))
    return Dt[:, None] * W1, Dt[:, None] * WG


# ----------------------------------------------------------------------------
# Algorithm 1 with a nodal tensor coefficient
# ----------------------------------------------------------------------------

def nodal_on_subtriangle(ops: RefOps, pi, f: int, values) -> np.ndarray:
    """An element's nodal field [..., Np] evaluated at the nodes of its
    sub-triangle (the total projection followed by the sub-triangle's
    Vandermonde): V V^{-1} V_p V_rf^{-1} values."""
    return np.asarray(values) @ (ops.V @ total_projection(ops, pi, f)).T


def alg1_tensor_flux(ops: RefOps, eg: EdgeGeometry, m1, m2, Dp1, Dp2) -> np.ndarray:
    """Algorithm 1 with nodal tensor coefficients: m_k modal data on Omega'_k
    [Np], Dp_k [3, Np] = (Dxx, Dxy, Dyy) at Omega'_k's nodes.  Returns the
    flux n1 . (D grad u~)~ at the diagonal nodes [Nfp]."""
    N, Np = ops.N, ops.Np
    R = recon_pinv(N)
    c = R[:, :Np] @ m1 + R[:, Np:] @ m2                  # u~ = RDG(u1, u2)
    rs = nodes(N)
    u1n = phi(rs[:, 0], rs[:, 1], N) @ c                 # Separation
    u2n = phi(-rs[:, 0], -rs[:, 1], N) @ c
    g1x = eg.Rx * (ops.Dr @ u1n) + eg.Sx * (ops.Ds @ u1n)   # Grad, own frames
    g1y = eg.Ry * (ops.Dr @ u1n) + eg.Sy * (ops.Ds @ u1n)
    g2x = eg.Rx2 * (ops.Dr @ u2n) + eg.Sx2 * (ops.Ds @ u2n)
    g2y = eg.Ry2 * (ops.Dr @ u2n) + eg.Sy2 * (ops.Ds @ u2n)
    q1x, q1y = Dp1[0] * g1x + Dp1[1] * g1y, Dp1[1] * g1x + Dp1[2] * g1y
    q2x, q2y = Dp2[0] * g2x + Dp2[1] * g2y, Dp2[1] * g2x + Dp2[2] * g2y
    cx = R[:, :Np] @ (ops.Vinv @ q1x) + R[:, Np:] @ (ops.Vinv @ q2x)   # second RDG
    cy = R[:, :Np] @ (ops.Vinv @ q1y) + R[:, Np:] @ (ops.Vinv @ q2y)
    E0, _, _ = diagonal_eval(N)
    return eg.n1[0] * (E0 @ cx) + eg.n1[1] * (E0 @ cy)


def mirrored_on_ghost(ops: RefOps, geom, k1, eg: EdgeGeometry, values) -> np.ndarray:
    """An element's nodal field evaluated at the mirror images of the nodes of
    the ghost sub-triangle (P2, B, A): the even reflection of a coefficient
    (the ghost's data is minus this for the solution)."""
    return -(np.asarray(values) @ _boundary_ghost_data_operator(ops, geom, k1, eg).T)
