"""Physical-domain brute force for the reconstruction and the RHS (tests only).

Nothing here uses the reference-domain operators of the oracle (no V_p, no
rotations, no reference reconstruction matrix): polynomials are handled as
monomials in physical coordinates, integrals use Gauss rules mapped onto the
physical triangles, and the reconstruction space Q_N is spanned by monomials
R^a S^b of the parallelogram's own affine coordinates.  Only the node layout
(an input convention) and the enclosed parallelogram apex are taken as given.
"""
from __future__ import annotations

import numpy as np
from scipy.special import roots_jacobi, roots_legendre


def tri_rule(n, v):
    """Collapsed Gauss rule mapped to the physical triangle v [3,2]."""
    a, wa = roots_legendre(n)
    b, wb = roots_jacobi(n, 1.0, 0.0)
    A, B = np.meshgrid(a, b, indexing="ij")
    # unit-simplex coordinates
    xi = 0.25 * (1 + A) * (1 - B)
    eta = 0.5 * (1 + B)
    w = np.outer(wa, wb) * 0.125
    x = v[0] + np.multiply.outer(xi.ravel(), v[1] - v[0]) + np.multiply.outer(eta.ravel(), v[2] - v[0])
    area2 = abs((v[1, 0] - v[0, 0]) * (v[2, 1] - v[0, 1]) - (v[2, 0] - v[0, 0]) * (v[1, 1] - v[0, 1]))
    return x, w.ravel() * area2


class PhysPoly:
    """Degree-N polynomial through nodal values at physical points (monomial
    fit in coordinates centred and scaled on the element)."""

    def __init__(self, N, xy_nodes, values):
        self.N = N
        self.c0 = xy_nodes.mean(axis=0)
        self.h = np.abs(xy_nodes - self.c0).max()
        self.terms = [(a, b) for a in range(N + 1) for b in range(N + 1 - a)]
        Vm = self._mono(xy_nodes)
        self.coef = np.linalg.solve(Vm, values)

    def _mono(self, X):
        z = (X - self.c0) / self.h
        return np.stack([z[:, 0] ** a * z[:, 1] ** b for (a, b) in self.terms], axis=1)

    def __call__(self, X):
        return self._mono(X) @ self.coef

    def grad(self, X):
        """Physical gradient [len(X), 2] of the fitted polynomial."""
        z = (X - self.c0) / self.h
        gx = np.stack([a * z[:, 0] ** max(a - 1, 0) * z[:, 1] ** b if a else 0 * z[:, 0]
                       for (a, b) in self.terms], axis=1) @ self.coef / self.h
        gy = np.stack([b * z[:, 0] ** a * z[:, 1] ** max(b - 1, 0) if b else 0 * z[:, 0]
                       for (a, b) in self.terms], axis=1) @ self.coef / self.h
        return np.stack([gx, gy], axis=1)

    def basis(self, X):
        """Values of the Lagrange basis (nodal) at X: [len(X), Np]."""
        return self._mono(X) @ np.linalg.inv(self._Vn)

    def set_nodes(self, xy_nodes):
        self._Vn = self._mono(xy_nodes)
        return self

    def basis_grad(self, X):
        z = (X - self.c0) / self.h
        gx = np.stack([a * z[:, 0] ** max(a - 1, 0) * z[:, 1] ** b if a else 0 * z[:, 0]
                       for (a, b) in self.terms], axis=1) / self.h
        gy = np.stack([b * z[:, 0] ** a * z[:, 1] ** max(b - 1, 0) if b else 0 * z[:, 0]
                       for (a, b) in self.terms], axis=1) / self.h
        Vi = np.linalg.inv(self._Vn)
        return gx @ Vi, gy @ Vi


def _orthonormal_PN(N, X, w, c0, h):
    """Orthonormal basis of P_N on a sub-triangle (Cholesky of the Gram matrix)."""
    z = (X - c0) / h
    terms = [(a, b) for a in range(N + 1) for b in range(N + 1 - a)]
    Mo = np.stack([z[:, 0] ** a * z[:, 1] ** b for (a, b) in terms], axis=1)
    G = (Mo * w[:, None]).T @ Mo
    L = np.linalg.cholesky(G)
    return np.linalg.solve(L, Mo.T).T          # [Q, Np], orthonormal under w


def _mirror(p, A, B):
    d = B - A
    t = ((p - A) @ d) / (d @ d)
    foot = A + np.outer(t, d)
    return 2 * foot - p


class ParallelogramLS:
    """Least-squares fit of Q_N on the enclosed parallelogram, in physical
    coordinates.

    The unknowns are the coefficients of the monomials R^a S^b (0 <= a, b <= N)
    of the parallelogram's own affine coordinates, X(R, S) = -(R+S)/2 P1 +
    (R+1)/2 A + (S+1)/2 B; the equations are the L2 moments against an
    orthonormal basis of P_N on each physical sub-triangle (P1, A, B) and
    (P2, B, A), integrated with Gauss rules mapped onto them.
    """

    def __init__(self, N, eg):
        self.N = N
        self.P1, self.P2, self.A, self.B = eg.P1, eg.P2, eg.A, eg.B
        nq = 2 * N + 3
        self.X1, self.w1 = tri_rule(nq, np.array([self.P1, self.A, self.B]))
        self.X2, self.w2 = tri_rule(nq, np.array([self.P2, self.B, self.A]))
        Jm = 0.5 * np.column_stack([self.A - self.P1, self.B - self.P1])
        self.Jinv = np.linalg.inv(Jm)
        self.centre = 0.5 * (self.A + self.B)     # X(0, 0) is the midpoint of AB
        self.qterms = [(a, b) for a in range(N + 1) for b in range(N + 1)]
        self.T = []
        rows = []
        for (X, w) in ((self.X1, self.w1), (self.X2, self.w2)):
            c0 = X.mean(axis=0)
            h = np.abs(X - c0).max()
            T = _orthonormal_PN(N, X, w, c0, h)
            self.T.append(T)
            rows.append((T * w[:, None]).T @ self.qbasis(X))
        self.Amat = np.vstack(rows)

    def RS(self, X):
        return (X - self.centre) @ self.Jinv.T

    def qbasis(self, X):
        rs = self.RS(X)
        return np.stack([rs[:, 0] ** a * rs[:, 1] ** b for (a, b) in self.qterms], axis=1)

    def fit(self, f1, f2):
        """Q_N coefficients of the fit to data f1 on (P1, A, B) and f2 on
        (P2, B, A) (callables of physical points)."""
        rhs = [(self.T[0] * self.w1[:, None]).T @ f1(self.X1),
               (self.T[1] * self.w2[:, None]).T @ f2(self.X2)]
        return np.linalg.lstsq(self.Amat, np.concatenate(rhs), rcond=None)[0]

    def value(self, c, X):
        return self.qbasis(X) @ c

    def grad(self, c, X):
        """Physical gradient [len(X), 2] of the fit (chain rule through J^-T)."""
        rs = self.RS(X)
        dR = np.stack([a * rs[:, 0] ** max(a - 1, 0) * rs[:, 1] ** b if a else 0 * rs[:, 0]
                       for (a, b) in self.qterms], axis=1) @ c
        dS = np.stack([b * rs[:, 0] ** a * rs[:, 1] ** max(b - 1, 0) if b else 0 * rs[:, 0]
                       for (a, b) in self.qterms], axis=1) @ c
        return np.stack([dR, dS], axis=1) @ self.Jinv

    def diagonal(self):
        """The edge's LGL points from A to B (the interface nodes)."""
        from oracle.reference_element import lgl_nodes   # 1D LGL points only
        t = lgl_nodes(self.N)[::-1]
        return ((1 + t) / 2)[:, None] * self.A + ((1 - t) / 2)[:, None] * self.B


def _side_data(N, eg, xy1, u1, xy2, u2):
    p1 = PhysPoly(N, xy1, u1)
    if xy2 is None:
        A, B = eg.A, eg.B

        def p2(X):
            return -p1(_mirror(X, A, B))
    else:
        p2 = PhysPoly(N, xy2, u2)
    return p1, p2


def physical_edge_flux(N, eg, xy1, u1, v1, xy2, u2, v2):
    """n1 . grad u~ at the edge's LGL points (A -> B), by physical LS.

    Side 2 given as None means a boundary face: the ghost is the mirror image
    carrying -u1 at mirrored points.
    """
    p1, p2 = _side_data(N, eg, xy1, u1, xy2, u2)
    ls = ParallelogramLS(N, eg)
    c = ls.fit(p1, p2)
    return ls.grad(c, ls.diagonal()) @ eg.n1


def _map_nodes(rs, V):
    """Reference nodes mapped affinely onto the physical triangle V [3, 2]."""
    r, s = rs[:, 0], rs[:, 1]
    return (-(r + s)[:, None] / 2 * V[0] + (r + 1)[:, None] / 2 * V[1]
            + (s + 1)[:, None] / 2 * V[2])


def physical_edge_flux_alg1(N, eg, rs_nodes, xy1, u1, xy2, u2, D1, D2):
    """Algorithm 1 (reconstruction of D grad u~) assembled in physical
    coordinates, D1 and D2 the constant coefficients of the two elements.

    1. u~ = least-squares fit of the two elements' polynomials on the
       parallelogram (physical moments);
    2. separation: u~ sampled at the nodes of each physical sub-triangle
       (the node layout rs_nodes is the input convention) and interpolated
       there by a degree-N polynomial;
    3. each sub-triangle's polynomial is differentiated in x and y and
       multiplied by its element's D;
    4. a second least-squares fit of each component of D grad u~ on the
       parallelogram;
    5. n1 . (result) at the edge's LGL points.
    Side 2 given as None is a boundary face: the mirror ghost carries -u1 at
    mirrored points and the element's own D.
    """
    p1, p2 = _side_data(N, eg, xy1, u1, xy2, u2)
    ls = ParallelogramLS(N, eg)
    c = ls.fit(p1, p2)
    flux_parts = []
    for V, Dk in ((np.array([eg.P1, eg.A, eg.B]), D1), (np.array([eg.P2, eg.B, eg.A]), D2)):
        Xn = _map_nodes(rs_nodes, V)
        pk = PhysPoly(N, Xn, ls.value(c, Xn))
        flux_parts.append((pk, Dk))

    def comp(k, d):
        pk, Dk = flux_parts[k]
        return lambda X: Dk * pk.grad(X)[:, d]

    cx = ls.fit(comp(0, 0), comp(1, 0))
    cy = ls.fit(comp(0, 1), comp(1, 1))
    Xd = ls.diagonal()
    return eg.n1[0] * ls.value(cx, Xd) + eg.n1[1] * ls.value(cy, Xd)


def physical_edge_flux_alg1_tensor(N, eg, rs_nodes, xy1, u1, D1, xy2, u2, D2, D0=None):
    """Algorithm 1 with a nodal tensor coefficient, in physical coordinates.

    D_k: callable X -> [len(X), 3] (Dxx, Dxy, Dyy) of side k's coefficient
    (the element's coefficient polynomial, evaluated anywhere); with D0
    given instead, the coefficient of each side is D0 times that side's state.
    Side 2 given as xy2 = None: the mirror ghost carrying -u1, with the
    coefficient at mirrored points (or D0 times the ghost's state).
    """
    p1 = PhysPoly(N, xy1, u1)
    if xy2 is None:
        A, B = eg.A, eg.B

        def p2(X):
            return -p1(_mirror(X, A, B))

        def D2(X, D1=D1):
            return D1(_mirror(X, A, B))
    else:
        p2 = PhysPoly(N, xy2, u2)
    if D0 is not None:
        D1 = lambda X: p1(X)[:, None] * np.asarray(D0)[None, :]
        D2 = lambda X: p2(X)[:, None] * np.asarray(D0)[None, :]
    ls = ParallelogramLS(N, eg)
    c = ls.fit(p1, p2)
    parts = []
    for V, Dk in ((np.array([eg.P1, eg.A, eg.B]), D1), (np.array([eg.P2, eg.B, eg.A]), D2)):
        Xn = _map_nodes(rs_nodes, V)
        pk = PhysPoly(N, Xn, ls.value(c, Xn))         # separation
        g = pk.grad(Xn)
        Dn = Dk(Xn)                                    # coefficient at the sub-triangle's nodes
        qx = Dn[:, 0] * g[:, 0] + Dn[:, 1] * g[:, 1]
        qy = Dn[:, 1] * g[:, 0] + Dn[:, 2] * g[:, 1]
        parts.append((PhysPoly(N, Xn, qx), PhysPoly(N, Xn, qy)))
    cx = ls.fit(parts[0][0], parts[1][0])
    cy = ls.fit(parts[0][1], parts[1][1])
    Xd = ls.diagonal()
    return eg.n1[0] * ls.value(cx, Xd) + eg.n1[1] * ls.value(cy, Xd)
