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


def physical_edge_flux(N, eg, xy1, u1, v1, xy2, u2, v2):
    """n1 . grad u~ at the edge's LGL points (A -> B), by physical LS.

    Side 2 given as None means a boundary face: the ghost is the mirror image
    carrying -u1 at mirrored points.
    """
    from oracle.reference_element import lgl_nodes   # 1D LGL points only
    P1, P2, A, B = eg.P1, eg.P2, eg.A, eg.B
    p1 = PhysPoly(N, xy1, u1)
    if xy2 is None:
        def p2(X):
            return -p1(_mirror(X, A, B))
    else:
        p2 = PhysPoly(N, xy2, u2)
    nq = 2 * N + 3
    X1, w1 = tri_rule(nq, np.array([P1, A, B]))
    X2, w2 = tri_rule(nq, np.array([P2, B, A]))
    # parallelogram affine coordinates: X(R,S) = -(R+S)/2 P1 + (R+1)/2 A + (S+1)/2 B
    Jm = 0.5 * np.column_stack([A - P1, B - P1])
    Jinv = np.linalg.inv(Jm)
    centre = 0.5 * (A + B)

    def RS(X):
        return (X - centre) @ Jinv.T       # X(0,0) is the midpoint of AB

    qterms = [(a, b) for a in range(N + 1) for b in range(N + 1)]

    def qbasis(X):
        rs = RS(X)
        return np.stack([rs[:, 0] ** a * rs[:, 1] ** b for (a, b) in qterms], axis=1)

    rows, rhs = [], []
    for (X, w, p) in ((X1, w1, p1), (X2, w2, p2)):
        c0 = X.mean(axis=0)
        h = np.abs(X - c0).max()
        T = _orthonormal_PN(N, X, w, c0, h)
        rows.append((T * w[:, None]).T @ qbasis(X))
        rhs.append((T * w[:, None]).T @ p(X))
    Amat = np.vstack(rows)
    bvec = np.concatenate(rhs)
    c = np.linalg.lstsq(Amat, bvec, rcond=None)[0]
    t = lgl_nodes(N)[::-1]
    Xd = ((1 + t) / 2)[:, None] * A + ((1 - t) / 2)[:, None] * B
    rs = RS(Xd)
    dR = np.stack([a * rs[:, 0] ** max(a - 1, 0) * rs[:, 1] ** b if a else 0 * rs[:, 0]
                   for (a, b) in qterms], axis=1) @ c
    dS = np.stack([b * rs[:, 0] ** a * rs[:, 1] ** max(b - 1, 0) if b else 0 * rs[:, 0]
                   for (a, b) in qterms], axis=1) @ c
    grad = np.stack([dR, dS], axis=1) @ Jinv          # chain rule: d/dx = J^{-T} d/dR
    return grad @ eg.n1
