"""Reference-triangle operators, FP64.  TEST INFRASTRUCTURE ONLY.

Follows the section "Nodal discontinuous Galerkin method": nodal Lagrange
expansion on LGL-type nodes, orthonormal modal basis psi, the Vandermonde
matrix (eq. Vandermonde), reference mass and stiffness (via Dr, Ds), and the
reference LIFT operator (eq. lift_physicalDomain_ardg).

Reference triangle I = {(r,s): r,s >= -1, r+s <= 0} with vertices
a1=(-1,-1), a2=(1,-1), a3=(-1,1).

Node order (the state layout shared with the library): lattice points (i,j),
i,j >= 0, i+j <= N, row by row in j (rows of increasing s), within a row in i
(increasing r).  Lattice point (i,j) has barycentric coordinates
((N-i-j)/N, i/N, j/N) with respect to (a1, a2, a3) before warping.

Reading of the node set (the paper only says "LGL nodes"): Warburton's
warp-and-blend nodes with blend parameter alpha = 0, whose edge nodes are
exactly the 1D LGL points.  This oracle builds them on the equilateral
triangle and maps them back to I.
"""
from __future__ import annotations

import math
from functools import lru_cache

import numpy as np
from scipy.special import eval_jacobi, gammaln, roots_jacobi


# ----------------------------------------------------------------------------
# 1D: LGL nodes and normalised Jacobi polynomials
# ----------------------------------------------------------------------------

def lgl_nodes(N: int) -> np.ndarray:
    """Legendre-Gauss-Lobatto points: -1, +1 and the roots of P'_N.

    The roots of P'_N are the Gauss-Jacobi points with alpha=beta=1.
    Returned in increasing order.
    """
    if N < 1:
        raise ValueError("N >= 1")
    if N == 1:
        return np.array([-1.0, 1.0])
    x, _ = roots_jacobi(N - 1, 1.0, 1.0)
    return np.concatenate([[-1.0], np.sort(x), [1.0]])


def jacobi_normalised(x, n: int, alpha: float, beta: float):
    """P_n^{(alpha,beta)}(x) scaled to unit norm under (1-x)^alpha (1+x)^beta."""
    x = np.asarray(x, dtype=np.float64)
    if n < 0:
        return np.zeros_like(x)
    log_h = ((alpha + beta + 1) * math.log(2.0) - math.log(2 * n + alpha + beta + 1)
             + gammaln(n + alpha + 1) + gammaln(n + beta + 1)
             - gammaln(n + alpha + beta + 1) - gammaln(n + 1))
    return eval_jacobi(n, alpha, beta, x) / math.exp(0.5 * log_h)


def jacobi_normalised_deriv(x, n: int, alpha: float, beta: float):
    """d/dx of jacobi_normalised, from d/dx P_n^{(a,b)} = (n+a+b+1)/2 P_{n-1}^{(a+1,b+1)}."""
    x = np.asarray(x, dtype=np.float64)
    if n == 0:
        return np.zeros_like(x)
    log_h = ((alpha + beta + 1) * math.log(2.0) - math.log(2 * n + alpha + beta + 1)
             + gammaln(n + alpha + 1) + gammaln(n + beta + 1)
             - gammaln(n + alpha + beta + 1) - gammaln(n + 1))
    raw = 0.5 * (n + alpha + beta + 1) * eval_jacobi(n - 1, alpha + 1, beta + 1, x)
    return raw / math.exp(0.5 * log_h)


def vandermonde_1d(N: int, t: np.ndarray) -> np.ndarray:
    return np.stack([jacobi_normalised(t, n, 0.0, 0.0) for n in range(N + 1)], axis=1)


def mass_1d(N: int) -> np.ndarray:
    """1D mass matrix of the Lagrange basis on the LGL points, M1 = (V1 V1^T)^{-1}."""
    V1 = vandermonde_1d(N, lgl_nodes(N))
    return np.linalg.inv(V1 @ V1.T)


# ----------------------------------------------------------------------------
# Triangle nodes (warp & blend, alpha = 0), built on the equilateral triangle
# ----------------------------------------------------------------------------

_EQ = np.array([[-1.0, -1.0 / math.sqrt(3.0)],
                [1.0, -1.0 / math.sqrt(3.0)],
                [0.0, 2.0 / math.sqrt(3.0)]])  # equilateral images of a1, a2, a3
_REF = np.array([[-1.0, -1.0], [1.0, -1.0], [-1.0, 1.0]])  # a1, a2, a3


def _lagrange_eval(xnodes: np.ndarray, j: int, x: np.ndarray) -> np.ndarray:
    out = np.ones_like(x)
    for m, xm in enumerate(xnodes):
        if m != j:
            out = out * (x - xm) / (xnodes[j] - xm)
    return out


def _warp(N: int, r: np.ndarray) -> np.ndarray:
    """1D displacement that moves equispaced points onto LGL points, as a
    polynomial interpolating (LGL_k - equi_k) at the equispaced points."""
    lgl = lgl_nodes(N)
    eq = np.linspace(-1.0, 1.0, N + 1)
    w = np.zeros_like(r)
    for k in range(N + 1):
        w = w + (lgl[k] - eq[k]) * _lagrange_eval(eq, k, r)
    return w


@lru_cache(maxsize=None)
def nodes(N: int) -> np.ndarray:
    """[Np, 2] reference coordinates (r, s) of the triangle nodes."""
    lam = []
    for j in range(N + 1):
        for i in range(N + 1 - j):
            lam.append(((N - i - j) / N, i / N, j / N))
    lam = np.array(lam)
    X = lam @ _EQ
    for (a, b) in ((0, 1), (1, 2), (2, 0)):
        r = lam[:, b] - lam[:, a]
        blend = 4.0 * lam[:, a] * lam[:, b]
        w = _warp(N, r)
        denom = 1.0 - r * r
        safe = np.abs(denom) > 1e-12
        wf = np.where(safe, w / np.where(safe, denom, 1.0), 0.0)
        tangent = (_EQ[b] - _EQ[a]) / np.linalg.norm(_EQ[b] - _EQ[a])
        X = X + (blend * wf)[:, None] * tangent[None, :]
    # back to barycentric coordinates, then to (r, s)
    T = np.array([[_EQ[1, 0] - _EQ[0, 0], _EQ[2, 0] - _EQ[0, 0]],
                  [_EQ[1, 1] - _EQ[0, 1], _EQ[2, 1] - _EQ[0, 1]]])
    l23 = np.linalg.solve(T, (X - _EQ[0]).T).T
    lam_w = np.column_stack([1.0 - l23[:, 0] - l23[:, 1], l23[:, 0], l23[:, 1]])
    return lam_w @ _REF


# ----------------------------------------------------------------------------
# Orthonormal basis on I (collapsed coordinates) and its gradient
# ----------------------------------------------------------------------------

def mode_list(N: int):
    return [(i, j) for i in range(N + 1) for j in range(N + 1 - i)]


def _collapse(r, s):
    r = np.asarray(r, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    top = np.abs(1.0 - s) < 1e-14
    a = np.where(top, -1.0, 2.0 * (1.0 + r) / np.where(top, 1.0, 1.0 - s) - 1.0)
    return a, s


def psi(r, s, i: int, j: int):
    """psi_ij = sqrt(2) P_i(a) P_j^{(2i+1,0)}(b) (1-b)^i, orthonormal on I."""
    a, b = _collapse(r, s)
    return (math.sqrt(2.0) * jacobi_normalised(a, i, 0, 0)
            * jacobi_normalised(b, j, 2 * i + 1, 0) * (1.0 - b) ** i)


def grad_psi(r, s, i: int, j: int):
    a, b = _collapse(r, s)
    fa = jacobi_normalised(a, i, 0, 0)
    dfa = jacobi_normalised_deriv(a, i, 0, 0)
    gb = jacobi_normalised(b, j, 2 * i + 1, 0)
    dgb = jacobi_normalised_deriv(b, j, 2 * i + 1, 0)
    pw = (1.0 - b) ** (i - 1) if i >= 1 else np.zeros_like(b)
    dr = 2.0 * math.sqrt(2.0) * dfa * gb * pw
    ds = math.sqrt(2.0) * (dfa * (1.0 + a) * gb * pw + fa * dgb * (1.0 - b) ** i
                           - i * fa * gb * pw)
    return dr, ds


def vandermonde(N: int, r, s) -> np.ndarray:
    return np.stack([psi(r, s, i, j) for (i, j) in mode_list(N)], axis=-1)


def grad_vandermonde(N: int, r, s):
    cols = [grad_psi(r, s, i, j) for (i, j) in mode_list(N)]
    return (np.stack([c[0] for c in cols], axis=-1),
            np.stack([c[1] for c in cols], axis=-1))


# ----------------------------------------------------------------------------
# Face nodes, reference operators
# ----------------------------------------------------------------------------

def face_nodes(N: int):
    """Indices of the nodes on each face, listed counter-clockwise.

    f1 = (a1 -> a2) on s = -1; f2 = (a2 -> a3), the hypotenuse; f3 = (a3 -> a1)
    on r = -1.  Found from coordinates.
    """
    rs = nodes(N)
    r, s = rs[:, 0], rs[:, 1]
    tol = 1e-10
    f1 = np.where(np.abs(s + 1) < tol)[0]
    f1 = f1[np.argsort(r[f1])]
    f2 = np.where(np.abs(r + s) < tol)[0]
    f2 = f2[np.argsort(s[f2])]
    f3 = np.where(np.abs(r + 1) < tol)[0]
    f3 = f3[np.argsort(-s[f3])]
    return [f1, f2, f3]


class RefOps:
    """All reference-element matrices for order N."""

    def __init__(self, N: int):
        self.N = N
        self.Np = (N + 1) * (N + 2) // 2
        self.Nfp = N + 1
        self.rs = nodes(N)
        r, s = self.rs[:, 0], self.rs[:, 1]
        self.V = vandermonde(N, r, s)
        self.Vinv = np.linalg.inv(self.V)
        Vr, Vs = grad_vandermonde(N, r, s)
        self.Dr = Vr @ self.Vinv
        self.Ds = Vs @ self.Vinv
        self.M = np.linalg.inv(self.V @ self.V.T)
        self.Minv = self.V @ self.V.T
        self.fmask = face_nodes(N)
        M1 = mass_1d(N)
        E = np.zeros((self.Np, 3 * self.Nfp))
        for f in range(3):
            E[np.ix_(self.fmask[f], np.arange(f * self.Nfp, (f + 1) * self.Nfp))] = M1
        self.LIFT = self.Minv @ E
        # weak derivative matrices Drw = M^{-1} Dr^T M, Dsw likewise
        self.Drw = self.Minv @ self.Dr.T @ self.M
        self.Dsw = self.Minv @ self.Ds.T @ self.M
