"""Pins for the oracle's reference-element operators (CPU only).

Each check compares against something other than the oracle itself: closed-form
LGL points, closed-form monomial integrals on the triangle, exact derivatives
of monomials, the length of an edge, and integer symmetry facts.
"""
import json
import math
import os
from fractions import Fraction
from math import comb, factorial

import numpy as np
import pytest

from oracle import ardg
from oracle.reference_element import (RefOps, face_nodes, lgl_nodes, mass_1d, mode_list,
                                      nodes, vandermonde)

HERE = os.path.dirname(os.path.abspath(__file__))


def monomial_integral_I(a: int, b: int) -> float:
    """Exact int_I r^a s^b dr ds: r = 2 xi - 1, s = 2 eta - 1 on the unit
    simplex, int xi^i eta^j = i! j! / (i+j+2)!."""
    tot = Fraction(0)
    for i in range(a + 1):
        for j in range(b + 1):
            c = (comb(a, i) * 2 ** i * (-1) ** (a - i) * comb(b, j) * 2 ** j * (-1) ** (b - j))
            tot += c * Fraction(factorial(i) * factorial(j), factorial(i + j + 2))
    return float(4 * tot)


def test_lgl_closed_forms():
    assert np.allclose(lgl_nodes(1), [-1, 1], atol=1e-15)
    assert np.allclose(lgl_nodes(2), [-1, 0, 1], atol=1e-15)
    assert np.allclose(lgl_nodes(3), [-1, -1 / math.sqrt(5), 1 / math.sqrt(5), 1], atol=1e-15)
    assert np.allclose(lgl_nodes(4), [-1, -math.sqrt(3 / 7), 0, math.sqrt(3 / 7), 1], atol=1e-15)


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6])
def test_lgl_integrates_exactly(N):
    # Lobatto rule with the 1D mass matrix row sums as weights: exact to degree 2N-1
    t = lgl_nodes(N)
    w = mass_1d(N).sum(axis=1)
    for d in range(2 * N):
        exact = (1 - (-1) ** (d + 1)) / (d + 1)
        assert abs(np.dot(w, t ** d) - exact) < 1e-13


@pytest.mark.parametrize("n", [3, 6, 10])
def test_triangle_quadrature_matches_closed_form(n):
    r, s, w = ardg.triangle_quadrature(n)
    for a in range(2 * n - 1):
        for b in range(2 * n - 1 - a):
            ex = monomial_integral_I(a, b)
            assert abs(np.dot(w, r ** a * s ** b) - ex) < 1e-13 * max(1.0, abs(ex))


@pytest.mark.parametrize("N", [1, 2, 3, 4, 6])
def test_basis_orthonormal(N):
    r, s, w = ardg.triangle_quadrature(N + 2)
    V = vandermonde(N, r, s)
    G = (V * w[:, None]).T @ V
    assert np.abs(G - np.eye(len(mode_list(N)))).max() < 1e-13


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6])
def test_nodes_structure(N):
    rs = nodes(N)
    Np = (N + 1) * (N + 2) // 2
    assert rs.shape == (Np, 2)
    # inside I
    assert np.all(rs[:, 0] >= -1 - 1e-14) and np.all(rs[:, 1] >= -1 - 1e-14)
    assert np.all(rs.sum(axis=1) <= 1e-14)
    # every face carries exactly the LGL points, counter-clockwise
    t = lgl_nodes(N)
    f1, f2, f3 = face_nodes(N)
    assert np.allclose(rs[f1, 0], t, atol=1e-14)            # s=-1, r increasing
    assert np.allclose(rs[f2, 1], t, atol=1e-14)            # hypotenuse, s increasing
    assert np.allclose(rs[f3, 1], t[::-1], atol=1e-14)      # r=-1, s decreasing
    # row-by-row lattice order: first row is face 1
    assert list(f1) == list(range(N + 1))


@pytest.mark.parametrize("N", [1, 2, 3, 4, 6])
def test_nodes_unisolvent_and_lebesgue_reasonable(N):
    V = vandermonde(N, nodes(N)[:, 0], nodes(N)[:, 1])
    assert np.linalg.cond(V) < 1e3


@pytest.mark.parametrize("N", [1, 2, 3, 4, 6])
def test_derivative_matrices_exact_on_monomials(N):
    ops = RefOps(N)
    r, s = ops.rs[:, 0], ops.rs[:, 1]
    for a in range(N + 1):
        for b in range(N + 1 - a):
            p = r ** a * s ** b
            dr = a * r ** max(a - 1, 0) * s ** b
            ds = b * r ** a * s ** max(b - 1, 0)
            assert np.abs(ops.Dr @ p - dr).max() < 1e-12 * (N ** 2 + 1)
            assert np.abs(ops.Ds @ p - ds).max() < 1e-12 * (N ** 2 + 1)


@pytest.mark.parametrize("N", [1, 2, 3, 4, 6])
def test_mass_matrix_integrates_monomials(N):
    ops = RefOps(N)
    r, s = ops.rs[:, 0], ops.rs[:, 1]
    one = np.ones(ops.Np)
    for a in range(N + 1):
        for b in range(N + 1 - a):
            for c in range(N + 1):
                for d in range(N + 1 - c):
                    p, q = r ** a * s ** b, r ** c * s ** d
                    ex = monomial_integral_I(a + c, b + d)
                    assert abs(p @ ops.M @ q - ex) < 1e-12
            assert abs(one @ ops.M @ (r ** a * s ** b) - monomial_integral_I(a, b)) < 1e-13


@pytest.mark.parametrize("N", [1, 2, 3, 4, 6])
def test_lift_edge_integrals(N):
    """1^T M LIFT_f g = int_{-1}^{1} g dt for polynomial traces g, and with the
    surface scale |edge|/2 the lifted constant integrates to the edge length."""
    ops = RefOps(N)
    t = lgl_nodes(N)
    Nfp = ops.Nfp
    for f in range(3):
        Lf = ops.LIFT[:, f * Nfp:(f + 1) * Nfp]
        for d in range(N + 1):
            g = t ** d
            ex = (1 - (-1) ** (d + 1)) / (d + 1)
            assert abs(np.ones(ops.Np) @ ops.M @ Lf @ g - ex) < 1e-13
    # physical check on a random triangle: J 1^T M (sJ/J) LIFT_f 1 = |edge|
    rng = np.random.default_rng(3)
    v = rng.uniform(size=(3, 2))
    if (v[1, 0] - v[0, 0]) * (v[2, 1] - v[0, 1]) - (v[2, 0] - v[0, 0]) * (v[1, 1] - v[0, 1]) < 0:
        v = v[[0, 2, 1]]
    xr, yr = (v[1] - v[0]) / 2
    xs, ys = (v[2] - v[0]) / 2
    J = xr * ys - xs * yr
    for f, (a, b) in enumerate(((0, 1), (1, 2), (2, 0))):
        L = np.linalg.norm(v[b] - v[a])
        Lf = ops.LIFT[:, f * Nfp:(f + 1) * Nfp]
        val = J * np.ones(ops.Np) @ ops.M @ ((L / 2) / J * Lf @ np.ones(Nfp))
        assert abs(val - L) < 1e-13


@pytest.mark.parametrize("N", [1, 2, 3, 4, 6])
def test_rotations(N):
    ops = RefOps(N)
    f1, f2, f3 = ops.fmask
    for f, fm in enumerate(ops.fmask):
        p = ardg.rotation_perm(N, f)
        assert sorted(p.tolist()) == list(range(ops.Np))
        # face f (CCW) lands on the hypotenuse (CCW) of the rotated ordering
        assert list(p[f2]) == list(fm)
    p0, p2 = ardg.rotation_perm(N, 0), ardg.rotation_perm(N, 2)
    # rotating three times by the same cyclic relabelling is the identity
    assert list(p0[p0[p0]]) == list(range(ops.Np))
    assert list(p0[p2]) == list(range(ops.Np))


def test_storage_table_counts():
    """Table 1: (P+1)^2 modes on the parallelogram and a (P+1)^4 mass matrix,
    one J and four R_X values per interior edge, stored once."""
    with open(os.path.join(HERE, "golden", "paper_table1_storage.json")) as fh:
        t1 = json.load(fh)
    for P, Mp, mass in zip(t1["P"], t1["modes_on_parallelogram"], t1["mass_matrix_values"]):
        A = ardg.recon_system(P)
        Np = (P + 1) * (P + 2) // 2
        assert A.shape == (2 * Np, Mp)
        assert Mp * Mp == mass
    assert set(t1["parallelogram_J_per_edge"]) == {1}
    assert set(t1["parallelogram_RX_per_edge"]) == {4}
