"""Pins for the oracle's enclosed parallelogram, projection, reconstruction and
edge flux (CPU only)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import ardg
from oracle.mesh import Geometry
from oracle.reference_element import RefOps, lgl_nodes, nodes, vandermonde
from oracle.rhs import Problem

from physical_bruteforce import physical_edge_flux


def _tri_area(a, b, c):
    return 0.5 * ((b[0] - a[0]) * (c[1] - a[1]) - (c[0] - a[0]) * (b[1] - a[1]))


def _inside(p, a, b, c, tol=1e-12):
    return (_tri_area(a, b, p) >= -tol and _tri_area(b, c, p) >= -tol and _tri_area(c, a, p) >= -tol)


def _random_quad(rng):
    A = np.array([0.0, 0.0])
    B = np.array([1.0, 0.0]) + rng.uniform(-0.3, 0.3, 2)
    C1 = np.array([rng.uniform(-0.5, 1.5), rng.uniform(0.2, 1.2)])
    C2 = np.array([rng.uniform(-0.5, 1.5), rng.uniform(-1.2, -0.2)])
    # orient: (A, B, C1) CCW, (B, A, C2) CCW
    return A, B, C1, C2


# ----------------------------------------------------------------------------
# Enclosed parallelogram
# ----------------------------------------------------------------------------

def test_parallelogram_of_a_parallelogram_is_itself():
    A, B = np.array([0.0, 0.0]), np.array([1.0, 0.2])
    C1 = np.array([0.3, 0.9])
    C2 = A + B - C1
    P1 = ardg.parallelogram_apex(A, B, C1, C2)
    assert np.allclose(P1, C1, atol=1e-14)


@pytest.mark.parametrize("seed", range(12))
def test_parallelogram_matches_grid_search(seed):
    """Brute force over a fine grid of w: maximise the height of m+w above AB
    with m+w in Omega_1 and m-w in Omega_2."""
    rng = np.random.default_rng(seed)
    A, B, C1, C2 = _random_quad(rng)
    P1 = ardg.parallelogram_apex(A, B, C1, C2)
    m = 0.5 * (A + B)
    assert _inside(P1, A, B, C1, 1e-12) and _inside(A + B - P1, B, A, C2, 1e-12)
    nrm = np.array([-(B - A)[1], (B - A)[0]])
    best = -np.inf
    xs = np.linspace(-1.5, 1.5, 601)
    ys = np.linspace(0.0, 1.5, 301)
    X, Y = np.meshgrid(xs, ys)
    for x, y in zip(X.ravel(), Y.ravel()):
        p = np.array([x, y])
        if _inside(p, A, B, C1, 0) and _inside(2 * m - p, B, A, C2, 0):
            best = max(best, float(np.dot(p - A, nrm)))
    h = float(np.dot(P1 - A, nrm))
    assert h >= best - 1e-12
    assert h <= best + 0.02 * np.linalg.norm(nrm)   # grid spacing 0.005


@pytest.mark.parametrize("seed", range(8))
def test_parallelogram_swap_symmetry_and_area_bound(seed):
    rng = np.random.default_rng(100 + seed)
    A, B, C1, C2 = _random_quad(rng)
    P1 = ardg.parallelogram_apex(A, B, C1, C2)
    Q1 = ardg.parallelogram_apex(B, A, C2, C1)     # same edge seen from side 2
    assert np.allclose(Q1, A + B - P1, atol=1e-12)
    area_p = 2 * abs(_tri_area(A, B, P1))
    assert area_p <= 2 * min(abs(_tri_area(A, B, C1)), abs(_tri_area(B, A, C2))) + 1e-14


# ----------------------------------------------------------------------------
# Projection and reconstruction
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("N", [1, 2, 3, 4, 6])
def test_projection_exact_for_PN(N):
    """Restricting a degree-N polynomial to the sub-triangle (pi, a2, a3) and
    re-expanding gives its values at the sub-triangle's nodes."""
    ops = RefOps(N)
    rng = np.random.default_rng(N)
    pi = np.array([-0.7, -0.6])
    coef = rng.standard_normal((N + 1, N + 1))

    def p(r, s):
        return sum(coef[a, b] * r ** a * s ** b for a in range(N + 1) for b in range(N + 1 - a))
    u = p(ops.rs[:, 0], ops.rs[:, 1])
    uhat_sub = ops.Vinv @ ardg.projection_vandermonde(N, pi) @ ops.Vinv @ u
    pts = ardg.subtriangle_points(N, pi)
    assert np.abs(ops.V @ uhat_sub - p(pts[:, 0], pts[:, 1])).max() < 1e-12


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6])
def test_reconstruction_operator_is_pseudo_inverse(N):
    A = ardg.recon_system(N)
    R = ardg.recon_pinv(N)
    Mp = (N + 1) ** 2
    assert np.linalg.matrix_rank(A) == Mp
    assert np.abs(R @ A - np.eye(Mp)).max() < 1e-12
    # R v = 0 for v orthogonal to range(A)
    Q, _ = np.linalg.qr(A, mode="complete")
    Nperp = Q[:, Mp:]
    assert np.abs(R @ Nperp).max() < 1e-12
    # A R is the orthogonal projector onto range(A) (symmetric, idempotent)
    P = A @ R
    assert np.abs(P - P.T).max() < 1e-12 and np.abs(P @ P - P).max() < 1e-12


@pytest.mark.parametrize("N", [1, 2, 3, 4, 6])
def test_reconstruction_reproduces_QN(N):
    """Feeding the exact L2 projections (onto P_N of each sub-triangle) of any
    q in Q_N returns q: the LS residual is zero."""
    rng = np.random.default_rng(10 + N)
    c = rng.standard_normal((N + 1) ** 2)
    r, s, w = ardg.triangle_quadrature(3 * N + 3)
    Vq = vandermonde(N, r, s)
    q1 = ardg.phi(r, s, N) @ c            # q on the lower half, in its frame
    q2 = ardg.phi(-r, -s, N) @ c          # q on the upper half, in its own frame
    b = np.concatenate([(Vq * w[:, None]).T @ q1, (Vq * w[:, None]).T @ q2])
    assert np.abs(ardg.recon_pinv(N) @ b - c).max() < 1e-12


@pytest.mark.parametrize("N", [2, 3, 4])
def test_reconstruction_independent_of_QN_basis(N):
    """Monomials R^a S^b instead of Legendre products give the same function."""
    rng = np.random.default_rng(20 + N)
    b = rng.standard_normal(2 * ((N + 1) * (N + 2) // 2))
    r, s, w = ardg.triangle_quadrature(3 * N + 3)
    Vq = vandermonde(N, r, s)
    mono = [(a, c) for a in range(N + 1) for c in range(N + 1)]
    P1 = np.stack([r ** a * s ** c for (a, c) in mono], axis=1)
    P2 = np.stack([(-r) ** a * (-s) ** c for (a, c) in mono], axis=1)
    A_m = np.vstack([(Vq * w[:, None]).T @ P1, (Vq * w[:, None]).T @ P2])
    cm = np.linalg.lstsq(A_m, b, rcond=None)[0]
    cl = ardg.recon_pinv(N) @ b
    d = ardg.diagonal_points(N)
    pts = np.vstack([d, np.array([[0.3, -0.9], [-0.2, 0.7]])])
    vm = np.stack([pts[:, 0] ** a * pts[:, 1] ** c for (a, c) in mono], axis=1) @ cm
    vl = ardg.phi(pts[:, 0], pts[:, 1], N) @ cl
    assert np.abs(vm - vl).max() < 1e-11


# ----------------------------------------------------------------------------
# Edge flux
# ----------------------------------------------------------------------------

def _poly(N, seed):
    rng = np.random.default_rng(seed)
    terms = [(a, b) for a in range(N + 1) for b in range(N + 1 - a)]
    co = rng.standard_normal(len(terms))

    def p(x, y):
        return sum(c * x ** a * y ** b for c, (a, b) in zip(co, terms))

    def g(x, y):
        gx = sum(c * a * x ** (a - 1) * y ** b for c, (a, b) in zip(co, terms) if a > 0)
        gy = sum(c * b * x ** a * y ** (b - 1) for c, (a, b) in zip(co, terms) if b > 0)
        return gx + 0 * x, gy + 0 * x
    return p, g


def _diag_xy(eg, N):
    t = lgl_nodes(N)[::-1]
    return ((1 + t) / 2)[:, None] * eg.A + ((1 - t) / 2)[:, None] * eg.B


@pytest.mark.parametrize("N", [1, 2, 3, 4, 6])
def test_flux_reproduces_PN_on_jittered_mesh(N):
    mesh = W.split_square_mesh(4, 0.2, seed=5)
    pr = Problem(mesh.vxy, mesh.etov, N, 1.0)
    xy = pr.nodal_xy()
    p, g = _poly(N, 30 + N)
    Fi, _ = pr.diffusive_flux(p(xy[..., 0], xy[..., 1]))
    err, sc = 0.0, 0.0
    for e, eg in enumerate(pr.edge_geom):
        X = _diag_xy(eg, N)
        gx, gy = g(X[:, 0], X[:, 1])
        ex = eg.n1[0] * gx + eg.n1[1] * gy
        err = max(err, np.abs(Fi[e] - ex).max())
        sc = max(sc, np.abs(ex).max())
    assert err <= 5e-11 * max(sc, 1.0)


@pytest.mark.parametrize("N", [2, 3])
def test_flux_alg1_reproduces_D_grad_when_D_equal(N):
    mesh = W.split_square_mesh(4, 0.2, seed=6)
    pr = Problem(mesh.vxy, mesh.etov, N, np.full(mesh.K, 3.5), D_mode="element")
    xy = pr.nodal_xy()
    p, g = _poly(N, 40 + N)
    Fi, _ = pr.diffusive_flux(p(xy[..., 0], xy[..., 1]))
    for e, eg in enumerate(pr.edge_geom):
        X = _diag_xy(eg, N)
        gx, gy = g(X[:, 0], X[:, 1])
        ex = 3.5 * (eg.n1[0] * gx + eg.n1[1] * gy)
        assert np.abs(Fi[e] - ex).max() < 1e-10 * max(1.0, np.abs(ex).max())


@pytest.mark.parametrize("N", [2, 3, 4])
@pytest.mark.parametrize("alg1", [False, True])
def test_flux_swap_symmetry(N, alg1):
    """Exchanging the two sides gives the negated flux in reverse order: the
    two elements' surface terms cancel pairwise (conservation)."""
    mesh = W.split_square_mesh(3, 0.2, seed=8)
    g = Geometry(mesh.vxy, mesh.etov)
    ops = RefOps(N)
    rng = np.random.default_rng(N)
    D = rng.uniform(0.1, 10.0, g.K)
    u = rng.standard_normal((g.K, ops.Np))
    for (k1, f1, k2, f2) in g.interior:
        e12 = ardg.interior_edge_geometry(g, k1, f1, k2, f2)
        e21 = ardg.interior_edge_geometry(g, k2, f2, k1, f1)
        if alg1:
            a1, a2 = ardg.edge_operator_alg1(ops, e12, f1, f2, D[k1], D[k2])
            b1, b2 = ardg.edge_operator_alg1(ops, e21, f2, f1, D[k2], D[k1])
        else:
            a1, a2 = ardg.edge_operator(ops, e12, f1, f2)
            b1, b2 = ardg.edge_operator(ops, e21, f2, f1)
        F12 = a1 @ u[k1] + a2 @ u[k2]
        F21 = b1 @ u[k2] + b2 @ u[k1]
        assert np.abs(F12 + F21[::-1]).max() < 1e-10 * max(1.0, np.abs(F12).max())


@pytest.mark.parametrize("N", [2, 3])
def test_flux_affine_invariance(N):
    """(i) A similarity x -> sc Q x + c with the same nodal data maps the
    reconstruction to the transported function, so the normal derivative
    scales by 1/sc for any data.  (ii) A general affine map with positive
    determinant keeps area ratios, so the enclosed parallelogram and the
    least-squares fit commute with it: for transported P_N data the flux is
    n'.(G^{-T} grad p)."""
    mesh = W.split_square_mesh(3, 0.2, seed=9)
    c = np.array([0.7, -1.1])
    pr1 = Problem(mesh.vxy, mesh.etov, N, 1.0)
    rng = np.random.default_rng(1)
    u = rng.standard_normal((mesh.K, pr1.ops.Np))
    F1, _ = pr1.diffusive_flux(u)
    theta, sc = 0.6, 1.7
    Rm = sc * np.array([[math.cos(theta), -math.sin(theta)], [math.sin(theta), math.cos(theta)]])
    pr3 = Problem(mesh.vxy @ Rm.T + c, mesh.etov, N, 1.0)
    F3, _ = pr3.diffusive_flux(u)
    assert np.abs(F3 * sc - F1).max() < 1e-10 * np.abs(F1).max()

    G = np.array([[1.3, 0.4], [-0.2, 0.8]])
    pr2 = Problem(mesh.vxy @ G.T + c, mesh.etov, N, 1.0)
    p, g = _poly(N, 77)
    xy1 = pr1.nodal_xy()
    F2p, _ = pr2.diffusive_flux(p(xy1[..., 0], xy1[..., 1]))
    Ginv = np.linalg.inv(G)
    for e, eg in enumerate(pr2.edge_geom):
        X1 = (_diag_xy(eg, N) - c) @ Ginv.T
        gx, gy = g(X1[:, 0], X1[:, 1])
        ex = (np.stack([gx, gy], axis=1) @ Ginv) @ eg.n1
        assert np.abs(F2p[e] - ex).max() < 1e-10 * max(1.0, np.abs(ex).max())


@pytest.mark.parametrize("N", [1, 2, 3])
def test_flux_matches_physical_domain_bruteforce(N):
    """The reference-domain operator (one operator for every edge) equals a
    least-squares reconstruction assembled directly in physical coordinates
    with physical quadrature on each sub-triangle."""
    mesh = W.split_square_mesh(3, 0.25, seed=11)
    pr = Problem(mesh.vxy, mesh.etov, N, 1.0)
    rng = np.random.default_rng(N)
    u = rng.standard_normal((mesh.K, pr.ops.Np))
    Fi, Fb = pr.diffusive_flux(u)
    xy = pr.nodal_xy()
    for e, (k1, f1, k2, f2) in enumerate(pr.int_edges):
        eg = pr.edge_geom[e]
        Fbf = physical_edge_flux(N, eg, xy[k1], u[k1], mesh.vxy[mesh.etov[k1]],
                                 xy[k2], u[k2], mesh.vxy[mesh.etov[k2]])
        assert np.abs(Fbf - Fi[e]).max() < 1e-9 * max(1.0, np.abs(Fi[e]).max())
    for e, (k1, f1) in enumerate(pr.bdy_edges):
        eg = pr.bdy_geom[e]
        Fbf = physical_edge_flux(N, eg, xy[k1], u[k1], mesh.vxy[mesh.etov[k1]],
                                 None, None, None)
        assert np.abs(Fbf - Fb[e]).max() < 1e-9 * max(1.0, np.abs(Fb[e]).max())


@pytest.mark.parametrize("N", [2, 3, 4])
def test_boundary_flux_reproduces_odd_polynomials(N):
    """On y = 0 the mirror ghost is exact for data odd across the line:
    p = y q(x) with deg p <= N gives the exact normal derivative."""
    mesh = W.split_square_mesh(3, 0.2, seed=12)
    pr = Problem(mesh.vxy, mesh.etov, N, 1.0)
    xy = pr.nodal_xy()
    x, y = xy[..., 0], xy[..., 1]
    rng = np.random.default_rng(N)
    qc = rng.standard_normal(N)
    p = y * sum(qc[i] * x ** i for i in range(N))
    _, Fb = pr.diffusive_flux(p)
    checked = 0
    for e, eg in enumerate(pr.bdy_geom):
        if abs(eg.A[1]) < 1e-14 and abs(eg.B[1]) < 1e-14:
            X = _diag_xy(eg, N)
            dpdy = sum(qc[i] * X[:, 0] ** i for i in range(N))
            ex = eg.n1[1] * dpdy
            assert np.abs(Fb[e] - ex).max() < 1e-10 * max(1.0, np.abs(ex).max())
            checked += 1
    assert checked == 3


def _alg1_bruteforce_errors(N, D1v, D2v, mutate=None, seed=13):
    """Largest relative difference between the oracle's Algorithm 1 flux and
    the physical-domain brute force over every interior and boundary face of
    a jittered mesh whose elements alternate between two coefficients."""
    from physical_bruteforce import physical_edge_flux_alg1
    mesh = W.split_square_mesh(3, 0.25, seed=seed)
    K = mesh.K
    D = np.where(np.arange(K) % 2 == 0, D1v, D2v).astype(float)
    pr = Problem(mesh.vxy, mesh.etov, N, D, D_mode="element", build_edges=False)
    ops, g = pr.ops, pr.geom
    rng = np.random.default_rng(100 + N)
    u = rng.standard_normal((K, ops.Np))
    xy = pr.nodal_xy()
    rs = nodes(N)
    worst = 0.0
    for (k1, f1, k2, f2) in g.interior:
        eg = ardg.interior_edge_geometry(g, k1, f1, k2, f2)
        Da, Db = D[k1], D[k2]
        if mutate == "swap":
            Da, Db = Db, Da
        if mutate == "frame":
            # side 2 differentiated with side 1's parallelogram factors
            eg.Rx2, eg.Ry2, eg.Sx2, eg.Sy2 = eg.Rx, eg.Ry, eg.Sx, eg.Sy
        W1, W2 = ardg.edge_operator_alg1(ops, eg, f1, f2, Da, Db)
        F = W1 @ u[k1] + W2 @ u[k2]
        Fb = physical_edge_flux_alg1(N, eg, rs, xy[k1], u[k1], xy[k2], u[k2], D[k1], D[k2])
        worst = max(worst, np.abs(F - Fb).max() / max(np.abs(Fb).max(), 1e-300))
    for (k1, f1) in g.boundary:
        eg = ardg.boundary_edge_geometry(g, k1, f1)
        F = ardg.boundary_edge_operator_alg1(ops, g, k1, f1, eg, D[k1]) @ u[k1]
        Fb = physical_edge_flux_alg1(N, eg, rs, xy[k1], u[k1], None, None, D[k1], D[k1])
        worst = max(worst, np.abs(F - Fb).max() / max(np.abs(Fb).max(), 1e-300))
    return worst


@pytest.mark.parametrize("N", [1, 2, 3])
def test_flux_alg1_matches_physical_bruteforce_unequal_D(N):
    """Algorithm 1 with D1 != D2 (contrast 1e4) equals the same five steps
    carried out with physical monomials and physical quadrature: separation at
    the sub-triangles' physical nodes, physical gradients times each
    element's D, a second physical least-squares fit, n1 . (result) on the
    diagonal.  Boundary faces use the mirror ghost with the element's D."""
    assert _alg1_bruteforce_errors(N, 1e-2, 1e2) < 1e-9


@pytest.mark.parametrize("mutate", ["swap", "frame"])
def test_flux_alg1_bruteforce_detects_planted_mistakes(mutate):
    """The pin above is not vacuous: exchanging D1 and D2, or differentiating
    side 2 with side 1's parallelogram factors, moves the oracle's flux far
    from the brute force."""
    assert _alg1_bruteforce_errors(2, 1e-2, 1e2, mutate=mutate) > 1e-2


# ----------------------------------------------------------------------------
# Algorithm 2: reconstructed coefficient times the reconstructed gradient
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("N", [1, 2, 3, 4, 6])
def test_alg2_coefficient_is_arithmetic_mean_on_diagonal(N):
    """For element-wise constant D the reconstructed coefficient on the
    diagonal is (D1 + D2) / 2 at every node.  Closed form: the map
    (R, S) -> (-S, -R) swaps the two sub-triangles, fixes every diagonal point
    and leaves Q_N and the least-squares system invariant, so the fit of the
    odd part (D1 - D2)/2 * (indicator of side 1 - indicator of side 2) is odd
    under it and vanishes on the diagonal; the even part (D1 + D2)/2 is a
    constant, reproduced exactly."""
    mesh = W.split_square_mesh(4, 0.25, seed=17)
    g = Geometry(mesh.vxy, mesh.etov)
    ops = RefOps(N)
    one = np.ones(ops.Np)
    for (k1, f1, k2, f2) in g.interior:
        eg = ardg.interior_edge_geometry(g, k1, f1, k2, f2)
        Dt = ardg.coefficient_on_diagonal(ops, eg, f1, f2, 1e-2 * one, 1e2 * one)
        assert np.abs(Dt - 0.5 * (1e-2 + 1e2)).max() < 1e-11 * 1e2
    for (k1, f1) in g.boundary:
        eg = ardg.boundary_edge_geometry(g, k1, f1)
        Dt = ardg.boundary_coefficient_on_diagonal(ops, eg, f1, 3.0 * one)
        assert np.abs(Dt - 3.0).max() < 1e-12


@pytest.mark.parametrize("N", [1, 2, 3])
def test_alg2_matches_physical_bruteforce(N):
    """Algorithm 2 assembled in physical coordinates: the coefficient fitted by
    physical least squares on the parallelogram (data D1 on (P1, A, B), D2 on
    (P2, B, A)) times n1 . grad u~ of the physical fit, at the diagonal's LGL
    points; boundary faces with the mirror ghost carrying the element's D."""
    from physical_bruteforce import ParallelogramLS, physical_edge_flux
    mesh = W.split_square_mesh(3, 0.25, seed=19)
    K = mesh.K
    D = np.where(np.arange(K) % 2 == 0, 1e-2, 1e2)
    pr = Problem(mesh.vxy, mesh.etov, N, D, D_mode="element", alg=2)
    rng = np.random.default_rng(200 + N)
    u = rng.standard_normal((K, pr.ops.Np))
    Fi, Fb = pr.diffusive_flux(u)
    xy = pr.nodal_xy()
    for e, (k1, f1, k2, f2) in enumerate(pr.int_edges):
        eg = pr.edge_geom[e]
        ls = ParallelogramLS(N, eg)
        cD = ls.fit(lambda X: np.full(len(X), D[k1]), lambda X: np.full(len(X), D[k2]))
        Dt = ls.value(cD, ls.diagonal())
        Fbf = Dt * physical_edge_flux(N, eg, xy[k1], u[k1], None, xy[k2], u[k2], None)
        assert np.abs(Fbf - Fi[e]).max() < 1e-9 * max(1.0, np.abs(Fi[e]).max())
    for e, (k1, f1) in enumerate(pr.bdy_edges):
        eg = pr.bdy_geom[e]
        Fbf = D[k1] * physical_edge_flux(N, eg, xy[k1], u[k1], None, None, None, None)
        assert np.abs(Fbf - Fb[e]).max() < 1e-9 * max(1.0, np.abs(Fb[e]).max())


@pytest.mark.parametrize("N", [2, 3])
def test_alg2_equal_D_reduces_to_constant_form(N):
    """D1 = D2 = D: Algorithm 2 is D times the constant-coefficient flux."""
    mesh = W.split_square_mesh(4, 0.2, seed=23)
    pc = Problem(mesh.vxy, mesh.etov, N, 2.5)
    p2 = Problem(mesh.vxy, mesh.etov, N, np.full(mesh.K, 2.5), D_mode="element", alg=2)
    u = np.random.default_rng(N).standard_normal((mesh.K, pc.ops.Np))
    assert np.abs(p2.rhs(u) - pc.rhs(u)).max() < 1e-12 * np.abs(pc.rhs(u)).max()


@pytest.mark.parametrize("N", [2, 3])
def test_alg2_swap_symmetry(N):
    """Exchanging the sides gives the negated flux in reverse order."""
    mesh = W.split_square_mesh(3, 0.2, seed=29)
    g = Geometry(mesh.vxy, mesh.etov)
    ops = RefOps(N)
    rng = np.random.default_rng(N)
    D = rng.uniform(0.1, 10.0, g.K)
    u = rng.standard_normal((g.K, ops.Np))
    for (k1, f1, k2, f2) in g.interior:
        e12 = ardg.interior_edge_geometry(g, k1, f1, k2, f2)
        e21 = ardg.interior_edge_geometry(g, k2, f2, k1, f1)
        a1, a2 = ardg.edge_operator_alg2(ops, e12, f1, f2, D[k1], D[k2])
        b1, b2 = ardg.edge_operator_alg2(ops, e21, f2, f1, D[k2], D[k1])
        F12 = a1 @ u[k1] + a2 @ u[k2]
        F21 = b1 @ u[k2] + b2 @ u[k1]
        assert np.abs(F12 + F21[::-1]).max() < 1e-10 * max(1.0, np.abs(F12).max())
