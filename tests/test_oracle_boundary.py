"""Pins for the oracle's boundary faces with prescribed exterior data, its
time-dependent integration, and the paper's grid families (CPU only).

* Exactness: with the exterior state equal to a global polynomial p of
  degree <= N, the reconstruction at a boundary face sees p on both halves,
  so the right-hand side is D lap p - v . grad p on every element, boundary
  elements included.
* Physical brute force: the boundary-face flux equals the least-squares fit
  assembled in physical coordinates with the exterior state interpolated at
  the ghost sub-triangle's nodes.
* Time integration with a time-dependent right-hand side: fourth order for
  classic RK4 and for the low-storage scheme with its stage times (which
  follow from its coefficients and match the published ones); without stage
  times the low-storage scheme drops to first order (planted mistake).
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import ardg
from oracle.rhs import LSERK_A, LSERK_B, LSERK_C, Problem, lserk_step, rk4_step

from physical_bruteforce import PhysPoly, physical_edge_flux


def _poly(N, seed):
    rng = np.random.default_rng(seed)
    terms = [(a, b) for a in range(N + 1) for b in range(N + 1 - a)]
    co = rng.standard_normal(len(terms))

    def p(x, y):
        return sum(c * x ** a * y ** b for c, (a, b) in zip(co, terms)) + 0 * x

    def lap(x, y):
        v = 0 * x
        for c, (a, b) in zip(co, terms):
            if a >= 2:
                v = v + c * a * (a - 1) * x ** (a - 2) * y ** b
            if b >= 2:
                v = v + c * b * (b - 1) * x ** a * y ** (b - 2)
        return v

    def grad(x, y):
        gx = sum(c * a * x ** (a - 1) * y ** b for c, (a, b) in zip(co, terms) if a > 0) + 0 * x
        gy = sum(c * b * x ** a * y ** (b - 1) for c, (a, b) in zip(co, terms) if b > 0) + 0 * x
        return gx, gy
    return p, lap, grad


@pytest.mark.parametrize("N", [1, 2, 3, 4])
@pytest.mark.parametrize("alg", [0, 1, 2])
def test_prescribed_exterior_polynomial_is_exact_everywhere(N, alg):
    mesh = W.split_square_mesh(4, 0.2, seed=51)
    p, lap, grad = _poly(N, 60 + N)
    D = 0.7
    Dv = np.full(mesh.K, D) if alg else D
    pr = Problem(mesh.vxy, mesh.etov, N, Dv, D_mode="element" if alg else "const", alg=max(alg, 1),
                 ghost=lambda x, y, t, f: p(x, y))
    xy = pr.nodal_xy()
    r = pr.rhs(p(xy[..., 0], xy[..., 1]))
    ex = D * lap(xy[..., 0], xy[..., 1])
    assert np.abs(r - ex).max() < 1e-9 * max(1.0, np.abs(ex).max())


@pytest.mark.parametrize("N", [2, 3])
def test_prescribed_exterior_polynomial_with_convection(N):
    """Constant velocity: v u stays in P_N and the upwind flux takes the
    exterior state at inflow faces, so rhs = D lap p - v . grad p exactly."""
    mesh = W.split_square_mesh(4, 0.2, seed=52)
    p, lap, grad = _poly(N, 70 + N)
    v = (0.8, -0.45)
    pr = Problem(mesh.vxy, mesh.etov, N, 0.3, velocity=(v[0], v[1], 0, 0, 0, 0),
                 ghost=lambda x, y, t, f: p(x, y))
    xy = pr.nodal_xy()
    x, y = xy[..., 0], xy[..., 1]
    gx, gy = grad(x, y)
    ex = 0.3 * lap(x, y) - (v[0] * gx + v[1] * gy)
    r = pr.rhs(p(x, y))
    assert np.abs(r - ex).max() < 1e-9 * max(1.0, np.abs(ex).max())
    # the sampled evaluator agrees, boundary elements included
    els = [0, 3, mesh.K - 1]
    assert np.abs(pr.rhs_elements(p(x, y), els) - r[els]).max() < 1e-12 * np.abs(r).max()


@pytest.mark.parametrize("N", [1, 2, 3])
def test_prescribed_exterior_flux_matches_physical_bruteforce(N):
    mesh = W.split_square_mesh(3, 0.25, seed=53)
    g = lambda x, y, t, f: np.sin(1.3 * x + 0.4) * np.cos(0.7 * y) + t * x * y
    pr = Problem(mesh.vxy, mesh.etov, N, 1.0, ghost=g)
    rng = np.random.default_rng(N)
    u = rng.standard_normal((mesh.K, pr.ops.Np))
    t = 0.37
    _, Fb = pr.diffusive_flux(u, 0, t)
    xy = pr.nodal_xy()
    for e, (k1, f1) in enumerate(pr.bdy_edges):
        eg = pr.bdy_geom[e]
        X2 = ardg.ghost_nodes(N, eg)
        Fbf = physical_edge_flux(N, eg, xy[k1], u[k1], None, X2, g(X2[:, 0], X2[:, 1], t, 0), None)
        assert np.abs(Fbf - Fb[e]).max() < 1e-9 * max(1.0, np.abs(Fb[e]).max())


def test_lserk_stage_times_match_published():
    """c_s from the recursion on the coefficients against the published
    stage times of the Carpenter-Kennedy five-stage scheme."""
    published = np.array([0.0, 1432997174477.0 / 9575080441755.0, 2526269341429.0 / 6820363962896.0,
                          2006345519317.0 / 3224310063776.0, 2802321613138.0 / 2924317926251.0])
    assert np.abs(LSERK_C - published).max() < 1e-12


def _ode_errors(step, dts, T=1.0):
    """Errors of du/dt = -u + cos(t) + sin(t) from u(0) = 0 (exact: sin t) at T."""
    errs = []
    for dt in dts:
        u, t = np.array([0.0]), 0.0
        n = int(round(T / dt))
        for _ in range(n):
            u = step(lambda v, s: -v + np.cos(s) + np.sin(s), u, dt, t)
            t += dt
        errs.append(abs(u[0] - math.sin(T)))
    return errs


@pytest.mark.parametrize("step", [rk4_step, lserk_step])
def test_time_dependent_integration_is_fourth_order(step):
    e = _ode_errors(step, [0.1, 0.05])
    assert math.log2(e[0] / e[1]) > 3.8


def test_lserk_without_stage_times_drops_order(monkeypatch):
    import oracle.rhs as R
    monkeypatch.setattr(R, "LSERK_C", np.zeros(5))
    e = _ode_errors(R.lserk_step, [0.1, 0.05])
    assert math.log2(e[0] / e[1]) < 1.5


@pytest.mark.parametrize("a", [(0.0, 0.0), (6.0, 6.0)])
def test_gaussian_is_an_exact_solution(a):
    """The input generator's Gaussian satisfies u_t + a . grad u = D lap u
    (finite differences)."""
    x, y, t, h = 4.3, -0.7, 0.21, 1e-4
    D = 1.0
    f = lambda x, y, t: W.gaussian(x, y, t, D=D, x0=(4.0, -1.0), a=a)
    ut = (f(x, y, t + h) - f(x, y, t - h)) / (2 * h)
    ux = (f(x + h, y, t) - f(x - h, y, t)) / (2 * h)
    uy = (f(x, y + h, t) - f(x, y - h, t)) / (2 * h)
    lap = (f(x + h, y, t) + f(x - h, y, t) + f(x, y + h, t) + f(x, y - h, t) - 4 * f(x, y, t)) / h ** 2
    assert abs(ut + a[0] * ux + a[1] * uy - D * lap) < 1e-6 * abs(ut)


@pytest.mark.parametrize("kind,n,K", [("a", 4, 32), ("b", 2, 16), ("c", 4, 64)])
def test_paper_grids(kind, n, K):
    """Element counts of the paper's series, total area 100, equal element
    areas on grid c, and parallelograms everywhere on grid a only."""
    from oracle.mesh import Geometry
    m = W.paper_grid(kind, n)
    g = Geometry(m.vxy, m.etov)
    assert m.K == K
    assert abs(float(np.sum(2 * g.J)) - 100.0) < 1e-9
    if kind == "c":
        assert np.ptp(2 * g.J) < 1e-9
    nonpar = 0
    for (k1, f1, k2, f2) in g.interior:
        eg = ardg.interior_edge_geometry(g, k1, f1, k2, f2)
        nonpar += int(np.abs(eg.P1 - eg.C1).max() > 1e-9)
    assert (nonpar == 0) == (kind == "a")
