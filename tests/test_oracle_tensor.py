"""Pins for the oracle's Algorithm 1 with a nodal tensor coefficient
(space-varying, anisotropic with the shear cross term, or proportional to
the solution) (CPU only)."""
import numpy as np
import pytest

import workloads as W
from oracle import ardg
from oracle.reference_element import nodes
from oracle.rhs import Problem

from physical_bruteforce import PhysPoly, physical_edge_flux_alg1_tensor


def _monomials(N, seed):
    rng = np.random.default_rng(seed)
    terms = [(a, b) for a in range(N + 1) for b in range(N + 1 - a)]
    return terms, rng.standard_normal(len(terms))


def _eval(terms, co, x, y, dx=0, dy=0):
    """d^dx/dx d^dy/dy of sum c x^a y^b."""
    out = 0 * x
    for c, (a, b) in zip(co, terms):
        if a < dx or b < dy:
            continue
        fa = np.prod([a - i for i in range(dx)]) if dx else 1.0
        fb = np.prod([b - i for i in range(dy)]) if dy else 1.0
        out = out + c * fa * fb * x ** (a - dx) * y ** (b - dy)
    return out


def _interior(pr):
    return np.all(pr.geom.EToE >= 0, axis=1)


@pytest.mark.parametrize("N", [2, 3])
def test_tensor_reduces_to_elementwise_alg1(N):
    mesh = W.split_square_mesh(3, 0.2, seed=81)
    D = W.loguniform_per_element(mesh.K, 1e-2, 1e1, seed=82)
    Np = (N + 1) * (N + 2) // 2
    Dn = np.zeros((mesh.K, Np, 3))
    Dn[:, :, 0] = D[:, None]
    Dn[:, :, 2] = D[:, None]
    pe = Problem(mesh.vxy, mesh.etov, N, D, D_mode="element")
    pn = Problem(mesh.vxy, mesh.etov, N, Dn, D_mode="nodal")
    u = np.random.default_rng(N).standard_normal((mesh.K, Np))
    re, rn = pe.rhs(u), pn.rhs(u)
    assert np.abs(re - rn).max() < 1e-11 * np.abs(re).max()


@pytest.mark.parametrize("N", [2, 3, 4])
@pytest.mark.parametrize("prescribed", [False, True])
def test_constant_anisotropic_tensor_with_cross_term_is_exact(N, prescribed):
    """D = [[a, b], [b, c]] constant (the shear equation's cross term is the
    off-diagonal): rhs = a p_xx + 2 b p_xy + c p_yy for p in P_N, on interior
    elements (mirror ghost) or on every element (exterior state p)."""
    mesh = W.split_square_mesh(4, 0.2, seed=83)
    terms, co = _monomials(N, 90 + N)
    p = lambda x, y: _eval(terms, co, x, y)
    a, b, c = 0.9, 0.3, 0.5
    Np = (N + 1) * (N + 2) // 2
    Dn = np.tile(np.array([a, b, c]), (mesh.K, Np, 1))
    pr = Problem(mesh.vxy, mesh.etov, N, Dn, D_mode="nodal",
                 ghost=(lambda x, y, t, f: p(x, y)) if prescribed else None)
    xy = pr.nodal_xy()
    x, y = xy[..., 0], xy[..., 1]
    r = pr.rhs(p(x, y))
    ex = a * _eval(terms, co, x, y, 2, 0) + 2 * b * _eval(terms, co, x, y, 1, 1) + c * _eval(terms, co, x, y, 0, 2)
    sel = slice(None) if prescribed else _interior(pr)
    assert np.abs(r[sel] - ex[sel]).max() < 1e-9 * max(1.0, np.abs(ex).max())


@pytest.mark.parametrize("N", [3, 4])
def test_linear_tensor_field_is_exact(N):
    """Each tensor entry linear in x, y and p in P_{N-1}: D grad p has degree
    N - 1, every step of Algorithm 1 is exact, and rhs = div(D grad p)."""
    mesh = W.split_square_mesh(4, 0.2, seed=84)
    terms, co = _monomials(N - 1, 100 + N)
    coef = np.array([[1.0, 0.3, -0.2], [0.2, 0.1, 0.15], [0.8, -0.25, 0.3]])   # rows: Dxx, Dxy, Dyy

    def Dfun(x, y):
        return [coef[i, 0] + coef[i, 1] * x + coef[i, 2] * y for i in range(3)]
    pr0 = Problem(mesh.vxy, mesh.etov, N, 1.0, build_edges=False)
    xy = pr0.nodal_xy()
    x, y = xy[..., 0], xy[..., 1]
    Dn = np.stack(Dfun(x, y), axis=-1)
    pr = Problem(mesh.vxy, mesh.etov, N, Dn, D_mode="nodal")
    r = pr.rhs(_eval(terms, co, x, y))
    px, py = _eval(terms, co, x, y, 1, 0), _eval(terms, co, x, y, 0, 1)
    pxx, pxy, pyy = _eval(terms, co, x, y, 2, 0), _eval(terms, co, x, y, 1, 1), _eval(terms, co, x, y, 0, 2)
    Dxx, Dxy, Dyy = Dfun(x, y)
    # div(D grad p) = d/dx (Dxx px + Dxy py) + d/dy (Dxy px + Dyy py)
    ex = (coef[0, 1] * px + Dxx * pxx + coef[1, 1] * py + Dxy * pxy
          + coef[1, 2] * px + Dxy * pxy + coef[2, 2] * py + Dyy * pyy)
    inner = _interior(pr)
    assert np.abs(r[inner] - ex[inner]).max() < 1e-9 * max(1.0, np.abs(ex).max())


@pytest.mark.parametrize("N", [3, 5])
def test_solution_dependent_tensor_is_exact(N):
    """D = u D0 with D0 = [[a, b], [b, c]] and u = p of degree M, 2M - 1 <= N:
    rhs = div(p D0 grad p) = p (D0 : hess p) + grad p . D0 grad p."""
    M = (N + 1) // 2
    mesh = W.split_square_mesh(4, 0.2, seed=85)
    terms, co = _monomials(M, 110 + N)
    a, b, c = 0.7, 0.2, 0.4
    pr = Problem(mesh.vxy, mesh.etov, N, (a, b, c), D_mode="solution")
    xy = pr.nodal_xy()
    x, y = xy[..., 0], xy[..., 1]
    p = _eval(terms, co, x, y)
    px, py = _eval(terms, co, x, y, 1, 0), _eval(terms, co, x, y, 0, 1)
    pxx, pxy, pyy = _eval(terms, co, x, y, 2, 0), _eval(terms, co, x, y, 1, 1), _eval(terms, co, x, y, 0, 2)
    ex = p * (a * pxx + 2 * b * pxy + c * pyy) + (a * px * px + 2 * b * px * py + c * py * py)
    r = pr.rhs(p)
    inner = _interior(pr)
    assert np.abs(r[inner] - ex[inner]).max() < 1e-9 * max(1.0, np.abs(ex).max())


@pytest.mark.parametrize("N", [1, 2, 3])
@pytest.mark.parametrize("mode", ["nodal", "solution"])
def test_tensor_flux_matches_physical_bruteforce(N, mode):
    """Every face of a jittered mesh, random data and a random nodal tensor
    field (or u D0): the oracle's flux equals the same steps in physical
    coordinates (coefficient polynomials fitted to each element's nodal
    values and evaluated at the sub-triangle's physical nodes)."""
    mesh = W.split_square_mesh(3, 0.25, seed=86)
    rng = np.random.default_rng(120 + N)
    Np = (N + 1) * (N + 2) // 2
    u = rng.standard_normal((mesh.K, Np))
    if mode == "nodal":
        Dn = np.stack([rng.uniform(0.5, 2.0, (mesh.K, Np)), rng.uniform(-0.3, 0.3, (mesh.K, Np)),
                       rng.uniform(0.5, 2.0, (mesh.K, Np))], axis=-1)
        pr = Problem(mesh.vxy, mesh.etov, N, Dn, D_mode="nodal")
    else:
        D0 = np.array([0.8, 0.25, 0.6])
        pr = Problem(mesh.vxy, mesh.etov, N, D0, D_mode="solution")
    Fi, Fb = pr.diffusive_flux(u)
    xy = pr.nodal_xy()
    rs = nodes(N)

    def coef(k):
        if mode == "nodal":
            polys = [PhysPoly(N, xy[k], Dn[k, :, i]) for i in range(3)]
            return lambda X: np.stack([q(X) for q in polys], axis=1)
        return None
    d0 = D0 if mode == "solution" else None
    for e, (k1, f1, k2, f2) in enumerate(pr.int_edges):
        F = physical_edge_flux_alg1_tensor(N, pr.edge_geom[e], rs, xy[k1], u[k1], coef(k1), xy[k2], u[k2], coef(k2),
                                           D0=d0)
        assert np.abs(F - Fi[e]).max() < 1e-9 * max(1.0, np.abs(Fi[e]).max())
    for e, (k1, f1) in enumerate(pr.bdy_edges):
        F = physical_edge_flux_alg1_tensor(N, pr.bdy_geom[e], rs, xy[k1], u[k1], coef(k1), None, None, None, D0=d0)
        assert np.abs(F - Fb[e]).max() < 1e-9 * max(1.0, np.abs(Fb[e]).max())


@pytest.mark.parametrize("mode", ["nodal", "solution"])
def test_tensor_conservation_and_sampled_evaluator(mode):
    from oracle.reference_element import mass_1d
    N = 3
    mesh = W.split_square_mesh(4, 0.2, seed=87)
    rng = np.random.default_rng(5)
    Np = (N + 1) * (N + 2) // 2
    if mode == "nodal":
        D = np.stack([rng.uniform(0.5, 2.0, (mesh.K, Np)), rng.uniform(-0.3, 0.3, (mesh.K, Np)),
                      rng.uniform(0.5, 2.0, (mesh.K, Np))], axis=-1)
    else:
        D = (0.8, 0.25, 0.6)
    pr = Problem(mesh.vxy, mesh.etov, N, D, D_mode=mode)
    ops, g = pr.ops, pr.geom
    u = rng.standard_normal((g.K, Np)) + 2.0
    r = pr.rhs(u)
    total = float(np.sum(g.J * (r @ ops.M @ np.ones(Np))))
    _, Fb = pr.diffusive_flux(u)
    w = mass_1d(N).sum(axis=1)
    bsum = sum(g.sJ[k1, f1] * float(w @ Fb[e]) for e, (k1, f1) in enumerate(pr.bdy_edges))
    assert abs(total - bsum) < 1e-12 * float(np.sum(np.abs(g.J[:, None] * r)))
    els = [0, 5, g.K - 1]
    assert np.abs(pr.rhs_elements(u, els) - r[els]).max() < 1e-12 * np.abs(r).max()
