"""Pins for the oracle's right-hand side, time integrators and the whole
method (CPU only)."""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import ardg
from oracle.reference_element import lgl_nodes, mass_1d
from oracle.rhs import (LSERK_A, LSERK_B, Problem, error_norms, lserk_step, mass_norm,
                        rk4_step)

from physical_bruteforce import PhysPoly, physical_edge_flux, tri_rule

HERE = os.path.dirname(os.path.abspath(__file__))


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


def _interior(pr):
    return np.all(pr.geom.EToE >= 0, axis=1)


@pytest.mark.parametrize("N", [1, 2, 3, 4, 6])
def test_interior_rhs_is_D_laplacian_for_PN(N):
    mesh = W.split_square_mesh(5, 0.2, seed=2)
    pr = Problem(mesh.vxy, mesh.etov, N, 0.7)
    xy = pr.nodal_xy()
    p, lap, _ = _poly(N, N)
    r = pr.rhs(p(xy[..., 0], xy[..., 1]))
    ex = 0.7 * lap(xy[..., 0], xy[..., 1])
    inner = _interior(pr)
    scale = np.abs(pr.rhs(np.abs(p(xy[..., 0], xy[..., 1])))).max() + 1.0
    assert np.abs(r[inner] - ex[inner]).max() < 1e-12 * scale * 100


@pytest.mark.parametrize("N", [2, 3, 4])
def test_weak_equals_strong_form(N):
    """Integrating the volume term by parts once more (strong form) gives the
    same RHS up to rounding."""
    mesh = W.split_square_mesh(4, 0.2, seed=3)
    rng = np.random.default_rng(N)
    D = rng.uniform(0.1, 2.0, mesh.K)
    pr = Problem(mesh.vxy, mesh.etov, N, D, D_mode="element")
    ops, g = pr.ops, pr.geom
    u = rng.standard_normal((g.K, ops.Np))
    rw = pr.rhs(u)
    rx, ry, sx, sy = (a[:, None] for a in (g.rx, g.ry, g.sx, g.sy))
    qx = rx * (u @ ops.Dr.T) + sx * (u @ ops.Ds.T)
    qy = ry * (u @ ops.Dr.T) + sy * (u @ ops.Ds.T)
    div = (rx * (qx @ ops.Dr.T) + sx * (qx @ ops.Ds.T) + ry * (qy @ ops.Dr.T)
           + sy * (qy @ ops.Ds.T))
    Ff = pr.face_fluxes(*pr.diffusive_flux(u))
    rs_ = D[:, None] * div
    for f in range(3):
        fm = ops.fmask[f]
        nq = g.nx[:, f:f + 1] * qx[:, fm] + g.ny[:, f:f + 1] * qy[:, fm]
        jump = Ff[:, f, :] - D[:, None] * nq
        rs_ += (g.sJ[:, f] / g.J)[:, None] * (jump @ ops.LIFT[:, f * ops.Nfp:(f + 1) * ops.Nfp].T)
    assert np.abs(rw - rs_).max() < 1e-11 * np.abs(rw).max()


@pytest.mark.parametrize("N", [2, 3, 4])
@pytest.mark.parametrize("alg", [0, 1, 2])
def test_conservation(N, alg):
    """sum_k J_k 1^T M rhs_k equals the integral of the boundary fluxes:
    interior edges cancel pairwise (constant D, Algorithm 1, Algorithm 2)."""
    mesh = W.split_square_mesh(4, 0.2, seed=4)
    rng = np.random.default_rng(N)
    D = rng.uniform(0.1, 2.0, mesh.K) if alg else 1.3
    pr = Problem(mesh.vxy, mesh.etov, N, D, D_mode="element" if alg else "const", alg=max(alg, 1))
    ops, g = pr.ops, pr.geom
    u = rng.standard_normal((g.K, ops.Np))
    r = pr.rhs(u)
    total = float(np.sum(g.J * (r @ ops.M @ np.ones(ops.Np))))
    _, Fb = pr.diffusive_flux(u)
    w = mass_1d(N).sum(axis=1)
    bsum = 0.0
    for e, (k1, f1) in enumerate(pr.bdy_edges):
        bsum += g.sJ[k1, f1] * float(w @ Fb[e])
    assert abs(total - bsum) < 1e-12 * float(np.sum(np.abs(g.J[:, None] * r)))


def _bruteforce_operator(N, mesh, D=1.0):
    """Dense global operator from physical-domain quadrature and the physical
    least-squares flux."""
    pr = Problem(mesh.vxy, mesh.etov, N, D)       # only for connectivity / parallelograms
    xy = pr.nodal_xy()
    K, Np, Nfp = mesh.K, pr.ops.Np, pr.ops.Nfp
    n = K * Np
    L = np.zeros((n, n))
    t = lgl_nodes(N)
    ga, gw = np.polynomial.legendre.leggauss(2 * N + 2)

    def lag1d(j, x):
        out = np.ones_like(x)
        for m, tm in enumerate(t):
            if m != j:
                out = out * (x - tm) / (t[j] - tm)
        return out
    # per-edge flux operators (physical LS applied to unit vectors)
    I = np.eye(Np)
    face_ops = {}   # (k, f) -> list of (k_src, matrix [Nfp, Np]) in k's CCW order
    for e, (k1, f1, k2, f2) in enumerate(pr.int_edges):
        eg = pr.edge_geom[e]
        W1 = np.stack([physical_edge_flux(N, eg, xy[k1], I[j], mesh.vxy[mesh.etov[k1]],
                                          xy[k2], 0 * I[j], mesh.vxy[mesh.etov[k2]]) for j in range(Np)], 1)
        W2 = np.stack([physical_edge_flux(N, eg, xy[k1], 0 * I[j], mesh.vxy[mesh.etov[k1]],
                                          xy[k2], I[j], mesh.vxy[mesh.etov[k2]]) for j in range(Np)], 1)
        face_ops[(k1, f1)] = [(k1, D * W1), (k2, D * W2)]
        face_ops[(k2, f2)] = [(k1, -D * W1[::-1]), (k2, -D * W2[::-1])]
    for e, (k1, f1) in enumerate(pr.bdy_edges):
        eg = pr.bdy_geom[e]
        WB = np.stack([physical_edge_flux(N, eg, xy[k1], I[j], mesh.vxy[mesh.etov[k1]],
                                          None, None, None) for j in range(Np)], 1)
        face_ops[(k1, f1)] = [(k1, D * WB)]
    for k in range(K):
        v = mesh.vxy[mesh.etov[k]]
        poly = PhysPoly(N, xy[k], np.zeros(Np)).set_nodes(xy[k])
        X, w = tri_rule(N + 2, v)
        B = poly.basis(X)
        gx, gy = poly.basis_grad(X)
        Mk = (B * w[:, None]).T @ B
        Sk = (gx * w[:, None]).T @ gx + (gy * w[:, None]).T @ gy
        rows = slice(k * Np, (k + 1) * Np)
        L[rows, rows] += np.linalg.solve(Mk, -D * Sk)
        for f, (a, b) in enumerate(((0, 1), (1, 2), (2, 0))):
            A_, B_ = v[a], v[b]
            Xe = ((1 - ga) / 2)[:, None] * A_ + ((1 + ga) / 2)[:, None] * B_
            we = gw * np.linalg.norm(B_ - A_) / 2
            Bl = poly.basis(Xe)                                    # [Q, Np]
            L1 = np.stack([lag1d(j, ga) for j in range(Nfp)], 1)   # [Q, Nfp]
            Ef = (Bl * we[:, None]).T @ L1                         # [Np, Nfp]
            for (ks, Wm) in face_ops[(k, f)]:
                L[rows, ks * Np:(ks + 1) * Np] += np.linalg.solve(Mk, Ef @ Wm)
    return L, pr


@pytest.mark.parametrize("N", [1, 2, 3])
def test_global_operator_matches_physical_bruteforce(N):
    mesh = W.split_square_mesh(2, 0.25, seed=21)
    Lbf, pr = _bruteforce_operator(N, mesh, D=1.0)
    K, Np = mesh.K, pr.ops.Np
    Lor = np.zeros_like(Lbf)
    for j in range(K * Np):
        e = np.zeros(K * Np)
        e[j] = 1.0
        Lor[:, j] = pr.rhs(e.reshape(K, Np)).ravel()
    assert np.abs(Lor - Lbf).max() < 1e-8 * np.abs(Lbf).max()


@pytest.mark.parametrize("N", [1, 2, 3])
def test_spectrum_is_stable(N):
    """Reported property (the paper claims no stability proof): the linear
    operator on a tiny jittered mesh has no eigenvalue with positive real part
    beyond rounding."""
    mesh = W.split_square_mesh(3, 0.2, seed=22)
    pr = Problem(mesh.vxy, mesh.etov, N, 1.0)
    n = mesh.K * pr.ops.Np
    L = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        L[:, j] = pr.rhs(e.reshape(mesh.K, -1)).ravel()
    lam = np.linalg.eigvals(L)
    rho = np.abs(lam).max()
    assert lam.real.max() <= 1e-10 * rho


# ----------------------------------------------------------------------------
# Convection
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("N", [2, 3])
def test_convection_exact_for_polynomials(N):
    """Interior elements: -div(v p) exactly when v p stays in P_N (constant v
    with p in P_N; rotation v = (-y, x) with p in P_{N-1})."""
    mesh = W.split_square_mesh(4, 0.2, seed=31)
    for vel, deg in (((0.7, -1.3, 0, 0, 0, 0), N), ((0.0, 0.0, 0, -1.0, 1.0, 0), N - 1)):
        pr = Problem(mesh.vxy, mesh.etov, N, 0.0, velocity=vel)
        xy = pr.nodal_xy()
        x, y = xy[..., 0], xy[..., 1]
        p, _, grad = _poly(deg, 50 + deg)
        r = pr.rhs(p(x, y))
        gx, gy = grad(x, y)
        vx, vy = pr.velocity_at(xy)
        ex = -(vx * gx + vy * gy)          # both fields are divergence free
        inner = _interior(pr)
        assert np.abs(r[inner] - ex[inner]).max() < 1e-11 * max(1.0, np.abs(ex).max()) * 100


def test_convection_conserves_and_constant_state():
    N = 3
    mesh = W.split_square_mesh(4, 0.2, seed=32)
    pr = Problem(mesh.vxy, mesh.etov, N, 0.0, velocity=(0.0, 0.0, 0.0, -1.0, 1.0, 0.0))
    ops, g = pr.ops, pr.geom
    r = pr.rhs(np.ones((g.K, ops.Np)))
    assert np.abs(r[_interior(pr)]).max() < 1e-11
    rng = np.random.default_rng(0)
    u = rng.standard_normal((g.K, ops.Np))
    r = pr.rhs(u)
    total = float(np.sum(g.J * (r @ ops.M @ np.ones(ops.Np))))
    fs = pr.upwind_face_flux(u)
    w = mass_1d(N).sum(axis=1)
    bsum = sum(g.sJ[k, f] * float(w @ fs[k, f]) for (k, f) in pr.bdy_edges)
    assert abs(total + bsum) < 1e-11 * float(np.sum(np.abs(g.J[:, None] * r)))


# ----------------------------------------------------------------------------
# Time integrators
# ----------------------------------------------------------------------------

def test_rk4_amplification_polynomial():
    for z in (0.1, -0.5 + 0.3j, -1.2):
        amp = rk4_step(lambda u: z * u, np.array([1.0 + 0j]), 1.0)[0]
        assert abs(amp - (1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24)) < 1e-15


def _lserk_butcher():
    """Butcher tableau of the 2N-storage scheme: u_s = u + sum_j a_sj dt k_j."""
    s = 5
    # res_i = A_i res_{i-1} + dt k_i ;  u_i = u_{i-1} + B_i res_i
    coeff_res = np.zeros((s, s))   # res_i in terms of dt k_j
    for i in range(s):
        if i > 0:
            coeff_res[i] = LSERK_A[i] * coeff_res[i - 1]
        coeff_res[i, i] += 1.0
    Au = np.zeros((s + 1, s))      # u after stage i (row i+1) in dt k_j
    for i in range(s):
        Au[i + 1] = Au[i] + LSERK_B[i] * coeff_res[i]
    return Au[:s], Au[s]           # stage inputs (a matrix), weights b


def test_lserk_order_conditions():
    a, b = _lserk_butcher()
    c = a.sum(axis=1)
    conds = [
        (b.sum(), 1.0), (b @ c, 1 / 2), (b @ c ** 2, 1 / 3), (b @ (a @ c), 1 / 6),
        (b @ c ** 3, 1 / 4), (b @ (c * (a @ c)), 1 / 8), (b @ (a @ c ** 2), 1 / 12),
        (b @ (a @ (a @ c)), 1 / 24),
    ]
    for got, want in conds:
        assert abs(got - want) < 1e-12
    # and it is not fifth order
    assert abs(b @ c ** 4 - 1 / 5) > 1e-6


def test_lserk_order_four_on_ode():
    f = lambda u: -u + np.cos(u)      # noqa: E731
    errs = []
    ref = np.array([1.0])
    for _ in range(2000):
        ref = rk4_step(f, ref, 1.0 / 2000)
    for n in (10, 20, 40):
        u = np.array([1.0])
        for _ in range(n):
            u = lserk_step(f, u, 1.0 / n)
        errs.append(abs(u[0] - ref[0]))
    for i in range(2):
        assert 3.7 < math.log2(errs[i] / errs[i + 1]) < 4.5


# ----------------------------------------------------------------------------
# Whole method: manufactured solution and the paper's order pattern
# ----------------------------------------------------------------------------

def observed_order_fixed_dt(e_coarse, e_medium, e_fine, r):
    """Three-level order with a fixed temporal error phi cancelled:
    eps(h) = g h^p + phi gives (e_{r^2 h} - e_{r h}) / (e_{r h} - e_h) = r^p."""
    return math.log((e_coarse - e_medium) / (e_medium - e_fine)) / math.log(r)


def test_observed_order_formula_reading():
    """The three-level formula as printed (difference to the coarse level in the
    denominator) is inconsistent with its own error model; the reading used
    here recovers p exactly."""
    g, phi, r, p = 0.3, 1e-4, 2.0, 3.0
    e = [g * (r ** 2) ** p + phi, g * r ** p + phi, g + phi]
    assert abs(observed_order_fixed_dt(*e, r) - p) < 1e-12
    printed = math.log((e[0] - e[1]) / (e[0] - e[2])) / math.log(r)
    assert printed < 0


def _spectral_radius(pr, it=60):
    rng = np.random.default_rng(0)
    v = rng.standard_normal((pr.geom.K, pr.ops.Np))
    lam = 0.0
    for _ in range(it):
        w = pr.rhs(v)
        lam = np.linalg.norm(w) / np.linalg.norm(v)
        v = w / np.linalg.norm(w)
    return lam


@pytest.mark.parametrize("N,mins,ms", [(1, 1.8, (4, 8, 16)), (2, 1.8, (4, 8, 16)),
                                       (3, 3.7, (4, 8, 16))])
def test_manufactured_solution_order(N, mins, ms):
    """u = exp(-2 pi^2 D t) sin(pi x) sin(pi y): L2 order about N+1 for odd N
    and at least N for even N (the paper's conclusion; Table 2 P1-P3 orders
    are 2.0 / 2.75-2.83 / 4.0)."""
    with open(os.path.join(HERE, "golden", "paper_table2_orders.json")) as fh:
        t2 = json.load(fh)
    errs = []
    T = 0.02
    for m in ms:
        mesh = W.split_square_mesh(m, 0.2, seed=7)
        pr = Problem(mesh.vxy, mesh.etov, N, 1.0)
        xy = pr.nodal_xy()
        u = W.manufactured(xy[..., 0], xy[..., 1])
        nst = int(math.ceil(T * _spectral_radius(pr)))
        dt = T / nst
        for _ in range(nst):
            u = rk4_step(pr.rhs, u, dt)
        l2, _ = error_norms(pr, u, lambda x, y: W.manufactured(x, y, T))
        errs.append(l2)
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert orders[-1] >= mins
    paper = [t2["L2"][g][N - 1] for g in ("a", "b", "c")]
    # same order class as the paper's P_N results (within 0.5)
    assert abs(orders[-1] - float(np.mean(paper))) < 0.5


def test_mass_norm_is_l2_norm_of_polynomial():
    mesh = W.split_square_mesh(3, 0.2, seed=1)
    pr = Problem(mesh.vxy, mesh.etov, 3, 1.0)
    xy = pr.nodal_xy()
    e = xy[..., 0] ** 2 - xy[..., 1]
    l2, _ = error_norms(pr, e, lambda x, y: 0 * x)
    assert abs(mass_norm(pr, e) - l2) < 1e-13
