"""Pins for the oracle's sampled evaluators and the upwind direction (CPU only).

``Problem.rhs_elements`` and ``Problem.rk4_step_elements`` are what the
full-size GPU parity tests and the CPU baseline of the benchmark call: they
recompute each sampled element's three edge operators on the spot instead of
assembling the whole mesh.  Here they are tied to the assembled ``rhs`` and
``rk4_step`` on small meshes, for every coefficient mode, with and without the
convective term, on boundary elements and the last element.

The upwind direction of the convective flux is pinned by the spectrum: with
inflow data zero and a divergence-free velocity the upwind discretisation is
dissipative, so no eigenvalue of the linear operator has a positive real part
(a downwind flux gives eigenvalues far in the right half plane, shown by
planting it).
"""
import numpy as np
import pytest

import workloads as W
from oracle.rhs import Problem, rk4_step

ROT = (0.0, 0.0, 0.0, -1.0, 1.0, 0.0)
ROT_SHIFT = (0.3, -0.2, 0.0, -1.0, 1.0, 0.0)


def _cases():
    return [
        ("const", 0.7, None, 1),
        ("const", [1e-3, 0.5], ROT, 2),
        ("element", "loguniform", None, 1),
        ("element", "loguniform", ROT_SHIFT, 1),
        ("element2", "loguniform", None, 1),
    ]


def _problem(N, mode, D, vel, nf, m=4, seed=41):
    mesh = W.split_square_mesh(m, 0.2, seed=seed)
    alg = 2 if mode == "element2" else 1
    if mode.startswith("element"):
        mode = "element"
        D = W.loguniform_per_element(mesh.K, 1e-3, 1e1, seed=seed + 1)
    return mesh, Problem(mesh.vxy, mesh.etov, N, D, D_mode=mode, velocity=vel, nfields=nf, alg=alg)


def _sample(pr):
    g = pr.geom
    bdy = [k for k in range(g.K) if np.any(g.EToE[k] < 0)]
    inner = [k for k in range(g.K) if np.all(g.EToE[k] >= 0)]
    return sorted({0, g.K - 1, bdy[len(bdy) // 2], inner[0], inner[-1]})


@pytest.mark.parametrize("N", [2, 3])
@pytest.mark.parametrize("case", range(5))
def test_rhs_elements_equals_assembled_rhs(N, case):
    mode, D, vel, nf = _cases()[case]
    mesh, pr = _problem(N, mode, D, vel, nf)
    rng = np.random.default_rng(N * 10 + case)
    u = rng.standard_normal((nf, mesh.K, pr.ops.Np))
    full = pr.rhs(u)
    els = _sample(pr)
    for f in range(nf):
        got = pr.rhs_elements(u[f], els, field=f)
        ref = full[f, els]
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(full[f]).max()


@pytest.mark.parametrize("case", range(5))
def test_rk4_step_elements_equals_full_step(case):
    N = 2
    mode, D, vel, nf = _cases()[case]
    mesh, pr = _problem(N, mode, D, vel, nf, m=5)
    rng = np.random.default_rng(7 + case)
    u = rng.standard_normal((nf, mesh.K, pr.ops.Np))
    # a step of the order of the inverse spectral radius: the increment is
    # of the size of the state, so the four stages all matter
    v = rng.standard_normal(u.shape)
    for _ in range(30):
        w = pr.rhs(v)
        rho = np.linalg.norm(w) / np.linalg.norm(v)
        v = w / np.linalg.norm(w)
    dt = 0.5 / rho
    full = rk4_step(pr.rhs, u, dt)
    els = _sample(pr)
    for f in range(nf):
        got = pr.rk4_step_elements(u[f], dt, els, field=f)
        inc_ref = full[f, els] - u[f, els]
        assert np.abs(got - full[f, els]).max() <= 1e-12 * np.abs(inc_ref).max() * 10


def _operator(pr):
    K, Np = pr.geom.K, pr.ops.Np
    L = np.zeros((K * Np, K * Np))
    for j in range(K * Np):
        e = np.zeros(K * Np)
        e[j] = 1.0
        L[:, j] = pr.rhs(e.reshape(K, Np)).ravel()
    return L


def _max_real_over_rho(pr):
    lam = np.linalg.eigvals(_operator(pr))
    return lam.real.max() / np.abs(lam).max()


CONST_V = (0.7, -0.3, 0.0, 0.0, 0.0, 0.0)


@pytest.mark.parametrize("N", [1, 2, 3, 4])
@pytest.mark.parametrize("D", [0.0, 1e-2])
def test_upwind_convection_spectrum_is_dissipative(N, D):
    """Constant velocity: v u is in P_N, the collocated flux is exact, and
    upwind DG with zero inflow data is dissipative, so max Re(lambda) <= 0 up
    to rounding."""
    mesh = W.split_square_mesh(3, 0.2, seed=43)
    pr = Problem(mesh.vxy, mesh.etov, N, D, velocity=CONST_V)
    assert _max_real_over_rho(pr) <= 1e-10


@pytest.mark.parametrize("N", [2, 3, 4])
def test_rotating_convection_spectrum_near_dissipative(N):
    """Rotating velocity v = v0 + (-y, x): v u has degree N + 1 and its nodal
    collocation aliases, which can lift a few eigenvalues slightly into the
    right half plane (measured max Re(lambda)/rho = 6.5e-4 at N = 3 on this
    mesh, without diffusion); a downwind flux gives 1.0."""
    mesh = W.split_square_mesh(3, 0.2, seed=43)
    pr = Problem(mesh.vxy, mesh.etov, N, 0.0, velocity=ROT_SHIFT)
    assert _max_real_over_rho(pr) <= 2e-3


def test_spectrum_detects_planted_downwind_flux(monkeypatch):
    """Planting a downwind flux in the oracle turns the spectrum test red."""
    mesh = W.split_square_mesh(3, 0.2, seed=43)
    pr = Problem(mesh.vxy, mesh.etov, 2, 0.0, velocity=CONST_V)
    pr_rot = Problem(mesh.vxy, mesh.etov, 2, 0.0, velocity=ROT_SHIFT)
    orig = Problem.upwind_face_flux

    def downwind(self, u, t=0.0, field=0):
        ops, g = self.ops, self.geom
        up = orig(self, u, t, field)
        # f* = min(n.v,0) u- + max(n.v,0) u+: recover u+ from the upwind form
        xyn = g.physical(ops.rs)
        vx, vy = self.velocity_at(xyn)
        out = np.zeros_like(up)
        for k in range(g.K):
            for f in range(3):
                idx = ops.fmask[f]
                vn = g.nx[k, f] * vx[k, idx] + g.ny[k, f] * vy[k, idx]
                k2 = g.EToE[k, f]
                uo = np.zeros(ops.Nfp) if k2 < 0 else u[k2, ops.fmask[g.EToF[k, f]]][::-1]
                out[k, f] = np.minimum(vn, 0.0) * u[k, idx] + np.maximum(vn, 0.0) * uo
        return out

    monkeypatch.setattr(Problem, "upwind_face_flux", downwind)
    assert _max_real_over_rho(pr) > 0.5
    assert _max_real_over_rho(pr_rot) > 0.5
