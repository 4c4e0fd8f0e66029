"""Parity of the library's compressible Navier-Stokes path with the oracle.

The state is the isentropic vortex on a distorted split-square mesh with a
seeded 2% perturbation; the exterior state is the unperturbed vortex scaled
by (1 + 0.05 t), linear in t, so the library's Chebyshev-in-time
representation reproduces it exactly.  Bars: FP64 1e-12 of max |rhs| (the
arithmetic differs from the oracle's only in rounding order); FP32 2e-5 of
max |rhs|, about ten times the largest error measured (1.9e-6; LSERK steps
1.5e-6 of the increment).
"""
import numpy as np
import pytest

import workloads as W
from boundary_data import chebyshev_coefficients
from gpu_common import to_dev, to_np

pytestmark = pytest.mark.gpu

PRECS = {"fp64": (0, 1e-12), "fp32": (1, 2e-5)}
LAWS = {"sutherland": 1, "constant": 2}


def vortex_state(x, y):
    return W.isentropic_vortex(x, y, beta=5.0, uinf=(0.3, 0.2), c0=(0.5, 0.5), L=0.15)


def exterior(x, y, t):
    return vortex_state(x, y) * (1.0 + 0.05 * t)


def _setup(N, m=6, jitter=0.2, seed=0, law="sutherland", mu=2e-3, ext=exterior, build_edges=True):
    from oracle.ns import Gas, NavierStokes
    from paper_1912_06221_amd import ardg
    mesh = W.split_square_mesh(m, jitter, seed=seed)
    ops = ardg.Ops(N)
    lm = ardg.Mesh(ops, mesh.vxy, mesh.etov, device=0)
    lm.set_navier_stokes(LAWS[law], mu_ref=mu)
    X = lm.export(ardg.MESH_BFACE_GHOST_NODES).reshape(lm.E_bdy, ops.Np, 2)
    lm.set_boundary_data(chebyshev_coefficients(lambda x, y, t, f: ext(x, y, t)[f], X, 0.0, 1.0, 2, 4),
                         0.0, 1.0)
    ns = NavierStokes(mesh.vxy, mesh.etov, N, Gas(mu_ref=mu, law=law), ext, build_edges=build_edges)
    return mesh, ops, lm, ns


def _state(ns, seed=1):
    xy = ns.nodal_xy()
    Q = vortex_state(xy[..., 0], xy[..., 1])
    rng = np.random.default_rng(seed)
    return Q * (1.0 + 0.02 * rng.standard_normal(Q.shape))


@pytest.mark.parametrize("N", [1, 2, 3, 4])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_ns_rhs_matches_oracle(N, prec):
    import torch
    code, tol = PRECS[prec]
    mesh, ops, lm, ns = _setup(N)
    Q = _state(ns)
    t = 0.3
    ref = ns.rhs(Q, t)
    dt = torch.float64 if prec == "fp64" else torch.float32
    u = to_dev(Q, dt)
    out = torch.empty_like(u)
    lm.rhs_eval(u, out, precision=code, nfields=4, t=t)
    got = to_np(out)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"NS rhs N={N} {prec}: max err / max |rhs| = {err:.2e}")
    assert err < tol


@pytest.mark.parametrize("law", ["sutherland", "constant"])
def test_ns_edge_flux_matches_oracle(law):
    """The interface flux sJ (F + G)* . n1 of every interior edge and boundary
    face, in the library's edge order (side 1's node order)."""
    import torch
    from paper_1912_06221_amd import ardg
    N = 3
    mesh, ops, lm, ns = _setup(N, law=law, mu=5e-3)
    Q = _state(ns, seed=4)
    t = 0.7
    H = ns.face_fluxes(Q, t)                       # [K, 3, 4, Nfp]
    u = to_dev(Q)
    E = lm.E_int + lm.E_bdy
    fl = torch.empty((4, E, ops.Nfp), dtype=torch.float64, device=u.device)
    lm.edge_flux_eval(u, fl, precision=ardg.FP64, nfields=4, t=t)
    got = to_np(fl)
    edges = lm.export(ardg.MESH_EDGES).reshape(-1, 4)
    bf = lm.export(ardg.MESH_BFACES).reshape(-1, 2)
    sJ = ns.geom.sJ
    ref = np.zeros_like(got)
    for e, (k1, f1, _, _) in enumerate(edges):
        ref[:, e] = sJ[k1, f1] * H[k1, f1]
    for b, (k1, f1) in enumerate(bf):
        ref[:, lm.E_int + b] = sJ[k1, f1] * H[k1, f1]
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"NS edge flux {law}: {err:.2e}")
    assert err < 1e-12


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_ns_lserk_steps_match_oracle(prec):
    """Three low-storage RK steps from t0 = 0.1: every stage evaluates the
    exterior state at its own time."""
    import torch
    from oracle.rhs import lserk_step
    from paper_1912_06221_amd import ardg
    code = PRECS[prec][0]
    N = 3
    mesh, ops, lm, ns = _setup(N, m=5)
    Q = _state(ns, seed=2)
    dt, t0, nsteps = 2e-3, 0.1, 3
    ref = Q.copy()
    t = t0
    for _ in range(nsteps):
        ref = lserk_step(lambda q, tt: ns.rhs(q, tt), ref, dt, t)
        t += dt
    u = to_dev(Q)
    work = ardg.alloc_workspace(lm.workspace_bytes(ardg.LSERK54, code, 4), u.device)
    lm.rk_step(u, work, dt, nsteps, scheme=ardg.LSERK54, precision=code, nfields=4, t0=t0)
    got = to_np(u)
    inc = np.abs(ref - Q).max()
    err = np.abs(got - ref).max() / inc
    print(f"NS LSERK {prec}: max err / max increment = {err:.2e}")
    assert err < (1e-11 if prec == "fp64" else 2e-5)


def test_ns_density_wave_is_exact_on_gpu():
    """Inviscid, rho linear, velocity and pressure constant: every flux is
    linear and dQ/dt = -U . grad Q to round-off (the oracle's exact pin)."""
    import torch
    from paper_1912_06221_amd import ardg
    U, a, p0, gam = (0.4, -0.25), (0.5, 0.3), 1.0, 1.4

    def wave(x, y, t):
        rho = 1.0 + a[0] * (x - U[0] * t) + a[1] * (y - U[1] * t)
        E = p0 / (gam - 1) + 0.5 * rho * (U[0] ** 2 + U[1] ** 2)
        return np.stack([rho, rho * U[0], rho * U[1], E])
    for N in (1, 2, 3):
        mesh, ops, lm, ns = _setup(N, law="constant", mu=0.0, ext=wave)
        xy = ns.nodal_xy()
        Q = wave(xy[..., 0], xy[..., 1], 0.25)
        exact = np.imag(wave(xy[..., 0] + 0j, xy[..., 1] + 0j, 0.25 + 1e-30j)) / 1e-30
        u = to_dev(Q)
        out = torch.empty_like(u)
        lm.rhs_eval(u, out, precision=ardg.FP64, nfields=4, t=0.25)
        err = np.abs(to_np(out) - exact).max()
        print(f"NS density wave N={N}: {err:.2e}")
        assert err < 1e-12


def test_ns_noalloc_matches_rhs_eval():
    import torch
    from paper_1912_06221_amd import ardg
    mesh, ops, lm, ns = _setup(2)
    u = to_dev(_state(ns, seed=5))
    a, b = torch.empty_like(u), torch.empty_like(u)
    lm.rhs_eval(u, a, precision=ardg.FP64, nfields=4, t=0.2)
    lm.rhs_eval_noalloc(u, b, precision=ardg.FP64, nfields=4, t=0.2)
    assert torch.equal(a, b)


def test_ns_refusals():
    import torch
    from paper_1912_06221_amd import ardg
    mesh, ops, lm, ns = _setup(2)
    u = to_dev(_state(ns))
    out = torch.empty_like(u)
    with pytest.raises(ardg.ArdgError):
        lm.rhs_eval(u, out, precision=ardg.FP64, nfields=1)
    with pytest.raises(ardg.ArdgError):
        lm.rhs_eval(u.float(), out.float(), precision=ardg.BF16X3, nfields=4)
    with pytest.raises(ardg.ArdgError):
        ardg.Batch([lm])
    lm.set_boundary_data(None, 0.0, 1.0)
    with pytest.raises(ardg.ArdgError):
        lm.rhs_eval(u, out, precision=ardg.FP64, nfields=4)
    # switched off, the mesh is a scalar problem again
    lm.set_navier_stokes(ardg.NS_OFF)
    lm.set_diffusion_const([1.0])
    one = torch.zeros((1, lm.K, ops.Np), dtype=torch.float64, device=u.device)
    lm.rhs_eval(one, torch.empty_like(one), precision=ardg.FP64, nfields=1)


def test_fullsize_ns_rhs_sampled():
    """The bench's Navier-Stokes workload (708 x 708 split square, 1 002 528
    elements, N = 3, four fields): the RHS of sampled elements, boundary
    elements included, against the oracle element by element."""
    import torch
    from paper_1912_06221_amd import ardg
    N = 3
    mesh, ops, lm, ns = _setup(N, m=708, jitter=0.2, seed=11, build_edges=False)
    K = mesh.K
    xy = ns.nodal_xy()
    Q = vortex_state(xy[..., 0], xy[..., 1])
    rng = np.random.default_rng(12)
    Q *= 1.0 + 0.01 * rng.standard_normal(Q.shape)
    t = 0.4
    u = to_dev(Q)
    out = torch.empty_like(u)
    lm.rhs_eval(u, out, precision=ardg.FP64, nfields=4, t=t)
    got = to_np(out)
    els = np.concatenate([rng.choice(K, 20, replace=False), [0, 1, 2 * 707, K - 1, K - 2]])
    ref = ns.rhs_elements(Q, els, t)
    err = np.abs(got[:, els] - ref).max() / np.abs(ref).max()
    print(f"NS full-size sampled rhs: {err:.2e}")
    assert err < 1e-12
