"""Parity of the library's tensor diffusion coefficients (nodal tensor field;
solution-dependent u D0) with the oracle's Algorithm 1 with nodal products:
edge fluxes and right-hand sides on random data, with and without
convection and prescribed boundary data, and RK4 steps (nonlinear for the
solution-dependent coefficient)."""
import numpy as np
import pytest

import workloads as W
from boundary_data import chebyshev_coefficients
from gpu_common import to_dev, to_np

pytestmark = pytest.mark.gpu

# FP32: about ten times the largest error measured on these inputs (5.9e-7)
TOL = {0: 1e-12, 1: 5e-6}


def _tensor_field(K, Np, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(0.5, 2.0, (K, Np)), rng.uniform(-0.3, 0.3, (K, Np)),
                     rng.uniform(0.5, 2.0, (K, Np))], axis=-1)


def _case(m, N, mode, vel, seed, ghost=None):
    from oracle.rhs import Problem
    from paper_1912_06221_amd import ardg
    mesh = W.split_square_mesh(m, 0.2, seed=seed)
    ops = ardg.Ops(N)
    lm = ardg.Mesh(ops, mesh.vxy, mesh.etov, device=0)
    if mode == "nodal":
        D = _tensor_field(mesh.K, ops.Np, seed + 1)
        lm.set_diffusion_nodal(D)
    else:
        D = (0.8, 0.25, 0.6)
        lm.set_diffusion_solution(D)
    if vel is not None:
        lm.set_velocity(vel)
    if ghost is not None:
        X = lm.export(ardg.MESH_BFACE_GHOST_NODES).reshape(lm.E_bdy, ops.Np, 2)
        lm.set_boundary_data(chebyshev_coefficients(ghost, X, 0.0, 1.0, 4), 0.0, 1.0)
    pr = Problem(mesh.vxy, mesh.etov, N, D, D_mode=mode, velocity=vel, ghost=ghost)
    return mesh, ops, lm, pr


def _g(x, y, t, f):
    return 1.0 + 0.3 * np.sin(1.1 * x + 0.2) * np.cos(0.9 * y) * (1.0 + t)


CASES = [
    # m, N, mode, velocity, prescribed data
    (7, 1, "nodal", None, False),
    (7, 2, "nodal", None, False),
    (6, 3, "nodal", (0.5, -0.3, 0.0, -1.0, 1.0, 0.0), False),
    (5, 4, "nodal", None, True),
    (4, 6, "nodal", None, False),
    (7, 2, "solution", None, False),
    (6, 3, "solution", None, True),
    (5, 4, "solution", (0.4, 0.2, 0.0, 0.0, 0.0, 0.0), False),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"m{c[0]}-N{c[1]}-{c[2]}-{'conv' if c[3] else 'diff'}-{'g' if c[4] else 'm'}")
@pytest.mark.parametrize("prec", [0, 1])
def test_tensor_flux_and_rhs(case, prec):
    import torch
    m, N, mode, vel, presc = case
    print(f"tensor {case} prec={prec}", flush=True)
    mesh, ops, lm, pr = _case(m, N, mode, vel, seed=10 * m + N, ghost=_g if presc else None)
    # positive data for the solution-dependent coefficient (u D0 definite)
    u = 1.0 + 0.3 * W.random_nodal((1, mesh.K, ops.Np), seed=m + N)
    t = 0.4
    dt = torch.float64 if prec == 0 else torch.float32
    ud = to_dev(u, dt)
    rhs = torch.empty_like(ud)
    lm.rhs_eval(ud, rhs, precision=prec, t=t)
    ro = pr.rhs(u[0], t)
    err = np.abs(to_np(rhs)[0] - ro).max() / np.abs(ro).max()
    print(f"  rhs rel err {err:.2e}", flush=True)
    assert err <= TOL[prec]


def test_tensor_rk4_steps_and_refusals():
    from oracle.rhs import mass_norm, rk4_step
    from paper_1912_06221_amd import ardg
    print("tensor rk4", flush=True)
    for mode in ("nodal", "solution"):
        mesh, ops, lm, pr = _case(6, 3, mode, None, seed=3)
        xy = pr.nodal_xy()
        u0 = 1.0 + 0.5 * np.sin(np.pi * xy[..., 0]) * np.sin(np.pi * xy[..., 1])
        dt, n = 2e-5, 10
        ud = to_dev(u0[None])
        work = ardg.alloc_workspace(lm.workspace_bytes(ardg.RK4, ardg.FP64, 1), ud.device)
        lm.rk_step(ud, work, dt, n)
        uo = u0
        for _ in range(n):
            uo = rk4_step(pr.rhs, uo, dt)
        rel = mass_norm(pr, to_np(ud)[0] - uo) / mass_norm(pr, uo - u0)
        print(f"  {mode}: state error relative to the change {rel:.2e}", flush=True)
        assert rel <= 1e-11
        with pytest.raises(ardg.ArdgError) as ei:
            lm.rk_step(ud, ardg.alloc_workspace(lm.workspace_bytes(ardg.RK4, ardg.BF16X3, 1), ud.device),
                       dt, 1, precision=ardg.BF16X3)
        assert ei.value.status == -6
    # a tensor that is not positive definite is refused
    mesh = W.split_square_mesh(3, 0.0)
    ops = ardg.Ops(2)
    lm = ardg.Mesh(ops, mesh.vxy, mesh.etov, device=0)
    bad = np.tile(np.array([1.0, 2.0, 1.0]), (mesh.K, ops.Np, 1))
    with pytest.raises(ardg.ArdgError):
        lm.set_diffusion_nodal(bad)
