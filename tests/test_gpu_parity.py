"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances:
* FP64: relative 1e-12.  On seeded uniform random data the measure is
  max|rhs_gpu - rhs_oracle| / max|rhs_oracle|.  On smooth data the
  difference is measured against the scale of the operator's terms,
  max|L u_r| for random data u_r of the same amplitude, because the discrete
  Laplacian's individual terms exceed its result by about N^4/h^2.  The RK
  state after k steps: ||du||_M / ||u||_M.
* FP32 (operators and arithmetic in FP32, built from FP64) and BF16X3 (FP32
  data, products on the BF16 matrix cores as hi*hi + hi*lo + lo*hi with
  hi = bf16(x), lo = bf16(x - hi), FP32 accumulation): about ten times the
  largest error measured on these inputs across the GPU suite (the kernels
  are deterministic and the inputs seeded, so the measured values repeat):
    FP32 flux / rhs measures 5e-6 (measured up to 5.9e-7), RK states 2e-6
    (measured up to 2.1e-7);
    BF16X3 flux / rhs measures 2.5e-4 (measured up to 2.4e-5), RK states
    2.5e-5 (measured up to 2.3e-6).
"""
import math

import numpy as np
import pytest

import workloads as W
from gpu_common import library_mesh, make_case, oracle_problem, to_dev, to_np

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 5e-6
TOLBF = 2.5e-4
TOL_STATE = {"fp64": 1e-12, "fp32": 2e-6, "bf16x3": 2.5e-5}

PRECS = {"fp64": (0, TOL64), "fp32": (1, TOL32), "bf16x3": (2, TOLBF)}


def _flux_oracle(pr, u, nfields):
    """Oracle edge fluxes times each edge's surface factor sJ = |edge| / 2,
    the scaling the library's edge_flux_eval returns."""
    sj = np.array([pr.geom.sJ[k1, f1] for (k1, f1, _, _) in pr.int_edges] +
                  [pr.geom.sJ[k, fb] for (k, fb) in pr.bdy_edges])[:, None]
    out = []
    for f in range(nfields):
        Fi, Fb = pr.diffusive_flux(u[f], f)
        if pr.velocity is not None:
            fs = pr.upwind_face_flux(u[f])
            ie = pr.int_edges
            Fi = Fi - np.array([fs[k1, f1] for (k1, f1, _, _) in ie]).reshape(Fi.shape)
            Fb = Fb - np.array([fs[k, fb] for (k, fb) in pr.bdy_edges]).reshape(Fb.shape)
        out.append(np.vstack([Fi, Fb]) * sj)
    return np.stack(out)


CASES = [
    # m, jitter, N, D_mode, velocity, nfields
    (12, 0.2, 1, "const", None, 1),
    (12, 0.2, 2, "const", None, 1),
    (11, 0.2, 3, "const", None, 1),
    (12, 0.25, 4, "const", None, 1),
    (9, 0.2, 5, "const", None, 1),
    (9, 0.2, 6, "const", None, 1),
    (12, 0.2, 2, "element", None, 1),
    (11, 0.2, 4, "element", None, 1),
    (8, 0.2, 6, "element", None, 1),
    (12, 0.2, 3, "const", (0.0, 0.0, 0.0, -1.0, 1.0, 0.0), 3),
    (10, 0.2, 2, "const", (0.6, -0.4, 0.2, -1.0, 1.0, 0.1), 2),
    (10, 0.2, 4, "const", (0.3, -0.2, 0.0, -1.0, 1.0, 0.0), 2),
    (12, 0.2, 2, "element2", None, 1),
    (11, 0.2, 3, "element2", None, 1),
    (8, 0.2, 6, "element2", None, 1),
    (10, 0.2, 4, "element2", (0.3, -0.2, 0.0, -1.0, 1.0, 0.0), 1),
]


def _ids(c):
    return f"m{c[0]}-N{c[2]}-{c[3]}-{'conv' if c[4] else 'diff'}-F{c[5]}"


@pytest.mark.parametrize("case", CASES, ids=_ids)
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_edge_flux_and_rhs_parity_random(case, prec):
    import torch
    from paper_1912_06221_amd import ardg
    m, jit, N, D_mode, vel, nf = case
    print(f"case {_ids(case)} {prec}", flush=True)
    mesh, D = make_case(m, jit, N, D_mode, velocity=vel, nfields=nf, seed=10 * m + N)
    if D_mode == "const":
        D = [0.3 + f for f in range(nf)]
    ops, lm = library_mesh(mesh, N, D_mode, D, vel, nf)
    pr = oracle_problem(mesh, N, D_mode, D, vel, nf)
    u = W.random_nodal((nf, mesh.K, ops.Np), seed=m + N)
    dt = torch.float64 if prec == "fp64" else torch.float32
    p, tol = PRECS[prec]
    ud = to_dev(u, dt)
    flux = torch.empty((nf, lm.E, ops.Nfp), dtype=dt, device=ud.device)
    lm.edge_flux_eval(ud, flux, precision=p, nfields=nf)
    Fo = _flux_oracle(pr, u, nf)
    Fg = to_np(flux)
    ef = np.abs(Fg - Fo).max() / np.abs(Fo).max()
    print(f"  flux rel err {ef:.2e}", flush=True)
    assert ef <= tol
    rhs = torch.empty_like(ud)
    lm.rhs_eval(ud, rhs, precision=p, nfields=nf)
    ro = pr.rhs(u)
    rg = to_np(rhs)
    err = np.abs(rg - ro).max() / np.abs(ro).max()
    print(f"  rhs rel err {err:.2e}", flush=True)
    assert err <= tol


@pytest.mark.parametrize("N", [2, 3, 4])
def test_rhs_parity_smooth_data(N):
    import torch
    from paper_1912_06221_amd import ardg
    print(f"smooth N={N}", flush=True)
    mesh = W.split_square_mesh(16, 0.2, seed=N)
    D = W.circle_contrast_D(mesh)
    ops, lm = library_mesh(mesh, N, "element", D, None, 1)
    pr = oracle_problem(mesh, N, "element", D, None, 1)
    xy = pr.nodal_xy()
    u = W.fourier_modes(xy[..., 0], xy[..., 1], seed=3)
    ur = W.random_nodal(u.shape, seed=4) * np.abs(u).max()
    scale = np.abs(pr.rhs(ur)).max()
    ud = to_dev(u)
    rhs = torch.empty_like(ud)
    lm.rhs_eval(ud, rhs, precision=ardg.FP64)
    assert np.abs(to_np(rhs) - pr.rhs(u)).max() <= TOL64 * scale


def test_empty_and_tiny_meshes():
    """One element (only boundary faces) and two elements (one interior edge)."""
    import torch
    from paper_1912_06221_amd import ardg
    print("tiny meshes", flush=True)
    for vxy, etov in ((np.array([[0, 0], [1, 0], [0, 1.0]]), np.array([[0, 1, 2]], dtype=np.int32)),
                      (np.array([[0, 0], [1, 0], [1, 1], [0, 1.0]]),
                       np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32))):
        for N in (1, 3):
            ops = ardg.Ops(N)
            lm = ardg.Mesh(ops, vxy, etov, device=0)
            lm.set_diffusion_const([0.7])
            from oracle.rhs import Problem
            pr = Problem(vxy, etov, N, 0.7)
            u = W.random_nodal((1, len(etov), ops.Np), seed=N)
            ud = to_dev(u)
            rhs = torch.empty_like(ud)
            lm.rhs_eval(ud, rhs)
            ro = pr.rhs(u)
            assert np.abs(to_np(rhs) - ro).max() <= TOL64 * np.abs(ro).max()


@pytest.mark.parametrize("N", [2, 3])
@pytest.mark.parametrize("scheme", ["rk4", "lserk"])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_time_stepping_heat_8x8(scheme, prec, N):
    """The plain heat problem: 8x8x2 unjittered, D=1, u0 = sin(pi x) sin(pi y),
    100 steps (N = 2 is the plain-method workload as configured); state parity
    with the oracle and the error against the exact solution."""
    import torch
    from oracle.rhs import lserk_step, mass_norm, rk4_step
    from paper_1912_06221_amd import ardg
    print(f"heat 8x8 N={N} {scheme} {prec}", flush=True)
    mesh = W.split_square_mesh(8, 0.0)
    ops, lm = library_mesh(mesh, N, "const", 1.0, None, 1)
    pr = oracle_problem(mesh, N, "const", 1.0, None, 1)
    xy = pr.nodal_xy()
    u0 = W.manufactured(xy[..., 0], xy[..., 1])
    dt, nsteps = 5e-5, 100
    uo = u0.copy()
    step = rk4_step if scheme == "rk4" else lserk_step
    for _ in range(nsteps):
        uo = step(pr.rhs, uo, dt)
    sch = ardg.RK4 if scheme == "rk4" else ardg.LSERK54
    p = PRECS[prec][0]
    ud = to_dev(u0[None])
    work = ardg.alloc_workspace(lm.workspace_bytes(sch, p, 1), ud.device)
    # capture the graph ahead (ardg_rk_prepare), then replay it
    lm.rk_prepare(ud, work, dt, nsteps, scheme=sch, precision=p)
    lm.rk_step(ud, work, dt, nsteps, scheme=sch, precision=p)
    ug = to_np(ud)[0]
    rel = mass_norm(pr, ug - uo) / mass_norm(pr, uo)
    print(f"  state rel err {rel:.2e}", flush=True)
    assert rel <= TOL_STATE[prec]
    # graph replay: a second call continues from the new state
    lm.rk_step(ud, work, dt, nsteps, scheme=sch, precision=p)
    for _ in range(nsteps):
        uo = step(pr.rhs, uo, dt)
    rel2 = mass_norm(pr, to_np(ud)[0] - uo) / mass_norm(pr, uo)
    assert rel2 <= TOL_STATE[prec]
    from oracle.rhs import error_norms
    l2, _ = error_norms(pr, to_np(ud)[0], lambda x, y: W.manufactured(x, y, 2 * nsteps * dt))
    assert l2 < 2e-3


@pytest.mark.parametrize("scheme", ["rk4", "lserk"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_time_stepping_several_fields(prec, scheme):
    """Three fields with their own D and a rotating velocity, stepped together
    over two calls (the second replays the graph from the new state): each
    field's state matches the oracle's and the same field stepped alone (bit
    for bit in FP64, where both use the same edge kernel; FP32 takes the
    multi-field edge kernel for several fields)."""
    import torch
    from oracle.rhs import lserk_step, mass_norm, rk4_step
    from paper_1912_06221_amd import ardg
    print(f"three fields {scheme} {prec}", flush=True)
    N, nf = 3, 3
    vel = (0.3, -0.2, 0.0, -1.0, 1.0, 0.0)
    Dc = [2e-3, 5e-3, 1e-2]
    mesh, _ = make_case(6, 0.2, N, velocity=vel, nfields=nf, seed=21)
    ops, lm = library_mesh(mesh, N, "const", np.array(Dc), vel, nf)
    pr = oracle_problem(mesh, N, "const", np.array(Dc), vel, nf)
    xy = pr.nodal_xy()
    u0 = np.stack([np.sin(xy[..., 0] * (1.1 + f)) * np.cos(xy[..., 1] * (1.7 - 0.4 * f)) for f in range(nf)])
    sch = ardg.RK4 if scheme == "rk4" else ardg.LSERK54
    step = rk4_step if scheme == "rk4" else lserk_step
    p = PRECS[prec][0]
    tol = 1e-11 if prec == "fp64" else 2e-5
    dt, n = 1e-5, 20
    ud = to_dev(u0)
    work = ardg.alloc_workspace(lm.workspace_bytes(sch, p, nf), ud.device)
    lm.rk_step(ud, work, dt, n, scheme=sch, precision=p, nfields=nf)
    lm.rk_step(ud, work, dt, n, scheme=sch, precision=p, nfields=nf)
    ug = to_np(ud)
    uo = u0.copy()
    for _ in range(2 * n):
        uo = step(pr.rhs, uo, dt)
    for f in range(nf):
        rel = mass_norm(pr, ug[f] - uo[f]) / mass_norm(pr, uo[f] - u0[f])
        print(f"  field {f}: state error relative to the change {rel:.2e}", flush=True)
        assert rel <= tol
        # the same field alone
        _, l1 = library_mesh(mesh, N, "const", np.array([Dc[f]]), vel, 1)
        u1 = to_dev(u0[f:f + 1])
        w1 = ardg.alloc_workspace(l1.workspace_bytes(sch, p, 1), u1.device)
        l1.rk_step(u1, w1, dt, n, scheme=sch, precision=p)
        l1.rk_step(u1, w1, dt, n, scheme=sch, precision=p)
        torch.cuda.synchronize()
        if prec == "fp64":
            assert torch.equal(u1[0], ud[f])
        else:
            u1n = to_np(u1)[0]
            assert mass_norm(pr, u1n - ug[f]) / mass_norm(pr, uo[f] - u0[f]) <= tol


def test_long_run_equals_short_runs():
    """A run longer than one captured graph (graphs of at most 256 steps,
    replayed, plus a remainder graph) gives the same state as the same steps
    taken in shorter calls."""
    import torch
    from paper_1912_06221_amd import ardg
    mesh = W.split_square_mesh(6, 0.2, seed=3)
    N = 2
    ops, lm = library_mesh(mesh, N, "const", 0.5, None, 1)
    u0 = W.random_nodal((1, mesh.K, ops.Np), seed=4)
    dt = 1e-5
    a = to_dev(u0)
    b = to_dev(u0)
    work = ardg.alloc_workspace(lm.workspace_bytes(ardg.RK4, ardg.FP64, 1), a.device)
    lm.rk_step(a, work, dt, 600, scheme=ardg.RK4, precision=ardg.FP64)
    for _ in range(6):
        lm.rk_step(b, work, dt, 100, scheme=ardg.RK4, precision=ardg.FP64)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert bool(torch.isfinite(a).all())


def test_determinism():
    import torch
    from paper_1912_06221_amd import ardg
    print("determinism", flush=True)
    mesh = W.split_square_mesh(20, 0.2, seed=1)
    D = W.circle_contrast_D(mesh)
    ops, lm = library_mesh(mesh, 4, "element", D, None, 1)
    u = to_dev(W.random_nodal((1, mesh.K, ops.Np), seed=5))
    a = torch.empty_like(u)
    b = torch.empty_like(u)
    lm.rhs_eval(u, a)
    lm.rhs_eval(u, b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_check_detects_nonfinite():
    import torch
    from paper_1912_06221_amd import ardg
    print("nonfinite check", flush=True)
    mesh = W.split_square_mesh(4, 0.0)
    ops, lm = library_mesh(mesh, 2, "const", 1.0, None, 1)
    u = to_dev(W.random_nodal((1, mesh.K, ops.Np), seed=1))
    lm.check(u)
    u[0, 3, 2] = float("nan")
    with pytest.raises(ardg.ArdgError) as ei:
        lm.check(u)
    assert ei.value.status == -9


VARIANT_CASES = [
    # m, N, D kind, velocity
    (10, 1, "blocks", None),
    (10, 2, "blocks", None),
    (11, 3, "blocks", None),
    (12, 4, "blocks", None),
    (9, 5, "blocks", None),
    (9, 6, "blocks", None),
    (12, 4, "const", None),
    (10, 3, "const", (0.0, 0.0, 0.0, -1.0, 1.0, 0.0)),
    (10, 4, "blocks", (0.3, -0.2, 0.0, -1.0, 1.0, 0.0)),
    (10, 2, "blocks2", None),
    (9, 5, "blocks2", None),
    (10, 3, "blocks2", (0.0, 0.0, 0.0, -1.0, 1.0, 0.0)),
]


def _blocks_D(mesh):
    # two values of D, split at the middle element index: edge tiles away from
    # the split see one value (equal-D form of Algorithm 1), tiles near it two
    k = np.arange(mesh.K)
    return np.where(k < mesh.K // 2, 0.7, 3.1)


@pytest.mark.parametrize("case", VARIANT_CASES,
                         ids=lambda c: f"m{c[0]}-N{c[1]}-{c[2]}-{'conv' if c[3] else 'diff'}")
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_matrix_core_and_vector_kernels_agree(case, prec):
    """The edge kernel implementations (ardg_mesh_set_kernels) -- chosen by
    grid size, edge tiles split by side (conversion on the vector unit or on
    the matrix cores), one thread per edge, one wave per tile on the matrix
    cores -- compute the same flux and RHS (to rounding), each matching the
    oracle."""
    import torch
    from paper_1912_06221_amd import ardg
    m, N, dk, vel = case
    print(f"variants m{m} N{N} {dk} {prec}", flush=True)
    mesh = W.split_square_mesh(m, 0.2, seed=100 + N)
    D_mode = {"blocks": "element", "blocks2": "element2"}.get(dk, "const")
    D = _blocks_D(mesh) if dk.startswith("blocks") else [0.9]
    pr = oracle_problem(mesh, N, D_mode, D, vel, 1)
    dt = torch.float64 if prec == "fp64" else torch.float32
    p = ardg.FP64 if prec == "fp64" else ardg.FP32
    tol = TOL64 if prec == "fp64" else TOL32
    outs = {}
    variants = {"default": ardg.EDGE_AUTO, "split": ardg.EDGE_SPLIT, "split-mfma": ardg.EDGE_SPLIT_MFMA,
                "lane": ardg.EDGE_LANE, "mfma": ardg.EDGE_MFMA, "fields": ardg.EDGE_FIELDS}
    if dk.startswith("blocks"):
        del variants["fields"]      # the multi-field lanes take constant D only
    for variant, kern in variants.items():
        ops, lm = library_mesh(mesh, N, D_mode, D, vel, 1)
        lm.set_kernels(kern)
        u = W.random_nodal((1, mesh.K, ops.Np), seed=7 * N + m)
        ud = to_dev(u, dt)
        flux = torch.empty((1, lm.E, ops.Nfp), dtype=dt, device=ud.device)
        lm.edge_flux_eval(ud, flux, precision=p)
        rhs = torch.empty_like(ud)
        lm.rhs_eval(ud, rhs, precision=p)
        outs[variant] = (to_np(flux), to_np(rhs))
    Fo = _flux_oracle(pr, u, 1)
    ro = pr.rhs(u)
    for variant, (Fg, rg) in outs.items():
        ef = np.abs(Fg - Fo).max() / np.abs(Fo).max()
        er = np.abs(rg - ro).max() / np.abs(ro).max()
        print(f"  {variant}: flux {ef:.2e} rhs {er:.2e}", flush=True)
        assert ef <= tol and er <= tol


def test_stage_timing_hook():
    """The timing hook returns positive per-kernel durations and leaves the
    state finite."""
    import torch
    from paper_1912_06221_amd import ardg
    print("stage timing", flush=True)
    mesh = W.split_square_mesh(16, 0.2, seed=3)
    ops, lm = library_mesh(mesh, 3, "const", 1.0, None, 1)
    u = to_dev(W.random_nodal((1, mesh.K, ops.Np), seed=2))
    for p in (ardg.FP64, ardg.FP32, ardg.BF16X3):
        work = ardg.alloc_workspace(lm.workspace_bytes(ardg.RK4, p, 1), u.device)
        te, tl = lm.stage_timing(u, work, 1e-6, 8, scheme=ardg.RK4, precision=p)
        assert te > 0 and tl > 0
    lm.check(u)
