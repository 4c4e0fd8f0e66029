"""Parity at the full workload sizes, in the benchmark's launch configuration,
on sampled outputs that the oracle computes one by one.

The oracle evaluates the RHS of sampled elements (each with its three
literal per-edge reconstructions) and one classic RK4 step on sampled
elements through the four neighbour layers each stage needs.
"""
import numpy as np
import pytest

import workloads as W
from gpu_common import to_dev, to_np

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
# about ten times the largest error measured on these inputs: FP32 rhs
# 4.9e-7, FP32 RK4 increment 1.3e-7, BF16X3 rhs 1.4e-5
TOL32 = 5e-6
TOL32_STATE = 2e-6
TOLBF = 2.5e-4


def _setup(name, alg=1):
    from oracle.rhs import Problem
    from paper_1912_06221_amd import ardg
    spec = W.WORKLOADS[name]
    cfg = spec["config"]
    mesh = W.split_square_mesh(spec["m"], spec["jitter"], seed=W.seed_for(cfg, "mesh"))
    N, nf = spec["N"], spec["fields"]
    vel = (0.0, 0.0, 0.0, -1.0, 1.0, 0.0) if spec.get("velocity") == "rotation" else None
    if spec["D"] == "circle":
        D, mode = W.circle_contrast_D(mesh), "element"
    elif spec["D"] == "loguniform":
        D, mode = W.loguniform_per_element(mesh.K, spec["Dlo"], spec["Dhi"], W.seed_for(cfg, "D")), "element"
    else:
        D, mode = np.array(spec["Dfield"], dtype=float), "const"
    ops = ardg.Ops(N)
    lm = ardg.Mesh(ops, mesh.vxy, mesh.etov, device=0)
    if mode == "element":
        lm.set_diffusion_element(D, alg=alg)
    else:
        lm.set_diffusion_const(D)
    if vel is not None:
        lm.set_velocity(vel)
    pr = Problem(mesh.vxy, mesh.etov, N, D, D_mode=mode, velocity=vel, nfields=nf,
                 build_edges=False, alg=alg)
    xy = pr.nodal_xy()
    u0 = np.stack([W.fourier_modes(xy[..., 0], xy[..., 1], seed=W.seed_for(cfg, "IC") + 10 * f)
                   for f in range(nf)])
    return spec, mesh, ops, lm, pr, u0


def _sample(K, n, seed):
    rng = np.random.default_rng(seed)
    s = set(rng.choice(K, size=n, replace=False).tolist())
    s.update([0, K - 1])          # first and last element (boundary, ragged tail)
    return sorted(s)


@pytest.mark.parametrize("name", ["contrast_256x256_N4", "convdiff_708x708_N3_4f",
                                  "loguniformD_512x512_N6"])
def test_fullsize_rhs_sampled(name):
    import torch
    from paper_1912_06221_amd import ardg
    print(f"full-size rhs {name}", flush=True)
    spec, mesh, ops, lm, pr, u0 = _setup(name)
    nf = spec["fields"]
    els = _sample(mesh.K, 24, seed=1)
    ur = W.random_nodal(u0.shape, seed=9)
    for data, label in ((u0, "smooth"), (ur, "random")):
        ud = to_dev(data)
        for prec, dt, tol in ((ardg.FP64, torch.float64, TOL64), (ardg.FP32, torch.float32, TOL32),
                              (ardg.BF16X3, torch.float32, TOLBF)):
            x = ud.to(dt)
            out = torch.empty_like(x)
            lm.rhs_eval(x, out, precision=prec, nfields=nf)
            got = to_np(out)
            for f in range(nf):
                ref = pr.rhs_elements(data[f], els, field=f)
                scale = np.abs(pr.rhs_elements(ur[f] * np.abs(data[f]).max(), els, field=f)).max()
                err = np.abs(got[f, els] - ref).max() / scale
                print(f"  {label} prec={prec} field={f} err/scale={err:.2e}", flush=True)
                assert err <= tol


@pytest.mark.parametrize("name,dt", [("contrast_256x256_N4", 2e-11), ("convdiff_708x708_N3_4f", 5e-10)])
def test_fullsize_rk4_step_sampled(name, dt):
    """One RK4 step of a benchmark workload through ardg_rk_step (the
    graph-captured path the benchmark times), FP64 and mixed FP32, every
    field."""
    import torch
    from paper_1912_06221_amd import ardg
    print(f"full-size rk4 step {name}", flush=True)
    spec, mesh, ops, lm, pr, u0 = _setup(name)
    nf = spec["fields"]
    els = _sample(mesh.K, 6, seed=2)
    # random data and a step of the order of the inverse spectral radius, so
    # that the increment is of the size of the state (no cancellation)
    u0 = W.random_nodal(u0.shape, seed=11)
    refs = [pr.rk4_step_elements(u0[f], dt, els, field=f) for f in range(nf)]
    for prec, tol in ((ardg.FP64, TOL64), (ardg.FP32, TOL32_STATE)):
        ud = to_dev(u0)
        work = ardg.alloc_workspace(lm.workspace_bytes(ardg.RK4, prec, nf), ud.device)
        lm.rk_step(ud, work, dt, 1, scheme=ardg.RK4, precision=prec, nfields=nf)
        got = to_np(ud)
        for f in range(nf):
            # compare the increment u1 - u0 (the state itself is O(1)).  The
            # new state is stored in FP64, so an increment far below the state
            # (the four-field workload's D = 1e-4 field moves by 3e-5 of it)
            # is known only to a few units in the last place of the state:
            # the bound adds 4 eps max|u0| / max|inc| to the tolerance.
            inc_ref = refs[f] - u0[f, els]
            inc_got = got[f, els] - u0[f, els]
            scale = np.abs(inc_ref).max()
            err = np.abs(inc_got - inc_ref).max() / scale
            bound = tol + 4 * np.finfo(np.float64).eps * np.abs(u0[f, els]).max() / scale
            print(f"  prec={prec} field {f} increment rel err {err:.2e} (bound {bound:.2e})", flush=True)
            assert err <= bound
        del ud, work


@pytest.mark.parametrize("name", ["contrast_256x256_N4", "loguniformD_512x512_N6"])
def test_fullsize_alg2_rhs_sampled(name):
    """Algorithm 2 (reconstructed coefficient times the reconstructed
    gradient) at the full sizes of the two element-wise-D workloads, FP64 and
    FP32, on sampled elements."""
    import torch
    from paper_1912_06221_amd import ardg
    print(f"full-size rhs, Algorithm 2, {name}", flush=True)
    spec, mesh, ops, lm, pr, u0 = _setup(name, alg=2)
    els = _sample(mesh.K, 16, seed=3)
    ur = W.random_nodal(u0.shape, seed=9)
    for data, label in ((u0, "smooth"), (ur, "random")):
        ud = to_dev(data)
        for prec, dt, tol in ((ardg.FP64, torch.float64, TOL64), (ardg.FP32, torch.float32, TOL32)):
            x = ud.to(dt)
            out = torch.empty_like(x)
            lm.rhs_eval(x, out, precision=prec)
            got = to_np(out)
            ref = pr.rhs_elements(data[0], els)
            scale = np.abs(pr.rhs_elements(ur[0] * np.abs(data[0]).max(), els)).max()
            err = np.abs(got[0, els] - ref).max() / scale
            print(f"  {label} prec={prec} err/scale={err:.2e}", flush=True)
            assert err <= tol


@pytest.mark.parametrize("name", ["convdiff_708x708_N3_4f", "contrast_256x256_N4"])
def test_fullsize_edge_kernels_agree(name):
    """The vector-unit edge kernels at the full sizes: the side-split tiles'
    (and, with per-field constant D, the multi-field lanes') whole flux
    array agrees with the one-lane-per-edge kernel's (every edge, including
    the last, ragged tile and the boundary faces), and the RHS through the
    last of them matches the oracle on sampled elements."""
    import torch
    from paper_1912_06221_amd import ardg
    print(f"full-size edge kernels {name}", flush=True)
    spec, mesh, ops, lm, pr, u0 = _setup(name)
    nf = spec["fields"]
    els = _sample(mesh.K, 12, seed=4)
    ur = W.random_nodal(u0.shape, seed=12)
    ud = to_dev(ur)
    for prec, dt, tol in ((ardg.FP64, torch.float64, TOL64), (ardg.FP32, torch.float32, TOL32)):
        x = ud.to(dt)
        fl = {}
        kerns = (ardg.EDGE_LANE, ardg.EDGE_SPLIT) + ((ardg.EDGE_FIELDS,) if spec["D"] == "perfield" else ())
        for kern in kerns:
            lm.set_kernels(kern)
            f = torch.empty((nf, lm.E, ops.Nfp), dtype=dt, device=ud.device)
            lm.edge_flux_eval(x, f, precision=prec, nfields=nf)
            fl[kern] = to_np(f)
        for kern in kerns[1:]:
            d = np.abs(fl[kern] - fl[ardg.EDGE_LANE]).max() / np.abs(fl[ardg.EDGE_LANE]).max()
            print(f"  prec={prec} kernel {kern} vs lane flux {d:.2e}", flush=True)
            assert d <= tol
        out = torch.empty_like(x)
        lm.rhs_eval(x, out, precision=prec, nfields=nf)
        got = to_np(out)
        for f in range(nf):
            ref = pr.rhs_elements(ur[f], els, field=f)
            err = np.abs(got[f, els] - ref).max() / np.abs(ref).max()
            print(f"  prec={prec} field={f} rhs rel err {err:.2e}", flush=True)
            assert err <= tol
    lm.set_kernels(ardg.EDGE_AUTO)
