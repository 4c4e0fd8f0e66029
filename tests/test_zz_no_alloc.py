"""The right-hand side entry point that allocates nothing
(ardg_rhs_eval_noalloc) against ardg_rhs_eval, through the C ABI.

Two calls in a row, the second on a smaller mesh, each compared with the
allocating entry point on the same input (the same kernels run, so the results
agree to the FP64 parity bar, 1e-12 relative, and in fact bit for bit), and
the size check that refuses fluxes larger than the scratch array.
"""
import numpy as np
import pytest

import workloads as W
from gpu_common import library_mesh, to_dev, to_np

pytestmark = pytest.mark.gpu


def _compare(m, N, D_mode, nf, vel, prec, seed):
    import torch
    from paper_1912_06221_amd import ardg
    mesh = W.split_square_mesh(m, 0.2, seed=seed)
    D = W.loguniform_per_element(mesh.K, 1e-3, 1e1, seed=seed + 1) if D_mode == "element" else \
        [0.5 + f for f in range(nf)]
    ops, lm = library_mesh(mesh, N, D_mode, D, vel, nf)
    u = W.random_nodal((nf, mesh.K, ops.Np), seed=seed + 2)
    dt = torch.float64 if prec == ardg.FP64 else torch.float32
    ud = to_dev(u, dt)
    ref = torch.empty_like(ud)
    got = torch.full_like(ud, float("nan"))
    lm.rhs_eval(ud, ref, precision=prec, nfields=nf)
    lm.rhs_eval_noalloc(ud, got, precision=prec, nfields=nf)
    a, b = to_np(ref), to_np(got)
    err = np.abs(a - b).max() / np.abs(a).max()
    print(f"  m={m} N={N} {D_mode} F={nf} prec={prec}: rel diff {err:.1e}, "
          f"bitwise equal {np.array_equal(a, b)}", flush=True)
    return err


def test_noalloc_matches_rhs_eval_two_calls():
    from paper_1912_06221_amd import ardg
    print("no-alloc rhs: larger mesh, then a smaller one", flush=True)
    # first call: 96 x 96 x 2 elements, N = 4, Algorithm 1, FP64
    assert _compare(96, 4, "element", 1, None, ardg.FP64, seed=61) <= 1e-12
    # second call: 20 x 20 x 2 elements, N = 2, two fields with convection, FP64
    assert _compare(20, 2, "const", 2, (0.0, 0.0, 0.0, -1.0, 1.0, 0.0), ardg.FP64, seed=62) <= 1e-12
    # and the FP32 path on a third, smaller mesh
    assert _compare(12, 3, "const", 1, None, ardg.FP32, seed=63) <= 2e-4


def test_noalloc_refuses_fluxes_beyond_scratch():
    import torch
    from paper_1912_06221_amd import ardg
    print("no-alloc rhs: size check", flush=True)
    # 256 x 256 x 2 elements, N = 6, 16 fields: 16 * 197120 * 7 * 8 bytes of
    # fluxes = 176.6 MB, beyond the 64 MiB array
    mesh = W.split_square_mesh(256, 0.0)
    ops, lm = library_mesh(mesh, 6, "const", [1.0] * 16, None, 16)
    u = torch.zeros((16, mesh.K, ops.Np), dtype=torch.float64, device="cuda:0")
    out = torch.empty_like(u)
    with pytest.raises(ardg.ArdgError) as ei:
        lm.rhs_eval_noalloc(u, out, precision=ardg.FP64, nfields=16)
    assert ei.value.status == -1
    assert "scratch" in str(ei.value)
    # the same mesh in one field fits (11 MB) and works
    u1 = to_dev(W.random_nodal((1, mesh.K, ops.Np), seed=5))
    ref, got = torch.empty_like(u1), torch.empty_like(u1)
    lm.rhs_eval(u1, ref, precision=ardg.FP64, nfields=1)
    lm.rhs_eval_noalloc(u1, got, precision=ardg.FP64, nfields=1)
    a, b = to_np(ref), to_np(got)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()
