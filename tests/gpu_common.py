"""Shared helpers of the GPU tests: build the same problem for the library and
the oracle from the seeded generators, and move data between NumPy and torch."""
from __future__ import annotations

import numpy as np

import workloads as W


def torch_dev():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU test collected without a GPU")
    return torch, torch.device("cuda:0")


def make_case(m, jitter, N, D_mode="const", D=1.0, velocity=None, nfields=1, seed=0):
    """Returns (mesh, D array/values) for both sides.  D_mode: "const",
    "element" (Algorithm 1) or "element2" (Algorithm 2)."""
    mesh = W.split_square_mesh(m, jitter, seed=seed)
    if D_mode.startswith("element") and np.isscalar(D):
        D = W.loguniform_per_element(mesh.K, 1e-3, 1e1, seed=seed + 1)
    return mesh, D


def library_mesh(mesh, N, D_mode, D, velocity, nfields):
    from paper_1912_06221_amd import ardg
    ops = ardg.Ops(N)
    lm = ardg.Mesh(ops, mesh.vxy, mesh.etov, device=0)
    if D_mode.startswith("element"):
        lm.set_diffusion_element(D, alg=2 if D_mode == "element2" else 1)
    else:
        lm.set_diffusion_const(np.broadcast_to(np.asarray(D, dtype=float), (nfields,)).copy())
    if velocity is not None:
        lm.set_velocity(velocity)
    return ops, lm


def oracle_problem(mesh, N, D_mode, D, velocity, nfields, build_edges=True):
    from oracle.rhs import Problem
    alg = 2 if D_mode == "element2" else 1
    mode = "element" if D_mode.startswith("element") else D_mode
    return Problem(mesh.vxy, mesh.etov, N, D, D_mode=mode, velocity=velocity,
                   nfields=nfields, build_edges=build_edges, alg=alg)


def to_dev(a, dtype=None):
    torch, dev = torch_dev()
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev)


def to_np(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().to("cpu").double().numpy()
