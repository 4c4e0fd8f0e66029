"""Benchmark: DOF x RK-stage per second of the aRDG right-hand side on one MI355X.

Workload (default): unit square 256 x 256 x 2 = 131072 triangles, interior
vertices jittered by +-0.2 h (seeded), N = 4 (Np = 15), element-wise D with
contrast 1e4 (1e-2 outside, 1e2 inside a circle of radius 0.25; Algorithm 1
flux), initial data a seeded sum of 16 Fourier modes, classic RK4.  The FP64
path is the headline value; the mixed modes (FP32 operators and arithmetic,
and split-BF16 products on the matrix cores with FP32 accumulation, both with
the FP64 RK state) are reported beside it with their L2 difference to the
FP64 path.

One bench step = one RK4 time step = 4 passes of the whole hot path (edge
reconstruction kernel + element kernel with the fused RK update).  Inputs are
resident in HBM before timing starts; the K timed steps are one HIP graph,
captured before the timed region and launched once inside it.

`cpu_baseline` times the FP64 NumPy oracle (test infrastructure) on a bounded
sample: one RHS stage on the first S elements of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def log(msg):
    print(msg, file=sys.stderr, flush=True)


KERNEL_SOURCES = ("kernels.hip", "kernels_mfma.hip", "kernels_edge_mfma.hip", "kernel_common.hpp",
                  "edge_common.hpp", "mfma.hpp", "device.hpp")


def kernel_source_hash():
    """SHA-256 over the device-code sources, to tie stored counter data to the
    kernels it was measured on."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1912_06221_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stored_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary of
    this workload (FETCH_SIZE and WRITE_SIZE scaled by a copy-kernel
    calibration), or None when there is none or the kernels changed since."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    src, val = None, None
    with open(path) as fh:
        for line in fh:
            line = line.strip().strip("`")
            if line.startswith("kernel-source-sha256:"):
                src = line.split(":", 1)[1].strip()
            elif line.startswith(f"traffic-bytes-per-launch {kernel}:"):
                val = float(line.split(":", 1)[1])
    if src is None or val is None or src != kernel_source_hash():
        return None
    return val


def build_workload(name):
    spec = W.WORKLOADS[name]
    cfg = spec["config"]
    mesh = W.split_square_mesh(spec["m"], spec["jitter"], seed=W.seed_for(cfg, "mesh"))
    return spec, mesh


def nodal_xy(mesh, rs):
    v = mesh.vxy[mesh.etov]
    r, s = rs[:, 0], rs[:, 1]
    x = 0.5 * (-(r + s)[None] * v[:, 0:1, 0] + (r + 1)[None] * v[:, 1:2, 0] + (s + 1)[None] * v[:, 2:3, 0])
    y = 0.5 * (-(r + s)[None] * v[:, 0:1, 1] + (r + 1)[None] * v[:, 1:2, 1] + (s + 1)[None] * v[:, 2:3, 1])
    return x, y


def algorithmic_bytes(K, Np, Nfp, E_int, E_bdy, s, alg1, nfields=1):
    """Bytes each kernel must move per launch (each value counted once).

    edge kernel:    state read F*K*Np*s, edge table 56 B per interior edge
                    (int2 elements+faces, 3 x double2: apex weights of both
                    sides, gamma_R/gamma_S), 36 B per boundary face, D per
                    element (Algorithm 1) 8K, flux write F*E*Nfp*s.
    element kernel: RK4 stage averaged over the 4 stages: stage input read
                    F*K*Np*s, flux read F*E*Nfp*s, vertices 48K, face map
                    12K, D 8K, FP64 state/accumulator traffic 34 B per DOF on
                    average (stage 0: u, acc w, v w; 1-2: v, u, acc r/w, v w;
                    3: v, u r/w, acc r) with the FP64 v counted in the 34 B
                    when s = 8, and 26 + 4*... per DOF otherwise.
    """
    E = E_int + E_bdy
    dof = nfields * K * Np
    edge = dof * s + 56 * E_int + 36 * E_bdy + (8 * K if alg1 else 0) + nfields * E * Nfp * s
    if s == 8:
        state = 34.0 * dof          # includes the FP64 stage vector
        vin = 0.0
    else:
        # FP32: v read (4), u read 8 (stages 0-2) / r+w 16 (stage 3), acc as FP64,
        # v write 4 (all stages)
        state = (8 + 16 + 16 + 8) / 4.0 * dof + (8 * 3 + 16) / 4.0 * dof + 4.0 * dof
        vin = 4.0 * dof
    elem = vin + state + nfields * E * Nfp * s + 48 * K + 12 * K + (8 * K if alg1 else 0)
    return edge, elem


def edge_flops(K, Np, Nfp, N, E_int, E_bdy, alg1, nfields=1):
    """Algorithmic FLOPs of the edge kernel per launch: nodal->Bernstein and
    de Casteljau on both sides, the constant operator(s), the gamma/D combine."""
    dec = 3 * N * (N + 1) * (N + 2) // 6 * 2
    per_side = 2 * Np * Np + dec
    c = 2 if alg1 else 1
    per_edge = 2 * per_side + 2 * 2 * Nfp * 2 * Np * c + 6 * Nfp
    per_bdy = per_side + 2 * 2 * Nfp * Np + 6 * Nfp
    return nfields * (E_int * per_edge + E_bdy * per_bdy)


def bench_batch(args, dev):
    """512 independent heat problems of 200-20000 triangles, N in {2,3,4},
    constant D per problem: one graph launch per step for all of them (FP64 and
    FP32 operators with FP64 state) against the plain per-mesh path (one
    ardg_rk_step graph per mesh)."""
    import torch
    from paper_1912_06221_amd import ardg
    specs = W.batch_problems()
    meshes, states, dts, dof = [], [], [], 0
    for sp in specs:
        mesh = W.split_square_mesh(sp["m"], 0.2, seed=sp["mesh_seed"])
        ops = ardg.Ops(sp["N"])
        lm = ardg.Mesh(ops, mesh.vxy, mesh.etov, device=0)
        lm.set_diffusion_const([sp["D"]])
        rs = ops.export(ardg.OPS_NODES).reshape(-1, 2)
        x, y = nodal_xy(mesh, rs)
        states.append(W.fourier_modes(x, y, seed=sp["ic_seed"])[None])
        h = 1.0 / sp["m"]
        dts.append(0.02 * h * h / (sp["D"] * (sp["N"] + 1) ** 4))
        meshes.append(lm)
        dof += mesh.K * ops.Np
    out = {"workload": "512 heat problems, K_i 200-20000 (log-uniform), N in {2,3,4}, D per problem",
           "problems": len(specs), "DOF": dof}
    b = ardg.Batch(meshes)
    for name, prec in (("fp64", ardg.FP64), ("fp32", ardg.FP32)):
        us = [torch.from_numpy(u.copy()).to(dev) for u in states]
        work = ardg.alloc_workspace(b.workspace_bytes(ardg.RK4, prec), dev)
        for _ in range(max(1, args.warmup)):
            b.step(us, work, dts, 1, scheme=ardg.RK4, precision=prec)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        steps = max(5, args.steps // 2)
        e0.record()
        for _ in range(steps):
            b.step(us, work, dts, 1, scheme=ardg.RK4, precision=prec)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        out[f"batched_{name}"] = {"ms_per_step": ms, "value": dof * 4 / (ms * 1e-3)}
        tiles = {}
        for N in (2, 3, 4):
            et, lt, gm = b.tiles(prec, N)
            tiles[f"N{N}"] = {"edge_tile": et, "elem_tile": lt, "grid_per_cu": gm}
        out[f"batched_{name}"]["tiles"] = tiles
    # plain path: one graph launch per mesh per step, FP64
    us = [torch.from_numpy(u.copy()).to(dev) for u in states]
    works = [ardg.alloc_workspace(m.workspace_bytes(ardg.RK4, ardg.FP64, 1), dev) for m in meshes]
    for m, u, w, dt in zip(meshes, us, works, dts):
        m.rk_step(u, w, dt, 1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    steps = 3
    e0.record()
    for _ in range(steps):
        for m, u, w, dt in zip(meshes, us, works, dts):
            m.rk_step(u, w, dt, 1)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    out["per_mesh_fp64"] = {"ms_per_step": ms, "value": dof * 4 / (ms * 1e-3)}
    out["speedup_batched_fp32_vs_per_mesh_fp64"] = ms / out["batched_fp32"]["ms_per_step"]
    return out


def cpu_baseline(spec, mesh, D, u, budget_s=12.0):
    from oracle.rhs import Problem
    t0 = time.time()
    pr = Problem(mesh.vxy, mesh.etov, spec["N"], D, D_mode="element", build_edges=False)
    setup = time.time() - t0
    # calibrate on 50 elements, then run a sample sized to the budget
    t0 = time.time()
    pr.rhs_elements(u, list(range(50)))
    per = (time.time() - t0) / 50
    S = int(max(200, min(mesh.K, budget_s / max(per, 1e-6))))
    t0 = time.time()
    pr.rhs_elements(u, list(range(S)))
    dt = time.time() - t0
    Np = pr.ops.Np
    return {"value": S * Np / dt, "unit": "DOF*stage/s", "cores": 1, "kind": "oracle",
            "sample": f"one RHS stage (literal per-edge aRDG / Algorithm 1 operators) on the first "
                      f"{S} of {mesh.K} elements of the same workload; {dt:.1f} s; geometry setup "
                      f"{setup:.1f} s excluded; single-threaded NumPy"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="contrast_256x256_N4")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-fp32", action="store_true", help="time the FP64 path only")
    ap.add_argument("--power-iters", type=int, default=30)
    ap.add_argument("--no-batch", action="store_true", help="skip the 512-problem batched workload")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one device copy of 512 MiB first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported "
              f"(sharding the mesh over several GPUs is a design, not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1912_06221_amd import ardg

    dev = torch.device("cuda:0")
    spec, mesh = build_workload(args.workload)
    N = spec["N"]
    cfg = spec["config"]
    log(f"bench: workload {args.workload} K={mesh.K} N={N}")
    ops = ardg.Ops(N)
    lm = ardg.Mesh(ops, mesh.vxy, mesh.etov, device=0)
    alg1 = spec["D"] in ("circle", "loguniform")
    if spec["D"] == "circle":
        D = W.circle_contrast_D(mesh)
    elif spec["D"] == "loguniform":
        D = W.loguniform_per_element(mesh.K, spec["Dlo"], spec["Dhi"], W.seed_for(cfg, "D"))
    else:
        D = np.array(spec.get("Dfield", [spec.get("Dval", 1.0)]))
    nf = spec["fields"]
    if alg1:
        lm.set_diffusion_element(D)
    else:
        lm.set_diffusion_const(D)
    if spec.get("velocity") == "rotation":
        lm.set_velocity([0.0, 0.0, 0.0, -1.0, 1.0, 0.0])
    rs = ops.export(ardg.OPS_NODES).reshape(-1, 2)
    x, y = nodal_xy(mesh, rs)
    u0 = np.stack([W.fourier_modes(x, y, seed=W.seed_for(cfg, "IC") + 10 * f) for f in range(nf)])
    K, Np, Nfp = mesh.K, ops.Np, ops.Nfp
    dof = nf * K * Np

    if args.calib_copy:
        a = torch.empty(64 * 1024 * 1024, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"bench: calibration copy of {a.numel() * 8} bytes done")
        del a, b

    # time step from a power-iteration estimate of the spectral radius (setup)
    v = torch.from_numpy(W.random_nodal((nf, K, Np), seed=7)).to(dev)
    w = torch.empty_like(v)
    rho = 0.0
    for _ in range(args.power_iters):
        lm.rhs_eval(v, w, nfields=nf)
        nrm = float(torch.linalg.vector_norm(w))
        rho = nrm / float(torch.linalg.vector_norm(v))
        v = w / nrm
    # half the explicit limit of the estimate: power iteration approaches the
    # spectral radius from below, and the L2 differences between precisions
    # are only meaningful on a stable run
    dt = 0.5 / rho
    log(f"bench: spectral radius ~{rho:.3e}, dt={dt:.3e}")

    results = {}
    for prec_name, prec in (("fp64", ardg.FP64), ("fp32", ardg.FP32), ("bf16x3", ardg.BF16X3)):
        if prec_name != "fp64" and args.skip_fp32:
            continue
        u = torch.from_numpy(u0.copy()).to(dev)
        work = ardg.alloc_workspace(lm.workspace_bytes(ardg.RK4, prec, nf), dev)
        for _ in range(args.warmup):
            lm.rk_step(u, work, dt, 1, scheme=ardg.RK4, precision=prec, nfields=nf)
        # the K timed steps are one graph (captured here, outside the timing)
        lm.rk_prepare(u, work, dt, args.steps, scheme=ardg.RK4, precision=prec, nfields=nf)
        torch.cuda.synchronize()
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        lm.rk_step(u, work, dt, args.steps, scheme=ardg.RK4, precision=prec, nfields=nf)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        lm.check(u, nfields=nf)
        un = u.detach().cpu().numpy()
        # per-kernel durations: HIP events on the launch stream around replays
        # of a 40-stage graph and of its element kernels alone (alters u, so
        # it comes after the state is read)
        t_edge, t_elem = lm.stage_timing(u, work, dt, 40, scheme=ardg.RK4, precision=prec, nfields=nf)
        results[prec_name] = dict(ms=ms, t_edge=t_edge, t_elem=t_elem, u=un,
                                  norm_ratio=float(np.linalg.norm(un) / np.linalg.norm(u0)))
        log(f"bench: {prec_name}: {ms:.3f} ms/step, edge {t_edge*1e3:.1f} us, elem {t_elem*1e3:.1f} us")

    r64 = results["fp64"]
    value = dof * 4 / (r64["ms"] * 1e-3)
    s64 = 8
    b_edge, b_elem = algorithmic_bytes(K, Np, Nfp, lm.E_int, lm.E_bdy, s64, alg1, nf)
    bw_edge = b_edge / (r64["t_edge"] * 1e-3) / 1e9
    bw_elem = b_elem / (r64["t_elem"] * 1e-3) / 1e9
    dom = "element" if r64["t_elem"] >= r64["t_edge"] else "edge"
    bw = bw_elem if dom == "element" else bw_edge
    traffic = stored_traffic(args.workload, f"{dom}-fp64")
    fl = edge_flops(K, Np, Nfp, N, lm.E_int, lm.E_bdy, alg1, nf)
    line = {
        "metric": "DOF*RK-stage/s per MI355X (FP64 path; mixed FP32 and BF16x3 paths beside it with L2 difference)",
        "value": value,
        "unit": "DOF*stage/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms"],
        "step": "one classic RK4 time step = 4 RHS stages (edge kernel + element kernel each)",
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded jittered mesh, seeded D field and Fourier initial data)",
        "config": {"workload": args.workload, "K": K, "N": N, "Np": Np, "DOF": dof,
                   "E_int": lm.E_int, "E_bdy": lm.E_bdy, "D": spec["D"], "scheme": "RK4",
                   "dt": dt, "fields": nf},
        "state_norm_ratio": r64["norm_ratio"],
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": bw, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": bw / HBM_PEAK_GBS, "traffic": traffic,
                     "edge_kernel_us": r64["t_edge"] * 1e3, "element_kernel_us": r64["t_elem"] * 1e3,
                     "edge_GBps": bw_edge, "element_GBps": bw_elem,
                     "edge_algorithmic_bytes": b_edge, "element_algorithmic_bytes": b_elem,
                     "edge_TFLOPs": fl / (r64["t_edge"] * 1e-3) / 1e12,
                     "edge_fp64_frac": fl / (r64["t_edge"] * 1e-3) / 1e12 / FP64_PEAK_TFLOPS},
    }
    for mode in ("fp32", "bf16x3"):
        if mode not in results:
            continue
        r32 = results[mode]
        d = r32["u"] - r64["u"]
        l2 = float(np.sqrt(np.sum(d * d) / np.sum(r64["u"] ** 2)))
        b_edge32, b_elem32 = algorithmic_bytes(K, Np, Nfp, lm.E_int, lm.E_bdy, 4, alg1, nf)
        line["mixed_" + mode] = {
            "value": dof * 4 / (r32["ms"] * 1e-3), "ms_per_step": r32["ms"],
            "speedup_vs_fp64": r64["ms"] / r32["ms"],
            "rel_l2_diff_vs_fp64_after_steps": l2,
            "edge_kernel_us": r32["t_edge"] * 1e3, "element_kernel_us": r32["t_elem"] * 1e3,
            "edge_GBps": b_edge32 / (r32["t_edge"] * 1e-3) / 1e9,
            "element_GBps": b_elem32 / (r32["t_elem"] * 1e-3) / 1e9,
        }
    if not args.no_batch:
        log("bench: batched workload (512 problems)")
        line["batch"] = bench_batch(args, dev)
        bb = line["batch"]
        log(f"bench: batch fp64 {bb['batched_fp64']['ms_per_step']:.3f} ms, fp32 "
            f"{bb['batched_fp32']['ms_per_step']:.3f} ms, per-mesh fp64 {bb['per_mesh_fp64']['ms_per_step']:.3f} ms")
    if not args.no_cpu_baseline:
        log("bench: timing the oracle on a bounded sample (cpu_baseline)")
        line["cpu_baseline"] = cpu_baseline(spec, mesh, D, u0[0])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
