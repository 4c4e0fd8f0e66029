"""Benchmark: DOF x RK-stage per second of the aRDG right-hand side on one MI355X.

Headline workload: 4 independent scalar fields on the unit square cut into
708 x 708 cells of two triangles (1,002,528 elements, interior vertices
jittered by +-0.2 h, seeded), N = 3 (Np = 10), rotating velocity v = (-y, x)
with upwind convective flux, per-field constant D in {1e-4, 1e-3, 1e-2, 1},
initial data a seeded sum of 16 Fourier modes per field, classic RK4.  The
FP64 path is `value`; the reduced-precision modes (FP32 operators and
arithmetic, and split-BF16 products on the matrix cores with FP32
accumulation, both with the FP64 RK state) are reported beside it with their
L2 error after the workload's 200 steps.

One bench step = one RK4 time step = 4 passes of the whole hot path (edge
reconstruction kernel + element kernel with the fused RK update).  Inputs are
resident in HBM before timing starts; the K timed steps are HIP graphs
captured before the timed region and launched inside it.

Extra keys: the 256 x 256 x 2, N = 4 workload with element-wise D (contrast
1e4, Algorithm 1 flux), the 512 x 512 x 2, N = 6 workload with log-uniform D
(the precision workload: every mode's L2 error after 50 steps), the 512
independent problems advanced as one batch, and the compressible
Navier-Stokes workload (708 x 708 x 2, N = 3, four conserved fields, the
isentropic vortex, low-storage RK) with its kernels' HBM fractions.

`cpu_baseline` times the FP64 NumPy oracle (test infrastructure): its
assembled right-hand side with the per-edge operators prebuilt, on strips of
the headline mesh, one strip per worker process on the host's cores, before
the GPU is used.
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
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0}
HEADLINE = "convdiff_708x708_N3_4f"
ROTATION = (0.0, 0.0, 0.0, -1.0, 1.0, 0.0)
# edge kernel implementations (ardg_mesh_set_kernels)
EDGE_KERNELS = {"auto": 0, "split": 1, "lane": 2, "mfma": 3, "split_mfma": 4, "fields": 5}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# device sources each workload's kernels are compiled from (a stored counter
# summary is used only while these hash to the value it records)
KERNEL_SOURCES = ("kernels.hip", "kernels_mfma.hip", "kernels_edge_mfma.hip",
                  "kernel_common.hpp", "edge_common.hpp", "mfma.hpp", "device.hpp")
NS_KERNEL_SOURCES = ("kernels_ns.hip", "kernel_common.hpp", "edge_common.hpp", "device.hpp")


def sources_of(workload):
    return NS_KERNEL_SOURCES if workload.startswith("ns_") else KERNEL_SOURCES


def kernel_source_hash(workload=None):
    """SHA-256 over the device-code sources of a workload's kernels, to tie
    stored counter data to the kernels it was measured on."""
    import hashlib
    h = hashlib.sha256()
    for f in (sources_of(workload) if workload else KERNEL_SOURCES):
        with open(os.path.join(ROOT, "paper_1912_06221_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stored_counters(workload):
    """Per-launch counter values of the committed profile summary of this
    workload (`profiles/counters_<workload>.md`: lines `name: value`), or {}
    when there is none or the kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"counters_{workload}.md")
    if not os.path.exists(path):
        return {}
    src, vals = None, {}
    with open(path) as fh:
        for line in fh:
            line = line.strip().strip("`")
            if line.startswith("kernel-source-sha256:"):
                src = line.split(":", 1)[1].strip()
            elif line.startswith("per-launch "):
                k, v = line[len("per-launch "):].split(":", 1)
                vals[k.strip()] = float(v)
    if src != kernel_source_hash(workload):
        return {}
    return vals


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

def nodal_xy(mesh, rs):
    v = mesh.vxy[mesh.etov]
    r, s = rs[:, 0], rs[:, 1]
    x = 0.5 * (-(r + s)[None] * v[:, 0:1, 0] + (r + 1)[None] * v[:, 1:2, 0] + (s + 1)[None] * v[:, 2:3, 0])
    y = 0.5 * (-(r + s)[None] * v[:, 0:1, 1] + (r + 1)[None] * v[:, 1:2, 1] + (s + 1)[None] * v[:, 2:3, 1])
    return x, y


def workload_D(spec, mesh):
    """(D values, "element" | "const") of a named workload."""
    cfg = spec["config"]
    if spec["D"] == "circle":
        return W.circle_contrast_D(mesh), "element"
    if spec["D"] == "loguniform":
        return W.loguniform_per_element(mesh.K, spec["Dlo"], spec["Dhi"], W.seed_for(cfg, "D")), "element"
    return np.array(spec.get("Dfield", [spec.get("Dval", 1.0)]), dtype=float), "const"


def algorithmic_bytes(K, Np, Nfp, E_int, s, alg1, nfields):
    """Bytes each kernel must move per launch by the survey's model (each
    value counted once, neighbour reuse in L2 assumed):
    edge    F K Np s (state) + 60 E_int (edge table, FP64 parameters) + 8 K
            (element D, Algorithm 1) + F E_int Nfp s (flux write);
    element F K Np s (stage input) + F E_int Nfp s (flux) + 48 K (affine map)
            + F K Np (8 + 16) (u^n read, accumulator read and write, FP64)
            + F K Np s (next stage input)."""
    dof = nfields * K * Np
    edge = dof * s + 60 * E_int + (8 * K if alg1 else 0) + nfields * E_int * Nfp * s
    elem = dof * s + nfields * E_int * Nfp * s + 48 * K + dof * 24 + dof * s
    return edge, elem


def rk4_dof_bytes(s, f64):
    """Bytes per degree of freedom of one classic RK4 stage's element kernel
    outside the operator data, averaged over the four stages: stage input,
    state and accumulator reads, accumulator or state write, next stage
    input (s bytes per value of the stage vectors; FP64 reads the state
    itself at stage 0 and writes no stage vector at stage 3; the accumulator
    carries the new state as it forms, so stage 3 reads no state):
      stage 0: [s] + 8 (u) + 8 (A write) + s
      stage 1, 2: s + 8 (u) + 8 (A) + 8 (A write) + s
      stage 3: s + 8 (A) + 8 (u write) + [s]."""
    st0 = (0 if f64 else s) + 16 + s
    st12 = s + 24 + s
    st3 = s + 16 + (0 if f64 else s)
    return (st0 + 2 * st12 + st3) / 4.0


def stored_bytes(K, Np, Nfp, E_int, E_bdy, s, alg1, nfields, conv):
    """The same per launch for the data as this library stores and moves it:
    edge    F K Np s + 56 E_int + 36 E_bdy (edge and boundary-face tables) +
            16 E (n.v at the edge's ends, with convection) + 8 K (element D)
            + F E Nfp s (flux write, boundary faces included);
    element F E Nfp s (fluxes) + 60 K (vertices, face map) + 8 K (element D)
            + F K Np rk4_dof_bytes (stage vectors, state and accumulator,
            averaged over the stages as the timing is; the survey's model
            charges every launch the heaviest stage)."""
    E = E_int + E_bdy
    dof = nfields * K * Np
    f64 = s == 8
    edge = dof * s + 56 * E_int + 36 * E_bdy + (16 * E if conv else 0) + (8 * K if alg1 else 0) \
        + nfields * E * Nfp * s
    elem = nfields * E * Nfp * s + 60 * K + (8 * K if alg1 else 0) + dof * rk4_dof_bytes(s, f64)
    return edge, elem


def algorithmic_flops(K, Np, Nfp, N, E_int, alg1, nfields):
    """FLOPs per launch: edge, per field and interior edge, 2*2*(Np^2 +
    N(N+1)(N+2)/2) (nodal -> Bernstein and de Casteljau, both sides) +
    2*(2 Nfp)(2 Np)*c (c = 2 with Algorithm 1); element, per field and
    element, 2*(4 Np^2 + 3 Np Nfp)."""
    c = 2 if alg1 else 1
    edge = nfields * E_int * (4 * (Np * Np + N * (N + 1) * (N + 2) // 2) + 2 * (2 * Nfp) * (2 * Np) * c)
    elem = nfields * K * 2 * (4 * Np * Np + 3 * Np * Nfp)
    return edge, elem


class Case:
    """One workload on the device: library mesh, initial data, time step."""

    def __init__(self, name, dev, power_iters, edge_kernel="auto"):
        import torch
        from paper_1912_06221_amd import ardg
        self.name = name
        self.edge_kernel = edge_kernel
        spec = W.WORKLOADS[name]
        self.spec = spec
        cfg = spec["config"]
        t0 = time.time()
        self.mesh = W.split_square_mesh(spec["m"], spec["jitter"], seed=W.seed_for(cfg, "mesh"))
        self.N = spec["N"]
        self.nf = spec["fields"]
        self.ops = ardg.Ops(self.N)
        self.lm = ardg.Mesh(self.ops, self.mesh.vxy, self.mesh.etov, device=0)
        self.lm.set_kernels(EDGE_KERNELS[edge_kernel])
        self.D, self.D_mode = workload_D(spec, self.mesh)
        self.alg1 = self.D_mode == "element"
        if self.alg1:
            self.lm.set_diffusion_element(self.D)
        else:
            self.lm.set_diffusion_const(self.D)
        self.vel = ROTATION if spec.get("velocity") == "rotation" else None
        if self.vel is not None:
            self.lm.set_velocity(self.vel)
        rs = self.ops.export(ardg.OPS_NODES).reshape(-1, 2)
        x, y = nodal_xy(self.mesh, rs)
        self.u0 = np.stack([W.fourier_modes(x, y, seed=W.seed_for(cfg, "IC") + 10 * f)
                            for f in range(self.nf)])
        self.K, self.Np, self.Nfp = self.mesh.K, self.ops.Np, self.ops.Nfp
        self.dof = self.nf * self.K * self.Np
        self.setup_s = time.time() - t0
        # time step: the explicit limit from a power-iteration estimate of the
        # spectral radius (setup, outside any timing)
        v = torch.from_numpy(W.random_nodal((self.nf, self.K, self.Np), seed=7)).to(dev)
        w = torch.empty_like(v)
        rho = 0.0
        for _ in range(power_iters):
            self.lm.rhs_eval(v, w, nfields=self.nf)
            nrm = float(torch.linalg.vector_norm(w))
            rho = nrm / float(torch.linalg.vector_norm(v))
            v = w / nrm
        self.rho = rho
        # RK4's stability region reaches 2.78/|lambda| on the negative real
        # axis and less off it, and the power iteration approaches rho from
        # below: take 1/rho (halved by run_steps if a run still blows up)
        self.dt = 1.0 / rho
        log(f"bench: {name}: K={self.K} N={self.N} fields={self.nf} setup {self.setup_s:.1f} s, "
            f"rho~{rho:.3e}, dt={self.dt:.3e}")

    def config(self):
        return {"workload": self.name, "K": self.K, "N": self.N, "Np": self.Np, "DOF": self.dof,
                "E_int": self.lm.E_int, "E_bdy": self.lm.E_bdy, "fields": self.nf,
                "D": self.spec["D"], "velocity": self.spec.get("velocity"), "scheme": "RK4",
                "dt": self.dt, "config_steps": self.spec["steps"], "edge_kernel": self.edge_kernel}

    def time_mode(self, prec, steps, warmup, dev):
        """ms per RK4 step over `steps` graph-replayed steps, and the per-kernel
        average durations (HIP events on the launch stream, from replays of a
        40-stage graph and of its element kernels alone; median of three)."""
        import torch
        from paper_1912_06221_amd import ardg
        u = torch.from_numpy(self.u0.copy()).to(dev)
        work = ardg.alloc_workspace(self.lm.workspace_bytes(ardg.RK4, prec, self.nf), dev)
        for _ in range(warmup):
            self.lm.rk_step(u, work, self.dt, 1, scheme=ardg.RK4, precision=prec, nfields=self.nf)
        self.lm.rk_prepare(u, work, self.dt, steps, scheme=ardg.RK4, precision=prec, nfields=self.nf)
        torch.cuda.synchronize()
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        self.lm.rk_step(u, work, self.dt, steps, scheme=ardg.RK4, precision=prec, nfields=self.nf)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        self.lm.check(u, nfields=self.nf)
        # the median of three timing-hook runs (single runs of the same
        # kernels scatter by several per cent)
        runs = [self.lm.stage_timing(u, work, self.dt, 40, scheme=ardg.RK4, precision=prec, nfields=self.nf)
                for _ in range(3)]
        t_edge = float(np.median([r[0] for r in runs]))
        t_elem = float(np.median([r[1] for r in runs]))
        return ms, t_edge, t_elem

    def run_steps(self, prec, nsteps, dev, dt):
        """The state after nsteps RK4 steps of size dt from u0 (host array), or
        None if it is not finite (dt beyond the stability limit)."""
        import torch
        from paper_1912_06221_amd import ardg
        u = torch.from_numpy(self.u0.copy()).to(dev)
        work = ardg.alloc_workspace(self.lm.workspace_bytes(ardg.RK4, prec, self.nf), dev)
        self.lm.rk_step(u, work, dt, nsteps, scheme=ardg.RK4, precision=prec, nfields=self.nf)
        try:
            self.lm.check(u, nfields=self.nf)
        except ardg.ArdgError as e:
            if e.status != -9:
                raise
            return None
        return u.cpu().numpy()

    def rhs_vs_oracle(self, prec, dev, nsample=12):
        """max |rhs_mode - rhs_oracle| / scale on sampled elements per field
        (scale: max |L u_r| for random data of the same amplitude, the size of
        the operator's terms), one RHS of the initial data."""
        import torch
        from oracle.rhs import Problem
        from paper_1912_06221_amd import ardg
        if getattr(self, "_pr", None) is None:
            self._pr = Problem(self.mesh.vxy, self.mesh.etov, self.N, self.D, D_mode=self.D_mode,
                               velocity=self.vel, nfields=self.nf, build_edges=False)
        pr = self._pr
        rng = np.random.default_rng(3)
        els = sorted(set(rng.choice(self.K, size=nsample, replace=False).tolist()) | {0, self.K - 1})
        dt = torch.float64 if prec == ardg.FP64 else torch.float32
        x = torch.from_numpy(self.u0).to(dev).to(dt)
        out = torch.empty_like(x)
        self.lm.rhs_eval(x, out, precision=prec, nfields=self.nf)
        got = out.double().cpu().numpy()
        ur = W.random_nodal(self.u0.shape, seed=9)
        worst = 0.0
        for f in range(self.nf):
            ref = pr.rhs_elements(self.u0[f], els, field=f)
            scale = np.abs(pr.rhs_elements(ur[f] * np.abs(self.u0[f]).max(), els, field=f)).max()
            worst = max(worst, float(np.abs(got[f, els] - ref).max() / scale))
        return worst


def kernel_rates(case, t_edge_ms, t_elem_ms, s, prec_name):
    b_edge, b_elem = algorithmic_bytes(case.K, case.Np, case.Nfp, case.lm.E_int, s, case.alg1, case.nf)
    s_edge, s_elem = stored_bytes(case.K, case.Np, case.Nfp, case.lm.E_int, case.lm.E_bdy, s, case.alg1,
                                  case.nf, case.vel is not None)
    f_edge, f_elem = algorithmic_flops(case.K, case.Np, case.Nfp, case.N, case.lm.E_int, case.alg1, case.nf)
    te, tl = t_edge_ms * 1e-3, t_elem_ms * 1e-3
    peak = PEAK_TFLOPS[prec_name]
    return {
        "edge_us": t_edge_ms * 1e3, "element_us": t_elem_ms * 1e3,
        "edge_bytes": b_edge, "element_bytes": b_elem,
        "edge_GBps": b_edge / te / 1e9, "element_GBps": b_elem / tl / 1e9,
        "edge_frac": b_edge / te / 1e9 / HBM_PEAK_GBS, "element_frac": b_elem / tl / 1e9 / HBM_PEAK_GBS,
        "edge_TFLOPs": f_edge / te / 1e12, "element_TFLOPs": f_elem / tl / 1e12,
        "edge_flop_frac": f_edge / te / 1e12 / peak, "element_flop_frac": f_elem / tl / 1e12 / peak,
        "edge_stored_bytes": s_edge, "element_stored_bytes": s_elem,
        "edge_stored_frac": s_edge / te / 1e9 / HBM_PEAK_GBS, "element_stored_frac": s_elem / tl / 1e9 / HBM_PEAK_GBS,
    }


def mode_errors(case, states, u0):
    """L2 differences of each mode's state to the FP64 state after the
    workload's steps, relative to the state and to how far the FP64 state
    moved from the initial data."""
    u64 = states["fp64"]
    inc = float(np.linalg.norm(u64 - u0))
    out = {"fp64_evolution_rel_l2": inc / float(np.linalg.norm(u0)),
           "fp64_norm_growth": float(np.linalg.norm(u64) / np.linalg.norm(u0))}
    for mode, u in states.items():
        if mode == "fp64":
            continue
        d = float(np.linalg.norm(u - u64))
        out[mode] = {"rel_l2_vs_fp64_state": d / float(np.linalg.norm(u64)),
                     "rel_l2_vs_fp64_increment": d / inc if inc > 0 else None}
    return out


def measure_case(case, args, dev, modes, error_steps):
    from paper_1912_06221_amd import ardg
    prec_of = {"fp64": ardg.FP64, "fp32": ardg.FP32, "bf16x3": ardg.BF16X3}
    res = {}
    for mode in modes:
        ms, te, tl = case.time_mode(prec_of[mode], args.steps, args.warmup, dev)
        s = 8 if mode == "fp64" else 4
        r = {"ms_per_step": ms, "value": case.dof * 4 / (ms * 1e-3)}
        r.update(kernel_rates(case, te, tl, s, mode))
        res[mode] = r
        log(f"bench: {case.name} {mode}: {ms:.3f} ms/step, edge {te*1e3:.1f} us "
            f"({r['edge_frac']*100:.1f}% HBM), element {tl*1e3:.1f} us ({r['element_frac']*100:.1f}% HBM)")
    if error_steps:
        dt = case.dt
        while True:
            states = {m: case.run_steps(prec_of[m], error_steps, dev, dt) for m in modes}
            if all(s is not None for s in states.values()) or dt < case.dt / 64:
                break
            log(f"bench: {case.name}: dt={dt:.3e} is beyond the stability limit; halving it")
            dt *= 0.5
        if any(s is None for s in states.values()):
            raise RuntimeError(f"{case.name}: no stable time step found")
        err = mode_errors(case, states, case.u0)
        err["steps"] = error_steps
        err["dt"] = dt
        case.dt_stable = dt
        for m in modes:
            err.setdefault(m, {})
            err[m]["rhs_err_vs_oracle_sampled"] = case.rhs_vs_oracle(prec_of[m], dev)
        res["errors"] = err
        log(f"bench: {case.name} errors after {error_steps} steps: "
            + ", ".join(f"{m} {err[m].get('rel_l2_vs_fp64_increment', 0.0) or 0.0:.2e}" for m in modes))
    return res


def ns_algorithmic_bytes(K, Np, Nfp, E_int, E_bdy, s):
    """Bytes each Navier-Stokes kernel must move per launch (four fields,
    each value counted once, low-storage RK averaged over its five stages):
    edge    4 K Np s (state) + 88 E_int + 68 E_bdy (edge tables: element and
            face codes, apex weights, parallelogram metric, sJ n) + 4 E_bdy Np 8
            (exterior state) + 4 E Nfp s (flux write);
    element 4 K Np s (stage input) + 4 E Nfp s (flux) + 60 K (affine map and
            face map) + 4 K Np (8 + 8 + 8 + 6.4) (u^n write, u^n read beside
            the stage input in FP32 only, residual write, residual read in four
            of five stages) + 4 K Np s (next stage input, FP32 only)."""
    E = E_int + E_bdy
    dof = 4 * K * Np
    edge = dof * s + 88 * E_int + 68 * E_bdy + 4 * E_bdy * Np * 8 + 4 * E * Nfp * s
    if s == 8:      # the FP64 stage input is the state itself
        elem = dof * 8 + 4 * E * Nfp * 8 + 60 * K + dof * (8 + 8 + 6.4)
    else:
        elem = dof * s + 4 * E * Nfp * s + 60 * K + dof * (8 + 8 + 8 + 6.4) + dof * s
    return edge, elem


class NSCase:
    """The Navier-Stokes workload on the device (low-storage RK, the paper's
    integrator)."""

    def __init__(self, name, dev):
        import torch
        from paper_1912_06221_amd import ardg
        self.name = name
        spec = W.WORKLOADS[name]
        self.spec = spec
        cfg = spec["config"]
        t0 = time.time()
        self.mesh = W.split_square_mesh(spec["m"], spec["jitter"], seed=W.seed_for(cfg, "mesh"))
        self.N = spec["N"]
        self.nf = 4
        self.ops = ardg.Ops(self.N)
        self.lm = ardg.Mesh(self.ops, self.mesh.vxy, self.mesh.etov, device=0)
        self.gas = dict(gamma=1.4, R=1.0, Pr=0.7, mu_ref=spec["mu_ref"], T_ref=1.0, S=0.4)
        self.lm.set_navier_stokes(ardg.NS_SUTHERLAND, **self.gas)
        vp = spec["vortex"]
        X = self.lm.export(ardg.MESH_BFACE_GHOST_NODES).reshape(self.lm.E_bdy, self.ops.Np, 2)
        ext = W.isentropic_vortex(X[..., 0], X[..., 1], **vp)          # [4][E_bdy][Np]
        self.lm.set_boundary_data(ext[..., None], 0.0, 1.0)
        rs = self.ops.export(ardg.OPS_NODES).reshape(-1, 2)
        x, y = nodal_xy(self.mesh, rs)
        self.u0 = W.isentropic_vortex(x, y, **vp)
        self.K, self.Np, self.Nfp = self.mesh.K, self.ops.Np, self.ops.Nfp
        self.dof = self.nf * self.K * self.Np
        # explicit time step: the smaller of the acoustic limit h/((N+1)^2 (|u| + c))
        # and the viscous limit h^2/((N+1)^4 max(nu, gamma nu / Pr)), h the
        # smallest inscribed-circle diameter, with a safety factor 0.5
        v = self.mesh.vxy[self.mesh.etov]
        a = np.linalg.norm(v[:, 1] - v[:, 0], axis=1)
        b = np.linalg.norm(v[:, 2] - v[:, 1], axis=1)
        c = np.linalg.norm(v[:, 0] - v[:, 2], axis=1)
        area = 0.5 * np.abs((v[:, 1, 0] - v[:, 0, 0]) * (v[:, 2, 1] - v[:, 0, 1])
                            - (v[:, 2, 0] - v[:, 0, 0]) * (v[:, 1, 1] - v[:, 0, 1]))
        h = float(np.min(4.0 * area / (a + b + c)))
        rho, mx, my, E = self.u0
        uu, vv = mx / rho, my / rho
        p = 0.4 * (E - 0.5 * rho * (uu * uu + vv * vv))
        lam = float(np.max(np.hypot(uu, vv) + np.sqrt(1.4 * p / rho)))
        nu = float(np.max(spec["mu_ref"] * 1.5 / rho)) * max(1.0, 1.4 / 0.7)
        q = (self.N + 1) ** 2
        self.dt = 0.5 * min(h / (q * lam), h * h / (q * q * nu))
        self.setup_s = time.time() - t0
        log(f"bench: {name}: K={self.K} N={self.N} setup {self.setup_s:.1f} s, h={h:.3e}, dt={self.dt:.3e}")

    def config(self):
        return {"workload": self.name, "K": self.K, "N": self.N, "Np": self.Np, "DOF": self.dof,
                "E_int": self.lm.E_int, "E_bdy": self.lm.E_bdy, "fields": 4, "scheme": "LSERK(5,4)",
                "dt": self.dt, "gas": self.gas, "vortex": self.spec["vortex"]}

    def time_mode(self, prec, steps, warmup, dev):
        import torch
        from paper_1912_06221_amd import ardg
        u = torch.from_numpy(self.u0.copy()).to(dev)
        work = ardg.alloc_workspace(self.lm.workspace_bytes(ardg.LSERK54, prec, 4), dev)
        for _ in range(warmup):
            self.lm.rk_step(u, work, self.dt, 1, scheme=ardg.LSERK54, precision=prec, nfields=4)
        self.lm.rk_prepare(u, work, self.dt, steps, scheme=ardg.LSERK54, precision=prec, nfields=4)
        torch.cuda.synchronize()
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        self.lm.rk_step(u, work, self.dt, steps, scheme=ardg.LSERK54, precision=prec, nfields=4)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        self.lm.check(u, nfields=4)
        runs = [self.lm.stage_timing(u, work, self.dt, 40, scheme=ardg.LSERK54, precision=prec, nfields=4)
                for _ in range(3)]
        t_edge = float(np.median([r[0] for r in runs]))
        t_elem = float(np.median([r[1] for r in runs]))
        return ms, t_edge, t_elem

    def rhs_vs_oracle(self, prec, dev, nsample=12):
        """max |rhs - rhs_oracle| / max |rhs_oracle| on sampled elements (one
        right-hand side of the initial state)."""
        import torch
        from oracle.ns import Gas, NavierStokes
        from paper_1912_06221_amd import ardg
        g = self.gas
        vp = self.spec["vortex"]
        ns = NavierStokes(self.mesh.vxy, self.mesh.etov, self.N,
                          Gas(gamma=g["gamma"], R=g["R"], Pr=g["Pr"], mu_ref=g["mu_ref"], T_ref=g["T_ref"],
                              S=g["S"]),
                          lambda x, y, t: W.isentropic_vortex(x, y, **vp), build_edges=False)
        rng = np.random.default_rng(3)
        els = sorted(set(rng.choice(self.K, size=nsample, replace=False).tolist()) | {0, self.K - 1})
        dt = torch.float64 if prec == ardg.FP64 else torch.float32
        x = torch.from_numpy(self.u0).to(dev).to(dt)
        out = torch.empty_like(x)
        self.lm.rhs_eval(x, out, precision=prec, nfields=4)
        got = out.double().cpu().numpy()
        ref = ns.rhs_elements(self.u0, els, 0.0)
        return float(np.abs(got[:, els] - ref).max() / np.abs(ref).max())


def bench_ns(args, dev):
    from paper_1912_06221_amd import ardg
    c = NSCase("ns_vortex_708x708_N3", dev)
    out = {"config": c.config()}
    ctr = stored_counters(c.name)
    for mode, prec, s in (("fp64", ardg.FP64, 8), ("fp32", ardg.FP32, 4)):
        ms, te, tl = c.time_mode(prec, args.steps, args.warmup, dev)
        be, bl = ns_algorithmic_bytes(c.K, c.Np, c.Nfp, c.lm.E_int, c.lm.E_bdy, s)
        r = {"ms_per_step": ms, "value": c.dof * 5 / (ms * 1e-3), "unit": "DOF*stage/s",
             "edge_us": te * 1e3, "element_us": tl * 1e3, "edge_bytes": be, "element_bytes": bl,
             "edge_GBps": be / (te * 1e-3) / 1e9, "element_GBps": bl / (tl * 1e-3) / 1e9}
        r["edge_frac"] = r["edge_GBps"] / HBM_PEAK_GBS
        r["element_frac"] = r["element_GBps"] / HBM_PEAK_GBS
        r["edge_traffic"] = ctr.get(f"edge-{mode} hbm_bytes")
        r["element_traffic"] = ctr.get(f"element-{mode} hbm_bytes")
        vf = ctr.get(f"edge-{mode} valu_flops")
        if vf is not None:
            r[f"edge_valu_{mode}_frac"] = vf / (te * 1e-3) / 1e12 / PEAK_TFLOPS[mode]
        if not args.no_errors:
            r["rhs_err_vs_oracle_sampled"] = c.rhs_vs_oracle(prec, dev)
        out[mode] = r
        log(f"bench: {c.name} {mode}: {ms:.3f} ms/step (5 stages), edge {te*1e3:.1f} us "
            f"({r['edge_frac']*100:.1f}% HBM), element {tl*1e3:.1f} us ({r['element_frac']*100:.1f}% HBM)")
    return out


def alg2_compare(case, args, dev):
    """Algorithm 2 (reconstructed coefficient times the reconstructed
    gradient) beside Algorithm 1 on an element-wise-D workload: FP64 step
    time, the smallest reconstructed coefficient on the diagonals relative to
    the smallest element D, and the L2 difference of the two after the
    workload's steps."""
    from paper_1912_06221_amd import ardg
    w = case.ops.export(ardg.OPS_ALG2_W).reshape(2, case.Nfp)
    edges = case.lm.export(ardg.MESH_EDGES).reshape(-1, 4)
    D = np.asarray(case.D)
    Dt = D[edges[:, 0], None] * w[0][None, :] + D[edges[:, 2], None] * w[1][None, :]
    steps = case.spec["steps"]
    dt = getattr(case, "dt_stable", case.dt)
    u1 = case.run_steps(ardg.FP64, steps, dev, dt)
    case.lm.set_diffusion_element(D, alg=2)
    try:
        ms, te, tl = case.time_mode(ardg.FP64, args.steps, args.warmup, dev)
        u2 = case.run_steps(ardg.FP64, steps, dev, dt)
    finally:
        case.lm.set_diffusion_element(D, alg=1)
    out = {"fp64_ms_per_step": ms, "value": case.dof * 4 / (ms * 1e-3), "edge_us": te * 1e3,
           "element_us": tl * 1e3, "min_Dtilde": float(Dt.min()),
           "min_Dtilde_over_min_D": float(Dt.min() / D.min()), "steps": steps, "dt": dt}
    if u1 is not None and u2 is not None:
        n0 = float(np.linalg.norm(case.u0))
        out["alg1_norm_growth"] = float(np.linalg.norm(u1)) / n0
        out["alg2_norm_growth"] = float(np.linalg.norm(u2)) / n0
        out["rel_l2_alg2_vs_alg1_state"] = float(np.linalg.norm(u2 - u1) / np.linalg.norm(u1))
        inc = float(np.linalg.norm(u1 - case.u0))
        out["rel_l2_alg2_vs_alg1_increment"] = float(np.linalg.norm(u2 - u1)) / inc if inc > 0 else None
    log(f"bench: {case.name} Algorithm 2: {ms:.3f} ms/step, min D~ {out['min_Dtilde']:.3e}, "
        f"alg2 vs alg1 increment {out.get('rel_l2_alg2_vs_alg1_increment')}")
    return out


# ---------------------------------------------------------------------------
# Batched workload
# ---------------------------------------------------------------------------

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
    finals = {}
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
        finals[name] = [u.cpu().numpy() for u in us]
        out[f"batched_{name}"] = {"ms_per_step": ms, "value": dof * 4 / (ms * 1e-3)}
        tiles = {}
        for N in (2, 3, 4):
            et, lt, gm = b.tiles(prec, N)
            tiles[f"N{N}"] = {"edge_tile": et, "elem_tile": lt, "grid_per_cu": gm}
        out[f"batched_{name}"]["tiles"] = tiles
    num = sum(float(np.sum((a - c) ** 2)) for a, c in zip(finals["fp32"], finals["fp64"]))
    den = sum(float(np.sum(c ** 2)) for c in finals["fp64"])
    out["batched_fp32"]["rel_l2_vs_batched_fp64_state"] = math.sqrt(num / den)
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
    out["speedup_batched_fp64_vs_per_mesh_fp64"] = ms / out["batched_fp64"]["ms_per_step"]
    return out


# ---------------------------------------------------------------------------
# CPU baseline: the oracle on the host's cores
# ---------------------------------------------------------------------------

def _strip(mesh, m, j0, rows):
    """Sub-mesh of the cell rows [j0, j0 + rows) of an m x m split-square mesh
    (cell-major element numbering), vertices renumbered."""
    e = mesh.etov[2 * j0 * m: 2 * (j0 + rows) * m]
    used, inv = np.unique(e, return_inverse=True)
    return mesh.vxy[used], inv.reshape(e.shape).astype(np.int32)


def _oracle_worker(vxy, etov, N, D, D_mode, vel, nf, reps, seed, barrier, queue):
    os.environ["OMP_NUM_THREADS"] = "1"
    from oracle.rhs import Problem
    t0 = time.time()
    pr = Problem(vxy, etov, N, D, D_mode=D_mode, velocity=vel, nfields=nf)
    setup = time.time() - t0
    u = np.random.default_rng(seed).standard_normal((nf, etov.shape[0], pr.ops.Np))
    barrier.wait()
    t0 = time.time()
    for _ in range(reps):
        pr.rhs(u)
    queue.put((setup, time.time() - t0, reps * u.size))


def copy_bandwidth(dev, mib=1024, reps=20):
    """Achievable HBM rate on this device: the best of `reps` timed
    device-to-device copies of `mib` MiB (bytes read + written per second,
    GB/s; the best rather than the median, as single copies scatter by 10 %
    from box to box)."""
    import torch
    a = torch.empty(mib * 1024 * 1024 // 8, dtype=torch.float64, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    st = torch.cuda.current_stream()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        b.copy_(a)
        e1.record(st)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    del a, b
    torch.cuda.empty_cache()
    return 2 * mib * 1024 * 1024 / float(np.min(ts)) / 1e9


def cpu_baseline(name, rows_per_worker=2, reps=4):
    """The oracle's assembled RHS (edge operators prebuilt, setup reported
    apart) on strips of cell rows of the workload's mesh, one strip per worker
    process on the host's cores; DOF*stage/s = DOF evaluated / wall time
    between the common start and the last worker's end."""
    import multiprocessing as mp
    spec = W.WORKLOADS[name]
    cfg = spec["config"]
    m = spec["m"]
    mesh = W.split_square_mesh(m, spec["jitter"], seed=W.seed_for(cfg, "mesh"))
    D, D_mode = workload_D(spec, mesh)
    vel = ROTATION if spec.get("velocity") == "rotation" else None
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    workers = max(1, min(16, ncpu))
    ctx = mp.get_context("spawn")
    barrier = ctx.Barrier(workers + 1)
    queue = ctx.Queue()
    procs = []
    for w in range(workers):
        j0 = (w * rows_per_worker * 7) % (m - rows_per_worker)
        vxy, etov = _strip(mesh, m, j0, rows_per_worker)
        Dw = D if D_mode == "const" else D[2 * j0 * m: 2 * (j0 + rows_per_worker) * m]
        p = ctx.Process(target=_oracle_worker, args=(vxy, etov, spec["N"], Dw, D_mode, vel, spec["fields"],
                                                     reps, w, barrier, queue))
        p.start()
        procs.append(p)
    barrier.wait()
    t0 = time.time()
    res = [queue.get() for _ in range(workers)]
    wall = time.time() - t0
    for p in procs:
        p.join()
    dof = sum(r[2] for r in res)
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    K_strip = 2 * m * rows_per_worker
    return {"value": dof / wall, "unit": "DOF*stage/s", "cores": workers, "kind": "oracle",
            "cpu_model": model, "host_cpus": ncpu,
            "sample": (f"{workers} worker processes (one thread each), each evaluating the oracle's assembled "
                       f"RHS (literal per-edge aRDG operators prebuilt, weak-form volume term, upwind "
                       f"convection, {spec['fields']} fields) {reps} times on its own strip of "
                       f"{rows_per_worker} cell rows ({K_strip} elements) of the {name} mesh; "
                       f"{wall:.1f} s wall for {dof:.3g} DOF*stage; operator setup "
                       f"{max(r[0] for r in res):.1f} s per worker excluded")}


# ---------------------------------------------------------------------------

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default=HEADLINE, help="headline workload")
    ap.add_argument("--extras", default="contrast_256x256_N4,loguniformD_512x512_N6",
                    help="comma-separated extra workloads ('' for none)")
    ap.add_argument("--modes", default="fp64,fp32,bf16x3")
    ap.add_argument("--no-errors", action="store_true", help="skip the error runs (profiling)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 512-problem batched workload")
    ap.add_argument("--no-ns", action="store_true", help="skip the Navier-Stokes workload")
    ap.add_argument("--power-iters", type=int, default=60)
    ap.add_argument("--edge-kernel", default="auto", choices=sorted(EDGE_KERNELS),
                    help="edge kernel implementation (default: chosen by the library)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one device copy of 512 MiB first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {args.gpus} is not supported "
              f"(sharding the mesh over several GPUs is a design, not implemented)", file=sys.stderr)
        sys.exit(2)

    # the oracle's worker processes start before anything touches the GPU
    cpu = None
    if not args.no_cpu_baseline:
        log("bench: timing the oracle on the host cores (cpu_baseline)")
        cpu = cpu_baseline(args.workload)
        log(f"bench: cpu_baseline {cpu['value']:.3e} DOF*stage/s on {cpu['cores']} cores")

    import torch
    dev = torch.device("cuda:0")
    if args.calib_copy:
        a = torch.empty(64 * 1024 * 1024, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"bench: calibration copy of {a.numel() * 8} bytes done")
        del a, b

    modes = [m for m in args.modes.split(",") if m]
    if "fp64" not in modes:
        sys.exit("bench: --modes must include fp64 (the headline path)")
    head = Case(args.workload, dev, args.power_iters, args.edge_kernel)
    hr = measure_case(head, args, dev, modes, 0 if args.no_errors else head.spec["steps"])
    r64 = hr["fp64"]
    dom = "element" if r64["element_us"] >= r64["edge_us"] else "edge"
    ctr = stored_counters(args.workload)
    roof = {"bound": "hbm", "kernel": dom, "achieved": r64[f"{dom}_GBps"], "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": r64[f"{dom}_frac"],
            "traffic": ctr.get(f"{dom}-fp64 hbm_bytes"),
            "edge_frac": r64["edge_frac"], "edge_GBps": r64["edge_GBps"], "edge_us": r64["edge_us"],
            "edge_bytes": r64["edge_bytes"], "edge_traffic": ctr.get("edge-fp64 hbm_bytes"),
            "element_frac": r64["element_frac"], "element_GBps": r64["element_GBps"],
            "element_us": r64["element_us"], "element_bytes": r64["element_bytes"],
            "element_traffic": ctr.get("element-fp64 hbm_bytes"),
            "edge_fp64_flop_frac": r64["edge_flop_frac"], "element_fp64_flop_frac": r64["element_flop_frac"],
            # the same kernels' fractions for the bytes as stored and moved
            # (tables as laid out, RK traffic averaged over the stages)
            "edge_stored_frac": r64["edge_stored_frac"], "element_stored_frac": r64["element_stored_frac"],
            "edge_stored_bytes": r64["edge_stored_bytes"], "element_stored_bytes": r64["element_stored_bytes"]}
    # the same rates against what a plain device copy reaches on this machine
    cbw = copy_bandwidth(dev)
    roof["copy_GBps"] = cbw
    roof["edge_frac_of_copy"] = r64["edge_GBps"] / cbw
    roof["element_frac_of_copy"] = r64["element_GBps"] / cbw
    log(f"bench: device copy {cbw:.0f} GB/s (read + write); FP64 edge {r64['edge_GBps'] / cbw:.1%}, "
        f"element {r64['element_GBps'] / cbw:.1%} of it")
    mf = ctr.get("element-fp64 mfma_flops")
    if mf is not None:
        roof["element_mfma_fp64_frac"] = mf / (r64["element_us"] * 1e-6) / 1e12 / PEAK_TFLOPS["fp64"]
    vf = ctr.get("edge-fp64 valu_flops")
    if vf is not None:
        roof["edge_valu_fp64_frac"] = vf / (r64["edge_us"] * 1e-6) / 1e12 / PEAK_TFLOPS["fp64"]
    line = {
        "metric": "DOF*RK-stage/s per MI355X (FP64 path; FP32 and split-BF16 paths beside it with their L2 "
                  "error after the workload's steps); % HBM roofline",
        "value": r64["value"],
        "unit": "DOF*stage/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms_per_step"],
        "step": "one classic RK4 time step = 4 RHS stages (edge kernel + element kernel each)",
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded jittered mesh, seeded Fourier initial data per field)",
        "config": head.config(),
        "roofline": roof,
        "modes": {m: hr[m] for m in modes},
    }
    for m in modes:
        if m != "fp64":
            line["modes"][m]["speedup_vs_fp64"] = r64["ms_per_step"] / hr[m]["ms_per_step"]
    if "errors" in hr:
        line["errors"] = hr["errors"]
    extras = {}
    for name in [x for x in args.extras.split(",") if x]:
        c = Case(name, dev, args.power_iters, args.edge_kernel)
        # the precision workload states every mode's error after its steps
        steps = c.spec["steps"] if (not args.no_errors and name.startswith("loguniform")) else 0
        r = measure_case(c, args, dev, modes, steps)
        r["config"] = c.config()
        if c.alg1 and not args.no_errors:
            r["algorithm2"] = alg2_compare(c, args, dev)
        for m in modes:
            if m != "fp64":
                r[m]["speedup_vs_fp64"] = r["fp64"]["ms_per_step"] / r[m]["ms_per_step"]
        extras[name] = r
        del c
        torch.cuda.empty_cache()
    if extras:
        line["extra_workloads"] = extras
    if not args.no_batch:
        log("bench: batched workload (512 problems)")
        line["batch"] = bench_batch(args, dev)
        bb = line["batch"]
        log(f"bench: batch fp64 {bb['batched_fp64']['ms_per_step']:.3f} ms, fp32 "
            f"{bb['batched_fp32']['ms_per_step']:.3f} ms, per-mesh fp64 {bb['per_mesh_fp64']['ms_per_step']:.3f} ms")
    if not args.no_ns:
        line["navier_stokes"] = bench_ns(args, dev)
        torch.cuda.empty_cache()
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
