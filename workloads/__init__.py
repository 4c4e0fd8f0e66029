"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the reconstruction method: it only builds
meshes (vertex coordinates and CCW vertex lists), coefficient fields, smooth
functions evaluated at caller-supplied points, and random nodal data.  Both the
oracle and the HIP library consume what it returns; neither side's operators,
node sets or geometry live here.

Input recipe (the paper runs on grids of split quadrilaterals; the workloads
below are synthetic stand-ins with the same structure):

* ``split_square_mesh(m, jitter)``: the unit square cut into m x m cells, each
  cell split along its (i,j)->(i+1,j+1) diagonal into two CCW triangles.  Every
  interior vertex is moved independently in x and y by U[-jitter*h, jitter*h]
  (h = 1/m); boundary vertices stay fixed.  Unjittered, every interior pair of
  triangles forms a parallelogram (the paper's grid-a situation).
* ``circle_contrast_D``: piecewise constant per element, ``inside`` within a
  circle and ``outside`` elsewhere, assigned by element centroid.
* ``loguniform_per_element``: per-element coefficient, log-uniform in [lo, hi].
* ``fourier_modes``: sum_{k,l=1..4} a_kl sin(k pi x) sin(l pi y) with
  a_kl = g_kl/(k^2+l^2), g ~ N(0,1); vanishes on the boundary of the square.
* ``manufactured``: exp(-2 pi^2 D t) sin(pi x) sin(pi y), an exact solution of
  the heat equation with zero Dirichlet data on the unit square.
* ``paper_grid(kind, n)``: the three grid families of the paper's results
  (its figure is missing; this is the reading the text supports).  Grid a:
  the square [0,10] x [-5,5] cut into n x n cells of two triangles (2 n^2
  elements, every interior pair a parallelogram).  Grids b and c: a
  quadrilateral (corners BL, BR, TR, TL) cut into the four triangles
  (BL, BR, C), (BR, TR, C), (TR, TL, C), (TL, BL, C) around a centre point C,
  each refined uniformly into n^2 congruent triangles (4 n^2 elements); pairs
  across the four corner-to-centre lines ("the diagonals") are not
  parallelograms.  Grid b: the square itself with C = (5, 0) (two triangles
  across a diagonal form one larger triangle).  Grid c: the bottom-left and
  top-right corners moved to (1.5, -3.5) and (11.5, 6.5) and C = (6.5, 1.5),
  which leaves all four blocks, hence all elements, the same area.
* ``gaussian``: the paper's travelling Gaussian pulse of mass M released at
  time -D0/D, M / (4 pi (D t + D0)) exp(-|x - a t - x0|^2 / (4 (D t + D0))),
  an exact solution of u_t + a . grad u = D lap u (a = 0: pure diffusion).
* ``isentropic_vortex``: the conserved variables (rho, rho u, rho v, E) of
  the isentropic vortex of strength beta and radius L centred at c0,
  convected with the free stream uinf (ideal gas, R = 1, p = rho^gamma), an
  exact solution of the Euler equations; the Navier-Stokes workload's
  initial and exterior state (the paper's Navier-Stokes tests use
  manufactured solutions and a cylinder flow whose fields it does not print).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Mesh", "split_square_mesh", "centroids", "circle_contrast_D",
    "loguniform_per_element", "fourier_modes", "manufactured",
    "random_nodal", "seed_for", "WORKLOADS", "batch_problems", "paper_grid", "gaussian",
    "isentropic_vortex",
]


def seed_for(config: int, what: str) -> int:
    """Seed convention: 1000*config + {mesh:1, D:2, IC:3, batch:4}."""
    return 1000 * int(config) + {"mesh": 1, "D": 2, "IC": 3, "batch": 4}[what]


@dataclass
class Mesh:
    vxy: np.ndarray    # [Nv, 2] float64 vertex coordinates
    etov: np.ndarray   # [K, 3] int32 vertex indices, counter-clockwise

    @property
    def K(self) -> int:
        return int(self.etov.shape[0])


def split_square_mesh(m: int, jitter: float = 0.0, seed: int = 0) -> Mesh:
    """m x m cells on [0,1]^2, each split along its (i,j)->(i+1,j+1) diagonal.

    Elements are numbered cell by cell in row-major order (cell (i,j) holds
    elements 2(j*m+i) and 2(j*m+i)+1), which keeps face neighbours close in
    memory.
    """
    if m < 1:
        raise ValueError("m must be >= 1")
    h = 1.0 / m
    ii, jj = np.meshgrid(np.arange(m + 1), np.arange(m + 1), indexing="xy")
    x = (ii * h).astype(np.float64).ravel()
    y = (jj * h).astype(np.float64).ravel()
    if jitter > 0.0:
        rng = np.random.Generator(np.random.PCG64(seed))
        d = rng.uniform(-jitter * h, jitter * h, size=(2, (m + 1) * (m + 1)))
        interior = ((ii > 0) & (ii < m) & (jj > 0) & (jj < m)).ravel()
        x = x + np.where(interior, d[0], 0.0)
        y = y + np.where(interior, d[1], 0.0)
    vxy = np.stack([x, y], axis=1)

    def vid(i, j):
        return j * (m + 1) + i

    ci, cj = np.meshgrid(np.arange(m), np.arange(m), indexing="xy")
    ci = ci.ravel()
    cj = cj.ravel()
    a = vid(ci, cj)
    b = vid(ci + 1, cj)
    c = vid(ci + 1, cj + 1)
    d = vid(ci, cj + 1)
    lower = np.stack([a, b, c], axis=1)   # (i,j),(i+1,j),(i+1,j+1)
    upper = np.stack([a, c, d], axis=1)   # (i,j),(i+1,j+1),(i,j+1)
    etov = np.empty((2 * m * m, 3), dtype=np.int32)
    etov[0::2] = lower
    etov[1::2] = upper
    return Mesh(vxy=vxy, etov=etov)


def centroids(mesh: Mesh) -> np.ndarray:
    return mesh.vxy[mesh.etov].mean(axis=1)


def circle_contrast_D(mesh: Mesh, inside: float = 1e2, outside: float = 1e-2,
                      radius: float = 0.25, centre=(0.5, 0.5)) -> np.ndarray:
    c = centroids(mesh)
    r2 = (c[:, 0] - centre[0]) ** 2 + (c[:, 1] - centre[1]) ** 2
    return np.where(r2 < radius * radius, inside, outside).astype(np.float64)


def loguniform_per_element(K: int, lo: float, hi: float, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size=K))


def fourier_modes(x: np.ndarray, y: np.ndarray, seed: int, modes: int = 4) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.standard_normal((modes, modes))
    out = np.zeros(np.broadcast(x, y).shape)
    for k in range(1, modes + 1):
        sx = np.sin(k * math.pi * x)
        for l in range(1, modes + 1):
            out = out + g[k - 1, l - 1] / (k * k + l * l) * sx * np.sin(l * math.pi * y)
    return out


def manufactured(x, y, t: float = 0.0, D: float = 1.0):
    return math.exp(-2.0 * math.pi ** 2 * D * t) * np.sin(math.pi * x) * np.sin(math.pi * y)


def random_nodal(shape, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-1.0, 1.0, size=shape)


# Named workloads (sizes as quoted for each configuration).
WORKLOADS = {
    "heat_8x8_N2": dict(config=0, m=8, jitter=0.0, N=2, D="const", Dval=1.0,
                        ic="manufactured", steps=100, fields=1),
    "contrast_256x256_N4": dict(config=1, m=256, jitter=0.2, N=4, D="circle",
                                ic="fourier", steps=100, fields=1),
    "loguniformD_512x512_N6": dict(config=2, m=512, jitter=0.2, N=6, D="loguniform",
                                   Dlo=1e-3, Dhi=1e1, ic="fourier", steps=50, fields=1),
    "convdiff_708x708_N3_4f": dict(config=4, m=708, jitter=0.2, N=3, D="perfield",
                                   Dfield=(1e-4, 1e-3, 1e-2, 1.0), ic="fourier",
                                   velocity="rotation", steps=200, fields=4),
    # compressible Navier-Stokes, four conserved fields: the vortex of radius
    # 0.1 at the centre of the unit square, free stream (0.3, 0.2), Sutherland
    # viscosity mu_ref = 1e-4 (Reynolds number 300 on the vortex radius),
    # Pr = 0.7, gamma = 1.4; the exterior state is the initial vortex
    "ns_vortex_708x708_N3": dict(config=5, m=708, jitter=0.2, N=3, D="navier-stokes",
                                 ic="vortex", steps=100, fields=4, mu_ref=1e-4,
                                 vortex=dict(beta=5.0, uinf=(0.3, 0.2), c0=(0.5, 0.5), L=0.1)),
}


def batch_problems(n: int = 512, seed: int = seed_for(3, "batch"),
                   kmin: int = 200, kmax: int = 20000):
    """Independent heat problems of uneven size and order.

    Returns a list of dicts with m (cells per side, K = 2 m^2 ~ n_i), N in
    {2,3,4} and a constant D log-uniform in [1e-3, 1].
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n):
        ni = math.exp(rng.uniform(math.log(kmin), math.log(kmax)))
        m = max(2, int(round(math.sqrt(ni / 2.0))))
        N = int(rng.integers(2, 5))
        D = math.exp(rng.uniform(math.log(1e-3), math.log(1.0)))
        out.append(dict(m=m, N=N, D=D, mesh_seed=seed * 1000 + 2 * i,
                        ic_seed=seed * 1000 + 2 * i + 1))
    return out


def _refined_triangle(V0, V1, V2, n):
    """Points and CCW triangles of the uniform n x n refinement of (V0,V1,V2)."""
    idx = {}
    pts = []
    for j in range(n + 1):
        for i in range(n + 1 - j):
            idx[(i, j)] = len(pts)
            pts.append(V0 + (i / n) * (V1 - V0) + (j / n) * (V2 - V0))
    tris = []
    for j in range(n):
        for i in range(n - j):
            tris.append((idx[(i, j)], idx[(i + 1, j)], idx[(i, j + 1)]))
            if i + j <= n - 2:
                tris.append((idx[(i + 1, j)], idx[(i + 1, j + 1)], idx[(i, j + 1)]))
    return np.array(pts), np.array(tris, dtype=np.int64)


def paper_grid(kind: str, n: int) -> Mesh:
    """Grid family a, b or c at refinement n (see the module docstring)."""
    if kind == "a":
        m = split_square_mesh(n, 0.0)
        vxy = m.vxy * np.array([10.0, 10.0]) + np.array([0.0, -5.0])
        return Mesh(vxy=vxy, etov=m.etov)
    if kind == "b":
        BL, BR, TR, TL, C = (0.0, -5.0), (10.0, -5.0), (10.0, 5.0), (0.0, 5.0), (5.0, 0.0)
    elif kind == "c":
        BL, BR, TR, TL, C = (1.5, -3.5), (10.0, -5.0), (11.5, 6.5), (0.0, 5.0), (6.5, 1.5)
    else:
        raise ValueError(kind)
    BL, BR, TR, TL, C = (np.array(p) for p in (BL, BR, TR, TL, C))
    allp, allt, off = [], [], 0
    for (A, B) in ((BL, BR), (BR, TR), (TR, TL), (TL, BL)):
        p, t = _refined_triangle(A, B, C, n)
        allp.append(p)
        allt.append(t + off)
        off += len(p)
    P = np.vstack(allp)
    T = np.vstack(allt)
    # merge the points the blocks share (their common edges)
    key = np.round(P, 9)
    _, first, inv = np.unique(key, axis=0, return_index=True, return_inverse=True)
    inv = inv.ravel()
    return Mesh(vxy=P[first], etov=inv[T].astype(np.int32))


def gaussian(x, y, t, D=1.0, D0=2.0, x0=(5.0, 0.0), a=(0.0, 0.0), M=1.0):
    """The Gaussian pulse of mass M released at time -D0/D at x0, advected with
    constant velocity a: M / (4 pi (D t + D0)) exp(-|x - a t - x0|^2 / (4 (D t + D0)))."""
    s = D * t + D0
    dx = x - a[0] * t - x0[0]
    dy = y - a[1] * t - x0[1]
    return M / (4.0 * math.pi * s) * np.exp(-(dx * dx + dy * dy) / (4.0 * s))


def isentropic_vortex(x, y, t=0.0, gamma=1.4, beta=5.0, uinf=(0.3, 0.2), c0=(0.5, 0.5), L=0.1):
    """(rho, rho u, rho v, E) [4, ...] of the isentropic vortex at time t:
    f = exp((1 - r^2) / 2) with r the distance to c0 + uinf t over L,
    u = uinf + beta / (2 pi) f (-y', x'), T = 1 - (gamma - 1) beta^2 f^2 /
    (8 gamma pi^2), rho = T^(1/(gamma - 1)), p = rho T."""
    xc = (x - c0[0] - uinf[0] * t) / L
    yc = (y - c0[1] - uinf[1] * t) / L
    f = np.exp(0.5 * (1.0 - xc * xc - yc * yc))
    u = uinf[0] - beta / (2.0 * math.pi) * f * yc
    v = uinf[1] + beta / (2.0 * math.pi) * f * xc
    T = 1.0 - (gamma - 1.0) * beta ** 2 / (8.0 * gamma * math.pi ** 2) * f * f
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho * T
    return np.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])
