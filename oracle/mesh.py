"""Element geometry and face connectivity, FP64.  TEST INFRASTRUCTURE ONLY.

Geometry follows the affine triangle map (eq. mapping_tri), its derivatives
(eq. mapping_tri_diff) and Jacobians (eqs. triangle_jacobian_a/b).  Faces are
f1 = (v1,v2), f2 = (v2,v3), f3 = (v3,v1), traversed counter-clockwise.
"""
from __future__ import annotations

import numpy as np


class Geometry:
    """Per-element affine data and the face-to-face connectivity of a mesh."""

    def __init__(self, vxy: np.ndarray, etov: np.ndarray):
        self.vxy = np.asarray(vxy, dtype=np.float64)
        self.etov = np.asarray(etov, dtype=np.int64)
        K = self.etov.shape[0]
        self.K = K
        v = self.vxy[self.etov]                       # [K, 3, 2]
        self.v = v
        # (x_r, y_r) = (v2 - v1)/2, (x_s, y_s) = (v3 - v1)/2
        xr, yr = 0.5 * (v[:, 1, 0] - v[:, 0, 0]), 0.5 * (v[:, 1, 1] - v[:, 0, 1])
        xs, ys = 0.5 * (v[:, 2, 0] - v[:, 0, 0]), 0.5 * (v[:, 2, 1] - v[:, 0, 1])
        J = xr * ys - xs * yr
        if np.any(J <= 0):
            raise ValueError("element with non-positive Jacobian (not CCW)")
        self.J = J
        self.rx, self.ry = ys / J, -xs / J
        self.sx, self.sy = -yr / J, xr / J
        # outward unit normals and surface scale sJ = |edge| / 2 per face
        self.nx = np.zeros((K, 3))
        self.ny = np.zeros((K, 3))
        self.sJ = np.zeros((K, 3))
        for f, (a, b) in enumerate(((0, 1), (1, 2), (2, 0))):
            tx = v[:, b, 0] - v[:, a, 0]
            ty = v[:, b, 1] - v[:, a, 1]
            L = np.hypot(tx, ty)
            self.nx[:, f] = ty / L
            self.ny[:, f] = -tx / L
            self.sJ[:, f] = 0.5 * L
        self._connect()

    def _connect(self):
        """Face neighbours by matching sorted vertex pairs (O(K log K))."""
        K = self.K
        self.EToE = -np.ones((K, 3), dtype=np.int64)
        self.EToF = -np.ones((K, 3), dtype=np.int64)
        seen = {}
        for k in range(K):
            for f, (a, b) in enumerate(((0, 1), (1, 2), (2, 0))):
                key = tuple(sorted((int(self.etov[k, a]), int(self.etov[k, b]))))
                if key in seen:
                    k2, f2 = seen.pop(key)
                    self.EToE[k, f], self.EToF[k, f] = k2, f2
                    self.EToE[k2, f2], self.EToF[k2, f2] = k, f
                else:
                    seen[key] = (k, f)
        # edge list: interior edges once (side 1 = lower element index), then
        # boundary faces
        inter, bdy = [], []
        for k in range(K):
            for f in range(3):
                k2 = self.EToE[k, f]
                if k2 < 0:
                    bdy.append((k, f))
                elif k < k2:
                    inter.append((k, f, int(k2), int(self.EToF[k, f])))
        self.interior = inter
        self.boundary = bdy

    def physical(self, rs: np.ndarray) -> np.ndarray:
        """[K, Np, 2] physical coordinates of reference points rs [Np, 2]."""
        r, s = rs[:, 0], rs[:, 1]
        v = self.v
        x = (-(r + s)[None, :] * v[:, 0:1, 0] + (r + 1)[None, :] * v[:, 1:2, 0]
             + (s + 1)[None, :] * v[:, 2:3, 0]) * 0.5
        y = (-(r + s)[None, :] * v[:, 0:1, 1] + (r + 1)[None, :] * v[:, 1:2, 1]
             + (s + 1)[None, :] * v[:, 2:3, 1]) * 0.5
        return np.stack([x, y], axis=-1)
