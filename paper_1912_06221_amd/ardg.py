"""ctypes binding of libardg.so (argument marshalling only).

Every computation runs in the library's HIP kernels; this module converts
NumPy host arrays and torch device tensors into the plain pointers and sizes
of the C ABI declared in include/ardg.h, and turns error codes into Python
exceptions.  There is no fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_void_p

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libardg.so")

OK = 0
FP64, FP32, BF16X3 = 0, 1, 2
RK4, LSERK54 = 0, 1
D_CONST, D_ELEMENT, D_ELEMENT_ALG2, D_NODAL, D_SOLUTION = 0, 1, 2, 3, 4
VEL_NONE, VEL_AFFINE = 0, 1
NS_OFF, NS_SUTHERLAND, NS_CONSTANT_MU = 0, 1, 2
EDGE_AUTO, EDGE_SPLIT, EDGE_LANE, EDGE_MFMA, EDGE_SPLIT_MFMA, EDGE_FIELDS = 0, 1, 2, 3, 4, 5

OPS_NODES, OPS_V, OPS_DR, OPS_DS, OPS_MASS, OPS_LIFT = 0, 1, 2, 3, 4, 5
OPS_FACE_NODES, OPS_ROT_PERM, OPS_RECON_A, OPS_RECON_R = 6, 7, 8, 9
OPS_RECON_GRAD, OPS_ALG1_GRAD, OPS_N2B, OPS_ALG2_W = 10, 11, 12, 13
OPS_RECON_VALUE = 14
MESH_EDGES, MESH_BFACES, MESH_EDGE_GEOM, MESH_BFACE_GEOM, MESH_ELEM_FACES = 0, 1, 2, 3, 4
MESH_BFACE_GHOST_NODES = 5


class ArdgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"ardg status {status}: {msg}")
        self.status = status


class MeshInfo(ctypes.Structure):
    _fields_ = [("K", c_int64), ("Np", c_int64), ("Nfp", c_int64), ("E_int", c_int64),
                ("E_bdy", c_int64), ("N", c_int32), ("device", c_int32),
                ("min_J", c_double), ("min_area_ratio", c_double)]


_lib = None

# name -> (restype, argtypes)
SIGNATURES = {
    "ardg_ops_create": (c_int32, [c_int32, c_int32, POINTER(c_void_p)]),
    "ardg_ops_export": (c_int32, [c_void_p, c_int32, POINTER(c_double), c_int64, POINTER(c_int64)]),
    "ardg_ops_destroy": (None, [c_void_p]),
    "ardg_mesh_create": (c_int32, [c_void_p, POINTER(c_double), c_int64, POINTER(c_int32), c_int64,
                                   POINTER(c_int32), c_int32, POINTER(c_void_p)]),
    "ardg_mesh_info": (c_int32, [c_void_p, POINTER(MeshInfo)]),
    "ardg_mesh_export": (c_int32, [c_void_p, c_int32, c_void_p, c_int64, POINTER(c_int64)]),
    "ardg_mesh_destroy": (None, [c_void_p]),
    "ardg_mesh_set_diffusion": (c_int32, [c_void_p, c_int32, c_int32, POINTER(c_double)]),
    "ardg_mesh_set_velocity": (c_int32, [c_void_p, c_int32, POINTER(c_double)]),
    "ardg_mesh_set_kernels": (c_int32, [c_void_p, c_int32]),
    "ardg_mesh_set_navier_stokes": (c_int32, [c_void_p, c_int32, POINTER(c_double)]),
    "ardg_mesh_set_boundary_data": (c_int32, [c_void_p, c_int32, c_int32, c_double, c_double, POINTER(c_double)]),
    "ardg_rhs_eval": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_double, c_void_p]),
    "ardg_rhs_eval_noalloc": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_double, c_void_p]),
    "ardg_edge_flux_eval": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_double, c_void_p]),
    "ardg_rk_workspace_bytes": (c_int32, [c_void_p, c_int32, c_int32, c_int32, POINTER(c_int64)]),
    "ardg_rk_step": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p, c_double,
                               c_double, c_int32, c_void_p]),
    "ardg_rk_prepare": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p, c_double, c_int32]),
    "ardg_stage_timing": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p, c_double,
                                    c_int32, c_void_p, POINTER(ctypes.c_float)]),
    "ardg_check": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p]),
    "ardg_batch_create": (c_int32, [POINTER(c_void_p), c_int32, c_char_p, POINTER(c_void_p)]),
    "ardg_batch_workspace_bytes": (c_int32, [c_void_p, c_int32, c_int32, POINTER(c_int64)]),
    "ardg_batch_step": (c_int32, [c_void_p, c_int32, c_int32, POINTER(c_void_p), c_void_p,
                                  POINTER(c_double), c_int32, c_void_p]),
    "ardg_batch_tiles": (c_int32, [c_void_p, c_int32, c_int32, POINTER(c_int32), POINTER(c_int32),
                                   POINTER(c_int32)]),
    "ardg_batch_destroy": (None, [c_void_p]),
    "ardg_batch_check": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "ardg_status_string": (c_char_p, [c_int32]),
    "ardg_last_error": (c_char_p, []),
}


def lib():
    """Load libardg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != OK:
        raise ArdgError(status, lib().ardg_last_error().decode(errors="replace"))


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(POINTER(c_double))


def _ptr(t):
    """Device pointer of a torch tensor (or an int / None)."""
    if t is None:
        return None
    if isinstance(t, int):
        return c_void_p(t)
    return c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return c_void_p(stream)
    return c_void_p(stream.cuda_stream)


class Ops:
    """Reference operators of order N (ardg_ops_create)."""

    def __init__(self, N: int, node_family: int = 0):
        h = c_void_p()
        _check(lib().ardg_ops_create(N, node_family, ctypes.byref(h)))
        self.handle = h
        self.N = N
        self.Np = (N + 1) * (N + 2) // 2
        self.Nfp = N + 1

    def export(self, which: int) -> np.ndarray:
        n = c_int64()
        lib().ardg_ops_export(self.handle, which, None, 0, ctypes.byref(n))
        out = np.empty(n.value, dtype=np.float64)
        _check(lib().ardg_ops_export(self.handle, which, _dptr(out), n.value, ctypes.byref(n)))
        return out

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.ardg_ops_destroy(self.handle)
            self.handle = None


class Mesh:
    """A mesh on one device (or host-only with device=-1)."""

    def __init__(self, ops: Ops, vxy, etov, device: int = 0):
        vxy = np.ascontiguousarray(vxy, dtype=np.float64)
        etov = np.ascontiguousarray(etov, dtype=np.int32)
        h = c_void_p()
        _check(lib().ardg_mesh_create(ops.handle, _dptr(vxy), vxy.shape[0],
                                      etov.ctypes.data_as(POINTER(c_int32)), etov.shape[0], None,
                                      device, ctypes.byref(h)))
        self.handle = h
        self.ops = ops
        self.device = device
        info = MeshInfo()
        _check(lib().ardg_mesh_info(h, ctypes.byref(info)))
        self.info = info
        self.K, self.Np, self.Nfp = info.K, info.Np, info.Nfp
        self.E_int, self.E_bdy = info.E_int, info.E_bdy
        self.E = self.E_int + self.E_bdy

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.ardg_mesh_destroy(self.handle)
            self.handle = None

    def export(self, which: int) -> np.ndarray:
        n = c_int64()
        lib().ardg_mesh_export(self.handle, which, None, 0, ctypes.byref(n))
        is_int = which in (MESH_EDGES, MESH_BFACES, MESH_ELEM_FACES)
        out = np.empty(n.value, dtype=np.int32 if is_int else np.float64)
        _check(lib().ardg_mesh_export(self.handle, which, out.ctypes.data_as(c_void_p),
                                      out.nbytes, ctypes.byref(n)))
        return out

    def set_diffusion_const(self, D):
        D = np.ascontiguousarray(np.atleast_1d(D), dtype=np.float64)
        _check(lib().ardg_mesh_set_diffusion(self.handle, D_CONST, D.size, _dptr(D)))

    def set_diffusion_element(self, D, alg: int = 1):
        """Element-wise D with the flux of Algorithm 1 (alg=1) or Algorithm 2
        (alg=2)."""
        D = np.ascontiguousarray(D, dtype=np.float64)
        mode = {1: D_ELEMENT, 2: D_ELEMENT_ALG2}[alg]
        _check(lib().ardg_mesh_set_diffusion(self.handle, mode, 1, _dptr(D)))

    def set_diffusion_nodal(self, D):
        """Tensor coefficient (Dxx, Dxy, Dyy) at every node: D [K][Np][3]."""
        D = np.ascontiguousarray(D, dtype=np.float64)
        if D.shape != (self.K, self.Np, 3):
            raise ValueError("D must be [K][Np][3]")
        _check(lib().ardg_mesh_set_diffusion(self.handle, D_NODAL, 1, _dptr(D)))

    def set_diffusion_solution(self, D0):
        """Solution-dependent coefficient u D0, D0 = (D0xx, D0xy, D0yy)."""
        D = np.ascontiguousarray(D0, dtype=np.float64).reshape(3)
        _check(lib().ardg_mesh_set_diffusion(self.handle, D_SOLUTION, 1, _dptr(D)))

    def set_velocity(self, params=None):
        if params is None:
            _check(lib().ardg_mesh_set_velocity(self.handle, VEL_NONE, None))
        else:
            p = np.ascontiguousarray(params, dtype=np.float64)
            _check(lib().ardg_mesh_set_velocity(self.handle, VEL_AFFINE, _dptr(p)))

    def set_kernels(self, edge_kernel: int = EDGE_AUTO):
        _check(lib().ardg_mesh_set_kernels(self.handle, edge_kernel))

    def set_navier_stokes(self, law: int = NS_SUTHERLAND, gamma: float = 1.4, R: float = 1.0,
                          Pr: float = 0.7, mu_ref: float = 1e-2, T_ref: float = 1.0, S: float = 0.4):
        """The compressible Navier-Stokes system on four fields (law NS_OFF
        switches back to the scalar equation)."""
        if law == NS_OFF:
            _check(lib().ardg_mesh_set_navier_stokes(self.handle, NS_OFF, None))
            return
        p = np.array([gamma, R, Pr, mu_ref, T_ref, S], dtype=np.float64)
        _check(lib().ardg_mesh_set_navier_stokes(self.handle, law, _dptr(p)))

    def set_boundary_data(self, coeffs, t_a: float, t_b: float):
        """Prescribed exterior state: coeffs [F][E_bdy][Np][nt] Chebyshev
        coefficients in time on [t_a, t_b] (None clears)."""
        if coeffs is None:
            _check(lib().ardg_mesh_set_boundary_data(self.handle, 1, 0, 0.0, 1.0, None))
            return
        c = np.ascontiguousarray(coeffs, dtype=np.float64)
        if c.ndim != 4 or c.shape[1] != self.E_bdy or c.shape[2] != self.Np:
            raise ValueError("coeffs must be [F][E_bdy][Np][nt]")
        _check(lib().ardg_mesh_set_boundary_data(self.handle, c.shape[0], c.shape[3], t_a, t_b, _dptr(c)))

    # ---- device calls (torch tensors on this mesh's device) ---------------
    def rhs_eval(self, u, out, precision: int = FP64, nfields: int = 1, stream=None, t: float = 0.0):
        _check(lib().ardg_rhs_eval(self.handle, precision, nfields, _ptr(u), _ptr(out), t,
                                   _stream(stream)))
        return out

    def rhs_eval_noalloc(self, u, out, precision: int = FP64, nfields: int = 1, stream=None, t: float = 0.0):
        """rhs_eval with the fluxes in the library's device scratch array (no
        allocation)."""
        _check(lib().ardg_rhs_eval_noalloc(self.handle, precision, nfields, _ptr(u), _ptr(out), t,
                                           _stream(stream)))
        return out

    def edge_flux_eval(self, u, flux, precision: int = FP64, nfields: int = 1, stream=None, t: float = 0.0):
        _check(lib().ardg_edge_flux_eval(self.handle, precision, nfields, _ptr(u), _ptr(flux), t,
                                         _stream(stream)))
        return flux

    def workspace_bytes(self, scheme: int = RK4, precision: int = FP64, nfields: int = 1) -> int:
        n = c_int64()
        _check(lib().ardg_rk_workspace_bytes(self.handle, scheme, precision, nfields, ctypes.byref(n)))
        return n.value

    def rk_step(self, u, work, dt: float, nsteps: int, scheme: int = RK4, precision: int = FP64,
                nfields: int = 1, t0: float = 0.0, stream=None):
        _check(lib().ardg_rk_step(self.handle, scheme, precision, nfields, _ptr(u), _ptr(work), t0,
                                  dt, nsteps, _stream(stream)))

    def rk_prepare(self, u, work, dt: float, nsteps: int, scheme: int = RK4, precision: int = FP64,
                   nfields: int = 1):
        """Capture the graph rk_step would replay for these arguments, without
        running it."""
        _check(lib().ardg_rk_prepare(self.handle, scheme, precision, nfields, _ptr(u), _ptr(work),
                                     dt, nsteps))

    def stage_timing(self, u, work, dt: float, reps: int, scheme: int = RK4, precision: int = FP64,
                     nfields: int = 1, stream=None):
        """Average kernel duration (edge ms, element ms) from replays of a graph
        of `reps` RK stages and of one of their element kernels alone; alters u."""
        out = (ctypes.c_float * 2)()
        _check(lib().ardg_stage_timing(self.handle, scheme, precision, nfields, _ptr(u), _ptr(work),
                                       dt, reps, _stream(stream), out))
        return float(out[0]), float(out[1])

    def check(self, u, nfields: int = 1, stream=None):
        _check(lib().ardg_check(self.handle, nfields, _ptr(u), _stream(stream)))


class Batch:
    """Many independent meshes advanced together (ardg_batch_*)."""

    def __init__(self, meshes, tune_cache: str | None = None):
        self.meshes = list(meshes)          # keeps the handles alive
        arr = (c_void_p * len(self.meshes))(*[m.handle.value for m in self.meshes])
        h = c_void_p()
        _check(lib().ardg_batch_create(arr, len(self.meshes),
                                       tune_cache.encode() if tune_cache else None, ctypes.byref(h)))
        self.handle = h

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.ardg_batch_destroy(self.handle)
            self.handle = None

    def workspace_bytes(self, scheme: int = RK4, precision: int = FP64) -> int:
        n = c_int64()
        _check(lib().ardg_batch_workspace_bytes(self.handle, scheme, precision, ctypes.byref(n)))
        return n.value

    def tiles(self, precision: int, N: int):
        a, b, c = c_int32(), c_int32(), c_int32()
        _check(lib().ardg_batch_tiles(self.handle, precision, N, ctypes.byref(a), ctypes.byref(b),
                                      ctypes.byref(c)))
        return a.value, b.value, c.value

    def step(self, us, work, dts, nsteps: int, scheme: int = RK4, precision: int = FP64, stream=None):
        ptrs = (c_void_p * len(us))(*[u.data_ptr() for u in us])
        dt = np.ascontiguousarray(dts, dtype=np.float64)
        _check(lib().ardg_batch_step(self.handle, scheme, precision, ptrs, _ptr(work), _dptr(dt),
                                     nsteps, _stream(stream)))

    def check(self, us, stream=None):
        """Synchronise and scan every mesh's FP64 state for non-finite values."""
        ptrs = (c_void_p * len(us))(*[u.data_ptr() for u in us])
        _check(lib().ardg_batch_check(self.handle, ptrs, _stream(stream)))


def alloc_workspace(nbytes: int, device):
    """A 256-byte aligned device buffer (torch uint8) of at least nbytes."""
    import torch
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf[off:off + nbytes]
