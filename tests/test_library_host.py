"""The C-ABI library without a GPU: it loads, exports every declared symbol,
and its independent FP64 host setup (reference operators, connectivity,
enclosed parallelograms, per-edge parameters) agrees with the oracle.  Error
paths are exercised with host-only meshes (device -1)."""
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import ardg as oa
from oracle.mesh import Geometry
from oracle.reference_element import RefOps

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

ardg = pytest.importorskip("paper_1912_06221_amd.ardg")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(ardg.LIB_PATH):
        pytest.fail("libardg.so is not built (run __graft_entry__.build())")
    return ardg.lib()


def test_exports_every_declared_symbol(L):
    hdr = open(os.path.join(ROOT, "include", "ardg.h")).read()
    names = set(re.findall(r"\b(ardg_[a-z0-9_]+)\s*\(", hdr))
    assert len(names) >= 15
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert not missing, missing
    assert set(ardg.SIGNATURES) <= names


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6])
def test_reference_operators_match_oracle(L, N):
    o = ardg.Ops(N)
    ro = RefOps(N)
    Np, Nfp = o.Np, o.Nfp
    assert np.abs(o.export(ardg.OPS_NODES).reshape(Np, 2) - ro.rs).max() < 1e-14
    for w, ref in ((ardg.OPS_DR, ro.Dr), (ardg.OPS_DS, ro.Ds), (ardg.OPS_MASS, ro.M),
                   (ardg.OPS_LIFT, ro.LIFT)):
        A = o.export(w).reshape(ref.shape)
        assert np.abs(A - ref).max() < 1e-13 * np.abs(ref).max()
    fm = o.export(ardg.OPS_FACE_NODES).reshape(3, Nfp).astype(int)
    for f in range(3):
        assert list(fm[f]) == list(ro.fmask[f])
    rp = o.export(ardg.OPS_ROT_PERM).reshape(3, Np).astype(int)
    for f in range(3):
        assert list(rp[f]) == list(oa.rotation_perm(N, f))


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6])
def test_face_rotation_commutes_with_bernstein_conversion(L, N):
    """Relabelling the vertices permutes Bernstein coefficients by the same
    lattice permutation that it applies to the (symmetric) nodes, so the
    nodal->Bernstein matrix commutes with each face's reordering: an element
    can store its Bernstein coefficients once and every edge rotates them by
    index, as it rotates nodal values."""
    o = ardg.Ops(N)
    Np = o.Np
    n2b = o.export(ardg.OPS_N2B).reshape(Np, Np)
    rp = o.export(ardg.OPS_ROT_PERM).reshape(3, Np).astype(int)
    for f in range(3):
        P = np.zeros((Np, Np))
        P[np.arange(Np), rp[f]] = 1.0
        assert np.abs(n2b @ P - P @ n2b).max() < 1e-12 * np.abs(n2b).max()


@pytest.mark.parametrize("N", [1, 2, 3, 4, 6])
def test_reconstruction_operators_match_oracle(L, N):
    o = ardg.Ops(N)
    ro = RefOps(N)
    Np, Nfp = o.Np, o.Nfp
    R = oa.recon_pinv(N)
    E0, ER, ES = oa.diagonal_eval(N)
    Vb = np.kron(np.eye(2), ro.Vinv)
    ref = np.vstack([ER @ R @ Vb, ES @ R @ Vb])
    G = o.export(ardg.OPS_RECON_GRAD).reshape(2 * Nfp, 2 * Np)
    assert np.abs(G - ref).max() < 1e-12 * np.abs(ref).max()
    # values of u~ at the diagonal nodes (the Navier-Stokes interface)
    Vv = o.export(ardg.OPS_RECON_VALUE).reshape(Nfp, 2 * Np)
    refv = E0 @ R @ Vb
    assert np.abs(Vv - refv).max() < 1e-12 * np.abs(refv).max()
    # library A^+ is a pseudo-inverse of its own A
    A = o.export(ardg.OPS_RECON_A).reshape(2 * Np, (N + 1) ** 2)
    Rl = o.export(ardg.OPS_RECON_R).reshape((N + 1) ** 2, 2 * Np)
    assert np.abs(Rl @ A - np.eye((N + 1) ** 2)).max() < 1e-12


def test_alg1_blocks_match_oracle(L):
    """Algorithm 1 blocks: apply the oracle's Algorithm 1 to an edge whose
    sub-triangles are the elements themselves and compare the nodal maps."""
    N = 3
    o = ardg.Ops(N)
    Np, Nfp = o.Np, o.Nfp
    U = o.export(ardg.OPS_ALG1_GRAD).reshape(4 * Nfp, 2 * Np)
    U1R, U1S, U2R, U2S = (U[i * Nfp:(i + 1) * Nfp] for i in range(4))
    ro = RefOps(N)
    # a parallelogram edge: projection = rotation only; choose f1 = f2 = hypotenuse
    A, B = np.array([1.0, 0.0]), np.array([0.0, 1.0])
    C1 = np.array([0.1, 0.2])
    C2 = A + B - C1
    eg = oa.EdgeGeometry(A, B, C1, C2, n1=np.array([1.0, 1.0]) / np.sqrt(2.0))
    for D1, D2 in ((1.0, 0.0), (0.0, 1.0), (2.5, 0.7)):
        W1, W2 = oa.edge_operator_alg1(ro, eg, 1, 1, D1, D2)
        gR, gS = eg.n1[0] * eg.Rx + eg.n1[1] * eg.Ry, eg.n1[0] * eg.Sx + eg.n1[1] * eg.Sy
        lib = D1 * (gR * U1R + gS * U1S) - D2 * (gR * U2R + gS * U2S)
        # sub-triangle nodal data = the element's rotated nodal data (identity projection)
        assert np.abs(lib[:, :Np] - W1).max() < 1e-11 * max(1.0, np.abs(W1).max())
        assert np.abs(lib[:, Np:] - W2).max() < 1e-11 * max(1.0, np.abs(W2).max())


def _bary(w1, w2, w3, P):
    rs = oa.ref_coords(w1, w2, w3, P)
    return np.array([(rs[0] + 1) / 2, (rs[1] + 1) / 2])


@pytest.mark.parametrize("m,jit", [(4, 0.0), (6, 0.2), (5, 0.25)])
def test_mesh_setup_matches_oracle(L, m, jit):
    mesh = W.split_square_mesh(m, jit, seed=m)
    o = ardg.Ops(2)
    lm = ardg.Mesh(o, mesh.vxy, mesh.etov, device=-1)
    g = Geometry(mesh.vxy, mesh.etov)
    edges = lm.export(ardg.MESH_EDGES).reshape(-1, 4)
    assert [tuple(e) for e in edges] == [tuple(e) for e in g.interior]
    bf = lm.export(ardg.MESH_BFACES).reshape(-1, 2)
    assert [tuple(e) for e in bf] == [tuple(e) for e in g.boundary]
    geo = lm.export(ardg.MESH_EDGE_GEOM).reshape(-1, 8)
    for e, (k1, f1, k2, f2) in enumerate(g.interior):
        eg = oa.interior_edge_geometry(g, k1, f1, k2, f2)
        assert np.abs(geo[e, 0:2] - eg.P1).max() < 1e-13
        assert np.abs(geo[e, 2:4] - _bary(eg.C1, eg.A, eg.B, eg.P1)).max() < 1e-12
        assert np.abs(geo[e, 4:6] - _bary(eg.C2, eg.B, eg.A, eg.P2)).max() < 1e-12
        gR = eg.n1[0] * eg.Rx + eg.n1[1] * eg.Ry
        gS = eg.n1[0] * eg.Sx + eg.n1[1] * eg.Sy
        assert np.abs(geo[e, 6:8] - [gR, gS]).max() < 1e-11 * max(1.0, abs(gR) + abs(gS))
    bgeo = lm.export(ardg.MESH_BFACE_GEOM).reshape(-1, 6)
    for b, (k, f) in enumerate(g.boundary):
        eg = oa.boundary_edge_geometry(g, k, f)
        assert np.abs(bgeo[b, 0:2] - eg.P1).max() < 1e-13
        gR = eg.n1[0] * eg.Rx + eg.n1[1] * eg.Ry
        gS = eg.n1[0] * eg.Sx + eg.n1[1] * eg.Sy
        assert np.abs(bgeo[b, 4:6] - [gR, gS]).max() < 1e-11 * max(1.0, abs(gR) + abs(gS))
    ef = lm.export(ardg.MESH_ELEM_FACES).reshape(-1, 3)
    for e, (k1, f1, k2, f2) in enumerate(g.interior):
        assert ef[k1, f1] == 2 * e and ef[k2, f2] == 2 * e + 1
    assert lm.info.min_area_ratio > 0.2 and lm.info.min_J > 0
    if jit == 0.0:
        assert abs(lm.info.min_area_ratio - 1.0) < 1e-12   # all parallelograms


def test_error_paths(L):
    o = ardg.Ops(2)
    mesh = W.split_square_mesh(2, 0.0)
    bad = mesh.etov.copy()
    bad[0] = bad[0][[0, 2, 1]]                      # clockwise element
    with pytest.raises(ardg.ArdgError) as ei:
        ardg.Mesh(o, mesh.vxy, bad, device=-1)
    assert ei.value.status == -2
    v = mesh.vxy.copy()
    v[3, 0] = np.nan
    with pytest.raises(ardg.ArdgError) as ei:
        ardg.Mesh(o, v, mesh.etov, device=-1)
    assert ei.value.status == -1
    bad = mesh.etov.copy()
    bad[1, 2] = 10_000
    with pytest.raises(ardg.ArdgError) as ei:
        ardg.Mesh(o, mesh.vxy, bad, device=-1)
    assert ei.value.status == -1
    # three triangles on one edge
    vxy = np.array([[0, 0], [1, 0], [0.5, 1], [0.5, -1], [0.2, 0.9]], dtype=float)
    etov = np.array([[0, 1, 2], [1, 0, 3], [0, 1, 4]], dtype=np.int32)
    with pytest.raises(ardg.ArdgError) as ei:
        ardg.Mesh(o, vxy, etov, device=-1)
    assert ei.value.status == -3
    with pytest.raises(ardg.ArdgError) as ei:
        ardg.Ops(7)
    assert ei.value.status == -6
    with pytest.raises(ardg.ArdgError) as ei:
        ardg.Ops(0)
    assert ei.value.status == -6
    lm = ardg.Mesh(o, mesh.vxy, mesh.etov, device=-1)
    with pytest.raises(ardg.ArdgError):
        lm.set_diffusion_const([-1.0])
    Dbad = np.ones(mesh.K)
    Dbad[2] = 0.0
    with pytest.raises(ardg.ArdgError):
        lm.set_diffusion_element(Dbad)
    with pytest.raises(ardg.ArdgError):
        lm.set_velocity([0, 0, np.inf, 0, 0, 0])
    # kernels refuse a host-only mesh
    with pytest.raises(ardg.ArdgError):
        lm.rhs_eval(1, 1, stream=0)
    assert L.ardg_status_string(-4).decode().startswith("degenerate")


def test_batch_refuses_host_only_meshes(L):
    o = ardg.Ops(2)
    mesh = W.split_square_mesh(3, 0.0)
    lm = ardg.Mesh(o, mesh.vxy, mesh.etov, device=-1)
    with pytest.raises(ardg.ArdgError) as ei:
        ardg.Batch([lm])
    assert ei.value.status == -1
    with pytest.raises(ardg.ArdgError):
        ardg.Batch([])


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6])
def test_alg2_weights_match_oracle(L, N):
    """Algorithm 2's diagonal weights (reconstruction of a coefficient that is
    1 on one side and 0 on the other) from the library's host setup against
    the oracle's literal reconstruction on a jittered mesh's edges."""
    from paper_1912_06221_amd import ardg as A
    from oracle import ardg as OA
    from oracle.mesh import Geometry
    from oracle.reference_element import RefOps
    ops = A.Ops(N)
    w = ops.export(A.OPS_ALG2_W).reshape(2, N + 1)
    mesh = W.split_square_mesh(3, 0.2, seed=N)
    g = Geometry(mesh.vxy, mesh.etov)
    ro = RefOps(N)
    one, zero = np.ones(ro.Np), np.zeros(ro.Np)
    for (k1, f1, k2, f2) in g.interior[:6]:
        eg = OA.interior_edge_geometry(g, k1, f1, k2, f2)
        assert np.abs(OA.coefficient_on_diagonal(ro, eg, f1, f2, one, zero) - w[0]).max() < 1e-12
        assert np.abs(OA.coefficient_on_diagonal(ro, eg, f1, f2, zero, one) - w[1]).max() < 1e-12


@pytest.mark.parametrize("N", [1, 3, 5])
def test_ghost_nodes_match_oracle(L, N):
    """The physical points where the exterior state is sampled (the nodes of
    each boundary face's ghost sub-triangle) from the library's host setup
    against the oracle's."""
    from paper_1912_06221_amd import ardg as A
    mesh = W.split_square_mesh(4, 0.2, seed=N + 40)
    ops = A.Ops(N)
    lm = A.Mesh(ops, mesh.vxy, mesh.etov, device=-1)
    X = lm.export(A.MESH_BFACE_GHOST_NODES).reshape(lm.E_bdy, ops.Np, 2)
    g = Geometry(mesh.vxy, mesh.etov)
    bf = lm.export(A.MESH_BFACES).reshape(-1, 2)
    for b, (k, f) in enumerate(bf):
        eg = oa.boundary_edge_geometry(g, int(k), int(f))
        assert np.abs(X[b] - oa.ghost_nodes(N, eg)).max() < 1e-12
