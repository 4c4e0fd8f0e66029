// C ABI of the library: handles, validation, device uploads, launch sequences
// and the HIP-graph-captured Runge-Kutta loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <exception>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/ardg.h"
#include "device.hpp"
#include "meshsetup.hpp"
#include "noalloc.hpp"
#include "refops.hpp"

using namespace ardg;

namespace {

thread_local std::string g_err;

ardg_status fail(ardg_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

ardg_status hip_fail(hipError_t e, const char* what) {
  return fail(ARDG_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                         \
  do {                                              \
    hipError_t _e = (expr);                         \
    if (_e != hipSuccess) return hip_fail(_e, what); \
  } while (0)

struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = (hipSetDevice(dev) == hipSuccess);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

void pack_into(const RefOps& o, std::vector<double>& out) {
  const OpLayout L(o.N);
  out.assign(L.total, 0.0);
  auto put = [&](int off, const Mat& M) { std::copy(M.a.begin(), M.a.end(), out.begin() + off); };
  put(L.n2b, o.N2B);
  put(L.kr, o.KR);
  put(L.ks, o.KS);
  put(L.kbr, o.KBR);
  put(L.kbs, o.KBS);
  put(L.u1r, o.U1R);
  put(L.u1s, o.U1S);
  put(L.u2r, o.U2R);
  put(L.u2s, o.U2S);
  put(L.udr, add(o.U1R, o.U2R, -1.0));
  put(L.uds, add(o.U1S, o.U2S, -1.0));
  put(L.ubr, o.UBR);
  put(L.ubs, o.UBS);
  put(L.dr, o.Dr);
  put(L.ds, o.Ds);
  put(L.drsh, hcat(o.Dr, o.Ds));
  put(L.lift, o.LIFT);
  for (int j = 0; j < o.Nfp; ++j) out[L.tau + j] = 0.5 * (o.lgl[j] + 1.0);
  for (int n = 0; n < o.Np; ++n) {
    out[L.nr + n] = o.r[n];
    out[L.ns + n] = o.s[n];
  }
  // 1D Bernstein basis of degree N at the face's LGL nodes, tau = (x + 1)/2
  // measured from the face's first (counter-clockwise) vertex
  for (int j = 0; j < o.Nfp; ++j) {
    out[L.w1 + j] = o.alg2_w1[j];
    out[L.w2 + j] = o.alg2_w2[j];
  }
  put(L.tr1, o.TR1);
  put(L.ts1, o.TS1);
  put(L.tr2, o.TR2);
  put(L.ts2, o.TS2);
  put(L.g1, o.G1);
  put(L.g2, o.G2);
  put(L.b2n, o.Bv);
  put(L.kv, o.KV);
  for (int j = 0; j < o.Nfp; ++j) {
    const double tau = 0.5 * (o.lgl[j] + 1.0);
    for (int k = 0; k <= o.N; ++k) {
      double binom = 1.0;
      for (int q = 1; q <= k; ++q) binom = binom * (o.N - k + q) / q;
      out[L.bf2n + j * o.Nfp + k] = binom * std::pow(1.0 - tau, o.N - k) * std::pow(tau, k);
    }
  }
}

template <typename T>
ardg_status upload(const T* src, size_t n, T** dst) {
  if (n == 0) { *dst = nullptr; return ARDG_OK; }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, n * sizeof(T));
  if (e != hipSuccess) return fail(ARDG_E_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
  e = hipMemcpy(p, src, n * sizeof(T), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(p);
    return hip_fail(e, "hipMemcpy");
  }
  *dst = (T*)p;
  return ARDG_OK;
}

}  // namespace

struct ardg_ops_s {
  RefOps ro;
  std::vector<double> packed;
};

struct GraphKey {
  int scheme, precision, nfields, nsteps;
  const void* u;
  const void* work;
  double dt;
  uint64_t version;
  bool operator<(const GraphKey& o) const {
    return std::tie(scheme, precision, nfields, nsteps, u, work, dt, version) <
           std::tie(o.scheme, o.precision, o.nfields, o.nsteps, o.u, o.work, o.dt, o.version);
  }
};

struct ardg_mesh_s {
  int N = 0, device = -1;
  RefOps ro;
  std::vector<double> packed;
  HostMesh hm;
  DevMesh dm;
  std::vector<void*> allocs;      // device allocations owned by the mesh
  double* Delem_dev = nullptr;
  double* Dfield_dev = nullptr;     // device copy of dm.Dfield (owned through allocs)
  double2* vn_dev = nullptr;
  double* Dnodal_dev = nullptr;     // tensor coefficient [K][Np][3]
  double4* gp_dev = nullptr;        // per face: parallelogram inverse metric
  double2* sn_dev = nullptr;        // per face: sJ n1
  int nfields_D = 1;
  void* flux_scratch = nullptr;
  size_t flux_scratch_bytes = 0;
  // prescribed exterior data: Chebyshev coefficients in time [F][E_bdy][Np][nt]
  // on [ghost_ta, ghost_tb], the state at the current stage time, and the
  // start time of the current step (device scalar advanced by the step graphs)
  double* ghost_coef = nullptr;
  double* ghost_val = nullptr;
  double* tdev = nullptr;
  int ghost_nt = 0, ghost_nf = 0;
  double ghost_ta = 0.0, ghost_tb = 0.0;
  hipStream_t cap_stream = nullptr;
  std::map<GraphKey, hipGraphExec_t> graphs;
  uint64_t version = 0;

  ~ardg_mesh_s() {
    if (device >= 0) {
      DeviceGuard g(device);
      for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
      if (cap_stream) (void)hipStreamDestroy(cap_stream);
      for (void* p : allocs) (void)hipFree(p);
      if (Delem_dev) (void)hipFree(Delem_dev);
      if (vn_dev) (void)hipFree(vn_dev);
      if (Dnodal_dev) (void)hipFree(Dnodal_dev);
      if (gp_dev) (void)hipFree(gp_dev);
      if (sn_dev) (void)hipFree(sn_dev);
      if (flux_scratch) (void)hipFree(flux_scratch);
      if (ghost_coef) (void)hipFree(ghost_coef);
      if (ghost_val) (void)hipFree(ghost_val);
      if (tdev) (void)hipFree(tdev);
    }
  }
  void drop_graphs() {
    // earlier launches of these graphs may still run
    (void)hipDeviceSynchronize();
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    graphs.clear();
    ++version;
  }
};

// Steps per captured graph: a longer run replays the graph of kGraphSteps
// steps (and one graph for the remainder), so that a graph stays a few
// thousand nodes whatever the step count.
constexpr int kGraphSteps = 256;

extern "C" {

const char* ardg_last_error(void) { return g_err.c_str(); }

const char* ardg_status_string(ardg_status s) {
  switch (s) {
    case ARDG_OK: return "ok";
    case ARDG_E_INVALID_ARG: return "invalid argument";
    case ARDG_E_MESH_ORIENTATION: return "element not counter-clockwise (J <= 0)";
    case ARDG_E_MESH_TOPOLOGY: return "non-manifold or inconsistently oriented mesh";
    case ARDG_E_DEGENERATE_PARALLELOGRAM: return "degenerate enclosed parallelogram";
    case ARDG_E_RECON_RANK: return "reconstruction system rank deficient";
    case ARDG_E_UNSUPPORTED: return "unsupported order or precision";
    case ARDG_E_HIP: return "HIP runtime error";
    case ARDG_E_OOM: return "out of device memory";
    case ARDG_E_NONFINITE: return "non-finite value in state";
    default: return "unknown status";
  }
}

ardg_status ardg_ops_create(int32_t N, int32_t node_family, ardg_ops* out) {
  if (!out) return fail(ARDG_E_INVALID_ARG, "ops_create: null out");
  *out = nullptr;
  if (N < 1 || N > 6) return fail(ARDG_E_UNSUPPORTED, "ops_create: N must be in 1..6");
  if (node_family != 0) return fail(ARDG_E_UNSUPPORTED, "ops_create: node_family must be 0");
  try {
    auto o = std::make_unique<ardg_ops_s>();
    bool rank_ok = true;
    o->ro = build_refops(N, &rank_ok);
    if (!rank_ok) return fail(ARDG_E_RECON_RANK, "ops_create: reconstruction system rank deficient");
    pack_into(o->ro, o->packed);
    *out = o.release();
    return ARDG_OK;
  } catch (const std::exception& ex) {
    return fail(ARDG_E_INVALID_ARG, std::string("ops_create: ") + ex.what());
  }
}

void ardg_ops_destroy(ardg_ops ops) { delete ops; }

ardg_status ardg_ops_export(ardg_ops ops, int32_t which, double* dst, int64_t cap, int64_t* n_written) {
  if (!ops) return fail(ARDG_E_INVALID_ARG, "ops_export: null handle");
  const RefOps& o = ops->ro;
  std::vector<double> v;
  auto mat = [&](const Mat& M) { v = M.a; };
  switch (which) {
    case ARDG_OPS_NODES:
      for (int n = 0; n < o.Np; ++n) { v.push_back(o.r[n]); v.push_back(o.s[n]); }
      break;
    case ARDG_OPS_V: mat(o.V); break;
    case ARDG_OPS_DR: mat(o.Dr); break;
    case ARDG_OPS_DS: mat(o.Ds); break;
    case ARDG_OPS_MASS: mat(o.M); break;
    case ARDG_OPS_LIFT: mat(o.LIFT); break;
    case ARDG_OPS_FACE_NODES:
      for (int f = 0; f < 3; ++f)
        for (int j = 0; j < o.Nfp; ++j) v.push_back(o.fmask[f][j]);
      break;
    case ARDG_OPS_ROT_PERM:
      for (int f = 0; f < 3; ++f)
        for (int n = 0; n < o.Np; ++n) v.push_back(o.rot[f][n]);
      break;
    case ARDG_OPS_RECON_A: mat(o.A); break;
    case ARDG_OPS_RECON_R: mat(o.Rop); break;
    case ARDG_OPS_RECON_GRAD: mat(o.recon_grad_nodal); break;
    case ARDG_OPS_ALG1_GRAD: mat(o.alg1_nodal); break;
    case ARDG_OPS_N2B: mat(o.N2B); break;
    case ARDG_OPS_RECON_VALUE: mat(o.recon_value_nodal); break;
    case ARDG_OPS_ALG2_W:
      v = o.alg2_w1;
      v.insert(v.end(), o.alg2_w2.begin(), o.alg2_w2.end());
      break;
    default: return fail(ARDG_E_INVALID_ARG, "ops_export: unknown selector");
  }
  if (n_written) *n_written = (int64_t)v.size();
  if (!dst || cap < (int64_t)v.size()) return fail(ARDG_E_INVALID_ARG, "ops_export: buffer too small");
  std::copy(v.begin(), v.end(), dst);
  return ARDG_OK;
}

ardg_status ardg_mesh_create(ardg_ops ops, const double* vxy, int64_t Nv, const int32_t* etov,
                             int64_t K, const int32_t* face_bc, int32_t device, ardg_mesh* out) {
  if (!out) return fail(ARDG_E_INVALID_ARG, "mesh_create: null out");
  *out = nullptr;
  if (!ops) return fail(ARDG_E_INVALID_ARG, "mesh_create: null ops");
  if (face_bc) return fail(ARDG_E_INVALID_ARG, "mesh_create: face_bc is reserved and must be NULL");
  try {
    auto m = std::make_unique<ardg_mesh_s>();
    m->N = ops->ro.N;
    m->ro = ops->ro;
    m->packed = ops->packed;
    std::string err;
    int st = build_host_mesh(vxy, Nv, etov, K, m->hm, err);
    if (st != ARDG_OK) return fail(st, err);
    m->dm.N = m->N;
    m->dm.edge_kernel = EDGE_AUTO;
    m->dm.K = m->hm.K;
    m->dm.E_int = m->hm.E_int;
    m->dm.E_bdy = m->hm.E_bdy;
    for (int f = 0; f < kMaxFields; ++f) m->dm.Dfield[f] = 1.0;
    if (device < 0) {
      m->device = -1;
      *out = m.release();
      return ARDG_OK;
    }
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
    if (device >= ndev) return fail(ARDG_E_INVALID_ARG, "mesh_create: no such device");
    DeviceGuard g(device);
    if (!g.ok) return fail(ARDG_E_HIP, "mesh_create: hipSetDevice failed");
    m->device = device;
    const HostMesh& h = m->hm;
    // device tables.  gamma (and below n.v) are stored times the edge's
    // surface factor sJ = |edge| / 2: the edge kernels then emit sJ * flux,
    // which is what the element's surface term lifts.
    const int rotv[3][3] = {{2, 0, 1}, {0, 1, 2}, {1, 2, 0}};
    auto half_len = [&](int64_t k, int f) {
      const int a = h.etov[3 * k + rotv[f][1]], b = h.etov[3 * k + rotv[f][2]];
      const double tx = h.vxy[2 * b] - h.vxy[2 * a], ty = h.vxy[2 * b + 1] - h.vxy[2 * a + 1];
      return 0.5 * std::sqrt(tx * tx + ty * ty);
    };
    std::vector<int2> ef(h.E_int);
    std::vector<double2> mu1(h.E_int), mu2(h.E_int), gam(h.E_int);
    for (int64_t e = 0; e < h.E_int; ++e) {
      ef[e].x = h.e1[e] | (h.f1[e] << 30);
      ef[e].y = h.e2[e] | (h.f2[e] << 30);
      mu1[e] = make_double2(h.mu1[2 * e], h.mu1[2 * e + 1]);
      mu2[e] = make_double2(h.mu2[2 * e], h.mu2[2 * e + 1]);
      const double sj = half_len(h.e1[e], h.f1[e]);
      gam[e] = make_double2(sj * h.gam[2 * e], sj * h.gam[2 * e + 1]);
    }
    std::vector<int> bk(h.E_bdy);
    std::vector<double2> bmu(h.E_bdy), bgam(h.E_bdy);
    for (int64_t b = 0; b < h.E_bdy; ++b) {
      bk[b] = h.bk[b] | (h.bf[b] << 30);
      bmu[b] = make_double2(h.bmu[2 * b], h.bmu[2 * b + 1]);
      const double sj = half_len(h.bk[b], h.bf[b]);
      bgam[b] = make_double2(sj * h.bgam[2 * b], sj * h.bgam[2 * b + 1]);
    }
    std::vector<double2> vert(3 * h.K);
    for (int64_t k = 0; k < h.K; ++k)
      for (int c = 0; c < 3; ++c) {
        const int v = h.etov[3 * k + c];
        vert[3 * k + c] = make_double2(h.vxy[2 * v], h.vxy[2 * v + 1]);
      }
    std::vector<int> efc(3 * h.K);
    for (int64_t k = 0; k < h.K; ++k)
      for (int f = 0; f < 3; ++f) efc[f * h.K + k] = h.elem_face[3 * k + f];
    std::vector<float> packed32(m->packed.begin(), m->packed.end());
    std::vector<double> Dinit(kMaxFields, 1.0);

    int2* d_ef; double2 *d_mu1, *d_mu2, *d_gam, *d_bmu, *d_bgam, *d_vert;
    double* d_Dfield;
    int *d_bk, *d_efc;
    double* d_ops64;
    float* d_ops32;
    ardg_status s;
#define UP(vec, ptr)                                           \
    s = upload(vec.data(), vec.size(), &ptr);                  \
    if (s != ARDG_OK) return s;                                \
    if (ptr) m->allocs.push_back((void*)ptr);
    UP(ef, d_ef) UP(mu1, d_mu1) UP(mu2, d_mu2) UP(gam, d_gam) UP(bk, d_bk) UP(bmu, d_bmu)
    UP(bgam, d_bgam) UP(vert, d_vert) UP(efc, d_efc) UP(m->packed, d_ops64) UP(packed32, d_ops32)
    UP(Dinit, d_Dfield)
#undef UP
    m->dm.ef = d_ef;
    m->dm.mu1 = d_mu1;
    m->dm.mu2 = d_mu2;
    m->dm.gam = d_gam;
    m->dm.bk = d_bk;
    m->dm.bmu = d_bmu;
    m->dm.bgam = d_bgam;
    m->dm.vert = d_vert;
    m->dm.elem_face = d_efc;
    m->dm.ops64 = d_ops64;
    m->dm.ops32 = d_ops32;
    m->dm.Dfield_dev = d_Dfield;
    m->Dfield_dev = d_Dfield;
    *out = m.release();
    return ARDG_OK;
  } catch (const std::bad_alloc&) {
    return fail(ARDG_E_OOM, "mesh_create: host allocation failed");
  } catch (const std::exception& ex) {
    return fail(ARDG_E_INVALID_ARG, std::string("mesh_create: ") + ex.what());
  }
}

void ardg_mesh_destroy(ardg_mesh mesh) { delete mesh; }

ardg_status ardg_mesh_info(ardg_mesh mesh, ardg_mesh_info_t* out) {
  if (!mesh || !out) return fail(ARDG_E_INVALID_ARG, "mesh_info: null argument");
  out->K = mesh->hm.K;
  out->Np = mesh->ro.Np;
  out->Nfp = mesh->ro.Nfp;
  out->E_int = mesh->hm.E_int;
  out->E_bdy = mesh->hm.E_bdy;
  out->N = mesh->N;
  out->device = mesh->device;
  out->min_J = mesh->hm.min_J;
  out->min_area_ratio = mesh->hm.min_area_ratio;
  return ARDG_OK;
}

ardg_status ardg_mesh_export(ardg_mesh mesh, int32_t which, void* dst, int64_t cap, int64_t* n_written) {
  if (!mesh) return fail(ARDG_E_INVALID_ARG, "mesh_export: null handle");
  const HostMesh& h = mesh->hm;
  std::vector<int32_t> iv;
  std::vector<double> dv;
  bool is_int = true;
  switch (which) {
    case ARDG_MESH_EDGES:
      for (int64_t e = 0; e < h.E_int; ++e) {
        iv.push_back(h.e1[e]); iv.push_back(h.f1[e]); iv.push_back(h.e2[e]); iv.push_back(h.f2[e]);
      }
      break;
    case ARDG_MESH_BFACES:
      for (int64_t b = 0; b < h.E_bdy; ++b) { iv.push_back(h.bk[b]); iv.push_back(h.bf[b]); }
      break;
    case ARDG_MESH_ELEM_FACES: iv = h.elem_face; break;
    case ARDG_MESH_EDGE_GEOM:
      is_int = false;
      for (int64_t e = 0; e < h.E_int; ++e) {
        const double row[8] = {h.P1[2 * e], h.P1[2 * e + 1], h.mu1[2 * e], h.mu1[2 * e + 1],
                               h.mu2[2 * e], h.mu2[2 * e + 1], h.gam[2 * e], h.gam[2 * e + 1]};
        dv.insert(dv.end(), row, row + 8);
      }
      break;
    case ARDG_MESH_BFACE_GHOST_NODES: {
      is_int = false;
      const int rotv[3][3] = {{2, 0, 1}, {0, 1, 2}, {1, 2, 0}};
      const RefOps& o = mesh->ro;
      for (int64_t b = 0; b < h.E_bdy; ++b) {
        const int64_t k = h.bk[b];
        const int f = h.bf[b];
        const int ia = h.etov[3 * k + rotv[f][1]], ib = h.etov[3 * k + rotv[f][2]];
        const double ax = h.vxy[2 * ia], ay = h.vxy[2 * ia + 1], bx = h.vxy[2 * ib], by = h.vxy[2 * ib + 1];
        // the ghost sub-triangle (P2, B, A) with P2 = A + B - P1
        const double p2x = ax + bx - h.bP1[2 * b], p2y = ay + by - h.bP1[2 * b + 1];
        for (int n = 0; n < o.Np; ++n) {
          const double l1 = -0.5 * (o.r[n] + o.s[n]), l2 = 0.5 * (o.r[n] + 1.0), l3 = 0.5 * (o.s[n] + 1.0);
          dv.push_back(l1 * p2x + l2 * bx + l3 * ax);
          dv.push_back(l1 * p2y + l2 * by + l3 * ay);
        }
      }
      break;
    }
    case ARDG_MESH_BFACE_GEOM:
      is_int = false;
      for (int64_t b = 0; b < h.E_bdy; ++b) {
        const double row[6] = {h.bP1[2 * b], h.bP1[2 * b + 1], h.bmu[2 * b], h.bmu[2 * b + 1],
                               h.bgam[2 * b], h.bgam[2 * b + 1]};
        dv.insert(dv.end(), row, row + 6);
      }
      break;
    default: return fail(ARDG_E_INVALID_ARG, "mesh_export: unknown selector");
  }
  const int64_t bytes = is_int ? (int64_t)(iv.size() * 4) : (int64_t)(dv.size() * 8);
  if (n_written) *n_written = is_int ? (int64_t)iv.size() : (int64_t)dv.size();
  if (!dst || cap < bytes) return fail(ARDG_E_INVALID_ARG, "mesh_export: buffer too small");
  if (bytes) std::memcpy(dst, is_int ? (const void*)iv.data() : (const void*)dv.data(), bytes);
  return ARDG_OK;
}

// Per face (interior edges, then boundary faces) the inverse metric of the
// enclosed parallelogram in the frame (P1, A, B) and sJ n1 = (t_y, -t_x) / 2
// for the edge vector t = B - A: the tensor-coefficient kernel forms
// physical gradients with them.
static ardg_status upload_face_metric(ardg_mesh mesh) {
  if (mesh->gp_dev || mesh->device < 0) return ARDG_OK;
  const HostMesh& h = mesh->hm;
  const int rotv[3][3] = {{2, 0, 1}, {0, 1, 2}, {1, 2, 0}};
  const int64_t E = h.E_int + h.E_bdy;
  std::vector<double4> gp(E);
  std::vector<double2> sn(E);
  auto face = [&](int64_t e, int64_t k, int f, double p1x, double p1y) {
    const int ia = h.etov[3 * k + rotv[f][1]], ib = h.etov[3 * k + rotv[f][2]];
    const double ax = h.vxy[2 * ia], ay = h.vxy[2 * ia + 1], bx = h.vxy[2 * ib], by = h.vxy[2 * ib + 1];
    const double xr = 0.5 * (ax - p1x), yr = 0.5 * (ay - p1y), xs = 0.5 * (bx - p1x), ys = 0.5 * (by - p1y);
    const double J = xr * ys - xs * yr;
    gp[e] = make_double4(ys / J, -xs / J, -yr / J, xr / J);
    sn[e] = make_double2(0.5 * (by - ay), -0.5 * (bx - ax));
  };
  for (int64_t e = 0; e < h.E_int; ++e) face(e, h.e1[e], h.f1[e], h.P1[2 * e], h.P1[2 * e + 1]);
  for (int64_t b = 0; b < h.E_bdy; ++b) face(h.E_int + b, h.bk[b], h.bf[b], h.bP1[2 * b], h.bP1[2 * b + 1]);
  DeviceGuard g(mesh->device);
  ardg_status s = upload(gp.data(), gp.size(), &mesh->gp_dev);
  if (s != ARDG_OK) return s;
  s = upload(sn.data(), sn.size(), &mesh->sn_dev);
  if (s != ARDG_OK) return s;
  mesh->dm.gp = mesh->gp_dev;
  mesh->dm.sn = mesh->sn_dev;
  return ARDG_OK;
}

static bool spd(double a, double b, double c) {
  return std::isfinite(a) && std::isfinite(b) && std::isfinite(c) && a > 0 && c > 0 && a * c - b * b > 0;
}

ardg_status ardg_mesh_set_diffusion(ardg_mesh mesh, int32_t mode, int32_t nfields, const double* D) {
  if (!mesh || !D) return fail(ARDG_E_INVALID_ARG, "set_diffusion: null argument");
  if (mode == ARDG_D_NODAL || mode == ARDG_D_SOLUTION) {
    if (nfields != 1) return fail(ARDG_E_INVALID_ARG, "set_diffusion: a tensor coefficient needs nfields == 1");
    const int64_t n = mode == ARDG_D_NODAL ? mesh->hm.K * mesh->ro.Np : 1;
    for (int64_t i = 0; i < n; ++i)
      if (!spd(D[3 * i], D[3 * i + 1], D[3 * i + 2]))
        return fail(ARDG_E_INVALID_ARG, "set_diffusion: every tensor (Dxx, Dxy, Dyy) must be symmetric positive definite");
    ardg_status s = upload_face_metric(mesh);
    if (s != ARDG_OK) return s;
    if (mode == ARDG_D_NODAL && mesh->device >= 0) {
      DeviceGuard g(mesh->device);
      if (mesh->Dnodal_dev) { (void)hipFree(mesh->Dnodal_dev); mesh->Dnodal_dev = nullptr; }
      s = upload(D, (size_t)(3 * n), &mesh->Dnodal_dev);
      if (s != ARDG_OK) return s;
      mesh->dm.Dnodal = mesh->Dnodal_dev;
    }
    if (mode == ARDG_D_SOLUTION)
      for (int i = 0; i < 3; ++i) mesh->dm.D0[i] = D[i];
    mesh->dm.dmode = mode == ARDG_D_NODAL ? DM_NODAL : DM_SOLUTION;
    mesh->nfields_D = 1;
    mesh->drop_graphs();
    return ARDG_OK;
  }
  if (mode == ARDG_D_CONST) {
    if (nfields < 1 || nfields > kMaxFields) return fail(ARDG_E_INVALID_ARG, "set_diffusion: nfields");
    for (int f = 0; f < nfields; ++f)
      if (!(std::isfinite(D[f]) && D[f] > 0)) return fail(ARDG_E_INVALID_ARG, "set_diffusion: D must be finite > 0");
    for (int f = 0; f < kMaxFields; ++f) mesh->dm.Dfield[f] = D[std::min(f, nfields - 1)];
    if (mesh->device >= 0) {
      DeviceGuard g(mesh->device);
      HIP_TRY(hipMemcpy(mesh->Dfield_dev, mesh->dm.Dfield, sizeof(mesh->dm.Dfield), hipMemcpyHostToDevice),
              "set_diffusion: hipMemcpy");
    }
    mesh->dm.dmode = DM_CONST;
    mesh->nfields_D = nfields;
  } else if (mode == ARDG_D_ELEMENT || mode == ARDG_D_ELEMENT_ALG2) {
    if (nfields != 1) return fail(ARDG_E_INVALID_ARG, "set_diffusion: element-wise D needs nfields == 1");
    const int64_t K = mesh->hm.K;
    for (int64_t k = 0; k < K; ++k)
      if (!(std::isfinite(D[k]) && D[k] > 0)) return fail(ARDG_E_INVALID_ARG, "set_diffusion: D must be finite > 0");
    if (mesh->device >= 0) {
      DeviceGuard g(mesh->device);
      if (mesh->Delem_dev) { (void)hipFree(mesh->Delem_dev); mesh->Delem_dev = nullptr; }
      ardg_status s = upload(D, (size_t)K, &mesh->Delem_dev);
      if (s != ARDG_OK) return s;
      mesh->dm.Delem = mesh->Delem_dev;
    }
    mesh->dm.dmode = mode == ARDG_D_ELEMENT ? DM_ALG1 : DM_ALG2;
    mesh->nfields_D = 1;
  } else {
    return fail(ARDG_E_INVALID_ARG, "set_diffusion: unknown mode");
  }
  mesh->drop_graphs();
  return ARDG_OK;
}

ardg_status ardg_mesh_set_velocity(ardg_mesh mesh, int32_t kind, const double* params) {
  if (!mesh) return fail(ARDG_E_INVALID_ARG, "set_velocity: null handle");
  if (kind == ARDG_VEL_NONE) {
    mesh->dm.conv = 0;
    mesh->drop_graphs();
    return ARDG_OK;
  }
  if (kind != ARDG_VEL_AFFINE || !params) return fail(ARDG_E_INVALID_ARG, "set_velocity: bad kind or params");
  for (int i = 0; i < 6; ++i)
    if (!std::isfinite(params[i])) return fail(ARDG_E_INVALID_ARG, "set_velocity: non-finite parameter");
  const HostMesh& h = mesh->hm;
  const int rotv[3][3] = {{2, 0, 1}, {0, 1, 2}, {1, 2, 0}};
  auto vel = [&](double x, double y, double* v) {
    v[0] = params[0] + params[2] * x + params[3] * y;
    v[1] = params[1] + params[4] * x + params[5] * y;
  };
  std::vector<double2> vn(h.E_int + h.E_bdy);
  auto edge_vn = [&](int64_t k, int f) {
    const int a = h.etov[3 * k + rotv[f][1]], b = h.etov[3 * k + rotv[f][2]];
    const double ax = h.vxy[2 * a], ay = h.vxy[2 * a + 1], bx = h.vxy[2 * b], by = h.vxy[2 * b + 1];
    // sJ n = (ty, -tx) / 2 with sJ = |edge| / 2: the stored n.v carries the
    // edge's surface factor like gamma
    const double tx = bx - ax, ty = by - ay;
    const double nx = 0.5 * ty, ny = -0.5 * tx;
    double va[2], vb[2];
    vel(ax, ay, va);
    vel(bx, by, vb);
    return make_double2(nx * va[0] + ny * va[1], nx * vb[0] + ny * vb[1]);
  };
  for (int64_t e = 0; e < h.E_int; ++e) vn[e] = edge_vn(h.e1[e], h.f1[e]);
  for (int64_t b = 0; b < h.E_bdy; ++b) vn[h.E_int + b] = edge_vn(h.bk[b], h.bf[b]);
  if (mesh->device >= 0) {
    DeviceGuard g(mesh->device);
    if (mesh->vn_dev) { (void)hipFree(mesh->vn_dev); mesh->vn_dev = nullptr; }
    ardg_status s = upload(vn.data(), vn.size(), &mesh->vn_dev);
    if (s != ARDG_OK) return s;
    mesh->dm.vn = mesh->vn_dev;
  }
  for (int i = 0; i < 6; ++i) mesh->dm.vel[i] = params[i];
  mesh->dm.conv = 1;
  mesh->drop_graphs();
  return ARDG_OK;
}

ardg_status ardg_mesh_set_boundary_data(ardg_mesh mesh, int32_t nfields, int32_t nt, double t_a, double t_b,
                                        const double* coeffs) {
  if (!mesh) return fail(ARDG_E_INVALID_ARG, "set_boundary_data: null handle");
  if (nt == 0) {
    mesh->dm.ghost = nullptr;
    mesh->ghost_nt = mesh->ghost_nf = 0;
    mesh->drop_graphs();
    return ARDG_OK;
  }
  if (nt < 1 || nt > 64) return fail(ARDG_E_INVALID_ARG, "set_boundary_data: nt must be in 1..64 (0 clears)");
  if (nfields < 1 || nfields > kMaxFields) return fail(ARDG_E_INVALID_ARG, "set_boundary_data: nfields");
  if (!coeffs) return fail(ARDG_E_INVALID_ARG, "set_boundary_data: null coefficients");
  if (!(std::isfinite(t_a) && std::isfinite(t_b) && t_b > t_a))
    return fail(ARDG_E_INVALID_ARG, "set_boundary_data: need finite t_a < t_b");
  const size_t nv = (size_t)nfields * mesh->hm.E_bdy * mesh->ro.Np;
  for (size_t i = 0; i < nv * nt; ++i)
    if (!std::isfinite(coeffs[i])) return fail(ARDG_E_INVALID_ARG, "set_boundary_data: non-finite coefficient");
  mesh->drop_graphs();
  if (mesh->device >= 0) {
    DeviceGuard g(mesh->device);
    if (mesh->ghost_coef) (void)hipFree(mesh->ghost_coef);
    if (mesh->ghost_val) (void)hipFree(mesh->ghost_val);
    mesh->ghost_coef = mesh->ghost_val = nullptr;
    mesh->dm.ghost = nullptr;
    ardg_status s = upload(coeffs, nv * nt, &mesh->ghost_coef);
    if (s != ARDG_OK) return s;
    if (nv) {
      hipError_t e = hipMalloc((void**)&mesh->ghost_val, nv * sizeof(double));
      if (e != hipSuccess) return fail(ARDG_E_OOM, "set_boundary_data: allocation failed");
    }
    if (!mesh->tdev) {
      hipError_t e = hipMalloc((void**)&mesh->tdev, sizeof(double));
      if (e != hipSuccess) return fail(ARDG_E_OOM, "set_boundary_data: allocation failed");
    }
    // E_bdy == 0: a non-null marker still routes the launches through the
    // (empty) evaluation; no boundary face reads it
    mesh->dm.ghost = mesh->ghost_val ? mesh->ghost_val : mesh->tdev;
  }
  mesh->ghost_nt = nt;
  mesh->ghost_nf = nfields;
  mesh->ghost_ta = t_a;
  mesh->ghost_tb = t_b;
  return ARDG_OK;
}

ardg_status ardg_mesh_set_navier_stokes(ardg_mesh mesh, int32_t law, const double* params) {
  if (!mesh) return fail(ARDG_E_INVALID_ARG, "set_navier_stokes: null handle");
  if (law == ARDG_NS_OFF) {
    mesh->dm.ns = NS_OFF;
    mesh->drop_graphs();
    return ARDG_OK;
  }
  if (law != ARDG_NS_SUTHERLAND && law != ARDG_NS_CONSTANT_MU)
    return fail(ARDG_E_INVALID_ARG, "set_navier_stokes: unknown law");
  if (!params) return fail(ARDG_E_INVALID_ARG, "set_navier_stokes: null params");
  for (int i = 0; i < 6; ++i)
    if (!std::isfinite(params[i])) return fail(ARDG_E_INVALID_ARG, "set_navier_stokes: non-finite parameter");
  const double gamma = params[0], R = params[1], Pr = params[2], mu_ref = params[3], T_ref = params[4],
               S = params[5];
  if (!(gamma > 1.0 && R > 0.0 && Pr > 0.0 && mu_ref >= 0.0 && T_ref > 0.0 && S >= 0.0))
    return fail(ARDG_E_INVALID_ARG, "set_navier_stokes: need gamma > 1, R, Pr, T_ref > 0 and mu_ref, S >= 0");
  ardg_status s = upload_face_metric(mesh);
  if (s != ARDG_OK) return s;
  for (int i = 0; i < 6; ++i) mesh->dm.gas[i] = params[i];
  mesh->dm.ns = law == ARDG_NS_SUTHERLAND ? NS_SUTHERLAND : NS_CONSTANT_MU;
  mesh->drop_graphs();
  return ARDG_OK;
}

// Exterior state at time toff (+ the device step time when tbase is used).
static hipError_t ghost_eval(ardg_mesh mesh, int nfields, bool use_tbase, double toff, hipStream_t st) {
  if (!mesh->dm.ghost) return hipSuccess;
  const int64_t n = (int64_t)nfields * mesh->hm.E_bdy * mesh->ro.Np;
  return launch_ghost_eval(mesh->ghost_coef, mesh->ghost_val, n, mesh->ghost_nt, mesh->ghost_ta, mesh->ghost_tb,
                           use_tbase ? mesh->tdev : nullptr, toff, st);
}

static bool time_in_range(ardg_mesh mesh, double t0, double t1) {
  if (!mesh->dm.ghost) return true;
  const double tol = 1e-9 * std::max(1.0, std::fabs(mesh->ghost_tb - mesh->ghost_ta));
  return t0 >= mesh->ghost_ta - tol && t1 <= mesh->ghost_tb + tol;
}

static ardg_status check_compute(ardg_mesh mesh, int32_t precision, int32_t nfields) {
  if (!mesh) return fail(ARDG_E_INVALID_ARG, "null mesh");
  if (mesh->device < 0) return fail(ARDG_E_INVALID_ARG, "mesh was created host-only (device -1)");
  if (precision != ARDG_FP64 && precision != ARDG_FP32 && precision != ARDG_BF16X3)
    return fail(ARDG_E_UNSUPPORTED, "unknown precision");
  if (nfields < 1 || nfields > kMaxFields) return fail(ARDG_E_INVALID_ARG, "nfields out of range");
  if (mesh->dm.ns != NS_OFF) {
    if (nfields != 4) return fail(ARDG_E_INVALID_ARG, "the Navier-Stokes system has four fields");
    if (precision == ARDG_BF16X3)
      return fail(ARDG_E_UNSUPPORTED, "the Navier-Stokes system has no split-BF16 form (FP64 and FP32 only)");
    if (!mesh->dm.ghost || mesh->ghost_nf < 4)
      return fail(ARDG_E_INVALID_ARG, "the Navier-Stokes system needs the exterior state of all four fields "
                                      "(ardg_mesh_set_boundary_data)");
    return ARDG_OK;
  }
  if (mesh->dm.dmode != DM_CONST && nfields != 1) return fail(ARDG_E_INVALID_ARG, "element-wise D is for one field");
  if ((mesh->dm.dmode == DM_NODAL || mesh->dm.dmode == DM_SOLUTION) && precision == ARDG_BF16X3)
    return fail(ARDG_E_UNSUPPORTED, "a tensor coefficient has no split-BF16 form (FP64 and FP32 only)");
  if (mesh->dm.dmode == DM_CONST && nfields > mesh->nfields_D && mesh->nfields_D != 1)
    return fail(ARDG_E_INVALID_ARG, "more fields than diffusion coefficients");
  if (mesh->dm.ghost && nfields > mesh->ghost_nf)
    return fail(ARDG_E_INVALID_ARG, "more fields than the boundary data was given for");
  return ARDG_OK;
}

static ardg_status ensure_scratch(ardg_mesh mesh, size_t bytes) {
  if (mesh->flux_scratch_bytes >= bytes) return ARDG_OK;
  if (mesh->flux_scratch) (void)hipFree(mesh->flux_scratch);
  mesh->flux_scratch = nullptr;
  mesh->flux_scratch_bytes = 0;
  hipError_t e = hipMalloc(&mesh->flux_scratch, bytes);
  if (e != hipSuccess) return fail(ARDG_E_OOM, "flux scratch allocation failed");
  mesh->flux_scratch_bytes = bytes;
  return ARDG_OK;
}

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

ardg_status ardg_mesh_set_kernels(ardg_mesh mesh, int32_t edge_kernel) {
  if (!mesh) return fail(ARDG_E_INVALID_ARG, "set_kernels: null handle");
  if (edge_kernel < ARDG_EDGE_AUTO || edge_kernel > ARDG_EDGE_FIELDS)
    return fail(ARDG_E_INVALID_ARG, "set_kernels: unknown edge kernel");
  mesh->dm.edge_kernel = edge_kernel;
  mesh->drop_graphs();
  return ARDG_OK;
}

ardg_status ardg_edge_flux_eval(ardg_mesh mesh, int32_t precision, int32_t nfields, const void* u_dev,
                                void* flux_dev, double t, void* hip_stream) {
  ardg_status s = check_compute(mesh, precision, nfields);
  if (s != ARDG_OK) return s;
  if (!u_dev || !flux_dev) return fail(ARDG_E_INVALID_ARG, "edge_flux_eval: null buffer");
  if (!time_in_range(mesh, t, t)) return fail(ARDG_E_INVALID_ARG, "edge_flux_eval: t outside the boundary data's interval");
  DeviceGuard g(mesh->device);
  hipStream_t st = (hipStream_t)hip_stream;
  HIP_TRY(ghost_eval(mesh, nfields, false, t, st), "boundary data launch");
  HIP_TRY(launch_edge_flux(mesh->dm, precision, nfields, u_dev, flux_dev, st), "edge flux launch");
  return ARDG_OK;
}

ardg_status ardg_rhs_eval(ardg_mesh mesh, int32_t precision, int32_t nfields, const void* u_dev,
                          void* rhs_dev, double t, void* hip_stream) {
  ardg_status s = check_compute(mesh, precision, nfields);
  if (s != ARDG_OK) return s;
  if (!u_dev || !rhs_dev) return fail(ARDG_E_INVALID_ARG, "rhs_eval: null buffer");
  if (!time_in_range(mesh, t, t)) return fail(ARDG_E_INVALID_ARG, "rhs_eval: t outside the boundary data's interval");
  DeviceGuard g(mesh->device);
  const size_t ts = precision == ARDG_FP64 ? 8 : 4;
  const size_t fb = align256((size_t)nfields * (mesh->hm.E_int + mesh->hm.E_bdy) * mesh->ro.Nfp * ts);
  s = ensure_scratch(mesh, fb);
  if (s != ARDG_OK) return s;
  hipStream_t st = (hipStream_t)hip_stream;
  void* flux = mesh->flux_scratch;
  HIP_TRY(ghost_eval(mesh, nfields, false, t, st), "boundary data launch");
  HIP_TRY(launch_edge_flux(mesh->dm, precision, nfields, u_dev, flux, st), "edge flux launch");
  Epilogue epi;
  epi.kind = EPI_RHS;
  epi.rhs_out = rhs_dev;
  HIP_TRY(launch_element(mesh->dm, precision, nfields, u_dev, flux, epi, st), "element launch");
  return ARDG_OK;
}

ardg_status ardg_rhs_eval_noalloc(ardg_mesh mesh, int32_t precision, int32_t nfields, const void* u_dev,
                                  void* rhs_dev, double t, void* hip_stream) {
  ardg_status s = check_compute(mesh, precision, nfields);
  if (s != ARDG_OK) return s;
  if (!u_dev || !rhs_dev) return fail(ARDG_E_INVALID_ARG, "rhs_eval_noalloc: null buffer");
  if (!time_in_range(mesh, t, t))
    return fail(ARDG_E_INVALID_ARG, "rhs_eval_noalloc: t outside the boundary data's interval");
  const size_t ts = precision == ARDG_FP64 ? 8 : 4;
  const size_t fb = (size_t)nfields * (mesh->hm.E_int + mesh->hm.E_bdy) * mesh->ro.Nfp * ts;
  if (fb > kNoallocScratchBytes)
    return fail(ARDG_E_INVALID_ARG, "rhs_eval_noalloc: the edge fluxes need " + std::to_string(fb) +
                                        " bytes, more than the " + std::to_string(kNoallocScratchBytes) +
                                        "-byte scratch array");
  DeviceGuard g(mesh->device);
  if (!g.ok) return fail(ARDG_E_HIP, "rhs_eval_noalloc: hipSetDevice failed");
  void* flux = nullptr;
  HIP_TRY(noalloc_scratch(mesh->device, &flux), "rhs_eval_noalloc: scratch address");
  hipStream_t st = (hipStream_t)hip_stream;
  HIP_TRY(ghost_eval(mesh, nfields, false, t, st), "boundary data launch");
  HIP_TRY(launch_edge_flux(mesh->dm, precision, nfields, u_dev, flux, st), "edge flux launch");
  Epilogue epi;
  epi.kind = EPI_RHS;
  epi.rhs_out = rhs_dev;
  HIP_TRY(launch_element(mesh->dm, precision, nfields, u_dev, flux, epi, st), "element launch");
  return ARDG_OK;
}

struct Work {
  double* acc;
  void* v;
  void* flux;
};

static void work_layout(ardg_mesh mesh, int precision, int nfields, size_t* total, Work* w, void* base) {
  const size_t ts = precision == ARDG_FP64 ? 8 : 4;
  const size_t n = (size_t)nfields * mesh->hm.K * mesh->ro.Np;
  const size_t nf = (size_t)nfields * (mesh->hm.E_int + mesh->hm.E_bdy) * mesh->ro.Nfp;
  const size_t b_acc = align256(n * 8), b_v = align256(n * ts), b_f = align256(nf * ts);
  if (total) *total = b_acc + b_v + b_f;
  if (w) {
    char* p = (char*)base;
    w->acc = (double*)p;
    w->v = p + b_acc;
    w->flux = p + b_acc + b_v;
  }
}

ardg_status ardg_rk_workspace_bytes(ardg_mesh mesh, int32_t scheme, int32_t precision, int32_t nfields,
                                    int64_t* bytes) {
  if (!mesh || !bytes) return fail(ARDG_E_INVALID_ARG, "rk_workspace_bytes: null argument");
  if (scheme != ARDG_RK4 && scheme != ARDG_LSERK54) return fail(ARDG_E_INVALID_ARG, "unknown scheme");
  if (precision != ARDG_FP64 && precision != ARDG_FP32 && precision != ARDG_BF16X3)
    return fail(ARDG_E_UNSUPPORTED, "unknown precision");
  size_t t = 0;
  work_layout(mesh, precision, nfields, &t, nullptr, nullptr);
  *bytes = (int64_t)t;
  return ARDG_OK;
}

// Carpenter & Kennedy (1994) five-stage fourth-order 2N-storage coefficients.
static const double kLsA[5] = {0.0, -567301805773.0 / 1357537059087.0,
                               -2404267990393.0 / 2016746695238.0,
                               -3550918686646.0 / 2091501179385.0,
                               -1275806237668.0 / 842570457699.0};
static const double kLsB[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                               1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                               2277821191437.0 / 14882151754819.0};

// Stage input and next-stage output of stage s.  FP64 stages read the state
// itself at RK4 stage 0 and at every LSERK stage and need no stage vector
// after the last RK4 stage; everything else goes through the stage vector v
// (FP32 copies in the reduced precisions).
struct StageIO {
  const void* vin;
  void* vnext;
};

static StageIO stage_io(int scheme, bool f64, int s, double* u, void* v) {
  StageIO io;
  io.vin = (f64 && (scheme == ARDG_LSERK54 || s == 0)) ? (const void*)u : v;
  if (scheme == ARDG_RK4)
    io.vnext = (s < 3 || !f64) ? v : nullptr;
  else
    io.vnext = f64 ? nullptr : v;
  return io;
}

// Stage time offsets c_s (in units of dt): classic RK4 0, 1/2, 1/2, 1; the
// low-storage scheme's from its coefficients (the stage values of
// du/dt = 1, integrated exactly: r_s = A_s r_{s-1} + 1, c_{s+1} = c_s + B_s r_s).
static double stage_time(int scheme, int s) {
  if (scheme == ARDG_RK4) return s == 0 ? 0.0 : (s == 3 ? 1.0 : 0.5);
  double c = 0.0, r = 0.0;
  for (int j = 0; j < s; ++j) {
    r = kLsA[j] * r + 1.0;
    c += kLsB[j] * r;
  }
  return c;
}

static void stage_epilogue(int scheme, int s, Epilogue& epi) {
  epi.stage = s;
  if (scheme == ARDG_RK4) {
    epi.kind = EPI_RK4;
  } else {
    epi.kind = EPI_LSERK;
    epi.a = kLsA[s];
    epi.b = kLsB[s];
  }
}

// First stage input from the FP64 state: an FP32 copy (nothing for FP64).
static hipError_t stage_vector_init(ardg_mesh mesh, int precision, int nfields, const double* u, void* v,
                                    hipStream_t st) {
  const int64_t n = (int64_t)nfields * mesh->hm.K * mesh->ro.Np;
  if (precision != ARDG_FP64) return launch_to_f32(u, (float*)v, n, st);
  return hipSuccess;
}

static hipError_t enqueue_steps(ardg_mesh mesh, int scheme, int precision, int nfields, double* u,
                                const Work& w, double dt, int nsteps, hipStream_t st) {
  const bool f64 = precision == ARDG_FP64;
  hipError_t e = stage_vector_init(mesh, precision, nfields, u, w.v, st);
  if (e != hipSuccess) return e;
  Epilogue epi;
  epi.u = u;
  epi.acc = w.acc;
  epi.dt = dt;
  const int nst = scheme == ARDG_RK4 ? 4 : 5;
  for (int step = 0; step < nsteps; ++step) {
    for (int s = 0; s < nst; ++s) {
      const StageIO io = stage_io(scheme, f64, s, u, w.v);
      e = ghost_eval(mesh, nfields, true, stage_time(scheme, s) * dt, st);
      if (e != hipSuccess) return e;
      e = launch_edge_flux(mesh->dm, precision, nfields, io.vin, w.flux, st);
      if (e != hipSuccess) return e;
      stage_epilogue(scheme, s, epi);
      epi.vnext = io.vnext;
      e = launch_element(mesh->dm, precision, nfields, io.vin, w.flux, epi, st);
      if (e != hipSuccess) return e;
    }
    if (mesh->dm.ghost) {
      e = launch_advance_time(mesh->tdev, dt, st);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

// The instantiated graph of `nsteps` steps for these arguments, captured on
// first use and cached on the mesh (a bounded cache).
static ardg_status step_graph(ardg_mesh mesh, int scheme, int precision, int nfields, double* u_dev,
                              void* work_dev, double dt, int nsteps, hipGraphExec_t* out) {
  Work w;
  work_layout(mesh, precision, nfields, nullptr, &w, work_dev);
  GraphKey key{scheme, precision, nfields, nsteps, u_dev, work_dev, dt, mesh->version};
  auto it = mesh->graphs.find(key);
  if (it == mesh->graphs.end()) {
    if (!mesh->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&mesh->cap_stream, hipStreamNonBlocking), "hipStreamCreate");
    HIP_TRY(hipStreamBeginCapture(mesh->cap_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    hipError_t e = enqueue_steps(mesh, scheme, precision, nfields, u_dev, w, dt, nsteps, mesh->cap_stream);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(mesh->cap_stream, &graph);
    if (e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return hip_fail(e, "rk_step: launch during capture");
    }
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    hipError_t e3 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) return hip_fail(e3, "hipGraphInstantiate");
    if (mesh->graphs.size() >= 8) {
      mesh->drop_graphs();
      key.version = mesh->version;
    }
    it = mesh->graphs.emplace(key, exec).first;
  }
  *out = it->second;
  return ARDG_OK;
}

// The graphs that run nsteps steps: *full of min(nsteps, kGraphSteps) steps,
// replayed nsteps / that many times, and *rem (null if none) of the
// remainder.  If capturing one of them evicted the cache, the other is
// captured again (the cache then holds room for both).
static ardg_status step_graphs(ardg_mesh mesh, int scheme, int precision, int nfields, double* u_dev,
                               void* work_dev, double dt, int nsteps, hipGraphExec_t* full, hipGraphExec_t* rem) {
  const int chunk = std::min<int>(nsteps, kGraphSteps);
  const int nrem = nsteps % chunk;
  *rem = nullptr;
  ardg_status s = ARDG_OK;
  if (nrem) {
    s = step_graph(mesh, scheme, precision, nfields, u_dev, work_dev, dt, nrem, rem);
    if (s != ARDG_OK) return s;
  }
  const uint64_t v0 = mesh->version;
  s = step_graph(mesh, scheme, precision, nfields, u_dev, work_dev, dt, chunk, full);
  if (s != ARDG_OK || !nrem || mesh->version == v0) return s;
  return step_graph(mesh, scheme, precision, nfields, u_dev, work_dev, dt, nrem, rem);
}

ardg_status ardg_rk_step(ardg_mesh mesh, int32_t scheme, int32_t precision, int32_t nfields, double* u_dev,
                         void* work_dev, double t0, double dt, int32_t nsteps, void* hip_stream) {
  ardg_status s = check_compute(mesh, precision, nfields);
  if (s != ARDG_OK) return s;
  if (scheme != ARDG_RK4 && scheme != ARDG_LSERK54) return fail(ARDG_E_INVALID_ARG, "unknown scheme");
  if (!u_dev || !work_dev) return fail(ARDG_E_INVALID_ARG, "rk_step: null buffer");
  if (((uintptr_t)work_dev & 255) != 0) return fail(ARDG_E_INVALID_ARG, "rk_step: work_dev not 256-byte aligned");
  if (nsteps < 0 || !std::isfinite(dt)) return fail(ARDG_E_INVALID_ARG, "rk_step: bad nsteps or dt");
  if (nsteps == 0) return ARDG_OK;
  if (!time_in_range(mesh, std::min(t0, t0 + nsteps * dt), std::max(t0, t0 + nsteps * dt)))
    return fail(ARDG_E_INVALID_ARG, "rk_step: the steps leave the boundary data's time interval");
  DeviceGuard g(mesh->device);
  hipGraphExec_t ex_full = nullptr, ex_rem = nullptr;
  s = step_graphs(mesh, scheme, precision, nfields, u_dev, work_dev, dt, nsteps, &ex_full, &ex_rem);
  if (s != ARDG_OK) return s;
  if (mesh->dm.ghost) HIP_TRY(launch_set_time(mesh->tdev, t0, (hipStream_t)hip_stream), "time launch");
  const int chunk = std::min<int>(nsteps, kGraphSteps);
  for (int i = 0; i < nsteps / chunk; ++i)
    HIP_TRY(hipGraphLaunch(ex_full, (hipStream_t)hip_stream), "hipGraphLaunch");
  if (ex_rem) HIP_TRY(hipGraphLaunch(ex_rem, (hipStream_t)hip_stream), "hipGraphLaunch");
  return ARDG_OK;
}

ardg_status ardg_rk_prepare(ardg_mesh mesh, int32_t scheme, int32_t precision, int32_t nfields, double* u_dev,
                            void* work_dev, double dt, int32_t nsteps) {
  ardg_status s = check_compute(mesh, precision, nfields);
  if (s != ARDG_OK) return s;
  if (scheme != ARDG_RK4 && scheme != ARDG_LSERK54) return fail(ARDG_E_INVALID_ARG, "unknown scheme");
  if (!u_dev || !work_dev) return fail(ARDG_E_INVALID_ARG, "rk_prepare: null buffer");
  if (((uintptr_t)work_dev & 255) != 0) return fail(ARDG_E_INVALID_ARG, "rk_prepare: work_dev not 256-byte aligned");
  if (nsteps < 1 || !std::isfinite(dt)) return fail(ARDG_E_INVALID_ARG, "rk_prepare: bad nsteps or dt");
  DeviceGuard g(mesh->device);
  hipGraphExec_t ex_full = nullptr, ex_rem = nullptr;
  return step_graphs(mesh, scheme, precision, nfields, u_dev, work_dev, dt, nsteps, &ex_full, &ex_rem);
}

// One graph of `reps` stages of the step sequence (edge kernel + element
// kernel each), or of the element kernels alone (with_edge false).
static hipError_t capture_stages(ardg_mesh mesh, int scheme, int precision, int nfields, double* u_dev,
                                 const Work& w, double dt, int reps, bool with_edge, hipGraphExec_t* out) {
  const bool f64 = precision == ARDG_FP64;
  const int nst = scheme == ARDG_RK4 ? 4 : 5;
  hipStream_t cs = mesh->cap_stream;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  hipError_t ec = stage_vector_init(mesh, precision, nfields, u_dev, w.v, cs);
  Epilogue epi;
  epi.u = u_dev;
  epi.acc = w.acc;
  epi.dt = dt;
  for (int r = 0; r < reps && ec == hipSuccess; ++r) {
    const int sidx = r % nst;
    const StageIO io = stage_io(scheme, f64, sidx, u_dev, w.v);
    stage_epilogue(scheme, sidx, epi);
    epi.vnext = io.vnext;
    if (with_edge) ec = ghost_eval(mesh, nfields, false, 0.0 + stage_time(scheme, sidx) * dt, cs);
    if (with_edge && ec == hipSuccess) ec = launch_edge_flux(mesh->dm, precision, nfields, io.vin, w.flux, cs);
    if (ec == hipSuccess) ec = launch_element(mesh->dm, precision, nfields, io.vin, w.flux, epi, cs);
  }
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(cs, &graph);
  if (ec != hipSuccess) e = ec;
  if (e == hipSuccess) e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  return e;
}

ardg_status ardg_stage_timing(ardg_mesh mesh, int32_t scheme, int32_t precision, int32_t nfields,
                              double* u_dev, void* work_dev, double dt, int32_t reps, void* hip_stream,
                              float* out_ms) {
  ardg_status s = check_compute(mesh, precision, nfields);
  if (s != ARDG_OK) return s;
  if (scheme != ARDG_RK4 && scheme != ARDG_LSERK54) return fail(ARDG_E_INVALID_ARG, "unknown scheme");
  const int nst = scheme == ARDG_RK4 ? 4 : 5;
  if (!u_dev || !work_dev || !out_ms || reps <= 0 || reps % nst != 0)
    return fail(ARDG_E_INVALID_ARG, "stage_timing: bad arguments (reps must be a multiple of the stage count)");
  if (((uintptr_t)work_dev & 255) != 0) return fail(ARDG_E_INVALID_ARG, "stage_timing: work_dev not 256-byte aligned");
  DeviceGuard g(mesh->device);
  Work w;
  work_layout(mesh, precision, nfields, nullptr, &w, work_dev);
  hipStream_t st = (hipStream_t)hip_stream;
  if (!mesh->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&mesh->cap_stream, hipStreamNonBlocking), "hipStreamCreate");
  // graph A: the stage sequence; graph B: its element kernels alone.  Events
  // on the launch stream bracket each replay: element = B / reps, edge =
  // (A - B) / reps (kernels in a graph follow each other without host gaps)
  hipGraphExec_t ga = nullptr, gb = nullptr;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  hipError_t e = capture_stages(mesh, scheme, precision, nfields, u_dev, w, dt, reps, true, &ga);
  if (e == hipSuccess) e = capture_stages(mesh, scheme, precision, nfields, u_dev, w, dt, reps, false, &gb);
  for (auto& x : ev)
    if (e == hipSuccess) e = hipEventCreate(&x);
  // one replay of each first (warm-up), then the timed replays
  if (e == hipSuccess) e = hipGraphLaunch(ga, st);
  if (e == hipSuccess) e = hipGraphLaunch(gb, st);
  if (e == hipSuccess) e = hipEventRecord(ev[0], st);
  if (e == hipSuccess) e = hipGraphLaunch(ga, st);
  if (e == hipSuccess) e = hipEventRecord(ev[1], st);
  if (e == hipSuccess) e = hipEventRecord(ev[2], st);
  if (e == hipSuccess) e = hipGraphLaunch(gb, st);
  if (e == hipSuccess) e = hipEventRecord(ev[3], st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  float ta = 0.f, tb = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ta, ev[0], ev[1]);
  if (e == hipSuccess) e = hipEventElapsedTime(&tb, ev[2], ev[3]);
  if (ga) (void)hipGraphExecDestroy(ga);
  if (gb) (void)hipGraphExecDestroy(gb);
  for (auto& x : ev)
    if (x) (void)hipEventDestroy(x);
  if (e != hipSuccess) return hip_fail(e, "stage_timing");
  out_ms[0] = (ta - tb) / reps;
  out_ms[1] = tb / reps;
  return ARDG_OK;
}

ardg_status ardg_check(ardg_mesh mesh, int32_t nfields, const double* u_dev, void* hip_stream) {
  if (!mesh || !u_dev) return fail(ARDG_E_INVALID_ARG, "check: null argument");
  if (mesh->device < 0) return fail(ARDG_E_INVALID_ARG, "check: host-only mesh");
  if (nfields < 1 || nfields > kMaxFields) return fail(ARDG_E_INVALID_ARG, "check: nfields");
  DeviceGuard g(mesh->device);
  hipStream_t st = (hipStream_t)hip_stream;
  int* cnt = nullptr;
  HIP_TRY(hipMalloc(&cnt, sizeof(int)), "hipMalloc");
  hipError_t e = hipMemsetAsync(cnt, 0, sizeof(int), st);
  if (e == hipSuccess) e = launch_nonfinite(u_dev, (int64_t)nfields * mesh->hm.K * mesh->ro.Np, cnt, st);
  int host = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&host, cnt, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(cnt);
  if (e != hipSuccess) return hip_fail(e, "check");
  if (host) return fail(ARDG_E_NONFINITE, "check: " + std::to_string(host) + " non-finite values");
  return ARDG_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batching
// ---------------------------------------------------------------------------

namespace {

struct Tiles {
  int edge_tile = 256, elem_tile = 256, grid_mult = 4;
};

struct GroupItems {
  int tile_e = 0, tile_l = 0;
  std::vector<int2> eitems, litems;
  int2* d_eitems = nullptr;
  int2* d_litems = nullptr;
};

struct BatchGroup {
  int N = 0;
  std::vector<int> probs;           // problem indices, largest first
  GroupItems items[2];              // per precision (0: FP64, 1: FP32)
  Tiles tiles[2];
  bool tuned[2] = {false, false};
};

}  // namespace

struct ardg_batch_s {
  int device = -1;
  int ncu = 0;
  std::string arch;
  std::vector<ardg_mesh> meshes;
  std::string cache;
  std::vector<BatchGroup> groups;
  std::vector<BatchProb> hprobs;
  BatchProb* dprobs = nullptr;
  uint64_t version = 0;
  hipStream_t cap_stream = nullptr;
  std::map<GraphKey, hipGraphExec_t> graphs;
  ~ardg_batch_s() {
    DeviceGuard g(device);
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (auto& gr : groups)
      for (auto& it : gr.items) {
        if (it.d_eitems) (void)hipFree(it.d_eitems);
        if (it.d_litems) (void)hipFree(it.d_litems);
      }
    if (dprobs) (void)hipFree(dprobs);
  }
  void drop_graphs() {
    // earlier launches of these graphs may still run
    (void)hipDeviceSynchronize();
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    graphs.clear();
    ++version;
  }
};

namespace {

void batch_layout(ardg_batch b, int precision, std::vector<size_t>* offs, size_t* total) {
  const size_t ts = precision == ARDG_FP64 ? 8 : 4;
  size_t off = 0;
  if (offs) offs->clear();
  for (ardg_mesh m : b->meshes) {
    const size_t n = (size_t)m->hm.K * m->ro.Np;
    const size_t nf = (size_t)(m->hm.E_int + m->hm.E_bdy) * m->ro.Nfp;
    const size_t a = align256(n * 8), v = align256(n * ts), f = align256(nf * ts);
    if (offs) {
      offs->push_back(off);
      offs->push_back(off + a);
      offs->push_back(off + a + v);
    }
    off += a + v + f;
  }
  if (total) *total = off;
}

ardg_status build_items(ardg_batch b, BatchGroup& g, int pi, int tile_e, int tile_l) {
  GroupItems& it = g.items[pi];
  if (it.tile_e == tile_e && it.tile_l == tile_l && it.d_eitems) return ARDG_OK;
  it.eitems.clear();
  it.litems.clear();
  // tile code 0: side-split edge tiles of 64 interior edges plus boundary
  // tiles of 128 faces (negative index), and 64-element MFMA tiles
  for (int p : g.probs) {
    ardg_mesh m = b->meshes[p];
    const int64_t E = m->hm.E_int + m->hm.E_bdy, K = m->hm.K;
    if (tile_e == 0) {
      for (int64_t t = 0; t * 64 < m->hm.E_int; ++t) it.eitems.push_back(make_int2(p, (int)t));
      for (int64_t t = 0; t * 128 < m->hm.E_bdy; ++t) it.eitems.push_back(make_int2(p, (int)(-1 - t)));
    } else {
      for (int64_t t = 0; t * tile_e < E; ++t) it.eitems.push_back(make_int2(p, (int)t));
    }
    const int tl = tile_l == 0 ? 64 : tile_l;
    for (int64_t t = 0; t * tl < K; ++t) it.litems.push_back(make_int2(p, (int)t));
  }
  if (it.d_eitems) (void)hipFree(it.d_eitems);
  if (it.d_litems) (void)hipFree(it.d_litems);
  it.d_eitems = it.d_litems = nullptr;
  ardg_status s = upload(it.eitems.data(), it.eitems.size(), &it.d_eitems);
  if (s != ARDG_OK) return s;
  s = upload(it.litems.data(), it.litems.size(), &it.d_litems);
  if (s != ARDG_OK) return s;
  it.tile_e = tile_e;
  it.tile_l = tile_l;
  return ARDG_OK;
}

int grid_for(ardg_batch b, int nitems, int mult) {
  const int g = std::max(1, b->ncu * mult);
  return std::max(1, std::min(nitems, g));
}

// One Runge-Kutta stage of one group.
hipError_t group_stage(ardg_batch b, BatchGroup& g, int pi, bool f64, int scheme, int s,
                       hipStream_t st) {
  GroupItems& it = g.items[pi];
  const Tiles& t = g.tiles[pi];
  const int in_u = f64 && (scheme == ARDG_LSERK54 || s == 0);
  hipError_t e = launch_batch_edge(g.N, f64, it.tile_e, grid_for(b, (int)it.eitems.size(), t.grid_mult),
                                   b->dprobs, it.d_eitems, (int)it.eitems.size(), in_u, st);
  if (e != hipSuccess) return e;
  Epilogue epi;
  epi.stage = s;
  int write_v;
  if (scheme == ARDG_RK4) {
    epi.kind = EPI_RK4;
    write_v = (s < 3) || !f64;
  } else {
    epi.kind = EPI_LSERK;
    epi.a = kLsA[s];
    epi.b = kLsB[s];
    write_v = !f64;
  }
  return launch_batch_element(g.N, f64, it.tile_l, grid_for(b, (int)it.litems.size(), t.grid_mult),
                              b->dprobs, it.d_litems, (int)it.litems.size(), epi, in_u, write_v, st);
}

std::string cache_key(ardg_batch b, int precision, int N) {
  return b->arch + " " + (precision == ARDG_FP64 ? "fp64" : "fp32") + " N=" + std::to_string(N);
}

bool cache_lookup(ardg_batch b, int precision, int N, Tiles& t) {
  if (b->cache.empty()) return false;
  std::ifstream in(b->cache);
  if (!in) return false;
  const std::string key = cache_key(b, precision, N);
  std::string line;
  bool found = false;
  while (std::getline(in, line)) {
    if (line.compare(0, key.size(), key) != 0 || line.size() <= key.size() || line[key.size()] != ' ')
      continue;
    std::istringstream ss(line.substr(key.size()));
    Tiles c;
    if (ss >> c.edge_tile >> c.elem_tile >> c.grid_mult) {
      t = c;
      found = true;   // the last matching line wins
    }
  }
  return found;
}

void cache_store(ardg_batch b, int precision, int N, const Tiles& t) {
  if (b->cache.empty()) return;
  std::ofstream out(b->cache, std::ios::app);
  if (out) out << cache_key(b, precision, N) << " " << t.edge_tile << " " << t.elem_tile << " "
               << t.grid_mult << "\n";
}

// Time one RK4 stage of group g (mean of reps) with the given tiles; the
// problems' buffers must be set up in dprobs.
ardg_status time_group(ardg_batch b, BatchGroup& g, int pi, bool f64, const Tiles& t, float* ms) {
  g.tiles[pi] = t;
  ardg_status s = build_items(b, g, pi, t.edge_tile, t.elem_tile);
  if (s != ARDG_OK) return s;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
  HIP_TRY(hipEventCreate(&e1), "hipEventCreate");
  hipError_t e = hipSuccess;
  for (int r = 0; r < 4 && e == hipSuccess; ++r) e = group_stage(b, g, pi, f64, ARDG_RK4, r, nullptr);
  if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
  const int reps = 8;
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = group_stage(b, g, pi, f64, ARDG_RK4, r % 4, nullptr);
  if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t_ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t_ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(e, "batch tuning");
  *ms = t_ms / reps;
  return ARDG_OK;
}

// Choose tiles for every group of a precision: coordinate search over the
// edge tile, the element tile and the persistent grid size, each candidate
// timed on scratch buffers (zero state, dt = 0) of the real problems.
ardg_status tune(ardg_batch b, int precision) {
  const int pi = precision == ARDG_FP64 ? 0 : 1;
  const bool f64 = precision == ARDG_FP64;
  std::vector<BatchGroup*> todo;
  for (auto& g : b->groups) {
    if (g.tuned[pi]) continue;
    Tiles t;
    if (cache_lookup(b, precision, g.N, t)) {
      g.tiles[pi] = t;
      g.tuned[pi] = true;
      ardg_status s = build_items(b, g, pi, t.edge_tile, t.elem_tile);
      if (s != ARDG_OK) return s;
    } else {
      todo.push_back(&g);
    }
  }
  if (todo.empty()) return ARDG_OK;
  // the descriptors are about to be overwritten: no earlier step may still read them
  HIP_TRY(hipDeviceSynchronize(), "batch tuning: synchronise");
  // scratch state and workspace for every problem
  std::vector<size_t> offs;
  size_t wbytes = 0;
  batch_layout(b, precision, &offs, &wbytes);
  size_t ubytes = 0;
  std::vector<size_t> uoffs;
  for (ardg_mesh m : b->meshes) {
    uoffs.push_back(ubytes);
    ubytes += align256((size_t)m->hm.K * m->ro.Np * 8);
  }
  char* scratch = nullptr;
  hipError_t e = hipMalloc((void**)&scratch, ubytes + wbytes);
  if (e != hipSuccess) return fail(ARDG_E_OOM, "batch tuning: scratch allocation failed");
  e = hipMemset(scratch, 0, ubytes + wbytes);
  std::vector<BatchProb> hp(b->meshes.size());
  for (size_t i = 0; i < b->meshes.size(); ++i) {
    hp[i].m = b->meshes[i]->dm;
    hp[i].u = (double*)(scratch + uoffs[i]);
    hp[i].acc = (double*)(scratch + ubytes + offs[3 * i]);
    hp[i].v = scratch + ubytes + offs[3 * i + 1];
    hp[i].flux = scratch + ubytes + offs[3 * i + 2];
    hp[i].dt = 0.0;
  }
  if (e == hipSuccess) e = hipMemcpy(b->dprobs, hp.data(), hp.size() * sizeof(BatchProb), hipMemcpyHostToDevice);
  ardg_status st = (e == hipSuccess) ? ARDG_OK : hip_fail(e, "batch tuning setup");
  // 0: side-split edge tiles / matrix-core element tiles
  const int cand_tile[4] = {64, 128, 256, 0};
  const int cand_grid[4] = {1, 2, 4, 8};
  for (BatchGroup* g : todo) {
    if (st != ARDG_OK) break;
    Tiles best;
    float best_ms = 1e30f, ms = 0.f;
    for (int c : cand_tile) {
      Tiles t = best;
      t.edge_tile = c;
      if ((st = time_group(b, *g, pi, f64, t, &ms)) != ARDG_OK) break;
      if (ms < best_ms) { best_ms = ms; best.edge_tile = c; }
    }
    best_ms = 1e30f;
    for (int c : cand_tile) {
      if (st != ARDG_OK) break;
      Tiles t = best;
      t.elem_tile = c;
      if ((st = time_group(b, *g, pi, f64, t, &ms)) != ARDG_OK) break;
      if (ms < best_ms) { best_ms = ms; best.elem_tile = c; }
    }
    best_ms = 1e30f;
    for (int c : cand_grid) {
      if (st != ARDG_OK) break;
      Tiles t = best;
      t.grid_mult = c;
      if ((st = time_group(b, *g, pi, f64, t, &ms)) != ARDG_OK) break;
      if (ms < best_ms) { best_ms = ms; best.grid_mult = c; }
    }
    if (st != ARDG_OK) break;
    g->tiles[pi] = best;
    st = build_items(b, *g, pi, best.edge_tile, best.elem_tile);
    g->tuned[pi] = true;
    cache_store(b, precision, g->N, best);
  }
  (void)hipFree(scratch);
  b->hprobs.clear();   // descriptors on the device now point at scratch
  b->drop_graphs();
  return st;
}

}  // namespace

extern "C" {

// What the batched kernels are built for: one field with constant D, no
// velocity, no exterior data (their boundary faces take the mirror-ghost
// path only), the scalar equation.
static bool batch_mesh_ok(ardg_mesh m) {
  return m->dm.dmode == DM_CONST && !m->dm.conv && m->nfields_D == 1 && !m->dm.ghost && m->dm.ns == NS_OFF;
}

ardg_status ardg_batch_create(const ardg_mesh* meshes, int32_t n, const char* tune_cache, ardg_batch* out) {
  if (!out) return fail(ARDG_E_INVALID_ARG, "batch_create: null out");
  *out = nullptr;
  if (!meshes || n < 1) return fail(ARDG_E_INVALID_ARG, "batch_create: no meshes");
  const int dev = meshes[0] ? meshes[0]->device : -1;
  for (int i = 0; i < n; ++i) {
    ardg_mesh m = meshes[i];
    if (!m) return fail(ARDG_E_INVALID_ARG, "batch_create: null mesh");
    if (m->device < 0 || m->device != dev)
      return fail(ARDG_E_INVALID_ARG, "batch_create: meshes must live on one device");
    if (!batch_mesh_ok(m))
      return fail(ARDG_E_UNSUPPORTED,
                  "batch_create: meshes need one field, constant D, no velocity and zero Dirichlet data");
  }
  try {
    auto b = std::make_unique<ardg_batch_s>();
    b->device = dev;
    b->meshes.assign(meshes, meshes + n);
    if (tune_cache) b->cache = tune_cache;
    DeviceGuard g(dev);
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
    b->ncu = prop.multiProcessorCount;
    b->arch = prop.gcnArchName;
    const size_t sp = b->arch.find(':');
    if (sp != std::string::npos) b->arch = b->arch.substr(0, sp);
    std::map<int, std::vector<int>> byN;
    for (int i = 0; i < n; ++i) byN[meshes[i]->N].push_back(i);
    for (auto& kv : byN) {
      BatchGroup gr;
      gr.N = kv.first;
      gr.probs = kv.second;
      std::stable_sort(gr.probs.begin(), gr.probs.end(), [&](int a, int c) {
        return meshes[a]->hm.K > meshes[c]->hm.K;
      });
      b->groups.push_back(gr);
    }
    void* p = nullptr;
    HIP_TRY(hipMalloc(&p, sizeof(BatchProb) * n), "hipMalloc");
    b->dprobs = (BatchProb*)p;
    *out = b.release();
    return ARDG_OK;
  } catch (const std::exception& ex) {
    return fail(ARDG_E_INVALID_ARG, std::string("batch_create: ") + ex.what());
  }
}

void ardg_batch_destroy(ardg_batch batch) { delete batch; }

ardg_status ardg_batch_workspace_bytes(ardg_batch batch, int32_t scheme, int32_t precision, int64_t* bytes) {
  if (!batch || !bytes) return fail(ARDG_E_INVALID_ARG, "batch_workspace_bytes: null argument");
  if (scheme != ARDG_RK4 && scheme != ARDG_LSERK54) return fail(ARDG_E_INVALID_ARG, "unknown scheme");
  if (precision != ARDG_FP64 && precision != ARDG_FP32)
    return fail(ARDG_E_UNSUPPORTED, "batched stepping is built for FP64 and FP32");
  size_t t = 0;
  batch_layout(batch, precision, nullptr, &t);
  *bytes = (int64_t)t;
  return ARDG_OK;
}

ardg_status ardg_batch_check(ardg_batch batch, double* const* u_devs, void* hip_stream) {
  if (!batch || !u_devs) return fail(ARDG_E_INVALID_ARG, "batch_check: null argument");
  DeviceGuard g(batch->device);
  hipStream_t st = (hipStream_t)hip_stream;
  int* cnt = nullptr;
  HIP_TRY(hipMalloc(&cnt, sizeof(int)), "hipMalloc");
  hipError_t e = hipMemsetAsync(cnt, 0, sizeof(int), st);
  for (size_t i = 0; i < batch->meshes.size() && e == hipSuccess; ++i) {
    if (!u_devs[i]) {
      (void)hipFree(cnt);
      return fail(ARDG_E_INVALID_ARG, "batch_check: null state pointer");
    }
    const ardg_mesh m = batch->meshes[i];
    e = launch_nonfinite(u_devs[i], m->hm.K * m->ro.Np, cnt, st);
  }
  int host = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&host, cnt, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(cnt);
  if (e != hipSuccess) return hip_fail(e, "batch_check");
  if (host) return fail(ARDG_E_NONFINITE, "batch_check: " + std::to_string(host) + " non-finite values");
  return ARDG_OK;
}

ardg_status ardg_batch_tiles(ardg_batch batch, int32_t precision, int32_t N, int32_t* edge_tile,
                             int32_t* elem_tile, int32_t* grid) {
  if (!batch) return fail(ARDG_E_INVALID_ARG, "batch_tiles: null batch");
  if (precision != ARDG_FP64 && precision != ARDG_FP32)
    return fail(ARDG_E_UNSUPPORTED, "batched stepping is built for FP64 and FP32");
  DeviceGuard g(batch->device);
  ardg_status s = tune(batch, precision);
  if (s != ARDG_OK) return s;
  const int pi = precision == ARDG_FP64 ? 0 : 1;
  for (auto& gr : batch->groups)
    if (gr.N == N) {
      if (edge_tile) *edge_tile = gr.tiles[pi].edge_tile;
      if (elem_tile) *elem_tile = gr.tiles[pi].elem_tile;
      if (grid) *grid = gr.tiles[pi].grid_mult;
      return ARDG_OK;
    }
  return fail(ARDG_E_INVALID_ARG, "batch_tiles: no mesh of that order in the batch");
}

// The graph of nsteps steps of the whole batch (captured on first use).
static ardg_status batch_graph(ardg_batch batch, int scheme, int precision, void* work_dev, int nsteps,
                               hipGraphExec_t* out) {
  const int pi = precision == ARDG_FP64 ? 0 : 1;
  const bool f64 = precision == ARDG_FP64;
  GraphKey key{scheme, precision, 1, nsteps, nullptr, work_dev, 0.0, batch->version};
  auto it = batch->graphs.find(key);
  if (it == batch->graphs.end()) {
    if (!batch->cap_stream)
      HIP_TRY(hipStreamCreateWithFlags(&batch->cap_stream, hipStreamNonBlocking), "hipStreamCreate");
    HIP_TRY(hipStreamBeginCapture(batch->cap_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    hipError_t e = hipSuccess;
    if (!f64)
      for (auto& gr : batch->groups) {
        if (e != hipSuccess) break;
        GroupItems& gi = gr.items[pi];
        const int Np = (gr.N + 1) * (gr.N + 2) / 2;
        // element items cover 64 elements each under tile code 0
        e = launch_batch_to_f32(batch->dprobs, gi.d_litems, (int)gi.litems.size(), gi.tile_l == 0 ? 64 : gi.tile_l, Np,
                                grid_for(batch, (int)gi.litems.size(), gr.tiles[pi].grid_mult), batch->cap_stream);
      }
    const int nst = scheme == ARDG_RK4 ? 4 : 5;
    for (int step = 0; step < nsteps && e == hipSuccess; ++step)
      for (int st = 0; st < nst && e == hipSuccess; ++st)
        for (auto& gr : batch->groups) {
          e = group_stage(batch, gr, pi, f64, scheme, st, batch->cap_stream);
          if (e != hipSuccess) break;
        }
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(batch->cap_stream, &graph);
    if (e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return hip_fail(e, "batch_step: launch during capture");
    }
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    hipError_t e3 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) return hip_fail(e3, "hipGraphInstantiate");
    if (batch->graphs.size() >= 8) {
      batch->drop_graphs();
      key.version = batch->version;
    }
    it = batch->graphs.emplace(key, exec).first;
  }
  *out = it->second;
  return ARDG_OK;
}

ardg_status ardg_batch_step(ardg_batch batch, int32_t scheme, int32_t precision, double* const* u_devs,
                            void* work_dev, const double* dt, int32_t nsteps, void* hip_stream) {
  if (!batch || !u_devs || !work_dev || !dt) return fail(ARDG_E_INVALID_ARG, "batch_step: null argument");
  if (scheme != ARDG_RK4 && scheme != ARDG_LSERK54) return fail(ARDG_E_INVALID_ARG, "unknown scheme");
  if (precision != ARDG_FP64 && precision != ARDG_FP32)
    return fail(ARDG_E_UNSUPPORTED, "batched stepping is built for FP64 and FP32");
  if (((uintptr_t)work_dev & 255) != 0) return fail(ARDG_E_INVALID_ARG, "batch_step: work_dev not 256-byte aligned");
  if (nsteps < 0) return fail(ARDG_E_INVALID_ARG, "batch_step: nsteps < 0");
  const size_t n = batch->meshes.size();
  for (size_t i = 0; i < n; ++i)
    if (!u_devs[i] || !std::isfinite(dt[i])) return fail(ARDG_E_INVALID_ARG, "batch_step: bad state pointer or dt");
  // the meshes are referenced: one changed since the batch was made may no
  // longer be one the batched kernels handle
  for (size_t i = 0; i < n; ++i)
    if (!batch_mesh_ok(batch->meshes[i]))
      return fail(ARDG_E_UNSUPPORTED, "batch_step: mesh " + std::to_string(i) +
                                          " no longer has one field, constant D, no velocity and zero Dirichlet data");
  if (nsteps == 0) return ARDG_OK;
  DeviceGuard g(batch->device);
  ardg_status s = tune(batch, precision);
  if (s != ARDG_OK) return s;
  std::vector<size_t> offs;
  batch_layout(batch, precision, &offs, nullptr);
  std::vector<BatchProb> hp(n);
  char* w = (char*)work_dev;
  for (size_t i = 0; i < n; ++i) {
    hp[i].m = batch->meshes[i]->dm;
    hp[i].u = u_devs[i];
    hp[i].acc = (double*)(w + offs[3 * i]);
    hp[i].v = w + offs[3 * i + 1];
    hp[i].flux = w + offs[3 * i + 2];
    hp[i].dt = dt[i];
  }
  if (batch->hprobs.size() != n ||
      std::memcmp(batch->hprobs.data(), hp.data(), n * sizeof(BatchProb)) != 0) {
    // earlier graph launches may still read the descriptors being replaced
    HIP_TRY(hipDeviceSynchronize(), "batch_step: synchronise");
    HIP_TRY(hipMemcpy(batch->dprobs, hp.data(), n * sizeof(BatchProb), hipMemcpyHostToDevice),
            "batch_step: descriptor upload");
    batch->hprobs = hp;
    batch->drop_graphs();
  }
  // the graph of min(nsteps, kGraphSteps) steps, replayed, and one of the
  // remainder (captured again if capturing the first evicted it)
  const int chunk = std::min<int>(nsteps, kGraphSteps);
  const int nrem = nsteps % chunk;
  hipGraphExec_t ex_full = nullptr, ex_rem = nullptr;
  if (nrem) {
    s = batch_graph(batch, scheme, precision, work_dev, nrem, &ex_rem);
    if (s != ARDG_OK) return s;
  }
  const uint64_t v0 = batch->version;
  s = batch_graph(batch, scheme, precision, work_dev, chunk, &ex_full);
  if (s != ARDG_OK) return s;
  if (nrem && batch->version != v0) {
    s = batch_graph(batch, scheme, precision, work_dev, nrem, &ex_rem);
    if (s != ARDG_OK) return s;
  }
  for (int i = 0; i < nsteps / chunk; ++i)
    HIP_TRY(hipGraphLaunch(ex_full, (hipStream_t)hip_stream), "hipGraphLaunch");
  if (ex_rem) HIP_TRY(hipGraphLaunch(ex_rem, (hipStream_t)hip_stream), "hipGraphLaunch");
  return ARDG_OK;
}

}  // extern "C"
