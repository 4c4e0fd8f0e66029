// Mesh setup in FP64: element Jacobians (eqs. mapping_tri_diff,
// triangle_jacobian_a/b), face connectivity, and for every edge the enclosed
// parallelogram (section "Enclosed parallelogram") and the per-edge constants
// the edge kernel needs:
//   * the apex P_k of sub-triangle k as barycentric weights in element k's
//     rotated frame (the node reordering of section "Reordering nodes in the
//     reference domain" puts the shared edge on the hypotenuse; element 1's
//     frame has vertices (C1, A, B), element 2's (C2, B, A));
//   * gamma_R, gamma_S = n1 . (r'_x, r'_y), n1 . (s'_x, s'_y), the constant
//     parallelogram factors contracted with element 1's outward normal.
// The parallelogram is the maximum-area one with diagonal AB: its apex P1 is
// the highest point above AB of the polygon  (A,B,C1) intersected with the
// point reflection of (B,A,C2) through the midpoint of AB, found here by
// clipping.  Boundary faces use the mirror image of the element as a ghost,
// which makes the parallelogram a rhombus symmetric about AB.
#include "meshsetup.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <unordered_map>

#include "../../include/ardg.h"

namespace ardg {

namespace {

struct P2 { double x, y; };
inline P2 operator+(P2 a, P2 b) { return {a.x + b.x, a.y + b.y}; }
inline P2 operator-(P2 a, P2 b) { return {a.x - b.x, a.y - b.y}; }
inline P2 operator*(double s, P2 a) { return {s * a.x, s * a.y}; }
inline double cross(P2 a, P2 b) { return a.x * b.y - a.y * b.x; }

// Keep the part of a convex polygon on the left of the directed line p->q.
std::vector<P2> clip_left(const std::vector<P2>& poly, P2 p, P2 q, double tol) {
  std::vector<P2> out;
  const size_t n = poly.size();
  for (size_t i = 0; i < n; ++i) {
    const P2 a = poly[i], b = poly[(i + 1) % n];
    const double da = cross(q - p, a - p), db = cross(q - p, b - p);
    const bool ina = da >= -tol, inb = db >= -tol;
    if (ina) out.push_back(a);
    if (ina != inb) {
      const double t = da / (da - db);
      out.push_back(a + t * (b - a));
    }
  }
  return out;
}

// Barycentric weights (of w2, w3) of point P in triangle (w1, w2, w3).
void bary23(P2 w1, P2 w2, P2 w3, P2 P, double* out) {
  const double area = cross(w2 - w1, w3 - w1);
  out[0] = cross(P - w1, w3 - w1) / area;
  out[1] = cross(w2 - w1, P - w1) / area;
}

// gamma_R, gamma_S of the parallelogram with vertices (P1, A, B) and normal n.
void gammas(P2 P1, P2 A, P2 B, P2 n, double* out) {
  const P2 XR = 0.5 * (A - P1), XS = 0.5 * (B - P1);
  const double Jp = XR.x * XS.y - XS.x * XR.y;
  out[0] = (n.x * XS.y - n.y * XS.x) / Jp;
  out[1] = (-n.x * XR.y + n.y * XR.x) / Jp;
}

}  // namespace

int build_host_mesh(const double* vxy, int64_t Nv, const int32_t* etov, int64_t K, HostMesh& m,
                    std::string& err) {
  if (!vxy || !etov || Nv < 3 || K < 1 || K >= (int64_t(1) << 29)) {
    err = "mesh_create: bad sizes or null arrays";
    return ARDG_E_INVALID_ARG;
  }
  m.K = K;
  m.Nv = Nv;
  m.vxy.assign(vxy, vxy + 2 * Nv);
  m.etov.assign(etov, etov + 3 * K);
  for (int64_t i = 0; i < 2 * Nv; ++i)
    if (!std::isfinite(vxy[i])) {
      err = "mesh_create: non-finite vertex coordinate at vertex " + std::to_string(i / 2);
      return ARDG_E_INVALID_ARG;
    }
  auto V = [&](int64_t k, int c) {
    const int32_t v = m.etov[3 * k + c];
    return P2{m.vxy[2 * (int64_t)v], m.vxy[2 * (int64_t)v + 1]};
  };
  m.J.resize(K);
  m.min_J = 1e300;
  for (int64_t k = 0; k < K; ++k) {
    for (int c = 0; c < 3; ++c) {
      const int32_t v = m.etov[3 * k + c];
      if (v < 0 || v >= Nv) {
        err = "mesh_create: vertex index out of range in element " + std::to_string(k);
        return ARDG_E_INVALID_ARG;
      }
    }
    const P2 a = V(k, 0), b = V(k, 1), c = V(k, 2);
    const double J = 0.25 * cross(b - a, c - a);
    if (!(J > 0.0)) {
      err = "mesh_create: element " + std::to_string(k) + " has J <= 0 (not counter-clockwise)";
      return ARDG_E_MESH_ORIENTATION;
    }
    m.J[k] = J;
    m.min_J = std::min(m.min_J, J);
  }

  // connectivity by hashing the undirected vertex pair of every face
  const int fv[3][2] = {{0, 1}, {1, 2}, {2, 0}};
  std::vector<int64_t> nbr(3 * K, -1);
  std::unordered_map<uint64_t, int64_t> seen;
  seen.reserve(size_t(3 * K));
  for (int64_t k = 0; k < K; ++k)
    for (int f = 0; f < 3; ++f) {
      const uint32_t va = (uint32_t)m.etov[3 * k + fv[f][0]], vb = (uint32_t)m.etov[3 * k + fv[f][1]];
      const uint64_t key = (uint64_t(std::min(va, vb)) << 32) | std::max(va, vb);
      auto it = seen.find(key);
      if (it == seen.end()) {
        seen.emplace(key, 3 * k + f);
        continue;
      }
      const int64_t other = it->second;
      if (other < 0) {
        err = "mesh_create: edge shared by more than two elements (element " + std::to_string(k) + ")";
        return ARDG_E_MESH_TOPOLOGY;
      }
      const int64_t k2 = other / 3;
      const int f2 = int(other % 3);
      if ((uint32_t)m.etov[3 * k2 + fv[f2][0]] != vb) {
        err = "mesh_create: elements " + std::to_string(k2) + " and " + std::to_string(k) +
              " traverse their shared edge in the same direction";
        return ARDG_E_MESH_TOPOLOGY;
      }
      nbr[3 * k + f] = other;
      nbr[other] = 3 * k + f;
      it->second = -1;
    }

  // edge lists
  m.elem_face.assign(3 * K, 0);
  for (int64_t k = 0; k < K; ++k)
    for (int f = 0; f < 3; ++f) {
      const int64_t o = nbr[3 * k + f];
      if (o >= 0 && o / 3 > k) {
        m.e1.push_back(int32_t(k));
        m.f1.push_back(f);
        m.e2.push_back(int32_t(o / 3));
        m.f2.push_back(int32_t(o % 3));
      }
    }
  m.E_int = (int64_t)m.e1.size();
  for (int64_t k = 0; k < K; ++k)
    for (int f = 0; f < 3; ++f)
      if (nbr[3 * k + f] < 0) {
        m.bk.push_back(int32_t(k));
        m.bf.push_back(f);
      }
  m.E_bdy = (int64_t)m.bk.size();

  // rotated frame (w1, w2, w3) for each face: face (v1,v2) -> (v3,v1,v2), ...
  const int rotv[3][3] = {{2, 0, 1}, {0, 1, 2}, {1, 2, 0}};
  m.P1.resize(2 * m.E_int);
  m.mu1.resize(2 * m.E_int);
  m.mu2.resize(2 * m.E_int);
  m.gam.resize(2 * m.E_int);
  m.min_area_ratio = 1.0;
  for (int64_t e = 0; e < m.E_int; ++e) {
    const int64_t k1 = m.e1[e], k2 = m.e2[e];
    const int fa = m.f1[e], fb = m.f2[e];
    const P2 C1 = V(k1, rotv[fa][0]), A = V(k1, rotv[fa][1]), B = V(k1, rotv[fa][2]);
    const P2 C2 = V(k2, rotv[fb][0]);
    const P2 C2r = A + B - C2;  // point reflection of C2 through the midpoint
    const P2 t = B - A;
    const double L2 = t.x * t.x + t.y * t.y;
    const double tol = 1e-13 * L2;
    std::vector<P2> poly = {A, B, C1};
    poly = clip_left(poly, B, C2r, tol);
    poly = clip_left(poly, C2r, A, tol);
    double best = -1e300;
    P2 P = C1;
    for (const P2& p : poly) {
      const double h = cross(t, p - A);
      if (h > best) { best = h; P = p; }
    }
    const double area_p = cross(t, P - A);          // parallelogram area
    const double area_q = 0.5 * (cross(t, C1 - A) + cross(A - B, C2 - B));
    const double ratio = area_p / area_q;
    if (!(ratio > 1e-8)) {
      err = "mesh_create: degenerate enclosed parallelogram at edge between elements " +
            std::to_string(k1) + " and " + std::to_string(k2);
      return ARDG_E_DEGENERATE_PARALLELOGRAM;
    }
    m.min_area_ratio = std::min(m.min_area_ratio, ratio);
    const P2 P2p = A + B - P;
    m.P1[2 * e] = P.x;
    m.P1[2 * e + 1] = P.y;
    bary23(C1, A, B, P, &m.mu1[2 * e]);
    bary23(C2, B, A, P2p, &m.mu2[2 * e]);
    const double Ln = std::sqrt(L2);
    const P2 n{t.y / Ln, -t.x / Ln};
    gammas(P, A, B, n, &m.gam[2 * e]);
    m.elem_face[3 * k1 + fa] = int32_t(e << 1);
    m.elem_face[3 * k2 + fb] = int32_t((e << 1) | 1);
  }

  m.bP1.resize(2 * m.E_bdy);
  m.bmu.resize(2 * m.E_bdy);
  m.bgam.resize(2 * m.E_bdy);
  for (int64_t b = 0; b < m.E_bdy; ++b) {
    const int64_t k = m.bk[b];
    const int fa = m.bf[b];
    const P2 C = V(k, rotv[fa][0]), A = V(k, rotv[fa][1]), B = V(k, rotv[fa][2]);
    const P2 t = B - A;
    const double Ln = std::sqrt(t.x * t.x + t.y * t.y);
    const P2 nin{-t.y / Ln, t.x / Ln};
    const P2 mid = 0.5 * (A + B);
    // largest s with mid + s nin inside (A, B, C): first crossing of B->C or C->A
    double smax = 1e300;
    const P2 segs[2][2] = {{B, C}, {C, A}};
    for (auto& sg : segs) {
      const P2 d = sg[1] - sg[0];
      const double den = cross(d, nin);
      if (std::fabs(den) > 0) {
        const double s = cross(d, sg[0] - mid) / den;
        if (s > 0) smax = std::min(smax, s);
      }
    }
    if (!(smax < 1e300) || !(smax > 0)) {
      err = "mesh_create: degenerate boundary rhombus at element " + std::to_string(k);
      return ARDG_E_DEGENERATE_PARALLELOGRAM;
    }
    const P2 P = mid + smax * nin;
    m.bP1[2 * b] = P.x;
    m.bP1[2 * b + 1] = P.y;
    bary23(C, A, B, P, &m.bmu[2 * b]);
    const P2 n{t.y / Ln, -t.x / Ln};
    gammas(P, A, B, n, &m.bgam[2 * b]);
    m.elem_face[3 * k + fa] = int32_t((m.E_int + b) << 1);
  }
  return ARDG_OK;
}

}  // namespace ardg
