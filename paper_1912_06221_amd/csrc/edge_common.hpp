// Per-edge aRDG flux on the vector unit (one lane per edge), shared by the
// thread-per-edge kernels, the batched kernels and the boundary faces of the
// matrix-core edge kernel, and the scalar-operand matrix-vector product used
// by the thread-per-element kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.hpp"
#include "kernel_common.hpp"

namespace ardg {

// y_v = A x_v (v < NV) for the ROWS x COLS block of a constant row-major
// operator with leading dimension LD.  The entries are wave-uniform scalar
// loads feeding scalar-operand FMAs, walked in steps of RB rows x CC columns
// (RB*CC <= E entries): the RB rows' accumulators are
// independent, so consecutive FMAs do not wait on each other, and the loads
// of the next step are issued before the FMAs of the current one, so their
// latency is covered by arithmetic.  The fence between steps keeps at most
// two steps of entries in SGPRs (without it the whole operator is hoisted
// into SGPRs and spilled).  With NV = 2 every loaded entry feeds two vectors.
template <int ROWS, int COLS, int LD, int NV, typename T, typename XA, typename YA, int RBX = 4, int E = 12>
__device__ inline void matvec_blk(cptr<T> A0, XA x, YA y) {
  constexpr int RB = ROWS < RBX ? ROWS : RBX;
  constexpr int CC = E / RB;
  constexpr int NRB = (ROWS + RB - 1) / RB;
  constexpr int NCC = (COLS + CC - 1) / CC;
  constexpr int NSTEP = NRB * NCC;
  T buf[2][RB][CC];
  {
    const cptr<T> A = fresh(A0);
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int q = 0; q < CC; ++q)
        if (r < ROWS && q < COLS) buf[0][r][q] = A[r * LD + q];
  }
  T acc[NV][RB];
#pragma unroll
  for (int st = 0; st < NSTEP; ++st) {
    const int r0 = (st / NCC) * RB, q0 = (st % NCC) * CC;
    const bool first = (st % NCC) == 0, last = (st % NCC) == NCC - 1;
    row_fence();
    if (st + 1 < NSTEP) {
      const int r1 = ((st + 1) / NCC) * RB, q1 = ((st + 1) % NCC) * CC;
      const cptr<T> A = fresh(A0);
#pragma unroll
      for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int q = 0; q < CC; ++q)
          if (r1 + r < ROWS && q1 + q < COLS) buf[(st + 1) & 1][r][q] = A[(r1 + r) * LD + q1 + q];
    }
#pragma unroll
    for (int q = 0; q < CC; ++q)
#pragma unroll
      for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int v = 0; v < NV; ++v)
          if (r0 + r < ROWS && q0 + q < COLS) {
            const T a = buf[st & 1][r][q];
            acc[v][r] = (first && q == 0) ? a * x[v][q0] : fma(a, x[v][q0 + q], acc[v][r]);
          }
    if (last) {
#pragma unroll
      for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int v = 0; v < NV; ++v)
          if (r0 + r < ROWS) y[v][r0 + r] = acc[v][r];
    }
  }
}

template <int ROWS, int COLS, int NV, typename T, typename XA, typename YA>
__device__ inline void matvec_n(cptr<T> A0, XA x, YA y) {
  matvec_blk<ROWS, COLS, COLS, NV, T>(A0, x, y);
}

// single-vector views for matvec_n: v[0][q] == p[q]
template <typename P>
struct OneVec {
  P p;
  __device__ P operator[](int) const { return p; }
};

template <int ROWS, int COLS, typename T, int RBX = 4, int E = 12>
__device__ inline void matvec_pf(cptr<T> A0, const T* x, T* y) {
  matvec_blk<ROWS, COLS, COLS, 1, T, OneVec<const T*>, OneVec<T*>, RBX, E>(A0, OneVec<const T*>{x}, OneVec<T*>{y});
}

// column slice of a wider row-major operator (leading dimension LD)
template <int ROWS, int COLS, int LD, typename T>
__device__ inline void matvec_ld(cptr<T> A0, const T* x, T* y) {
  matvec_blk<ROWS, COLS, LD, 1, T>(A0, OneVec<const T*>{x}, OneVec<T*>{y});
}

// Row groups of a constant operator block (row-major, leading dimension LD,
// the first COLS columns used): group g < NG is the G rows g + q GS (q < G).
// Each group's G dot products with x are formed in the prefetched
// scalar-operand steps of matvec_blk (E entries per step) and handed to
// emit(g, acc) as soon as the group is complete, so only G accumulators are
// live at a time.
template <int G, int NG, int GS, int COLS, int LD, typename T, typename Emit, int E = 12>
__device__ inline void matvec_groups(cptr<T> A0, const T* x, Emit emit) {
  constexpr int CC = E / G;
  constexpr int NCC = (COLS + CC - 1) / CC;
  constexpr int NSTEP = NG * NCC;
  T buf[2][G][CC];
  {
    const cptr<T> A = fresh(A0);
#pragma unroll
    for (int r = 0; r < G; ++r)
#pragma unroll
      for (int q = 0; q < CC; ++q)
        if (q < COLS) buf[0][r][q] = A[r * GS * LD + q];
  }
  T acc[G];
#pragma unroll
  for (int st = 0; st < NSTEP; ++st) {
    const int g = st / NCC, q0 = (st % NCC) * CC;
    const bool first = (st % NCC) == 0, last = (st % NCC) == NCC - 1;
    row_fence();
    if (st + 1 < NSTEP) {
      const int g1 = (st + 1) / NCC, q1 = ((st + 1) % NCC) * CC;
      const cptr<T> A = fresh(A0);
#pragma unroll
      for (int r = 0; r < G; ++r)
#pragma unroll
        for (int q = 0; q < CC; ++q)
          if (q1 + q < COLS) buf[(st + 1) & 1][r][q] = A[(g1 + r * GS) * LD + q1 + q];
    }
#pragma unroll
    for (int q = 0; q < CC; ++q)
#pragma unroll
      for (int r = 0; r < G; ++r)
        if (q0 + q < COLS) {
          const T a = buf[st & 1][r][q];
          acc[r] = (first && q == 0) ? a * x[q0] : fma(a, x[q0 + q], acc[r]);
        }
    if (last) emit(g, acc);
  }
}

// y = A x with one operator row in flight at a time (no prefetch): the row
// fence and the fresh pointer keep the row's scalar loads next to its FMAs.
// Used where many other values are live (the thread-per-element kernels).
template <int ROWS, int COLS, typename T>
__device__ inline void matvec(cptr<T> A0, const T* x, T* y) {
#pragma unroll
  for (int r = 0; r < ROWS; ++r) {
    row_fence();
    const cptr<T> A = fresh(A0);
    T s = A[r * COLS] * x[0];
#pragma unroll
    for (int q = 1; q < COLS; ++q) s = fma(A[r * COLS + q], x[q], s);
    y[r] = s;
  }
}

// In-place de Casteljau subdivision of Bernstein coefficients on I at the
// point with barycentric weights (1 - mu.x - mu.y, mu.x, mu.y) of (a1, a2, a3).
// Afterwards lattice slot (i,j) holds the coefficient with multi-index
// (N-i-j, i, j) of the same polynomial on the sub-triangle (point, a2, a3).
template <int N, typename T>
__device__ inline void decasteljau(T* c, double2 mu) {
  const T m2 = (T)mu.x, m3 = (T)mu.y;
  const T m1 = (T)(1.0 - mu.x - mu.y);
#pragma unroll
  for (int n = N; n >= 1; --n)
#pragma unroll
    for (int j = 0; j <= n - 1; ++j)
#pragma unroll
      for (int i = 0; i <= n - 1 - j; ++i)
        c[lat(N, i, j)] = m1 * c[lat(N, i, j)] + m2 * c[lat(N, i + 1, j)] + m3 * c[lat(N, i, j + 1)];
}

// Reorder one element's nodal values so that face f is the hypotenuse of the
// reference triangle (section "Reordering nodes in the reference domain"):
// rotated vertices (v3, v1, v2) for face 0, (v1, v2, v3) for face 1 and
// (v2, v3, v1) for face 2, a register permutation.  trace[j] receives the
// values on face f, counter-clockwise.
template <int N, typename T>
__device__ inline void rotate_to_face(const T* v, int f, T* t, T* trace) {
#pragma unroll
  for (int j = 0; j <= N; ++j)
#pragma unroll
    for (int i = 0; i <= N - j; ++i) {
      const T a0 = v[lat(N, j, N - i - j)];
      const T a1 = v[lat(N, i, j)];
      const T a2 = v[lat(N, N - i - j, i)];
      t[lat(N, i, j)] = (f == 0) ? a0 : ((f == 1) ? a1 : a2);
    }
#pragma unroll
  for (int j = 0; j <= N; ++j) trace[j] = t[lat(N, N - j, j)];
}

// The trace of a Bernstein-form polynomial on the hypotenuse of its
// (rotated) reference triangle: the face's Nfp coefficients, counter-
// clockwise, mapped to the values at the face's LGL nodes (in place).
template <int N, typename T>
__device__ inline void face_bernstein_to_nodal(cptr<T> op, T* tr) {
  constexpr OpLayout L(N);
  constexpr int Nfp = N + 1;
  T y[Nfp];
  matvec<Nfp, Nfp, T>(op + L.bf2n, tr, y);
#pragma unroll
  for (int j = 0; j < Nfp; ++j) tr[j] = y[j];
}

// Side k's Bernstein coefficients on its sub-triangle of one element field
// given by nodal values v (rotated to face f, converted, subdivided at mu).
template <int N, typename T>
__device__ inline void project_side(cptr<T> op, const T* v, int f, double2 mu, T* b, T* trace) {
  constexpr OpLayout L(N);
  constexpr int Np = L.Np;
  T t[Np];
  rotate_to_face<N, T>(v, f, t, trace);
  matvec<Np, Np, T>(op + L.n2b, t, b);
  decasteljau<N, T>(b, mu);
}

// The (r, s) swap of the lattice: the mirror image of a sub-triangle's
// Bernstein coefficients in the other half of the rhombus.
template <int N, typename T>
__device__ inline void lattice_swap(const T* b, T* out, T sign) {
#pragma unroll
  for (int j = 0; j <= N; ++j)
#pragma unroll
    for (int i = 0; i <= N - j; ++i) out[lat(N, i, j)] = sign * b[lat(N, j, i)];
}

// Pipelined products where registers allow it (moderate orders), the
// one-row-at-a-time form otherwise.
template <bool PF, int ROWS, int COLS, typename T>
__device__ inline void matvec_sel(cptr<T> A0, const T* x, T* y) {
  if constexpr (PF)
    matvec_pf<ROWS, COLS, T>(A0, x, y);
  else
    matvec<ROWS, COLS, T>(A0, x, y);
}

// Algorithm 2's reconstructed coefficient at diagonal node j of an edge
// with element coefficients D1, D2: D1 w1_j + D2 w2_j.
template <int N, typename T>
__device__ inline T alg2_coef(cptr<T> op, int j, T D1, T D2) {
  constexpr OpLayout L(N);
  return D1 * op[L.w1 + j] + D2 * op[L.w2 + j];
}

// Diffusive flux of boundary face e (index past the interior edges): the
// element's sub-triangle on its mirror-ghost rhombus and the boundary
// reconstruction operator (Algorithm 1: its boundary blocks; Algorithm 2:
// the constant-coefficient operator times the coefficient reconstructed
// from the element's D on both halves).  With prescribed exterior data the
// ghost sub-triangle carries that state instead of the mirror image: the
// reconstruction operator's side-2 columns act on its Bernstein
// coefficients, and gtrace receives its values on the face (side-1 order)
// for the upwind flux.  F receives sJ * flux, trace the element's values on
// the face, vn the stored n.v (convection).
template <int N, typename T, int DM, bool GH = true>
__device__ inline void boundary_flux(const DevMesh& m, cptr<T> op, int64_t e, int field,
                                     const T* __restrict__ uf, T* F, T* trace, double2& vn, T* gtrace) {
  constexpr OpLayout L(N);
  constexpr int Np = L.Np, Nfp = L.Nfp;
  const int64_t b = e - m.E_int;
  const int kb = m.bk[b];
  const double2 g = m.bgam[b], mu = m.bmu[b];
  if (m.conv) vn = m.vn[e];
  const int k = kb & 0x3fffffff, fa = (int)((unsigned)kb >> 30);
  T v[Np];
#pragma unroll
  for (int n = 0; n < Np; ++n) v[n] = uf[(int64_t)k * Np + n];
  const T D = DM != DM_CONST ? (T)m.Delem[k] : (T)field_D(m, field);
  const T gR = (T)g.x, gS = (T)g.y;
  if (GH && m.ghost) {
    // the element's sub-triangle (cb[0]) and the exterior state on the ghost
    // sub-triangle (P2, B, A), nodal -> Bernstein (cb[1]); the ghost carries
    // the element's D, so Algorithm 1 takes its equal-coefficient form
    // D (U1 - U2), as the constant-coefficient operator does.  One row of the
    // 2 Nfp x 2 Np operator at a time: this path shares its kernel's register
    // allocation with the interior edges.
    T cb[2][Np];
    {
      T t[Np];
      rotate_to_face<N, T>(v, fa, t, trace);
      matvec<Np, Np, T>(op + L.n2b, t, cb[0]);
    }
    decasteljau<N, T>(cb[0], mu);
    {
      T gv[Np];
      const double* gs = m.ghost + ((int64_t)field * m.E_bdy + b) * Np;
#pragma unroll
      for (int n = 0; n < Np; ++n) gv[n] = (T)gs[n];
#pragma unroll
      for (int j = 0; j <= N; ++j) gtrace[j] = gv[lat(N, j, N - j)];
      matvec<Np, Np, T>(op + L.n2b, gv, cb[1]);
    }
    T gg[2 * Nfp];
    matvec<2 * Nfp, 2 * Np, T>(op + (DM == DM_ALG1 ? L.udr : L.kr), &cb[0][0], gg);
#pragma unroll
    for (int j = 0; j < Nfp; ++j) {
      const T Dj = DM == DM_ALG2 ? alg2_coef<N, T>(op, j, D, D) : D;
      F[j] = Dj * (gR * gg[j] + gS * gg[Nfp + j]);
    }
    return;
  }
  T t[Np], c[Np];
  rotate_to_face<N, T>(v, fa, t, trace);
  matvec<Np, Np, T>(op + L.n2b, t, c);
  decasteljau<N, T>(c, mu);
#pragma unroll
  for (int j = 0; j <= N; ++j) gtrace[j] = T(0);   // u+ = 0 outside the domain
  T gb[2 * Nfp];
  matvec<2 * Nfp, Np, T>(op + (DM == DM_ALG1 ? L.ubr : L.kbr), c, gb);
#pragma unroll
  for (int j = 0; j < Nfp; ++j) {
    const T Dj = DM == DM_ALG2 ? alg2_coef<N, T>(op, j, D, D) : D;
    F[j] = Dj * (gR * gb[j] + gS * gb[Nfp + j]);
  }
}

// Upwind flux of a boundary face (u+ outside: 0, or the prescribed exterior
// state), subtracted from the diffusive flux F.
template <int N, typename T>
__device__ inline void boundary_upwind(const DevMesh& m, cptr<T> op, double2 vn, const T* tr, const T* gtr, T* F) {
  constexpr OpLayout L(N);
  constexpr int Nfp = L.Nfp;
#pragma unroll
  for (int j = 0; j < Nfp; ++j) {
    const T tau = op[L.tau + j];
    const T vnj = (T)vn.x + tau * (T)(vn.y - vn.x);
    F[j] -= vnj * ((vnj > (T)0) ? tr[j] : gtr[j]);
  }
}

// Boundary face e with its upwind convective flux (u+ outside: 0, or the
// prescribed exterior state), written to the flux array.  GH = false leaves
// out the prescribed-state path (its caller never sees exterior data), which
// holds about twice the registers of the mirror-ghost path.
template <int N, typename T, int DM, bool GH = true>
__device__ inline void boundary_body(const DevMesh& m, cptr<T> op, int64_t e, int field,
                                     const T* __restrict__ u, T* __restrict__ flux) {
  constexpr OpLayout L(N);
  constexpr int Np = L.Np, Nfp = L.Nfp;
  const int64_t E = m.E_int + m.E_bdy;
  const T* uf = u + (int64_t)field * m.K * Np;
  T F[Nfp], tr[Nfp], gtr[Nfp];
  double2 vn = make_double2(0.0, 0.0);
  boundary_flux<N, T, DM, GH>(m, op, e, field, uf, F, tr, vn, gtr);
  if (m.conv) boundary_upwind<N, T>(m, op, vn, tr, gtr, F);
  T* out = flux + ((int64_t)field * E + e) * Nfp;
#pragma unroll
  for (int j = 0; j < Nfp; ++j) out[j] = F[j];
}

// The flux of one interior edge from both sides' Bernstein coefficients in
// their rotated frames (c[0]: side 1, c[1]: side 2, before the subdivision):
// de Casteljau subdivision at each side's apex, the reconstruction operator
// (Algorithm 1's blocks with element-wise D, Algorithm 2's weights), and
// with convection the upwind flux from the sides' nodal traces tr1, tr2 (each
// in its own counter-clockwise order).  F receives sJ * flux.
template <int N, typename T, int DM, bool PF>
__device__ inline void interior_flux(const DevMesh& m, cptr<T> op, int field, T (&c)[2][(N + 1) * (N + 2) / 2],
                                     double2 mu1, double2 mu2, double2 g, double2 vn, double D1d, double D2d,
                                     const T* tr1, const T* tr2, T* F) {
  constexpr OpLayout L(N);
  constexpr int Np = L.Np, Nfp = L.Nfp;
  decasteljau<N, T>(c[0], mu1);
  decasteljau<N, T>(c[1], mu2);
  const T* cc = &c[0][0];
  const T gR = (T)g.x, gS = (T)g.y;
  if (DM == DM_ALG1) {
    const T D1 = (T)D1d, D2 = (T)D2d;
    if (D1d == D2d) {
      // equal coefficients: Algorithm 1 reduces exactly to D (U1 - U2) c
      T gg[2 * Nfp];
      matvec_sel<PF, 2 * Nfp, 2 * Np, T>(op + L.udr, cc, gg);
#pragma unroll
      for (int j = 0; j < Nfp; ++j) F[j] = D1 * (gR * gg[j] + gS * gg[Nfp + j]);
    } else {
      T gg[4 * Nfp];
      matvec_sel<PF, 4 * Nfp, 2 * Np, T>(op + L.u1r, cc, gg);
#pragma unroll
      for (int j = 0; j < Nfp; ++j)
        F[j] = D1 * (gR * gg[j] + gS * gg[Nfp + j]) - D2 * (gR * gg[2 * Nfp + j] + gS * gg[3 * Nfp + j]);
    }
  } else {
    const T D = (T)field_D(m, field);
    T gg[2 * Nfp];
    matvec_sel<PF, 2 * Nfp, 2 * Np, T>(op + L.kr, cc, gg);
#pragma unroll
    for (int j = 0; j < Nfp; ++j) {
      const T Dj = DM == DM_ALG2 ? alg2_coef<N, T>(op, j, (T)D1d, (T)D2d) : D;
      F[j] = Dj * (gR * gg[j] + gS * gg[Nfp + j]);
    }
  }
  if (m.conv) {
    // upwind flux f* = max(n.v,0) u- + min(n.v,0) u+, subtracted from the
    // diffusive flux; n.v is linear along the edge (affine velocity)
#pragma unroll
    for (int j = 0; j < Nfp; ++j) {
      const T tau = op[L.tau + j];
      const T vnj = (T)vn.x + tau * (T)(vn.y - vn.x);
      const T up = tr2[N - j];
      const T fs = (vnj > (T)0) ? vnj * tr1[j] : vnj * up;
      F[j] -= fs;
    }
  }
}

// One lane per edge (GH as for boundary_body).
template <int N, typename T, int DM, bool GH = true>
__device__ inline void edge_body(const DevMesh& m, cptr<T> op, int64_t e, int field,
                                 const T* __restrict__ u, T* __restrict__ flux) {
  constexpr OpLayout L(N);
  constexpr int Np = L.Np, Nfp = L.Nfp;
  constexpr bool kBoth = sizeof(T) == 8 ? N <= 4 : N <= 5;
  const int64_t E = m.E_int + m.E_bdy;
  const T* uf = u + (int64_t)field * m.K * Np;
  T F[Nfp];
  T tr1[Nfp], tr2[Nfp];
  double2 vn = make_double2(0.0, 0.0);
  if (e < m.E_int) {
    // one round of loads for the edge table, a second for both elements
    const int2 ef = m.ef[e];
    const double2 g = m.gam[e], mu1 = m.mu1[e], mu2 = m.mu2[e];
    if (m.conv) vn = m.vn[e];
    const int k1 = ef.x & 0x3fffffff, fa = (int)((unsigned)ef.x >> 30);
    const int k2 = ef.y & 0x3fffffff, fb = (int)((unsigned)ef.y >> 30);
    double D1d = 0.0, D2d = 0.0;
    if (DM != DM_CONST) {
      D1d = m.Delem[k1];
      D2d = m.Delem[k2];
    }
    // rotate, convert to Bernstein coefficients.  Up to moderate order both
    // elements are loaded at once and converted with one pass over the
    // conversion matrix; above it the sides go one after the other to stay
    // within the register file.
    T c[2][Np];
    if (kBoth) {
      T v[2][Np], t[2][Np];
#pragma unroll
      for (int n = 0; n < Np; ++n) v[0][n] = uf[(int64_t)k1 * Np + n];
#pragma unroll
      for (int n = 0; n < Np; ++n) v[1][n] = uf[(int64_t)k2 * Np + n];
      rotate_to_face<N, T>(v[0], fa, t[0], tr1);
      rotate_to_face<N, T>(v[1], fb, t[1], tr2);
      matvec_n<Np, Np, 2, T>(op + L.n2b, t, c);
    } else {
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        T v[Np], t[Np];
        const int64_t kk = sd ? k2 : k1;
#pragma unroll
        for (int n = 0; n < Np; ++n) v[n] = uf[kk * Np + n];
        rotate_to_face<N, T>(v, sd ? fb : fa, t, sd ? tr2 : tr1);
        matvec_sel<kBoth, Np, Np, T>(op + L.n2b, t, c[sd]);
      }
    }
    interior_flux<N, T, DM, kBoth>(m, op, field, c, mu1, mu2, g, vn, D1d, D2d, tr1, tr2, F);
  } else {
    T gtr[Nfp];
    boundary_flux<N, T, DM, GH>(m, op, e, field, uf, F, tr1, vn, gtr);
    if (m.conv) boundary_upwind<N, T>(m, op, vn, tr1, gtr, F);
  }
  T* out = flux + ((int64_t)field * E + e) * Nfp;
#pragma unroll
  for (int j = 0; j < Nfp; ++j) out[j] = F[j];
}

}  // namespace ardg
