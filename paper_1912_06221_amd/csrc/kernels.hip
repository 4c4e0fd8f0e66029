// gfx950 vector-unit kernels of the affine-reconstructed nodal DG
// right-hand side (the matrix-core ones are in kernels_mfma.hip and
// kernels_edge_mfma.hip).
//
// Edge kernels -- Algorithm aRDG for each edge and the flux on the diagonal
// of its enclosed parallelogram:
//   1. gather each side's Np values and apply the face's node reordering
//      (section "Reordering nodes in the reference domain") as a register
//      permutation;
//   2. project onto the sub-triangle (eq. NodalToModalProjection, eq.
//      totalProjection): nodal -> Bernstein coefficients on I (constant
//      matrix), then an in-place de Casteljau subdivision at the apex's
//      barycentric weights.  After the subdivision, lattice slot (i,j) holds
//      the Bernstein coefficient of the sub-triangle (apex, a2, a3) with
//      multi-index (N-i-j, i, j): the restriction of the polynomial, exactly;
//   3. apply the constant reconstruction-gradient operator (least squares on
//      the parallelogram, evaluated as d/dR, d/dS on the diagonal nodes; one
//      operator for every edge because the parallelogram map is affine) and
//      contract with the two per-edge factors gamma_R, gamma_S; with
//      element-wise D, Algorithm 1's four constant blocks weighted by D1, D2;
//   4. optionally subtract the upwind convective flux;
//   5. write Nfp values per edge, times the edge's sJ (no atomics: each edge
//      owns its slot).
// edge_flux_kernel runs one lane per edge; edge_split_kernel gives each side
// of a 64-edge tile its own wave.
// element_tile (one thread per element, the block's elements staged through
// LDS): strong-form volume term with the element's affine factors, LIFT of
// the face jumps and a fused Runge-Kutta update in FP64 over the block's
// degrees of freedom; one of the element tiles the batched stepping chooses
// from (the single-mesh element kernel runs on the matrix cores).
// batch_* kernels: the edge and element bodies over work items of many meshes.
//
// Constant operators are read through the constant address space with
// compile-time offsets, so every matrix entry is a wave-uniform scalar load
// broadcast to the FMA.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "device.hpp"
#include "kernel_common.hpp"
#include "edge_common.hpp"

namespace ardg {

template <int N, typename T, int DM>
__global__ __launch_bounds__(256) void edge_flux_kernel(DevMesh m, const T* __restrict__ u,
                                                        T* __restrict__ flux, int nf) {
  int64_t tile;
  int field;
  tile_and_field(blockIdx.x, gridDim.x, nf, tile, field);
  const int64_t e = tile * blockDim.x + threadIdx.x;
  if (e >= m.E_int + m.E_bdy) return;
  edge_body<N, T, DM>(m, opbase<T>(m), e, field, u, flux);
}

// Several fields with constant D: one lane per interior edge takes every
// field.  The edge's table (elements, faces, apex weights, gamma, n.v) is
// read once, and the next field's element values are loaded while the
// current field's flux is formed, so only the first field waits for its
// data.  Blocks [0, nb_bdy * nf) take the boundary faces (256 per block, one
// field each), the others 256 interior edges each, in contiguous ranges per
// XCD.
template <int N, typename T>
__global__ __launch_bounds__(256) void edge_fields_kernel(DevMesh m, const T* __restrict__ u,
                                                          T* __restrict__ flux, int nb_bdy, int nf) {
  constexpr OpLayout L(N);
  constexpr int Np = L.Np, Nfp = L.Nfp;
  constexpr bool kBoth = sizeof(T) == 8 ? N <= 4 : N <= 5;
  const cptr<T> op = opbase<T>(m);
  const int64_t b = blockIdx.x;
  const int64_t nbt = (int64_t)nb_bdy * nf;
  const int64_t E = m.E_int + m.E_bdy;
  if (b < nbt) {
    const int field = (int)(b % nf);
    const int64_t e = m.E_int + (b / nf) * 256 + threadIdx.x;
    if (e < E) boundary_body<N, T, DM_CONST>(m, op, e, field, u, flux);
    return;
  }
  // nb_bdy is a multiple of 8, so b - nbt keeps b's XCD
  const int64_t e = xcd_block(b - nbt, (int64_t)gridDim.x - nbt) * 256 + threadIdx.x;
  if (e >= m.E_int) return;
  const int2 ef = m.ef[e];
  const double2 g = m.gam[e], mu1 = m.mu1[e], mu2 = m.mu2[e];
  double2 vn = make_double2(0.0, 0.0);
  if (m.conv) vn = m.vn[e];
  const int64_t k1 = ef.x & 0x3fffffff, k2 = ef.y & 0x3fffffff;
  const int fa = (int)((unsigned)ef.x >> 30), fb = (int)((unsigned)ef.y >> 30);
  const int64_t KN = m.K * Np;
  const T* u1 = u + k1 * Np;
  const T* u2 = u + k2 * Np;
  T v[2][Np];
#pragma unroll
  for (int n = 0; n < Np; ++n) {
    v[0][n] = u1[n];
    v[1][n] = u2[n];
  }
  for (int f = 0; f < nf; ++f) {
    // the next field's values (the last field loads itself again: no branch)
    const int64_t on = (int64_t)(f + 1 < nf ? f + 1 : f) * KN;
    T w[2][Np];
#pragma unroll
    for (int n = 0; n < Np; ++n) {
      w[0][n] = u1[on + n];
      w[1][n] = u2[on + n];
    }
    T t[2][Np], c[2][Np], tr1[Nfp], tr2[Nfp];
    rotate_to_face<N, T>(v[0], fa, t[0], tr1);
    rotate_to_face<N, T>(v[1], fb, t[1], tr2);
    matvec_n<Np, Np, 2, T>(op + L.n2b, t, c);
    T F[Nfp];
    interior_flux<N, T, DM_CONST, kBoth>(m, op, f, c, mu1, mu2, g, vn, 0.0, 0.0, tr1, tr2, F);
    T* out = flux + ((int64_t)f * E + e) * Nfp;
#pragma unroll
    for (int j = 0; j < Nfp; ++j) out[j] = F[j];
#pragma unroll
    for (int n = 0; n < Np; ++n) {
      v[0][n] = w[0][n];
      v[1][n] = w[1][n];
    }
  }
}

// Interior edges split by side: a block of two waves takes a tile of 64
// edges; wave s (s = 0, 1) gathers, rotates, converts and subdivides element
// s+1 of every edge and applies the columns of the reconstruction operator
// that act on that side's sub-triangle coefficients.  The operator entries
// stay wave-uniform (one column slice per wave), the serial chain of each
// wave is half that of one lane per edge, and the two partial sums meet in
// LDS.
constexpr int kSplitTile = 64;

template <int N, typename T>
struct SplitShared {
  T part[N + 1][kSplitTile];   // side 2's flux shares
};

// One side of one tile of 64 interior edges: what the wave gathers from
// memory before any arithmetic.
template <int N, typename T>
struct SplitIn {
  static constexpr int Np = (N + 1) * (N + 2) / 2;
  T v[Np];               // the side's element values
  double2 mu, g, vn;     // apex weights of this side, (gamma_R, gamma_S) sJ, n.v sJ
  double D1, D2;         // element D of both sides (Algorithms 1 and 2)
  int f;                 // this side's face
  bool valid;
  int64_t e;
};

// Wave s of the block (side s + 1) issues the loads of the tile at e0.
template <int N, typename T, int DM, bool CONV>
__device__ inline void edge_split_gather(const DevMesh& m, int64_t e0, int field, const T* __restrict__ u,
                                         SplitIn<N, T>& in) {
  constexpr int Np = SplitIn<N, T>::Np;
  const int s = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  in.valid = e0 + l < m.E_int;
  // lanes past the last edge read the tile's first edge (e0 < E_int)
  in.e = in.valid ? e0 + l : e0;
  const int2 ef = m.ef[in.e];
  in.mu = s ? m.mu2[in.e] : m.mu1[in.e];
  in.g = m.gam[in.e];
  in.vn = make_double2(0.0, 0.0);
  if (CONV) in.vn = m.vn[in.e];
  const int k1 = ef.x & 0x3fffffff, fa = (int)((unsigned)ef.x >> 30);
  const int k2 = ef.y & 0x3fffffff, fb = (int)((unsigned)ef.y >> 30);
  const int k = s ? k2 : k1;
  in.f = s ? fb : fa;
  const T* uf = u + (int64_t)field * m.K * Np;
#pragma unroll
  for (int n = 0; n < Np; ++n) in.v[n] = uf[(int64_t)k * Np + n];
  in.D1 = 0.0;
  in.D2 = 0.0;
  if (DM != DM_CONST) {
    in.D1 = m.Delem[k1];
    in.D2 = m.Delem[k2];
  }
}

// The flux of the tile from the gathered inputs (all 128 threads of the
// block: wave s takes side s + 1).  The flux is linear in each side's
// coefficients, so each wave forms its side's share of it -- the
// reconstruction operator's columns of that side, contracted with the edge's
// gamma and D one flux node at a time, and the upwind term where this side is
// upstream -- and the two shares meet in LDS (part, Nfp x 64).
template <int N, typename T, int DM, bool CONV>
__device__ inline void edge_split_finish(const DevMesh& m, int field, T* __restrict__ flux, const SplitIn<N, T>& in,
                                         T (*part)[kSplitTile]) {
  constexpr OpLayout L(N);
  constexpr int Np = L.Np, Nfp = L.Nfp, K2 = 2 * Np;
  const int64_t E = m.E_int + m.E_bdy;
  const cptr<T> op = opbase<T>(m);
  const int s = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  T t[Np], tr[Nfp], c[Np];
  rotate_to_face<N, T>(in.v, in.f, t, tr);
  // 3 rows x 4 contiguous entries per step: one 32-byte scalar load per row
  matvec_pf<Np, Np, T, 3>(op + L.n2b, t, c);
  decasteljau<N, T>(c, in.mu);
  // Algorithm 1 reduces to D (U1 - U2) when every edge of the tile has
  // D1 == D2; both waves see the same tile and take the same branch
  const bool quad = DM == DM_ALG1 && __ballot(in.valid && in.D1 != in.D2) != 0;
  const T gR = (T)in.g.x, gS = (T)in.g.y;
  T F[Nfp];
  if (DM == DM_ALG2) {
    // Algorithm 2: the constant-coefficient gradient operator, weighted per
    // diagonal node by the reconstructed coefficient
    const T D1 = (T)in.D1, D2 = (T)in.D2;
    auto emit = [&](int j, const T* a) { F[j] = alg2_coef<N, T>(op, j, D1, D2) * (gR * a[0] + gS * a[1]); };
    matvec_groups<2, Nfp, Nfp, Np, K2, T, decltype(emit), 16>(op + L.kr + s * Np, c, emit);
  } else if (quad) {
    const T D1 = (T)in.D1, D2 = (T)in.D2;
    const T a1 = D1 * gR, b1 = D1 * gS, a2 = -D2 * gR, b2 = -D2 * gS;
    matvec_groups<4, Nfp, Nfp, Np, K2, T>(op + L.u1r + s * Np, c, [&](int j, const T* a) {
      F[j] = a1 * a[0] + b1 * a[1] + a2 * a[2] + b2 * a[3];
    });
  } else {
    const T D = DM == DM_ALG1 ? (T)in.D1 : (T)field_D(m, field);
    const T a1 = D * gR, b1 = D * gS;
    auto emit = [&](int j, const T* a) { F[j] = a1 * a[0] + b1 * a[1]; };
    matvec_groups<2, Nfp, Nfp, Np, K2, T, decltype(emit), 16>(op + (DM == DM_ALG1 ? L.udr : L.kr) + s * Np, c, emit);
  }
  if (CONV) {
    // upwind: node j of side 1 meets node N - j of side 2
#pragma unroll
    for (int j = 0; j < Nfp; ++j) {
      const T tau = op[L.tau + j];
      const T vnj = (T)in.vn.x + tau * (T)(in.vn.y - in.vn.x);
      const bool up = s ? !(vnj > (T)0) : (vnj > (T)0);
      F[j] -= up ? vnj * tr[s ? N - j : j] : T(0);
    }
  }
  if (s == 1) {
#pragma unroll
    for (int j = 0; j < Nfp; ++j) part[j][l] = F[j];
  }
  __syncthreads();
  if (s == 0 && in.valid) {
    T* out = flux + ((int64_t)field * E + in.e) * Nfp;
#pragma unroll
    for (int j = 0; j < Nfp; ++j) out[j] = F[j] + part[j][l];
  }
}

// Blocks [0, nb_bdy) take the boundary faces, 128 each (mirror-ghost
// operator, one lane per face): their serial chain is the longest of the
// launch, so they start first and run beside the interior tiles.  The other
// blocks take one tile of 64 interior edges each.
template <int N, typename T, int DM, bool CONV>
__global__ __launch_bounds__(2 * kSplitTile) void edge_split_kernel(DevMesh m, const T* __restrict__ u,
                                                                    T* __restrict__ flux, int nb_bdy, int nf) {
  __shared__ SplitShared<N, T> S;
  const int64_t b = blockIdx.x;
  const int64_t nbt = (int64_t)nb_bdy * nf;
  if (b < nbt) {
    // mirror-ghost faces only (with exterior data the faces take their own
    // launch and nb_bdy is 0)
    const int field = (int)(b % nf);
    const int64_t e = m.E_int + (b / nf) * (2 * kSplitTile) + threadIdx.x;
    if (e < m.E_int + m.E_bdy) boundary_body<N, T, DM, false>(m, opbase<T>(m), e, field, u, flux);
    return;
  }
  // nb_bdy is a multiple of 8, so b - nbt keeps b's XCD
  int64_t tile;
  int field;
  tile_and_field(b - nbt, (int64_t)gridDim.x - nbt, nf, tile, field);
  SplitIn<N, T> in;
  edge_split_gather<N, T, DM, CONV>(m, tile * kSplitTile, field, u, in);
  edge_split_finish<N, T, DM, CONV>(m, field, flux, in, S.part);
}

// Batched form: persistent blocks over items of many meshes (constant D, no
// convection, nodal stage vectors): item (problem, t) with t >= 0 is the
// interior-edge tile t, with t < 0 the boundary tile -1 - t of 128 faces.
template <int N, typename T>
__global__ __launch_bounds__(2 * kSplitTile) void batch_edge_split_kernel(const BatchProb* __restrict__ probs,
                                                                          const int2* __restrict__ items,
                                                                          int nitems, int in_u) {
  __shared__ SplitShared<N, T> S;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 w = items[it];
    const BatchProb* P = probs + __builtin_amdgcn_readfirstlane(w.x);
    const int t = __builtin_amdgcn_readfirstlane(w.y);
    const T* vin = in_u ? (const T*)(const void*)P->u : (const T*)P->v;
    if (t >= 0) {
      SplitIn<N, T> in;
      edge_split_gather<N, T, DM_CONST, false>(P->m, (int64_t)t * kSplitTile, 0, vin, in);
      edge_split_finish<N, T, DM_CONST, false>(P->m, 0, (T*)P->flux, in, S.part);
    } else {
      const int64_t e = P->m.E_int + (int64_t)(-1 - t) * (2 * kSplitTile) + threadIdx.x;
      // batched meshes carry no exterior data (mirror-ghost path only)
      if (e < P->m.E_int + P->m.E_bdy)
        boundary_body<N, T, DM_CONST, false>(P->m, opbase<T>(P->m), e, 0, vin, (T*)P->flux);
    }
    __syncthreads();
  }
}

template <int N, typename T>
hipError_t batch_edge_split_t(int grid, const BatchProb* probs, const int2* items, int nitems, int in_u,
                              hipStream_t st) {
  hipLaunchKernelGGL((batch_edge_split_kernel<N, T>), dim3(grid), dim3(2 * kSplitTile), 0, st, probs, items,
                     nitems, in_u);
  return hipGetLastError();
}

constexpr int kElemBlock = 256;

// Per-element inputs besides the nodal values, loaded ahead of the compute.
template <int Nfp, typename T>
struct ElemIn {
  double2 p1, p2, p3;     // vertices
  T fv[3][Nfp];           // face fluxes, already in this element's CCW order and sign
  double D;
};

template <int N, typename T>
__device__ inline void load_elem_in(const DevMesh& m, int64_t k, int field,
                                    const T* __restrict__ flux, ElemIn<N + 1, T>& in) {
  constexpr int Nfp = N + 1;
  const int64_t E = m.E_int + m.E_bdy;
  in.p1 = m.vert[3 * k];
  in.p2 = m.vert[3 * k + 1];
  in.p3 = m.vert[3 * k + 2];
  in.D = m.dmode != DM_CONST ? m.Delem[k] : field_D(m, field);
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const int code = m.elem_face[f * m.K + k];
    const T* fe = flux + ((int64_t)field * E + (code >> 1)) * Nfp;
    const bool side2 = code & 1;
    T v[Nfp];
#pragma unroll
    for (int j = 0; j < Nfp; ++j) v[j] = fe[j];
#pragma unroll
    for (int j = 0; j < Nfp; ++j) in.fv[f][j] = side2 ? -v[Nfp - 1 - j] : v[j];
  }
}

// du/dt of one element from its nodal values u (registers):
//   q = (r_x Dr u + s_x Ds u, r_y Dr u + s_y Ds u)
//   w_r = D (r_x q_x + r_y q_y) - v_r u,  w_s = D (s_x q_x + s_y q_y) - v_s u
//   rhs = [Dr Ds] [w_r; w_s] + LIFT [(1/J) (G_f - D (sJ n)_f.q + (sJ n)_f.v u)]_f
// (strong form; convection folded into the volume pass through the
// contravariant velocity v_r = r_x v_x + r_y v_y, v_s = s_x v_x + s_y v_y; the
// face fluxes G_f arrive multiplied by sJ_f).
template <int N, typename T, bool CONV>
__device__ inline void element_rhs(const DevMesh& m, cptr<T> op, const T* u,
                                   const ElemIn<N + 1, T>& in, T* rhs) {
  constexpr OpLayout L(N);
  constexpr int Np = L.Np, Nfp = L.Nfp;
  const ElemGeom gm = elem_geom(in.p1, in.p2, in.p3);
  const T rx = (T)gm.rx, ry = (T)gm.ry, sx = (T)gm.sx, sy = (T)gm.sy;
  ElemVel ev = {};
  if (CONV) ev = elem_vel(m.vel, in.p1, gm);

  T qx[Np], qy[Np];
  {
    T urs[2 * Np];
    matvec<2 * Np, Np, T>(op + L.dr, u, urs);          // [Dr; Ds] u
#pragma unroll
    for (int i = 0; i < Np; ++i) {
      qx[i] = rx * urs[i] + sx * urs[Np + i];
      qy[i] = ry * urs[i] + sy * urs[Np + i];
    }
  }
  const T D = (T)in.D;
  T vx[Np], vy[Np];
  if (CONV) {
#pragma unroll
    for (int n = 0; n < Np; ++n) {
      const T r1 = op[L.nr + n] + T(1), s1 = op[L.ns + n] + T(1);
      vx[n] = (T)ev.x1 + r1 * (T)ev.xr + s1 * (T)ev.xs;
      vy[n] = (T)ev.y1 + r1 * (T)ev.yr + s1 * (T)ev.ys;
    }
  }
  {
    T w[2 * Np];
#pragma unroll
    for (int i = 0; i < Np; ++i) {
      w[i] = D * (rx * qx[i] + ry * qy[i]);
      w[Np + i] = D * (sx * qx[i] + sy * qy[i]);
      if (CONV) {
        w[i] -= (rx * vx[i] + ry * vy[i]) * u[i];
        w[Np + i] -= (sx * vx[i] + sy * vy[i]) * u[i];
      }
    }
    matvec<Np, 2 * Np, T>(op + L.drsh, w, rhs);        // [Dr Ds] [w_r; w_s]
  }

  // surface terms, one LIFT pass
  T jump[3 * Nfp];
  const T iJ = (T)gm.iJ;
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const double2 sn = face_sjn(gm, f);
    const T nx = (T)sn.x, ny = (T)sn.y;
#pragma unroll
    for (int j = 0; j < Nfp; ++j) {
      const int nd = fnode(N, f, j);
      T jv = in.fv[f][j] - D * (nx * qx[nd] + ny * qy[nd]);
      if (CONV) jv += (nx * vx[nd] + ny * vy[nd]) * u[nd];
      jump[f * Nfp + j] = iJ * jv;
    }
  }
  {
    T lifted[Np];
    matvec<Np, 3 * Nfp, T>(op + L.lift, jump, lifted);
#pragma unroll
    for (int i = 0; i < Np; ++i) rhs[i] += lifted[i];
  }
}

// Thread-per-element tile (VALU, scalar-broadcast operators).
template <int N, typename T, bool CONV, int TILE>
__device__ inline void element_tile(const DevMesh& m, cptr<T> op, int64_t k0, int field,
                                    const T* __restrict__ vin, const T* __restrict__ flux,
                                    const Epilogue& epi, T* sh) {
  constexpr int Np = (N + 1) * (N + 2) / 2;
  constexpr bool kPre = ElemTune<N>::prefetch;
  const int t = threadIdx.x;
  TileIO<TileShape<N, TILE, TILE>::Q, T> io;
  tile_begin<N, T, TILE>(m, k0, field, vin, epi, sh, io, kPre);
  ElemIn<N + 1, T> in;
  if (t < io.nel) load_elem_in<N, T>(m, k0 + t, field, flux, in);
  __syncthreads();
  T u[Np];
  if (t < io.nel) {
#pragma unroll
    for (int n = 0; n < Np; ++n) u[n] = sh[t * Np + n];
  }
  __syncthreads();
  if (t < io.nel) {
    T rhs[Np];
    element_rhs<N, T, CONV>(m, op, u, in, rhs);
#pragma unroll
    for (int n = 0; n < Np; ++n) sh[t * Np + n] = rhs[n];
  }
  __syncthreads();
  tile_end<N, T, TILE>(epi, sh, io, kPre);
}

// ---------------------------------------------------------------------------
// Batching: many independent meshes.  Persistent blocks walk a list of work
// items (problem, tile); every item reads its problem's descriptor (tables,
// buffers, D, dt) through wave-uniform loads and runs the same edge and
// element bodies as the single-mesh kernels.
// ---------------------------------------------------------------------------

template <int N, typename T, int TILE>
__global__ __launch_bounds__(TILE) void batch_edge_kernel(const BatchProb* __restrict__ probs,
                                                          const int2* __restrict__ items, int nitems,
                                                          int in_u) {
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 w = items[it];
    const BatchProb* P = probs + __builtin_amdgcn_readfirstlane(w.x);
    const int64_t e = (int64_t)__builtin_amdgcn_readfirstlane(w.y) * TILE + threadIdx.x;
    if (e < P->m.E_int + P->m.E_bdy) {
      const T* vin = in_u ? (const T*)(const void*)P->u : (const T*)P->v;
      edge_body<N, T, DM_CONST, false>(P->m, opbase<T>(P->m), e, 0, vin, (T*)P->flux);
    }
  }
}

template <int N, typename T, int TILE>
__global__ __launch_bounds__(TILE) __attribute__((amdgpu_waves_per_eu(ElemTune<N>::waves)))
void batch_element_kernel(const BatchProb* __restrict__ probs, const int2* __restrict__ items,
                          int nitems, Epilogue epi0, int in_u, int write_v) {
  constexpr int Np = (N + 1) * (N + 2) / 2;
  __shared__ T sh[TILE * Np];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 w = items[it];
    const BatchProb* P = probs + __builtin_amdgcn_readfirstlane(w.x);
    Epilogue epi = epi0;
    epi.u = P->u;
    epi.acc = P->acc;
    epi.vnext = write_v ? P->v : nullptr;
    epi.dt = P->dt;
    const T* vin = in_u ? (const T*)(const void*)P->u : (const T*)P->v;
    const int64_t k0 = (int64_t)__builtin_amdgcn_readfirstlane(w.y) * TILE;
    element_tile<N, T, false, TILE>(P->m, opbase<T>(P->m), k0, 0, vin, (const T*)P->flux, epi, sh);
    __syncthreads();
  }
}

__global__ void batch_to_f32_kernel(const BatchProb* __restrict__ probs, const int2* __restrict__ items,
                                    int nitems, int tile, int Np) {
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 w = items[it];
    const BatchProb* P = probs + w.x;
    const int64_t k0 = (int64_t)w.y * tile;
    const int64_t k1 = (k0 + tile < P->m.K) ? k0 + tile : P->m.K;
    float* v = (float*)P->v;
    for (int64_t i = k0 * Np + threadIdx.x; i < k1 * Np; i += blockDim.x) v[i] = (float)P->u[i];
  }
}

// Chebyshev series of the prescribed exterior state in tau = (2t - ta - tb) /
// (tb - ta), one value per thread (Clenshaw's recurrence).
__global__ void ghost_eval_kernel(const double* __restrict__ coeffs, double* __restrict__ out, int64_t n,
                                  int nt, double ta, double tb, const double* __restrict__ tbase, double toff) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double t = (tbase ? tbase[0] : 0.0) + toff;
  const double tau = (2.0 * t - ta - tb) / (tb - ta);
  const double* c = coeffs + i * nt;
  double b1 = 0.0, b2 = 0.0;
  for (int k = nt - 1; k >= 1; --k) {
    const double b0 = c[k] + 2.0 * tau * b1 - b2;
    b2 = b1;
    b1 = b0;
  }
  out[i] = c[0] + tau * b1 - b2;
}

__global__ void set_time_kernel(double* t, double value) { t[0] = value; }
__global__ void advance_time_kernel(double* t, double dt) { t[0] += dt; }

__global__ void to_f32_kernel(const double* __restrict__ s, float* __restrict__ d, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = (float)s[i];
}

__global__ void nonfinite_kernel(const double* __restrict__ x, int64_t n, int* count) {
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    bad += !isfinite(x[i]);
  if (bad) atomicAdd(count, bad);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------


// One lane per boundary face, 64 faces of one field per block (field
// b % nf): the boundary faces of the tiled launches when exterior data
// is prescribed.
template <int N, typename T, int DM>
__global__ __launch_bounds__(64) void edge_bdy_kernel(DevMesh m, const T* __restrict__ u, T* __restrict__ flux,
                                                      int nf) {
  const int field = (int)(blockIdx.x % nf);
  const int64_t e = m.E_int + (int64_t)(blockIdx.x / nf) * 64 + threadIdx.x;
  if (e < m.E_int + m.E_bdy) boundary_body<N, T, DM>(m, opbase<T>(m), e, field, u, flux);
}

template <int N, typename T>
hipError_t bdy_launch_t(const DevMesh& m, int nfields, const void* u, void* flux, hipStream_t st) {
  if (m.E_bdy == 0) return hipSuccess;
  dim3 grid((unsigned)((m.E_bdy + 63) / 64 * nfields));
#define ARDG_BDY_LAUNCH(A) \
  hipLaunchKernelGGL((edge_bdy_kernel<N, T, A>), grid, dim3(64), 0, st, m, (const T*)u, (T*)flux, nfields)
  switch (m.dmode) {
    case DM_CONST: ARDG_BDY_LAUNCH(DM_CONST); break;
    case DM_ALG1: ARDG_BDY_LAUNCH(DM_ALG1); break;
    case DM_ALG2: ARDG_BDY_LAUNCH(DM_ALG2); break;
    default: return hipErrorInvalidValue;
  }
#undef ARDG_BDY_LAUNCH
  return hipGetLastError();
}

template <typename T>
hipError_t bdy_dispatch(const DevMesh& m, int nfields, const void* u, void* flux, hipStream_t st) {
  switch (m.N) {
    case 1: return bdy_launch_t<1, T>(m, nfields, u, flux, st);
    case 2: return bdy_launch_t<2, T>(m, nfields, u, flux, st);
    case 3: return bdy_launch_t<3, T>(m, nfields, u, flux, st);
    case 4: return bdy_launch_t<4, T>(m, nfields, u, flux, st);
    case 5: return bdy_launch_t<5, T>(m, nfields, u, flux, st);
    case 6: return bdy_launch_t<6, T>(m, nfields, u, flux, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_boundary_faces(const DevMesh& m, bool f64, int nfields, const void* u, void* flux,
                                 hipStream_t st) {
  return f64 ? bdy_dispatch<double>(m, nfields, u, flux, st) : bdy_dispatch<float>(m, nfields, u, flux, st);
}

template <int N, typename T>
hipError_t edge_launch_t(const DevMesh& m, int nfields, const void* u, void* flux, hipStream_t st) {
  const int64_t E = m.E_int + m.E_bdy;
  if (E == 0) return hipSuccess;
  // several FP32 fields with constant D: the multi-field lanes (708x708 N = 3,
  // four fields: 89.0 us against 92.4 us; no gain in FP64, whose lanes hold
  // more registers)
  if (m.edge_kernel == EDGE_FIELDS || (m.edge_kernel == EDGE_AUTO && sizeof(T) == 4 && nfields > 1 &&
                                        m.dmode == DM_CONST && N <= 4)) {
    if (m.dmode != DM_CONST) return hipErrorInvalidValue;
    const int64_t nbb = ((m.E_bdy + 255) / 256 + 7) / 8 * 8;
    const int64_t nbi = (m.E_int + 255) / 256;
    hipLaunchKernelGGL((edge_fields_kernel<N, T>), dim3((unsigned)(nbb * nfields + nbi)), dim3(256), 0, st, m,
                       (const T*)u, (T*)flux, (int)nbb, nfields);
    return hipGetLastError();
  }
  bool split = m.edge_kernel == EDGE_SPLIT;
  if (m.edge_kernel == EDGE_AUTO) {
    // one thread per edge: about 8 waves per SIMD (1024 SIMDs) hide the
    // latency of its serial chain; below that, or at orders whose register
    // use leaves few waves resident, the side-split tiles are faster
    const int64_t lane_waves = (m.E_int * nfields + 63) / 64;
    split = N >= 5 || lane_waves < 8 * 1024;
  }
  if (split) {
    const int64_t nbi = (m.E_int + kSplitTile - 1) / kSplitTile;
    int64_t nbb = ((m.E_bdy + 2 * kSplitTile - 1) / (2 * kSplitTile) + 7) / 8 * 8;
    if (m.ghost) {
      const hipError_t eb = launch_boundary_faces(m, sizeof(T) == 8, nfields, u, flux, st);
      if (eb != hipSuccess) return eb;
      nbb = 0;
    }
    if (nbi + nbb == 0) return hipSuccess;
    dim3 grid((unsigned)((nbi + nbb) * nfields));
#define ARDG_SPLIT_LAUNCH(A, C)                                                                  \
  hipLaunchKernelGGL((edge_split_kernel<N, T, A, C>), grid, dim3(2 * kSplitTile), 0, st, m,       \
                     (const T*)u, (T*)flux, (int)nbb, nfields)
    switch (m.dmode * 2 + (m.conv ? 1 : 0)) {
      case 0: ARDG_SPLIT_LAUNCH(DM_CONST, false); break;
      case 1: ARDG_SPLIT_LAUNCH(DM_CONST, true); break;
      case 2: ARDG_SPLIT_LAUNCH(DM_ALG1, false); break;
      case 3: ARDG_SPLIT_LAUNCH(DM_ALG1, true); break;
      case 4: ARDG_SPLIT_LAUNCH(DM_ALG2, false); break;
      case 5: ARDG_SPLIT_LAUNCH(DM_ALG2, true); break;
      default: return hipErrorInvalidValue;
    }
#undef ARDG_SPLIT_LAUNCH
    return hipGetLastError();
  }
  dim3 grid((unsigned)((E + 255) / 256 * nfields));
#define ARDG_LANE_LAUNCH(A) \
  hipLaunchKernelGGL((edge_flux_kernel<N, T, A>), grid, dim3(256), 0, st, m, (const T*)u, (T*)flux, nfields)
  switch (m.dmode) {
    case DM_CONST: ARDG_LANE_LAUNCH(DM_CONST); break;
    case DM_ALG1: ARDG_LANE_LAUNCH(DM_ALG1); break;
    case DM_ALG2: ARDG_LANE_LAUNCH(DM_ALG2); break;
    default: return hipErrorInvalidValue;
  }
#undef ARDG_LANE_LAUNCH
  return hipGetLastError();
}

#define ARDG_DISPATCH_N(FN, ...)                   \
  switch (m.N) {                                   \
    case 1: return FN<1, T>(__VA_ARGS__);          \
    case 2: return FN<2, T>(__VA_ARGS__);          \
    case 3: return FN<3, T>(__VA_ARGS__);          \
    case 4: return FN<4, T>(__VA_ARGS__);          \
    case 5: return FN<5, T>(__VA_ARGS__);          \
    case 6: return FN<6, T>(__VA_ARGS__);          \
    default: return hipErrorInvalidValue;          \
  }

template <typename T>
hipError_t edge_dispatch(const DevMesh& m, int nf, const void* u, void* flux, hipStream_t st) {
  ARDG_DISPATCH_N(edge_launch_t, m, nf, u, flux, st)
}

hipError_t launch_edge_flux(const DevMesh& m, int prec, int nfields, const void* u, void* flux, hipStream_t st) {
  // the Navier-Stokes system takes its four fields together
  if (m.ns != NS_OFF) return nfields == 4 ? launch_edge_ns(m, prec, u, flux, st) : hipErrorInvalidValue;
  // a nodal tensor coefficient has one kernel (whatever edge kernel is chosen)
  if (m.dmode == DM_NODAL || m.dmode == DM_SOLUTION) return launch_edge_tensor(m, prec, nfields, u, flux, st);
  // split-BF16 products exist only on the matrix cores: side-split tiles up
  // to N = 3, one wave per tile above (measured faster).  FP64 from N = 5 on
  // also converts on the matrix cores (512x512 N = 6: 238 us against 271 us
  // on the vector unit)
  if (m.edge_kernel == EDGE_SPLIT_MFMA ||
      (m.edge_kernel == EDGE_AUTO && ((prec == PREC_BF16X3 && m.N <= 3) || (prec == PREC_FP64 && m.N >= 5))))
    return launch_edge_split_mfma(m, prec, nfields, u, flux, st);
  if (m.edge_kernel == EDGE_MFMA || prec == PREC_BF16X3) return launch_edge_mfma(m, prec, nfields, u, flux, st);
  return prec == PREC_FP64 ? edge_dispatch<double>(m, nfields, u, flux, st)
                           : edge_dispatch<float>(m, nfields, u, flux, st);
}

hipError_t launch_element(const DevMesh& m, int prec, int nfields, const void* vin, const void* flux,
                          const Epilogue& epi, hipStream_t st) {
  if (m.ns != NS_OFF) return nfields == 4 ? launch_element_ns(m, prec, vin, flux, epi, st) : hipErrorInvalidValue;
  return launch_element_mfma(m, prec, nfields, vin, flux, epi, st);
}

template <int N, typename T>
hipError_t batch_edge_t(int tile, int grid, const BatchProb* probs, const int2* items, int nitems,
                        int in_u, hipStream_t st) {
  switch (tile) {
    case 64: hipLaunchKernelGGL((batch_edge_kernel<N, T, 64>), dim3(grid), dim3(64), 0, st, probs, items, nitems, in_u); break;
    case 128: hipLaunchKernelGGL((batch_edge_kernel<N, T, 128>), dim3(grid), dim3(128), 0, st, probs, items, nitems, in_u); break;
    case 256: hipLaunchKernelGGL((batch_edge_kernel<N, T, 256>), dim3(grid), dim3(256), 0, st, probs, items, nitems, in_u); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int N, typename T>
hipError_t batch_elem_t(int tile, int grid, const BatchProb* probs, const int2* items, int nitems,
                        const Epilogue& epi, int in_u, int write_v, hipStream_t st) {
  switch (tile) {
    case 64: hipLaunchKernelGGL((batch_element_kernel<N, T, 64>), dim3(grid), dim3(64), 0, st, probs, items, nitems, epi, in_u, write_v); break;
    case 128: hipLaunchKernelGGL((batch_element_kernel<N, T, 128>), dim3(grid), dim3(128), 0, st, probs, items, nitems, epi, in_u, write_v); break;
    case 256: hipLaunchKernelGGL((batch_element_kernel<N, T, 256>), dim3(grid), dim3(256), 0, st, probs, items, nitems, epi, in_u, write_v); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

#define ARDG_BATCH_N(FN, N, ...)                   \
  switch (N) {                                     \
    case 1: return FN<1, T>(__VA_ARGS__);          \
    case 2: return FN<2, T>(__VA_ARGS__);          \
    case 3: return FN<3, T>(__VA_ARGS__);          \
    case 4: return FN<4, T>(__VA_ARGS__);          \
    case 5: return FN<5, T>(__VA_ARGS__);          \
    case 6: return FN<6, T>(__VA_ARGS__);          \
    default: return hipErrorInvalidValue;          \
  }

template <typename T>
hipError_t batch_edge_dispatch(int N, int tile, int grid, const BatchProb* probs, const int2* items,
                               int nitems, int in_u, hipStream_t st) {
  ARDG_BATCH_N(batch_edge_t, N, tile, grid, probs, items, nitems, in_u, st)
}

template <typename T>
hipError_t batch_elem_dispatch(int N, int tile, int grid, const BatchProb* probs, const int2* items,
                               int nitems, const Epilogue& epi, int in_u, int write_v, hipStream_t st) {
  ARDG_BATCH_N(batch_elem_t, N, tile, grid, probs, items, nitems, epi, in_u, write_v, st)
}

hipError_t launch_batch_edge(int N, bool fp64, int tile, int grid, const BatchProb* probs,
                             const int2* items, int nitems, int in_u, hipStream_t st) {
  if (nitems == 0) return hipSuccess;
  if (tile == 0) {
    // side-split tiles (items as built for tile code 0)
    switch (N) {
      case 1: return fp64 ? batch_edge_split_t<1, double>(grid, probs, items, nitems, in_u, st)
                          : batch_edge_split_t<1, float>(grid, probs, items, nitems, in_u, st);
      case 2: return fp64 ? batch_edge_split_t<2, double>(grid, probs, items, nitems, in_u, st)
                          : batch_edge_split_t<2, float>(grid, probs, items, nitems, in_u, st);
      case 3: return fp64 ? batch_edge_split_t<3, double>(grid, probs, items, nitems, in_u, st)
                          : batch_edge_split_t<3, float>(grid, probs, items, nitems, in_u, st);
      case 4: return fp64 ? batch_edge_split_t<4, double>(grid, probs, items, nitems, in_u, st)
                          : batch_edge_split_t<4, float>(grid, probs, items, nitems, in_u, st);
      case 5: return fp64 ? batch_edge_split_t<5, double>(grid, probs, items, nitems, in_u, st)
                          : batch_edge_split_t<5, float>(grid, probs, items, nitems, in_u, st);
      case 6: return fp64 ? batch_edge_split_t<6, double>(grid, probs, items, nitems, in_u, st)
                          : batch_edge_split_t<6, float>(grid, probs, items, nitems, in_u, st);
      default: return hipErrorInvalidValue;
    }
  }
  return fp64 ? batch_edge_dispatch<double>(N, tile, grid, probs, items, nitems, in_u, st)
              : batch_edge_dispatch<float>(N, tile, grid, probs, items, nitems, 0, st);
}

hipError_t launch_batch_element(int N, bool fp64, int tile, int grid, const BatchProb* probs,
                                const int2* items, int nitems, const Epilogue& epi, int in_u,
                                int write_v, hipStream_t st) {
  // tile code 0: 64-element tiles on the matrix cores
  if (tile == 0) return launch_batch_element_mfma(N, fp64, grid, probs, items, nitems, epi, in_u, write_v, st);
  if (nitems == 0) return hipSuccess;
  return fp64 ? batch_elem_dispatch<double>(N, tile, grid, probs, items, nitems, epi, in_u, write_v, st)
              : batch_elem_dispatch<float>(N, tile, grid, probs, items, nitems, epi, 0, write_v, st);
}

hipError_t launch_batch_to_f32(const BatchProb* probs, const int2* items, int nitems, int tile,
                               int Np, int grid, hipStream_t st) {
  if (nitems == 0) return hipSuccess;
  hipLaunchKernelGGL(batch_to_f32_kernel, dim3(grid), dim3(256), 0, st, probs, items, nitems, tile, Np);
  return hipGetLastError();
}

hipError_t launch_ghost_eval(const double* coeffs, double* out, int64_t n, int nt, double ta, double tb,
                             const double* tbase, double toff, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(ghost_eval_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, coeffs, out, n, nt,
                     ta, tb, tbase, toff);
  return hipGetLastError();
}

hipError_t launch_set_time(double* t, double value, hipStream_t st) {
  hipLaunchKernelGGL(set_time_kernel, dim3(1), dim3(1), 0, st, t, value);
  return hipGetLastError();
}

hipError_t launch_advance_time(double* t, double dt, hipStream_t st) {
  hipLaunchKernelGGL(advance_time_kernel, dim3(1), dim3(1), 0, st, t, dt);
  return hipGetLastError();
}

hipError_t launch_to_f32(const double* src, float* dst, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(to_f32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_nonfinite(const double* x, int64_t n, int* count_dev, hipStream_t st) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(nonfinite_kernel, dim3((unsigned)blocks), dim3(256), 0, st, x, n, count_dev);
  return hipGetLastError();
}

}  // namespace ardg
