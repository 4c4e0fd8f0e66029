// Interior edges in tiles whose elements are staged through LDS.
//
// The interior edges are cut, in their stored order, into tiles of at most
// 256 edges that together touch at most 256 distinct elements (built once
// per mesh; the edges of one element row share most of their elements).  A
// block takes one (tile, field):
//   1. the tile's distinct elements are copied into LDS with wide, coalesced
//      loads (consecutive threads read consecutive chunks of the sorted
//      element list), instead of every lane gathering both of its edge's
//      elements value by value;
//   2. each distinct element is converted once from nodal values to
//      Bernstein coefficients on I (constant matrix, eq.
//      NodalToModalProjection in Bernstein form), instead of once per edge
//      side;
//   3. one lane per edge reads its two sides' coefficients in the face's
//      rotated frame (section "Reordering nodes in the reference domain"):
//      the vertex relabelling permutes Bernstein multi-indices exactly as it
//      permutes the lattice of nodes, so the rotation is an LDS address
//      permutation; then the de Casteljau subdivision at the apex (eq.
//      totalProjection), the reconstruction operator on the diagonal
//      (Algorithm aRDG; Algorithms 1 and 2 with element-wise D) and the upwind
//      flux from the sides' face traces (1D Bernstein -> LGL values) follow
//      as in the one-lane-per-edge kernel.
// Boundary faces take the first blocks of the launch, one lane per face.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.hpp"
#include "kernel_common.hpp"
#include "edge_common.hpp"

namespace ardg {

constexpr int kStageTile = 256;   // edges and distinct elements per tile, threads per block

template <int B> struct ChunkOf;
template <> struct ChunkOf<16> { typedef uint4 type; };
template <> struct ChunkOf<8> { typedef uint2 type; };
template <> struct ChunkOf<4> { typedef unsigned type; };

// One element's Np values move as CH chunks of CB bytes (the widest of 16,
// 8, 4 bytes dividing the element's size, so every chunk is aligned).
template <int N, typename T>
struct StageShape {
  static constexpr int Np = (N + 1) * (N + 2) / 2;
  static constexpr int BYTES = Np * (int)sizeof(T);
  static constexpr int CB = BYTES % 16 == 0 ? 16 : (BYTES % 8 == 0 ? 8 : 4);
  static constexpr int CH = BYTES / CB;
};

// Bernstein coefficients of one element (LDS, unrotated order) read in the
// frame that puts face f on the hypotenuse: slot (i, j) of the rotated
// lattice is slot (j, N-i-j) for face 0, (i, j) for face 1 and (N-i-j, i)
// for face 2 of the element's own lattice.
template <int N, typename T>
__device__ inline void read_rotated(const T* e, int f, T* t) {
#pragma unroll
  for (int j = 0; j <= N; ++j)
#pragma unroll
    for (int i = 0; i <= N - j; ++i) {
      const int o0 = lat(N, j, N - i - j), o1 = lat(N, i, j), o2 = lat(N, N - i - j, i);
      const int o = (f == 0) ? o0 : ((f == 1) ? o1 : o2);
      t[lat(N, i, j)] = e[o];
    }
}

template <int N, typename T, int DM, bool CONV>
__global__ __launch_bounds__(kStageTile) void edge_staged_kernel(DevMesh m, const T* __restrict__ u,
                                                                 T* __restrict__ flux, int nb_bdy, int nf) {
  using SS = StageShape<N, T>;
  constexpr OpLayout L(N);
  constexpr int Np = SS::Np, Nfp = N + 1, CH = SS::CH, CB = SS::CB, CE = CB / (int)sizeof(T);
  constexpr bool kPF = sizeof(T) == 8 ? N <= 4 : N <= 5;
  typedef typename ChunkOf<CB>::type C;
  __shared__ __align__(16) T sb[kStageTile * Np];
  __shared__ double sD[DM != DM_CONST ? kStageTile : 1];
  const cptr<T> op = opbase<T>(m);
  const int64_t b = blockIdx.x;
  const int64_t nbt = (int64_t)nb_bdy * nf;
  if (b < nbt) {
    const int field = (int)(b % nf);
    const int64_t e = m.E_int + (b / nf) * kStageTile + threadIdx.x;
    if (e < m.E_int + m.E_bdy) boundary_body<N, T, DM>(m, op, e, field, u, flux);
    return;
  }
  // nb_bdy is a multiple of 8, so b - nbt keeps b's XCD
  int64_t tile;
  int field;
  tile_and_field(b - nbt, (int64_t)gridDim.x - nbt, nf, tile, field);
  const int tid = threadIdx.x;
  const int2 t0 = m.stiles[tile], t1 = m.stiles[tile + 1];
  const int ne = t1.x - t0.x, nu = t1.y - t0.y;
  const int nchunk = nu * CH;

  // ---- loads: the distinct elements' indices, then their values in chunks
  // (clamped indices, masked at the LDS store), and this lane's edge ----
  const T* uf = u + (int64_t)field * m.K * Np;
  int g[CH];
#pragma unroll
  for (int q = 0; q < CH; ++q) {
    const int idx = tid + q * kStageTile;
    g[q] = m.sulist[t0.y + (idx < nchunk ? idx / CH : 0)];
  }
  const bool valid = tid < ne;
  const int64_t e = t0.x + (valid ? tid : 0);
  const unsigned loc = m.seloc[e];
  const double2 gm = m.gam[e], mu1 = m.mu1[e], mu2 = m.mu2[e];
  double2 vn = make_double2(0.0, 0.0);
  if (CONV) vn = m.vn[e];
  double Du = 0.0;
  if (DM != DM_CONST) Du = m.Delem[m.sulist[t0.y + (tid < nu ? tid : 0)]];
  C x[CH];
#pragma unroll
  for (int q = 0; q < CH; ++q) {
    const int idx = tid + q * kStageTile;
    const int c = idx - (idx / CH) * CH;
    x[q] = ((const C*)(uf + (int64_t)g[q] * Np))[c];
  }
#pragma unroll
  for (int q = 0; q < CH; ++q) {
    const int idx = tid + q * kStageTile;
    if (idx < nchunk) {
      const int j = idx / CH, c = idx - j * CH;
      ((C*)(sb + j * Np))[c] = x[q];
    }
  }
  if (DM != DM_CONST && tid < nu) sD[tid] = Du;
  (void)CE;
  __syncthreads();

  // ---- nodal -> Bernstein, once per distinct element ----
  if (tid < nu) {
    T v[Np], c[Np];
#pragma unroll
    for (int n = 0; n < Np; ++n) v[n] = sb[tid * Np + n];
    matvec_sel<kPF, Np, Np, T>(op + L.n2b, v, c);
#pragma unroll
    for (int n = 0; n < Np; ++n) sb[tid * Np + n] = c[n];
  }
  __syncthreads();
  if (!valid) return;

  // ---- one lane per edge ----
  const int l1 = loc & 0xff, l2 = (loc >> 8) & 0xff;
  const int fa = (loc >> 16) & 3, fb = (loc >> 18) & 3;
  T c[2][Np];
  read_rotated<N, T>(sb + l1 * Np, fa, c[0]);
  read_rotated<N, T>(sb + l2 * Np, fb, c[1]);
  T tr1[Nfp], tr2[Nfp];
#pragma unroll
  for (int j = 0; j <= N; ++j) {
    tr1[j] = CONV ? c[0][lat(N, N - j, j)] : T(0);
    tr2[j] = CONV ? c[1][lat(N, N - j, j)] : T(0);
  }
  if (CONV) {
    // nodal traces on the face from its 1D Bernstein coefficients
    face_bernstein_to_nodal<N, T>(op, tr1);
    face_bernstein_to_nodal<N, T>(op, tr2);
  }
  double D1d = 0.0, D2d = 0.0;
  if (DM != DM_CONST) {
    D1d = sD[l1];
    D2d = sD[l2];
  }
  T F[Nfp];
  interior_flux<N, T, DM, kPF>(m, op, field, c, mu1, mu2, gm, vn, D1d, D2d, tr1, tr2, F);
  T* out = flux + ((int64_t)field * (m.E_int + m.E_bdy) + e) * Nfp;
#pragma unroll
  for (int j = 0; j < Nfp; ++j) out[j] = F[j];
}

template <int N, typename T>
hipError_t edge_staged_t(const DevMesh& m, int nfields, const void* u, void* flux, hipStream_t st) {
  if (m.E_int + m.E_bdy == 0) return hipSuccess;
  if (m.E_int > 0 && (!m.stiles || m.ntiles <= 0)) return hipErrorInvalidValue;
  const int64_t nbb = ((m.E_bdy + kStageTile - 1) / kStageTile + 7) / 8 * 8;
  dim3 grid((unsigned)((nbb + m.ntiles) * nfields));
#define ARDG_STAGED_LAUNCH(A, CV)                                                                   \
  hipLaunchKernelGGL((edge_staged_kernel<N, T, A, CV>), grid, dim3(kStageTile), 0, st, m, (const T*)u, \
                     (T*)flux, (int)nbb, nfields)
  switch (m.dmode * 2 + (m.conv ? 1 : 0)) {
    case 0: ARDG_STAGED_LAUNCH(DM_CONST, false); break;
    case 1: ARDG_STAGED_LAUNCH(DM_CONST, true); break;
    case 2: ARDG_STAGED_LAUNCH(DM_ALG1, false); break;
    case 3: ARDG_STAGED_LAUNCH(DM_ALG1, true); break;
    case 4: ARDG_STAGED_LAUNCH(DM_ALG2, false); break;
    case 5: ARDG_STAGED_LAUNCH(DM_ALG2, true); break;
    default: return hipErrorInvalidValue;
  }
#undef ARDG_STAGED_LAUNCH
  return hipGetLastError();
}

template <typename T>
hipError_t edge_staged_dispatch(const DevMesh& m, int nf, const void* u, void* flux, hipStream_t st) {
  switch (m.N) {
    case 1: return edge_staged_t<1, T>(m, nf, u, flux, st);
    case 2: return edge_staged_t<2, T>(m, nf, u, flux, st);
    case 3: return edge_staged_t<3, T>(m, nf, u, flux, st);
    case 4: return edge_staged_t<4, T>(m, nf, u, flux, st);
    case 5: return edge_staged_t<5, T>(m, nf, u, flux, st);
    case 6: return edge_staged_t<6, T>(m, nf, u, flux, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_edge_staged(const DevMesh& m, int prec, int nfields, const void* u, void* flux,
                              hipStream_t st) {
  switch (prec) {
    case PREC_FP64: return edge_staged_dispatch<double>(m, nfields, u, flux, st);
    case PREC_FP32: return edge_staged_dispatch<float>(m, nfields, u, flux, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ardg
