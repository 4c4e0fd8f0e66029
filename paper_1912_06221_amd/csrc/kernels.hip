// gfx950 kernels of the affine-reconstructed nodal DG right-hand side.
//
// edge_flux_kernel (one thread per edge): Algorithm aRDG for one edge and the
// flux on the diagonal of its enclosed parallelogram.
//   1. gather the Np nodal values of each side and apply the face's node
//      reordering (section "Reordering nodes in the reference domain") as a
//      register permutation;
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
//   5. write Nfp values per edge (no atomics: each edge owns its slot).
// element_kernel (one thread per element, the block's elements staged through
// LDS): strong-form volume term with the element's affine factors,
// (J_f/J) LIFT_f of the face jumps, optional convective volume term, and a
// fused Runge-Kutta update in FP64 over the block's degrees of freedom.
//
// Constant operators are read through the constant address space with
// compile-time offsets, so every matrix entry is a wave-uniform scalar load
// broadcast to the FMA.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "device.hpp"
#include "kernel_common.hpp"

namespace ardg {
template <int ROWS, int COLS, typename T>
__device__ inline void matvec(cptr<T> A0, const T* x, T* y);

// Load one element, rotate so that face f is the hypotenuse, convert to
// Bernstein coefficients and subdivide at the apex (mu = weights of w2, w3).
// trace[j] receives the element's values on face f, counter-clockwise.
template <int N, typename T>
__device__ inline void subtriangle_coeffs(const T* __restrict__ ue, int f, double2 mu,
                                          cptr<T> n2b, T* c, T* trace) {
  constexpr int Np = (N + 1) * (N + 2) / 2;
  T v[Np];
#pragma unroll
  for (int n = 0; n < Np; ++n) v[n] = ue[n];
  T t[Np];
#pragma unroll
  for (int j = 0; j <= N; ++j)
#pragma unroll
    for (int i = 0; i <= N - j; ++i) {
      const T a0 = v[lat(N, j, N - i - j)];   // face (v1,v2): w = (v3, v1, v2)
      const T a1 = v[lat(N, i, j)];           // face (v2,v3): identity
      const T a2 = v[lat(N, N - i - j, i)];   // face (v3,v1): w = (v2, v3, v1)
      t[lat(N, i, j)] = (f == 0) ? a0 : ((f == 1) ? a1 : a2);
    }
#pragma unroll
  for (int j = 0; j <= N; ++j) trace[j] = t[lat(N, N - j, j)];
  matvec<Np, Np, T>(n2b, t, c);
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

// y = A x for a constant row-major ROWS x COLS operator A.  Each row's entries
// are wave-uniform scalar loads feeding scalar-operand FMAs; the row fence and
// the fresh pointer keep one row in flight at a time (without them the whole
// operator is hoisted into SGPRs and spilled).
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

template <int N, typename T, bool ALG1>
__device__ inline void edge_body(const DevMesh& m, cptr<T> op, int64_t e, int field,
                                 const T* __restrict__ u, T* __restrict__ flux) {
  constexpr OpLayout L(N);
  constexpr int Np = L.Np, Nfp = L.Nfp;
  const int64_t E = m.E_int + m.E_bdy;
  const T* uf = u + (int64_t)field * m.K * Np;
  T F[Nfp];
  T tr1[Nfp], tr2[Nfp];
  double2 vn = make_double2(0.0, 0.0);
  if (e < m.E_int) {
    const int2 ef = m.ef[e];
    const int k1 = ef.x & 0x3fffffff, fa = (int)((unsigned)ef.x >> 30);
    const int k2 = ef.y & 0x3fffffff, fb = (int)((unsigned)ef.y >> 30);
    const double2 g = m.gam[e];
    T c[2 * Np];
    subtriangle_coeffs<N, T>(uf + (int64_t)k1 * Np, fa, m.mu1[e], op + L.n2b, c, tr1);
    subtriangle_coeffs<N, T>(uf + (int64_t)k2 * Np, fb, m.mu2[e], op + L.n2b, c + Np, tr2);
    const T gR = (T)g.x, gS = (T)g.y;
    if (ALG1) {
      const double D1d = m.Delem[k1], D2d = m.Delem[k2];
      const T D1 = (T)D1d, D2 = (T)D2d;
      if (D1d == D2d) {
        // equal coefficients: Algorithm 1 reduces exactly to D (U1 - U2) c
        T g[2 * Nfp];
        matvec<2 * Nfp, 2 * Np, T>(op + L.udr, c, g);
#pragma unroll
        for (int j = 0; j < Nfp; ++j) F[j] = D1 * (gR * g[j] + gS * g[Nfp + j]);
      } else {
        T g[4 * Nfp];
        matvec<4 * Nfp, 2 * Np, T>(op + L.u1r, c, g);
#pragma unroll
        for (int j = 0; j < Nfp; ++j)
          F[j] = D1 * (gR * g[j] + gS * g[Nfp + j]) - D2 * (gR * g[2 * Nfp + j] + gS * g[3 * Nfp + j]);
      }
    } else {
      const T D = (T)m.Dfield[field];
      T g[2 * Nfp];
      matvec<2 * Nfp, 2 * Np, T>(op + L.kr, c, g);
#pragma unroll
      for (int j = 0; j < Nfp; ++j) F[j] = D * (gR * g[j] + gS * g[Nfp + j]);
    }
    if (m.conv) vn = m.vn[e];
  } else {
    const int64_t b = e - m.E_int;
    const int kb = m.bk[b];
    const int k = kb & 0x3fffffff, fa = (int)((unsigned)kb >> 30);
    const double2 g = m.bgam[b];
    T c[Np];
    subtriangle_coeffs<N, T>(uf + (int64_t)k * Np, fa, m.bmu[b], op + L.n2b, c, tr1);
    const T gR = (T)g.x, gS = (T)g.y;
    const T D = ALG1 ? (T)m.Delem[k] : (T)m.Dfield[field];
    T gb[2 * Nfp];
    matvec<2 * Nfp, Np, T>(op + (ALG1 ? L.ubr : L.kbr), c, gb);
#pragma unroll
    for (int j = 0; j < Nfp; ++j) F[j] = D * (gR * gb[j] + gS * gb[Nfp + j]);
#pragma unroll
    for (int j = 0; j < Nfp; ++j) tr2[j] = 0;   // u+ = 0 outside the domain
    if (m.conv) vn = m.vn[e];
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
  T* out = flux + ((int64_t)field * E + e) * Nfp;
#pragma unroll
  for (int j = 0; j < Nfp; ++j) out[j] = F[j];
}

template <int N, typename T, bool ALG1>
__global__ __launch_bounds__(256) void edge_flux_kernel(DevMesh m, const T* __restrict__ u,
                                                        T* __restrict__ flux) {
  const int64_t e = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (e >= m.E_int + m.E_bdy) return;
  edge_body<N, T, ALG1>(m, opbase<T>(m), e, blockIdx.y, u, flux);
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
  in.D = m.alg1 ? m.Delem[k] : m.Dfield[field];
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

// du/dt of one element from its nodal values u (registers).
template <int N, typename T, bool CONV>
__device__ inline void element_rhs(const DevMesh& m, cptr<T> op, const T* u,
                                   const ElemIn<N + 1, T>& in, T* rhs) {
  constexpr OpLayout L(N);
  constexpr int Np = L.Np, Nfp = L.Nfp;
  // affine factors of this element (eqs. mapping_tri_diff, triangle_jacobian_a/b)
  const double2 p1 = in.p1, p2 = in.p2, p3 = in.p3;
  const double xr = 0.5 * (p2.x - p1.x), yr = 0.5 * (p2.y - p1.y);
  const double xs = 0.5 * (p3.x - p1.x), ys = 0.5 * (p3.y - p1.y);
  const double J = xr * ys - xs * yr;
  const T rx = (T)(ys / J), ry = (T)(-xs / J), sx = (T)(-yr / J), sy = (T)(xr / J);

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
  {
    T w[2 * Np];
#pragma unroll
    for (int i = 0; i < Np; ++i) {
      w[i] = rx * qx[i] + ry * qy[i];
      w[Np + i] = sx * qx[i] + sy * qy[i];
    }
    T div[Np];
    matvec<Np, 2 * Np, T>(op + L.drsh, w, div);        // [Dr Ds] [wr; ws]
#pragma unroll
    for (int i = 0; i < Np; ++i) rhs[i] = D * div[i];
  }

  T vx[Np], vy[Np];
  if (CONV) {
#pragma unroll
    for (int n = 0; n < Np; ++n) {
      const double r = (double)op[L.nr + n], s = (double)op[L.ns + n];
      const double x = 0.5 * (-(r + s) * p1.x + (r + 1.0) * p2.x + (s + 1.0) * p3.x);
      const double y = 0.5 * (-(r + s) * p1.y + (r + 1.0) * p2.y + (s + 1.0) * p3.y);
      vx[n] = (T)(m.vel[0] + m.vel[2] * x + m.vel[3] * y);
      vy[n] = (T)(m.vel[1] + m.vel[4] * x + m.vel[5] * y);
    }
  }

  // surface terms: (J_f / J) LIFT_f (F_f - D n.q + [n.v u-]), one LIFT pass
  T jump[3 * Nfp];
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const double2 a = (f == 0) ? p1 : (f == 1 ? p2 : p3);
    const double2 b = (f == 0) ? p2 : (f == 1 ? p3 : p1);
    const double tx = b.x - a.x, ty = b.y - a.y;
    const double len = sqrt(tx * tx + ty * ty);
    const T nx = (T)(ty / len), ny = (T)(-tx / len);
    const T scale = (T)(0.5 * len / J);
#pragma unroll
    for (int j = 0; j < Nfp; ++j) {
      const T G = in.fv[f][j];
      const int nd = fnode(N, f, j);
      T jv = G - D * (nx * qx[nd] + ny * qy[nd]);
      if (CONV) jv += (nx * vx[nd] + ny * vy[nd]) * u[nd];
      jump[f * Nfp + j] = scale * jv;
    }
  }
  {
    T lifted[Np];
    matvec<Np, 3 * Nfp, T>(op + L.lift, jump, lifted);
#pragma unroll
    for (int i = 0; i < Np; ++i) rhs[i] += lifted[i];
  }

  if (CONV) {
    // -(d/dx (vx u) + d/dy (vy u)), nodal collocation of the flux vector
    T fx[Np], fy[Np];
#pragma unroll
    for (int n = 0; n < Np; ++n) {
      fx[n] = vx[n] * u[n];
      fy[n] = vy[n] * u[n];
    }
    T dfx[2 * Np], dfy[2 * Np];
    matvec<2 * Np, Np, T>(op + L.dr, fx, dfx);
    matvec<2 * Np, Np, T>(op + L.dr, fy, dfy);
#pragma unroll
    for (int i = 0; i < Np; ++i)
      rhs[i] -= rx * dfx[i] + sx * dfx[Np + i] + ry * dfy[i] + sy * dfy[Np + i];
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
  TileIO<Np> io;
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

template <int N, typename T, bool CONV>
__global__ __launch_bounds__(kElemBlock) __attribute__((amdgpu_waves_per_eu(ElemTune<N>::waves)))
void element_kernel(DevMesh m, const T* __restrict__ vin, const T* __restrict__ flux, Epilogue epi) {
  constexpr int Np = (N + 1) * (N + 2) / 2;
  __shared__ T sh[kElemBlock * Np];
  const int64_t k0 = xcd_block(blockIdx.x, gridDim.x) * kElemBlock;
  element_tile<N, T, CONV, kElemBlock>(m, opbase<T>(m), k0, blockIdx.y, vin, flux, epi, sh);
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
      edge_body<N, T, false>(P->m, opbase<T>(P->m), e, 0, vin, (T*)P->flux);
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

template <int N, typename T>
hipError_t edge_launch_t(const DevMesh& m, int nfields, const void* u, void* flux, hipStream_t st) {
  const int64_t E = m.E_int + m.E_bdy;
  if (E == 0) return hipSuccess;
  dim3 grid((unsigned)((E + 255) / 256), (unsigned)nfields);
  if (m.alg1)
    hipLaunchKernelGGL((edge_flux_kernel<N, T, true>), grid, dim3(256), 0, st, m, (const T*)u, (T*)flux);
  else
    hipLaunchKernelGGL((edge_flux_kernel<N, T, false>), grid, dim3(256), 0, st, m, (const T*)u, (T*)flux);
  return hipGetLastError();
}

template <int N, typename T>
hipError_t elem_launch_t(const DevMesh& m, int nfields, const void* vin, const void* flux,
                         const Epilogue& epi, hipStream_t st) {
  dim3 grid((unsigned)((m.K + kElemBlock - 1) / kElemBlock), (unsigned)nfields);
  if (m.conv)
    hipLaunchKernelGGL((element_kernel<N, T, true>), grid, dim3(kElemBlock), 0, st, m,
                       (const T*)vin, (const T*)flux, epi);
  else
    hipLaunchKernelGGL((element_kernel<N, T, false>), grid, dim3(kElemBlock), 0, st, m,
                       (const T*)vin, (const T*)flux, epi);
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

template <typename T>
hipError_t elem_dispatch(const DevMesh& m, int nf, const void* vin, const void* flux,
                         const Epilogue& epi, hipStream_t st) {
  ARDG_DISPATCH_N(elem_launch_t, m, nf, vin, flux, epi, st)
}

hipError_t launch_edge_flux(const DevMesh& m, bool fp64, int nfields, const void* u, void* flux,
                            hipStream_t st) {
  return fp64 ? edge_dispatch<double>(m, nfields, u, flux, st)
              : edge_dispatch<float>(m, nfields, u, flux, st);
}

hipError_t launch_element(const DevMesh& m, bool fp64, int nfields, const void* vin,
                          const void* flux, const Epilogue& epi, hipStream_t st) {
  if (m.elem_mfma) return launch_element_mfma(m, fp64, nfields, vin, flux, epi, st);
  return fp64 ? elem_dispatch<double>(m, nfields, vin, flux, epi, st)
              : elem_dispatch<float>(m, nfields, vin, flux, epi, st);
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
  return fp64 ? batch_edge_dispatch<double>(N, tile, grid, probs, items, nitems, in_u, st)
              : batch_edge_dispatch<float>(N, tile, grid, probs, items, nitems, 0, st);
}

hipError_t launch_batch_element(int N, bool fp64, int tile, int grid, const BatchProb* probs,
                                const int2* items, int nitems, const Epilogue& epi, int in_u,
                                int write_v, hipStream_t st) {
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
