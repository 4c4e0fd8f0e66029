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

namespace ardg {

template <typename T>
using cptr = const T __attribute__((address_space(4)))*;

__host__ __device__ constexpr int lat(int N, int i, int j) { return j * (N + 1) - (j * (j - 1)) / 2 + i; }

// node index of face f's j-th node (counter-clockwise)
__host__ __device__ constexpr int fnode(int N, int f, int j) {
  return f == 0 ? lat(N, j, 0) : (f == 1 ? lat(N, N - j, j) : lat(N, 0, N - j));
}

// Keeps the scalar loads of one operator row next to the FMAs that use them:
// without it the scheduler hoists whole matrices into SGPRs and spills.
// The operator pointer is also passed through an empty asm so that repeated
// uses of the same matrix are loaded again instead of being kept live.
__device__ inline void row_fence() { __builtin_amdgcn_sched_barrier(0); }

template <typename T>
__device__ inline cptr<T> fresh(cptr<T> p) {
  asm volatile("" : "+s"(p));
  return p;
}

template <typename T> __device__ inline cptr<T> opbase(const DevMesh& m);
template <> __device__ inline cptr<double> opbase<double>(const DevMesh& m) {
  return (cptr<double>)(m.ops64);
}
template <> __device__ inline cptr<float> opbase<float>(const DevMesh& m) {
  return (cptr<float>)(m.ops32);
}

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
#pragma unroll
  for (int r = 0; r < Np; ++r) {
    row_fence();
    const cptr<T> a = fresh(n2b);
    T s = 0;
#pragma unroll
    for (int q = 0; q < Np; ++q) s = fma(a[r * Np + q], t[q], s);
    c[r] = s;
  }
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

template <int ROWS, int COLS, typename T>
__device__ inline T rowdot(cptr<T> A0, int row, const T* x) {
  row_fence();
  const cptr<T> A = fresh(A0);
  T s = 0;
#pragma unroll
  for (int q = 0; q < COLS; ++q) s = fma(A[row * COLS + q], x[q], s);
  return s;
}

template <int N, typename T, bool ALG1>
__global__ __launch_bounds__(256) void edge_flux_kernel(DevMesh m, const T* __restrict__ u,
                                                        T* __restrict__ flux) {
  constexpr OpLayout L(N);
  constexpr int Np = L.Np, Nfp = L.Nfp;
  const int64_t E = m.E_int + m.E_bdy;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const int field = blockIdx.y;
  const cptr<T> op = opbase<T>(m);
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
#pragma unroll
        for (int j = 0; j < Nfp; ++j)
          F[j] = D1 * (gR * rowdot<Nfp, 2 * Np, T>(op + L.udr, j, c) +
                       gS * rowdot<Nfp, 2 * Np, T>(op + L.uds, j, c));
      } else {
#pragma unroll
        for (int j = 0; j < Nfp; ++j) {
          const T a = gR * rowdot<Nfp, 2 * Np, T>(op + L.u1r, j, c) +
                      gS * rowdot<Nfp, 2 * Np, T>(op + L.u1s, j, c);
          const T b = gR * rowdot<Nfp, 2 * Np, T>(op + L.u2r, j, c) +
                      gS * rowdot<Nfp, 2 * Np, T>(op + L.u2s, j, c);
          F[j] = D1 * a - D2 * b;
        }
      }
    } else {
      const T D = (T)m.Dfield[field];
#pragma unroll
      for (int j = 0; j < Nfp; ++j)
        F[j] = D * (gR * rowdot<Nfp, 2 * Np, T>(op + L.kr, j, c) +
                    gS * rowdot<Nfp, 2 * Np, T>(op + L.ks, j, c));
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
    const int orow = ALG1 ? L.ubr : L.kbr, srow = ALG1 ? L.ubs : L.kbs;
#pragma unroll
    for (int j = 0; j < Nfp; ++j)
      F[j] = D * (gR * rowdot<Nfp, Np, T>(op + orow, j, c) + gS * rowdot<Nfp, Np, T>(op + srow, j, c));
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

constexpr int kElemBlock = 256;

// du/dt of one element from its nodal values u (registers).
template <int N, typename T, bool CONV>
__device__ inline void element_rhs(const DevMesh& m, int64_t k, int field, const T* u,
                                   const T* __restrict__ flux, T* rhs) {
  constexpr OpLayout L(N);
  constexpr int Np = L.Np, Nfp = L.Nfp;
  const int64_t E = m.E_int + m.E_bdy;
  const cptr<T> op = opbase<T>(m);
  // affine factors of this element (eqs. mapping_tri_diff, triangle_jacobian_a/b)
  const double2 p1 = m.vert[3 * k], p2 = m.vert[3 * k + 1], p3 = m.vert[3 * k + 2];
  const double xr = 0.5 * (p2.x - p1.x), yr = 0.5 * (p2.y - p1.y);
  const double xs = 0.5 * (p3.x - p1.x), ys = 0.5 * (p3.y - p1.y);
  const double J = xr * ys - xs * yr;
  const T rx = (T)(ys / J), ry = (T)(-xs / J), sx = (T)(-yr / J), sy = (T)(xr / J);

  T qx[Np], qy[Np];
#pragma unroll
  for (int i = 0; i < Np; ++i) {
    const T ur = rowdot<Np, Np, T>(op + L.dr, i, u);
    const T us = rowdot<Np, Np, T>(op + L.ds, i, u);
    qx[i] = rx * ur + sx * us;
    qy[i] = ry * ur + sy * us;
  }
  const T D = m.alg1 ? (T)m.Delem[k] : (T)m.Dfield[field];
  {
    T wr[Np], ws[Np];
#pragma unroll
    for (int i = 0; i < Np; ++i) {
      wr[i] = rx * qx[i] + ry * qy[i];
      ws[i] = sx * qx[i] + sy * qy[i];
    }
#pragma unroll
    for (int i = 0; i < Np; ++i)
      rhs[i] = D * (rowdot<Np, Np, T>(op + L.dr, i, wr) + rowdot<Np, Np, T>(op + L.ds, i, ws));
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

  // surface terms: (J_f / J) LIFT_f (F_f - D n.q + [n.v u-])
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const double2 a = (f == 0) ? p1 : (f == 1 ? p2 : p3);
    const double2 b = (f == 0) ? p2 : (f == 1 ? p3 : p1);
    const double tx = b.x - a.x, ty = b.y - a.y;
    const double len = sqrt(tx * tx + ty * ty);
    const T nx = (T)(ty / len), ny = (T)(-tx / len);
    const T scale = (T)(0.5 * len / J);
    const int code = m.elem_face[f * m.K + k];
    const int64_t e = code >> 1;
    const bool side2 = code & 1;
    const T* fe = flux + ((int64_t)field * E + e) * Nfp;
    T fv[Nfp];
#pragma unroll
    for (int j = 0; j < Nfp; ++j) fv[j] = fe[j];
    T jump[Nfp];
#pragma unroll
    for (int j = 0; j < Nfp; ++j) {
      const T G = side2 ? -fv[Nfp - 1 - j] : fv[j];
      const int nd = fnode(N, f, j);
      T jv = G - D * (nx * qx[nd] + ny * qy[nd]);
      if (CONV) jv += (nx * vx[nd] + ny * vy[nd]) * u[nd];
      jump[j] = scale * jv;
    }
#pragma unroll
    for (int i = 0; i < Np; ++i) {
      row_fence();
      const cptr<T> lf = fresh(op);
      T s = 0;
#pragma unroll
      for (int j = 0; j < Nfp; ++j) s = fma(lf[L.lift + i * 3 * Nfp + f * Nfp + j], jump[j], s);
      rhs[i] += s;
    }
  }

  if (CONV) {
    // -(d/dx (vx u) + d/dy (vy u)), nodal collocation of the flux vector
    T fx[Np], fy[Np];
#pragma unroll
    for (int n = 0; n < Np; ++n) {
      fx[n] = vx[n] * u[n];
      fy[n] = vy[n] * u[n];
    }
#pragma unroll
    for (int i = 0; i < Np; ++i) {
      const T dxr = rowdot<Np, Np, T>(op + L.dr, i, fx), dxs = rowdot<Np, Np, T>(op + L.ds, i, fx);
      const T dyr = rowdot<Np, Np, T>(op + L.dr, i, fy), dys = rowdot<Np, Np, T>(op + L.ds, i, fy);
      rhs[i] -= rx * dxr + sx * dxs + ry * dyr + sy * dys;
    }
  }
}

// One block = kElemBlock consecutive elements.  Their nodal values form one
// contiguous chunk of the [F][K][Np] array: it is staged through LDS with
// coalesced loads, each thread computes one element from registers, the
// element results go back to LDS, and the Runge-Kutta update runs over the
// chunk's degrees of freedom with coalesced global traffic.
template <int N, typename T, bool CONV>
__global__ __launch_bounds__(kElemBlock) void element_kernel(DevMesh m, const T* __restrict__ vin,
                                                             const T* __restrict__ flux, Epilogue epi) {
  constexpr int Np = (N + 1) * (N + 2) / 2;
  __shared__ T sh[kElemBlock * Np];
  const int64_t k0 = (int64_t)blockIdx.x * kElemBlock;
  const int field = blockIdx.y;
  const int nel = (int)((m.K - k0) < kElemBlock ? (m.K - k0) : kElemBlock);
  const int ndof = nel * Np;
  const int64_t base = ((int64_t)field * m.K + k0) * Np;
  const int t = threadIdx.x;

  for (int i = t; i < ndof; i += kElemBlock) sh[i] = vin[base + i];
  __syncthreads();
  T u[Np];
  if (t < nel) {
#pragma unroll
    for (int n = 0; n < Np; ++n) u[n] = sh[t * Np + n];
  }
  __syncthreads();
  if (t < nel) {
    T rhs[Np];
    element_rhs<N, T, CONV>(m, k0 + t, field, u, flux, rhs);
#pragma unroll
    for (int n = 0; n < Np; ++n) sh[t * Np + n] = rhs[n];
  }
  __syncthreads();

  if (epi.kind == EPI_RHS) {
    T* o = (T*)epi.rhs_out + base;
    for (int i = t; i < ndof; i += kElemBlock) o[i] = sh[i];
    return;
  }
  double* U = epi.u + base;
  double* A = epi.acc + base;
  T* vn = epi.vnext ? (T*)epi.vnext + base : nullptr;
  const double dt = epi.dt;
  if (epi.kind == EPI_RK4) {
    const int s = epi.stage;
    if (s < 3) {
      const double c = (s < 2) ? 0.5 * dt : dt;
      for (int i = t; i < ndof; i += kElemBlock) {
        const double r = (double)sh[i];
        A[i] = (s == 0) ? r : A[i] + 2.0 * r;
        vn[i] = (T)(U[i] + c * r);
      }
    } else {
      for (int i = t; i < ndof; i += kElemBlock) {
        const double un = U[i] + dt / 6.0 * (A[i] + (double)sh[i]);
        U[i] = un;
        if (vn) vn[i] = (T)un;
      }
    }
  } else {
    for (int i = t; i < ndof; i += kElemBlock) {
      const double r = dt * (double)sh[i];
      const double res = (epi.stage == 0) ? r : epi.a * A[i] + r;
      A[i] = res;
      const double un = U[i] + epi.b * res;
      U[i] = un;
      if (vn) vn[i] = (T)un;
    }
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
  return fp64 ? elem_dispatch<double>(m, nfields, vin, flux, epi, st)
              : elem_dispatch<float>(m, nfields, vin, flux, epi, st);
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
