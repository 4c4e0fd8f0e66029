// Edge kernel for a nodal tensor diffusion coefficient (Algorithm 1 with
// nodal products; eq. NDG_diffusion_once_matrixForm_reference_general with D
// a function of space, anisotropic, or proportional to the solution).
//
// One lane per face (interior edges, then boundary faces):
//   1. each side's nodal values are rotated to its face, converted to
//      Bernstein coefficients and subdivided at its apex (as in the other
//      edge kernels); the coefficient's components (Dxx, Dxy, Dyy) take the
//      same path (nodal tensor), or the side's own coefficients stand for it
//      (D = u D0);
//   2. for each sub-triangle k: the reference gradient of the reconstruction
//      u~ at its nodes (one constant operator on both sides' coefficients:
//      least squares, separation, d/dr and d/ds in the sub-triangle's own
//      frame), the physical gradient with the parallelogram's inverse metric
//      (negated on side 2, whose frame is the point reflection), the
//      coefficient at its nodes (Bernstein -> nodal), and the nodal product
//      q = D grad(u~);
//   3. the second reconstruction of q, evaluated on the diagonal (one
//      constant operator per side), contracted with sJ n1;
//   4. the upwind convective flux where a velocity is set.
// A boundary face's ghost is the mirror image (data -u, coefficient D at
// mirrored points, i.e. minus / plus the side-1 coefficients with the
// (r, s) swap of the lattice), or carries the prescribed exterior state.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.hpp"
#include "edge_common.hpp"
#include "kernel_common.hpp"

namespace ardg {

template <int N, typename T, bool SOL>
__global__ __launch_bounds__(256) void edge_tensor_kernel(DevMesh m, const T* __restrict__ u, T* __restrict__ flux,
                                                          int nf) {
  constexpr OpLayout L(N);
  constexpr int Np = L.Np, Nfp = L.Nfp;
  int64_t tile;
  int field;
  tile_and_field(blockIdx.x, gridDim.x, nf, tile, field);
  const int64_t E = m.E_int + m.E_bdy;
  const int64_t e = tile * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const cptr<T> op = opbase<T>(m);
  const T* uf = u + (int64_t)field * m.K * Np;
  const bool interior = e < m.E_int;
  int k1, fa, k2 = 0, fb = 0;
  double2 mu1, mu2 = make_double2(0.0, 0.0);
  int64_t bi = 0;
  if (interior) {
    const int2 ef = m.ef[e];
    k1 = ef.x & 0x3fffffff;
    fa = (int)((unsigned)ef.x >> 30);
    k2 = ef.y & 0x3fffffff;
    fb = (int)((unsigned)ef.y >> 30);
    mu1 = m.mu1[e];
    mu2 = m.mu2[e];
  } else {
    bi = e - m.E_int;
    const int kb = m.bk[bi];
    k1 = kb & 0x3fffffff;
    fa = (int)((unsigned)kb >> 30);
    mu1 = m.bmu[bi];
  }
  const double4 g = m.gp[e];
  const double2 sn = m.sn[e];
  double2 vn = make_double2(0.0, 0.0);
  if (m.conv) vn = m.vn[e];

  // both sides' Bernstein coefficients c = [b1; b2] and face traces
  T c[2 * Np], tr1[Nfp], tr2[Nfp];
  {
    T v[Np];
#pragma unroll
    for (int n = 0; n < Np; ++n) v[n] = uf[(int64_t)k1 * Np + n];
    project_side<N, T>(op, v, fa, mu1, c, tr1);
  }
  if (interior) {
    T v[Np];
#pragma unroll
    for (int n = 0; n < Np; ++n) v[n] = uf[(int64_t)k2 * Np + n];
    project_side<N, T>(op, v, fb, mu2, c + Np, tr2);
  } else if (m.ghost) {
    T gv[Np];
    const double* gs = m.ghost + ((int64_t)field * m.E_bdy + bi) * Np;
#pragma unroll
    for (int n = 0; n < Np; ++n) gv[n] = (T)gs[n];
#pragma unroll
    for (int j = 0; j <= N; ++j) tr2[N - j] = gv[lat(N, j, N - j)];
    matvec<Np, Np, T>(op + L.n2b, gv, c + Np);
  } else {
    lattice_swap<N, T>(c, c + Np, T(-1));
#pragma unroll
    for (int j = 0; j < Nfp; ++j) tr2[j] = T(0);
  }

  const T rx = (T)g.x, ry = (T)g.y, sx = (T)g.z, sy = (T)g.w;
  T F[Nfp];
#pragma unroll
  for (int j = 0; j < Nfp; ++j) F[j] = T(0);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    // the coefficient's Bernstein coefficients on this sub-triangle
    T bD[SOL ? 1 : 3][Np];
    if (!SOL) {
      const bool mirror = s == 1 && !interior;
      const int kk = s ? (interior ? k2 : k1) : k1;
      const int ff = s ? (interior ? fb : fa) : fa;
      const double2 mu = s ? (interior ? mu2 : mu1) : mu1;
#pragma unroll
      for (int comp = 0; comp < 3; ++comp) {
        T v[Np], trd[Nfp], bd[Np];
#pragma unroll
        for (int n = 0; n < Np; ++n) v[n] = (T)m.Dnodal[((int64_t)kk * Np + n) * 3 + comp];
        project_side<N, T>(op, v, ff, mu, bd, trd);
        if (mirror)
          lattice_swap<N, T>(bd, bD[SOL ? 0 : comp], T(1));
        else
#pragma unroll
          for (int n = 0; n < Np; ++n) bD[SOL ? 0 : comp][n] = bd[n];
      }
    }
    // reference gradient of u~ at this sub-triangle's nodes, then physical
    T dR[Np], dS[Np];
    matvec<Np, 2 * Np, T>(op + (s ? L.tr2 : L.tr1), c, dR);
    matvec<Np, 2 * Np, T>(op + (s ? L.ts2 : L.ts1), c, dS);
    const T sg = s ? T(-1) : T(1);
    T qx[Np], qy[Np];
    {
      T Dn[SOL ? 1 : 3][Np];
      if (SOL) {
        matvec<Np, Np, T>(op + L.b2n, c + s * Np, Dn[0]);
      } else {
#pragma unroll
        for (int comp = 0; comp < 3; ++comp) matvec<Np, Np, T>(op + L.b2n, bD[SOL ? 0 : comp], Dn[SOL ? 0 : comp]);
      }
#pragma unroll
      for (int n = 0; n < Np; ++n) {
        const T gx = sg * (rx * dR[n] + sx * dS[n]);
        const T gy = sg * (ry * dR[n] + sy * dS[n]);
        T dxx, dxy, dyy;
        if (SOL) {
          dxx = (T)m.D0[0] * Dn[0][n];
          dxy = (T)m.D0[1] * Dn[0][n];
          dyy = (T)m.D0[2] * Dn[0][n];
        } else {
          dxx = Dn[0][n];
          dxy = Dn[SOL ? 0 : 1][n];
          dyy = Dn[SOL ? 0 : 2][n];
        }
        qx[n] = dxx * gx + dxy * gy;
        qy[n] = dxy * gx + dyy * gy;
      }
    }
    // second reconstruction on the diagonal, this side's part
    T ax[Nfp], ay[Nfp];
    matvec<Nfp, Np, T>(op + (s ? L.g2 : L.g1), qx, ax);
    matvec<Nfp, Np, T>(op + (s ? L.g2 : L.g1), qy, ay);
#pragma unroll
    for (int j = 0; j < Nfp; ++j) F[j] += (T)sn.x * ax[j] + (T)sn.y * ay[j];
  }
  if (m.conv) {
    // upwind flux f* = max(n.v,0) u- + min(n.v,0) u+ (node j of side 1 meets
    // node N - j of side 2)
#pragma unroll
    for (int j = 0; j < Nfp; ++j) {
      const T tau = op[L.tau + j];
      const T vnj = (T)vn.x + tau * (T)(vn.y - vn.x);
      F[j] -= (vnj > (T)0) ? vnj * tr1[j] : vnj * tr2[N - j];
    }
  }
  T* out = flux + ((int64_t)field * E + e) * Nfp;
#pragma unroll
  for (int j = 0; j < Nfp; ++j) out[j] = F[j];
}

template <int N, typename T>
hipError_t edge_tensor_t(const DevMesh& m, int nfields, const void* u, void* flux, hipStream_t st) {
  const int64_t E = m.E_int + m.E_bdy;
  if (E == 0) return hipSuccess;
  dim3 grid((unsigned)((E + 255) / 256 * nfields));
  if (m.dmode == DM_SOLUTION)
    hipLaunchKernelGGL((edge_tensor_kernel<N, T, true>), grid, dim3(256), 0, st, m, (const T*)u, (T*)flux, nfields);
  else
    hipLaunchKernelGGL((edge_tensor_kernel<N, T, false>), grid, dim3(256), 0, st, m, (const T*)u, (T*)flux, nfields);
  return hipGetLastError();
}

template <typename T>
hipError_t edge_tensor_dispatch(const DevMesh& m, int nf, const void* u, void* flux, hipStream_t st) {
  switch (m.N) {
    case 1: return edge_tensor_t<1, T>(m, nf, u, flux, st);
    case 2: return edge_tensor_t<2, T>(m, nf, u, flux, st);
    case 3: return edge_tensor_t<3, T>(m, nf, u, flux, st);
    case 4: return edge_tensor_t<4, T>(m, nf, u, flux, st);
    case 5: return edge_tensor_t<5, T>(m, nf, u, flux, st);
    case 6: return edge_tensor_t<6, T>(m, nf, u, flux, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_edge_tensor(const DevMesh& m, int prec, int nfields, const void* u, void* flux, hipStream_t st) {
  if (prec == PREC_FP64) return edge_tensor_dispatch<double>(m, nfields, u, flux, st);
  if (prec == PREC_FP32) return edge_tensor_dispatch<float>(m, nfields, u, flux, st);
  return hipErrorInvalidValue;   // no split-BF16 form
}

}  // namespace ardg
