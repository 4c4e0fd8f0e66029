// Compressible Navier-Stokes right-hand side (subsection on the Navier-Stokes
// equations: conserved Q = (rho, rho u, rho v, E), inviscid fluxes F_i and
// viscous fluxes G_i of eq. aRDG_Navier_Stokes, stress eq. NS_viscosity, heat
// flux eq. NS_heatflux, Sutherland's viscosity and kappa = Cp mu / Pr, a
// Lax-Friedrichs flux for the hyperbolic terms), for an ideal gas:
// p = (gamma - 1)(E - rho |u|^2 / 2), T = p / (rho R).
//
// Edge kernel (one lane per face, interior edges then boundary faces):
//   1. both sides' conserved values -> primitive u, v, T at their nodes;
//      each primitive field is rotated to the face, converted to Bernstein
//      coefficients and subdivided at its apex (as the scalar edge kernels);
//      a boundary face's ghost sub-triangle carries the prescribed exterior
//      state at its nodes;
//   2. per primitive field: the reconstruction's value and reference
//      gradient at the diagonal nodes (constant operators on both sides'
//      coefficients), the physical gradient with the parallelogram's inverse
//      metric;
//   3. at every diagonal node: mu and kappa from the reconstructed T, the
//      viscous flux G . (sJ n1) from the reconstructed values and gradients,
//      plus the Lax-Friedrichs flux of the two face traces (the exterior
//      state at a boundary face):
//        sJ F* . n = (F(Q-) + F(Q+)) . sn / 2 - lambda (Q+ - Q-) / 2,
//        lambda = max(|u- . sn| + c- |sn|, |u+ . sn| + c+ |sn|), sn = sJ n1;
//   4. stored per field in side 1's node order.
// Element kernel (one thread per element node, a tile of elements per block):
// the strong form of dQ/dt = -div(F + G),
//   rhs = -(Dx H_x + Dy H_y) + LIFT [ (1/J) (sn_f . H(Q-) - sJ H*_f . n_f) ],
// with H = F + G formed at the nodes from the element's own primitive values
// and their nodal gradients, followed by the Runge-Kutta epilogue.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.hpp"
#include "edge_common.hpp"
#include "kernel_common.hpp"

namespace ardg {

template <typename T>
struct GasC {
  T gamma, gm1, R, cp_pr, mu_ref, iTref, TrefS, S;
  bool sutherland;
};

template <typename T>
__device__ inline GasC<T> gas_consts(const DevMesh& m) {
  GasC<T> g;
  const double gamma = m.gas[0], R = m.gas[1], Pr = m.gas[2];
  g.gamma = (T)gamma;
  g.gm1 = (T)(gamma - 1.0);
  g.R = (T)R;
  g.cp_pr = (T)(gamma * R / ((gamma - 1.0) * Pr));
  g.mu_ref = (T)m.gas[3];
  g.iTref = (T)(1.0 / m.gas[4]);
  g.TrefS = (T)(m.gas[4] + m.gas[5]);
  g.S = (T)m.gas[5];
  g.sutherland = m.ns == NS_SUTHERLAND;
  return g;
}

// Sutherland: mu = mu_ref (T / T_ref)^(3/2) (T_ref + S) / (T + S)
template <typename T>
__device__ inline T viscosity(const GasC<T>& g, T Tt) {
  if (!g.sutherland) return g.mu_ref;
  const T t = Tt * g.iTref;
  return g.mu_ref * t * sqrt(t) * g.TrefS / (Tt + g.S);
}

template <typename T>
__device__ inline void primitives(const GasC<T>& g, T rho, T mx, T my, T E, T& u, T& v, T& p, T& Tt) {
  const T ir = T(1) / rho;
  u = mx * ir;
  v = my * ir;
  p = g.gm1 * (E - T(0.5) * (mx * u + my * v));
  Tt = p * ir / g.R;
}

// (G_x, G_y) of the momentum and energy rows (the mass row is zero).
template <typename T>
__device__ inline void viscous_flux(const GasC<T>& g, T u, T v, T Tt, T ux, T uy, T vx, T vy, T Tx, T Ty, T* Gx,
                                    T* Gy) {
  const T mu = viscosity(g, Tt);
  const T kap = g.cp_pr * mu;
  const T div = ux + vy;
  const T Pxx = mu * (T(2) * ux - T(2.0 / 3.0) * div);
  const T Pyy = mu * (T(2) * vy - T(2.0 / 3.0) * div);
  const T Pxy = mu * (uy + vx);
  Gx[0] = -Pxx;
  Gx[1] = -Pxy;
  Gx[2] = -(u * Pxx + v * Pxy) - kap * Tx;
  Gy[0] = -Pxy;
  Gy[1] = -Pyy;
  Gy[2] = -(u * Pxy + v * Pyy) - kap * Ty;
}

// ---------------------------------------------------------------------------
// Edge kernel
// ---------------------------------------------------------------------------

// Primitive field F (0: u, 1: v, 2: T) at the Np nodes of one element's
// conserved data q[c * stride + off + n] (T or double source).
template <int N, int F, typename T, typename S>
__device__ inline void primitive_field(const GasC<T>& g, const S* q, int64_t stride, int64_t off, T* pv) {
  constexpr int Np = (N + 1) * (N + 2) / 2;
#pragma unroll
  for (int n = 0; n < Np; ++n) {
    const T rho = (T)q[off + n], mx = (T)q[stride + off + n], my = (T)q[2 * stride + off + n];
    if (F == 0) {
      pv[n] = mx / rho;
    } else if (F == 1) {
      pv[n] = my / rho;
    } else {
      T u, v, p, Tt;
      primitives(g, rho, mx, my, (T)q[3 * stride + off + n], u, v, p, Tt);
      pv[n] = Tt;
    }
  }
}

// One side's share of the reconstruction of the three primitive fields on an
// edge.  The side's conserved values are read once; u, v and T at its nodes
// are rotated to the face, converted to Bernstein coefficients and
// subdivided at the apex (the ghost sub-triangle of a boundary face is
// already in its frame: GHOST), and the operator columns acting on this
// side's coefficients (SIDE 0: the first Np, 1: the last Np) are added into
// the value and the reference gradient at the diagonal nodes.  The flux is
// linear in each side's coefficients, so the two sides' shares add up.
template <int N, int SIDE, bool GHOST, typename T, typename S>
__device__ inline void recon_side(cptr<T> op, const GasC<T>& g, const S* q, int64_t stride, int64_t off, int f,
                                  double2 mu, T (&val)[3][N + 1], T (&dR)[3][N + 1], T (&dS)[3][N + 1]) {
  constexpr OpLayout L(N);
  constexpr int Np = L.Np, Nfp = L.Nfp;
  T pv[3][Np];
#pragma unroll
  for (int n = 0; n < Np; ++n) {
    const T rho = (T)q[off + n], mx = (T)q[stride + off + n], my = (T)q[2 * stride + off + n];
    const T E = (T)q[3 * stride + off + n];
    T p;
    primitives(g, rho, mx, my, E, pv[0][n], pv[1][n], p, pv[2][n]);
  }
#pragma unroll
  for (int F = 0; F < 3; ++F) {
    T c[Np];
    if (GHOST) {
      matvec<Np, Np, T>(op + L.n2b, pv[F], c);
    } else {
      T tr[Nfp];
      project_side<N, T>(op, pv[F], f, mu, c, tr);
    }
    T a[Nfp], b[Nfp], d[Nfp];
    matvec_ld<Nfp, Np, 2 * Np, T>(op + L.kv + SIDE * Np, c, a);
    matvec_ld<Nfp, Np, 2 * Np, T>(op + L.kr + SIDE * Np, c, b);
    matvec_ld<Nfp, Np, 2 * Np, T>(op + L.ks + SIDE * Np, c, d);
#pragma unroll
    for (int j = 0; j < Nfp; ++j) {
      val[F][j] += a[j];
      dR[F][j] += b[j];
      dS[F][j] += d[j];
    }
  }
}

template <int N, typename T>
__global__ __launch_bounds__(256) void edge_ns_kernel(DevMesh m, const T* __restrict__ q, T* __restrict__ flux) {
  constexpr OpLayout L(N);
  constexpr int Np = L.Np, Nfp = L.Nfp;
  const int64_t E = m.E_int + m.E_bdy;
  const int64_t e0 = xcd_block(blockIdx.x, gridDim.x) * blockDim.x;
  // lanes past the last face take the last face's data (every lane reaches
  // the block's barrier before the write-out)
  const int64_t e = (e0 + threadIdx.x < E) ? e0 + threadIdx.x : E - 1;
  const cptr<T> op = opbase<T>(m);
  const GasC<T> g = gas_consts<T>(m);
  const int64_t KN = m.K * Np;
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
  const double4 gpm = m.gp[e];
  const double2 snd = m.sn[e];
  const T rx = (T)gpm.x, ry = (T)gpm.y, sx = (T)gpm.z, sy = (T)gpm.w;
  const T snx = (T)snd.x, sny = (T)snd.y;

  // reconstructed (u, v, T) and their physical gradients at the diagonal
  // nodes: each side's share in turn, so that one side's values are live at
  // a time
  T val[3][Nfp], gx[3][Nfp], gy[3][Nfp];
  {
    T dR[3][Nfp], dS[3][Nfp];
#pragma unroll
    for (int F = 0; F < 3; ++F)
#pragma unroll
      for (int j = 0; j < Nfp; ++j) val[F][j] = dR[F][j] = dS[F][j] = T(0);
    recon_side<N, 0, false, T, T>(op, g, q, KN, (int64_t)k1 * Np, fa, mu1, val, dR, dS);
    if (interior)
      recon_side<N, 1, false, T, T>(op, g, q, KN, (int64_t)k2 * Np, fb, mu2, val, dR, dS);
    else
      recon_side<N, 1, true, T, double>(op, g, m.ghost, m.E_bdy * Np, bi * Np, 0, mu2, val, dR, dS);
#pragma unroll
    for (int F = 0; F < 3; ++F)
#pragma unroll
      for (int j = 0; j < Nfp; ++j) {
        gx[F][j] = rx * dR[F][j] + sx * dS[F][j];
        gy[F][j] = ry * dR[F][j] + sy * dS[F][j];
      }
  }

  // face traces: side 1's node j meets side 2's node N - j; at a boundary
  // face the exterior state at the ghost's node (j, N - j) of its lattice
  const T sJ = sqrt(snx * snx + sny * sny);
  // The fluxes wait in LDS, [field][face][node] with rows padded to Nfp + 1
  // (conflict-free node-by-node stores), until the block's faces are done;
  // then each field's block of 256 Nfp values leaves in coalesced writes.
  // Written node by node from the lanes, the FP64 fluxes cost 2.7 times
  // their bytes in HBM writes (partial lines).
  constexpr int RS = Nfp + 1;
  __shared__ T sOut[4][256 * RS];
  const int tid = threadIdx.x;
#pragma unroll
  for (int j = 0; j < Nfp; ++j) {
    const int64_t i1 = (int64_t)k1 * Np + fnode(N, fa, j);
    T QL[4], QR[4];
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) QL[cc] = q[cc * KN + i1];
    if (interior) {
      const int64_t i2 = (int64_t)k2 * Np + fnode(N, fb, N - j);
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) QR[cc] = q[cc * KN + i2];
    } else {
      const int64_t ig = bi * Np + lat(N, j, N - j);
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) QR[cc] = (T)m.ghost[cc * m.E_bdy * Np + ig];
    }
    T uL, vL, pL, TL, uR, vR, pR, TR;
    primitives(g, QL[0], QL[1], QL[2], QL[3], uL, vL, pL, TL);
    primitives(g, QR[0], QR[1], QR[2], QR[3], uR, vR, pR, TR);
    const T unL = uL * snx + vL * sny, unR = uR * snx + vR * sny;
    const T cL = sqrt(g.gamma * pL / QL[0]), cR = sqrt(g.gamma * pR / QR[0]);
    const T aL = fabs(unL) + cL * sJ, aR = fabs(unR) + cR * sJ;
    const T lam = aL > aR ? aL : aR;
    T H[4];
    H[0] = T(0.5) * (QL[0] * unL + QR[0] * unR);
    H[1] = T(0.5) * (QL[1] * unL + pL * snx + QR[1] * unR + pR * snx);
    H[2] = T(0.5) * (QL[2] * unL + pL * sny + QR[2] * unR + pR * sny);
    H[3] = T(0.5) * ((QL[3] + pL) * unL + (QR[3] + pR) * unR);
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) H[cc] -= T(0.5) * lam * (QR[cc] - QL[cc]);
    T Gx[3], Gy[3];
    viscous_flux(g, val[0][j], val[1][j], val[2][j], gx[0][j], gy[0][j], gx[1][j], gy[1][j], gx[2][j], gy[2][j],
                 Gx, Gy);
#pragma unroll
    for (int cc = 1; cc < 4; ++cc) H[cc] += Gx[cc - 1] * snx + Gy[cc - 1] * sny;
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) sOut[cc][tid * RS + j] = H[cc];
  }
  __syncthreads();
  const int nface = (int)((E - e0) < 256 ? (E - e0) : 256);
#pragma unroll
  for (int cc = 0; cc < 4; ++cc) {
    T* out = flux + ((int64_t)cc * E + e0) * Nfp;
#pragma unroll
    for (int r = 0; r < Nfp; ++r) {
      const int idx = tid + r * 256;
      const int f = idx / Nfp, j = idx - f * Nfp;
      if (f < nface) out[idx] = sOut[cc][f * RS + j];
    }
  }
}

template <int N, typename T>
hipError_t edge_ns_t(const DevMesh& m, const void* q, void* flux, hipStream_t st) {
  const int64_t E = m.E_int + m.E_bdy;
  if (E == 0) return hipSuccess;
  dim3 grid((unsigned)((E + 255) / 256));
  hipLaunchKernelGGL((edge_ns_kernel<N, T>), grid, dim3(256), 0, st, m, (const T*)q, (T*)flux);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Element kernel
// ---------------------------------------------------------------------------

template <int N>
struct NsTile {
  static constexpr int Np = (N + 1) * (N + 2) / 2, Nfp = N + 1;
  static constexpr int TE = 256 / Np;          // elements per block
  static constexpr int ND = TE * Np;           // nodes per block (<= 256)
  static constexpr int NJ = 3 * Nfp;           // face values per element
};

// Runge-Kutta epilogue for one degree of freedom (the same update as the
// scalar element kernels' tile epilogue), with the update operands U and A
// already loaded (A is read from stage 1 on).
template <typename T>
__device__ inline void epilogue_dof(const Epilogue& epi, int64_t i, T r_t, double U, double A, bool act) {
  if (epi.kind == EPI_RHS) {
    if (act) ((T*)epi.rhs_out)[i] = r_t;
    return;
  }
  const double r = (double)r_t, dt = epi.dt;
  T* vn = (T*)epi.vnext;
  if (epi.kind == EPI_RK4) {
    // the accumulator holds the new state as it forms (as in tile_end)
    const int s = epi.stage;
    if (s < 3) {
      const double c = (s < 2) ? 0.5 * dt : dt;
      const double w = dt * ((s == 0) ? (1.0 / 6.0) : (1.0 / 3.0));
      if (act) {
        epi.acc[i] = ((s == 0) ? U : A) + w * r;
        if (vn) vn[i] = (T)(U + c * r);
      }
    } else {
      const double un = A + dt * (1.0 / 6.0) * r;
      if (act) {
        epi.u[i] = un;
        if (vn) vn[i] = (T)un;
      }
    }
  } else {
    const double rr = dt * r;
    const double res = (epi.stage == 0) ? rr : epi.a * A + rr;
    const double un = U + epi.b * res;
    if (act) {
      epi.acc[i] = res;
      epi.u[i] = un;
      if (vn) vn[i] = (T)un;
    }
  }
}

// One block: TE elements, one thread per element node.  Every global load
// of the tile -- the operators for LDS, the conserved values, each
// element's vertices (by one thread per element), the face map and the
// interface fluxes of this thread's face nodes, and the update operands --
// is issued before the first wait; indices are clamped and results masked,
// so no load sits under a branch.  Per-element geometry (inverse metric, 1/J,
// sJ n of each face) is formed once and shared through LDS.
template <int N, typename T>
__global__ __launch_bounds__(256) void element_ns_kernel(DevMesh m, const T* __restrict__ vin,
                                                         const T* __restrict__ flux, Epilogue epi) {
  using Tl = NsTile<N>;
  constexpr OpLayout L(N);
  constexpr int Np = Tl::Np, Nfp = Tl::Nfp, TE = Tl::TE, ND = Tl::ND, NJ = Tl::NJ;
  constexpr int NO = 2 * Np * Np + Np * NJ;        // Dr, Ds, LIFT
  constexpr int QO = (NO + 255) / 256;
  constexpr int QJ = (TE * NJ + 255) / 256;        // face nodes per thread
  __shared__ T sQ[4][ND];
  __shared__ T sP[3][ND];        // u, v, T
  __shared__ T sH[8][ND];        // H_x then H_y of the four fields
  __shared__ T sJv[4][QJ * 256]; // lift inputs
  __shared__ T sOp[QO * 256];    // Dr, Ds, LIFT
  __shared__ double sG[TE][11];  // r_x, r_y, s_x, s_y, 1/J, sJ n of the three faces
  const cptr<T> op = opbase<T>(m);
  const GasC<T> g = gas_consts<T>(m);
  const int64_t tile = xcd_block(blockIdx.x, gridDim.x);
  const int64_t k0 = tile * TE;
  const int t = threadIdx.x;
  const int nel = (int)((m.K - k0) < TE ? (m.K - k0) : TE);
  const int ndof = nel * Np;
  const int64_t KN = m.K * Np;
  const int64_t E = m.E_int + m.E_bdy;
  const bool act = t < ndof;
  const int tc = act ? t : 0;
  const int el = tc / Np, n = tc - (tc / Np) * Np;

  // ---- loads ----
  int code[QJ];
#pragma unroll
  for (int r = 0; r < QJ; ++r) {
    const int idx = t + r * 256;
    const int ic = idx < nel * NJ ? idx : 0;
    const int e2 = ic / NJ, f = (ic - e2 * NJ) / Nfp;
    code[r] = m.elem_face[f * m.K + k0 + e2];
  }
  T ov[QO];
#pragma unroll
  for (int r = 0; r < QO; ++r) {
    const int i = t + r * 256;
    const int ic = i < NO ? i : 0;
    ov[r] = ic < 2 * Np * Np ? op[L.dr + ic] : op[L.lift + ic - 2 * Np * Np];
  }
  T Q[4];
#pragma unroll
  for (int cc = 0; cc < 4; ++cc) Q[cc] = vin[cc * KN + k0 * Np + tc];
  const int64_t kv = k0 + (t < nel ? t : 0);
  const double2 p1 = m.vert[3 * kv], p2 = m.vert[3 * kv + 1], p3 = m.vert[3 * kv + 2];
  // interface fluxes of this thread's face nodes, side 1's order and sign
  T Gs[QJ][4];
#pragma unroll
  for (int r = 0; r < QJ; ++r) {
    const int idx = t + r * 256;
    const int ic = idx < nel * NJ ? idx : 0;
    const int j = (ic - (ic / NJ) * NJ) % Nfp;
    const bool side2 = code[r] & 1;
    const int64_t fo = (int64_t)(code[r] >> 1) * Nfp + (side2 ? Nfp - 1 - j : j);
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) {
      const T x = flux[(int64_t)cc * E * Nfp + fo];
      Gs[r][cc] = side2 ? -x : x;
    }
  }

  // ---- LDS: operators, conserved and primitive values, geometry ----
#pragma unroll
  for (int r = 0; r < QO; ++r) sOp[t + r * 256] = ov[r];
  if (act) {
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) sQ[cc][t] = Q[cc];
    T u, v, p, Tt;
    primitives(g, Q[0], Q[1], Q[2], Q[3], u, v, p, Tt);
    sP[0][t] = u;
    sP[1][t] = v;
    sP[2][t] = Tt;
  }
  if (t < TE) {
    const ElemGeom gm = elem_geom(p1, p2, p3);
    double* G = sG[t];
    G[0] = gm.rx;
    G[1] = gm.ry;
    G[2] = gm.sx;
    G[3] = gm.sy;
    G[4] = gm.iJ;
    // sJ n of face f, (t_y, -t_x) / 2 for its counter-clockwise edge vector t
    G[5] = 0.5 * (p2.y - p1.y);
    G[6] = -0.5 * (p2.x - p1.x);
    G[7] = 0.5 * (p3.y - p2.y);
    G[8] = -0.5 * (p3.x - p2.x);
    G[9] = 0.5 * (p1.y - p3.y);
    G[10] = -0.5 * (p1.x - p3.x);
  }
  __syncthreads();

  const T* Dr = sOp;
  const T* Ds = sOp + Np * Np;
  const T* Lf = sOp + 2 * Np * Np;
  const T rx = (T)sG[el][0], ry = (T)sG[el][1], sx = (T)sG[el][2], sy = (T)sG[el][3];
  if (act) {
    // nodal gradients of u, v, T and the fluxes H = F + G at this node
    T gxv[3], gyv[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      T a = T(0), b = T(0);
#pragma unroll
      for (int j = 0; j < Np; ++j) {
        const T x = sP[f][el * Np + j];
        a = fma(Dr[n * Np + j], x, a);
        b = fma(Ds[n * Np + j], x, b);
      }
      gxv[f] = rx * a + sx * b;
      gyv[f] = ry * a + sy * b;
    }
    const T rho = sQ[0][t], mx = sQ[1][t], my = sQ[2][t], En = sQ[3][t];
    const T u = sP[0][t], v = sP[1][t], Tt = sP[2][t];
    const T p = Tt * rho * g.R;
    T Gx[3], Gy[3];
    viscous_flux(g, u, v, Tt, gxv[0], gyv[0], gxv[1], gyv[1], gxv[2], gyv[2], Gx, Gy);
    sH[0][t] = mx;
    sH[1][t] = mx * u + p + Gx[0];
    sH[2][t] = my * u + Gx[1];
    sH[3][t] = (En + p) * u + Gx[2];
    sH[4][t] = my;
    sH[5][t] = mx * v + Gy[0];
    sH[6][t] = my * v + p + Gy[1];
    sH[7][t] = (En + p) * v + Gy[2];
  }
  __syncthreads();

  // lift inputs (1/J) (sn_f . H(Q-) - sJ H* . n_f) of this thread's face nodes
#pragma unroll
  for (int r = 0; r < QJ; ++r) {
    const int idx = t + r * 256;
    if (idx < nel * NJ) {
      const int e2 = idx / NJ, qf = idx - e2 * NJ;
      const int f = qf / Nfp, j = qf - f * Nfp;
      const int nd = e2 * Np + fnode(N, f, j);
      const double* G = sG[e2];
      const T snx = (T)G[5 + 2 * f], sny = (T)G[6 + 2 * f], iJ = (T)G[4];
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) {
        const T hn = snx * sH[cc][nd] + sny * sH[4 + cc][nd];
        sJv[cc][idx] = iJ * (hn - Gs[r][cc]);
      }
    }
  }
  // update operands (read from the stage input's first value when there is
  // no update: no branch around the loads), issued here rather than with the
  // tile's other loads so that they hold no registers through the gradient
  // and flux phase (FP64 N = 3: 180 -> 162 registers, three waves per SIMD
  // instead of two; FP32: 108 -> 90, five instead of four)
  const bool rk = epi.kind != EPI_RHS;
  const bool need_acc = rk && epi.stage != 0;
  const double* Ub = rk ? (last_rk4(epi) ? epi.acc : epi.u) : (const double*)vin;
  const double* Ab = need_acc ? epi.acc : Ub;
  double Up[4], Ap[4];
#pragma unroll
  for (int cc = 0; cc < 4; ++cc) {
    const int64_t i = rk ? cc * KN + k0 * Np + tc : 0;
    Up[cc] = Ub[i];
    Ap[cc] = Ab[i];
  }
  __syncthreads();

#pragma unroll
  for (int cc = 0; cc < 4; ++cc) {
    T drx = T(0), dry = T(0), dsx = T(0), dsy = T(0);
#pragma unroll
    for (int j = 0; j < Np; ++j) {
      const T hx = sH[cc][el * Np + j], hy = sH[4 + cc][el * Np + j];
      drx = fma(Dr[n * Np + j], hx, drx);
      dry = fma(Dr[n * Np + j], hy, dry);
      dsx = fma(Ds[n * Np + j], hx, dsx);
      dsy = fma(Ds[n * Np + j], hy, dsy);
    }
    T r = -(rx * drx + ry * dry + sx * dsx + sy * dsy);
#pragma unroll
    for (int qf = 0; qf < NJ; ++qf) r = fma(Lf[n * NJ + qf], sJv[cc][el * NJ + qf], r);
    epilogue_dof<T>(epi, cc * KN + k0 * Np + tc, r, Up[cc], Ap[cc], act);
  }
}

template <int N, typename T>
hipError_t element_ns_t(const DevMesh& m, const void* vin, const void* flux, const Epilogue& epi, hipStream_t st) {
  if (m.K == 0) return hipSuccess;
  constexpr int TE = NsTile<N>::TE;
  dim3 grid((unsigned)((m.K + TE - 1) / TE));
  hipLaunchKernelGGL((element_ns_kernel<N, T>), grid, dim3(256), 0, st, m, (const T*)vin, (const T*)flux, epi);
  return hipGetLastError();
}

template <typename T>
hipError_t ns_dispatch(const DevMesh& m, bool edge, const void* in, const void* fl_in, void* fl_out,
                       const Epilogue& epi, hipStream_t st) {
  switch (m.N) {
#define ARDG_NS_CASE(NN)                                                                  \
  case NN:                                                                                \
    return edge ? edge_ns_t<NN, T>(m, in, fl_out, st) : element_ns_t<NN, T>(m, in, fl_in, epi, st);
    ARDG_NS_CASE(1)
    ARDG_NS_CASE(2)
    ARDG_NS_CASE(3)
    ARDG_NS_CASE(4)
    ARDG_NS_CASE(5)
    ARDG_NS_CASE(6)
#undef ARDG_NS_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_edge_ns(const DevMesh& m, int prec, const void* q, void* flux, hipStream_t st) {
  Epilogue none;
  if (prec == PREC_FP64) return ns_dispatch<double>(m, true, q, nullptr, flux, none, st);
  if (prec == PREC_FP32) return ns_dispatch<float>(m, true, q, nullptr, flux, none, st);
  return hipErrorInvalidValue;
}

hipError_t launch_element_ns(const DevMesh& m, int prec, const void* vin, const void* flux, const Epilogue& epi,
                             hipStream_t st) {
  if (prec == PREC_FP64) return ns_dispatch<double>(m, false, vin, flux, nullptr, epi, st);
  if (prec == PREC_FP32) return ns_dispatch<float>(m, false, vin, flux, nullptr, epi, st);
  return hipErrorInvalidValue;
}

}  // namespace ardg
