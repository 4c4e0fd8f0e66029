// Edge kernels on the matrix cores (gfx950 MFMA, 16x16 tiles).
//
// edge_mfma_kernel: one wave takes 64 consecutive interior edges, as four
// sub-tiles of 16 edges (the 16 columns of the MFMA tiles).  Per side:
//   1. gather + rotate: the B fragments are read straight from the stage
//      vector, the face's node reordering (section "Reordering nodes in the
//      reference domain") applied as an index remap;
//   2. nodal -> Bernstein on I: (Np x Np) x (Np x 16) products with the
//      constant conversion matrix held as A fragments;
//   3. projection onto the sub-triangle (eq. totalProjection): de Casteljau
//      subdivision at the edge's own apex weights, one lane per edge, on the
//      coefficients staged in LDS;
//   4. the constant reconstruction-gradient operator (least squares on the
//      enclosed parallelogram, d/dR and d/dS on the diagonal nodes) applied
//      to this side's half of the coefficient vector, accumulated over the
//      two sides on the matrix cores.
// The operator rows are laid out so that the values one flux node needs
// (d/dR and d/dS, and for Algorithm 1 the D1 and D2 blocks) arrive in the
// same lane; the flux of the 64 edges is formed there, staged in LDS and
// written as one contiguous block.  Boundary faces (mirror ghost) run the
// vector-unit body in the same launch, one lane per face.
//
// edge_smfma_kernel: the side-split tile (two waves per 64 edges, one per
// side) with only the conversion of step 2 on the matrix cores; see there.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "edge_common.hpp"
#include "kernel_common.hpp"
#include "mfma.hpp"

namespace ardg {

constexpr int kEdgeTile = 64;   // interior edges per block (one wave)

// Operator forms of step 4.
//   PAIR_K : constant D (or Algorithm 2's per-node coefficient), rows
//            (d/dR, d/dS) of the reconstruction gradient
//   PAIR_UD: Algorithm 1 with D1 == D2 on every edge of the wave: U1 - U2
//   QUAD   : Algorithm 1, rows (U1R, U1S, U2R, U2S)
enum EdgeForm { PAIR_K = 0, PAIR_UD = 1, QUAD = 2 };

template <int N, typename P, int FORM, int DM, bool CONV>
__device__ inline void edge_tile_mfma(const DevMesh& m, const typename Mma<P>::T* __restrict__ opg,
                                      int field, const typename Mma<P>::T* __restrict__ uf,
                                      typename Mma<P>::T* __restrict__ out, int nval, int k1, int fa,
                                      int k2, int fb, double2 mu1, double2 mu2, double2 gam, double D1,
                                      double D2, typename Mma<P>::T* cb, typename Mma<P>::T* fl,
                                      const int* rot) {
  using M = Mma<P>;
  using T = typename M::T;
  typedef typename M::acc acc_t;
  typedef typename M::frag frag_t;
  constexpr int KPL = M::KPL, KS = M::KSTEP;
  constexpr OpLayout L(N);
  constexpr int Np = L.Np, Nfp = L.Nfp, K2 = 2 * Np;
  constexpr int MT = (Np + 15) / 16;                       // row tiles of the conversion
  constexpr int KC = (Np + KS - 1) / KS;                   // k steps over one side's nodes
  constexpr int RPT = FORM == QUAD ? 4 : 8;                // flux nodes per row tile
  constexpr int MG = (Nfp + RPT - 1) / RPT;                // row tiles of step 4
  constexpr int base = FORM == PAIR_K ? L.kr : (FORM == PAIR_UD ? L.udr : L.u1r);
  const int l = threadIdx.x, col = l & 15, grp = l >> 4;
  const bool valid = l < nval;

  // conversion matrix as A fragments: row 16 mt + col, columns kidx(c, grp, .)
  frag_t aN[MT][KC];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      T v[KPL];
#pragma unroll
      for (int t = 0; t < KPL; ++t) {
        const int i = 16 * mt + col, k = kidx<M>(c, grp, t);
        v[t] = (i < Np && k < Np) ? opg[L.n2b + i * Np + k] : T(0);
      }
      aN[mt][c] = M::make(v);
    }
  // step-4 operator row held by this lane in tile mt: MFMA row `col`
  const int gi = M::grp_of(col), ri = M::reg_of(col);

  acc_t g[4][MG];
#pragma unroll
  for (int sb = 0; sb < 4; ++sb)
#pragma unroll
    for (int mt = 0; mt < MG; ++mt) g[sb][mt] = M::zero();

#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int kl = s ? k2 : k1, fl_ = s ? fb : fa;
    // 1 + 2: gather, rotate, convert to Bernstein coefficients
#pragma unroll
    for (int sb = 0; sb < 4; ++sb) {
      const int el = 16 * sb + col;
      const int kk = __shfl(kl, el), ff = __shfl(fl_, el);
      const bool ok = el < nval;
      const T* ue = uf + (int64_t)kk * Np;
      frag_t bu[KC];
#pragma unroll
      for (int c = 0; c < KC; ++c) {
        T v[KPL];
#pragma unroll
        for (int t = 0; t < KPL; ++t) {
          const int n = kidx<M>(c, grp, t);
          const int nc = n < Np ? n : 0;
          const T x = ue[ff == 1 ? nc : rot[(ff >> 1) * Np + nc]];
          v[t] = (ok && n < Np) ? x : T(0);
        }
        bu[c] = M::make(v);
      }
      acc_t b[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        b[mt] = M::zero();
#pragma unroll
        for (int c = 0; c < KC; ++c) b[mt] = M::mma(aN[mt][c], bu[c], b[mt]);
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * mt + M::row(grp, r);
          if (row < Np) cb[row * kEdgeTile + el] = b[mt][r];
        }
    }
    __syncthreads();
    // 3: subdivision at this edge's apex, one lane per edge
    if (valid) {
      T c[Np];
#pragma unroll
      for (int n = 0; n < Np; ++n) c[n] = cb[n * kEdgeTile + l];
      decasteljau<N, T>(c, s ? mu2 : mu1);
#pragma unroll
      for (int n = 0; n < Np; ++n) cb[n * kEdgeTile + l] = c[n];
    }
    __syncthreads();
    // 4: this side's columns of the step-4 operator
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      frag_t a[MG];
#pragma unroll
      for (int mt = 0; mt < MG; ++mt) {
        int jj, comp;
        if (FORM == QUAD) {
          jj = 4 * mt + gi;
          comp = ri;
        } else {
          jj = 8 * mt + 2 * gi + (ri >> 1);
          comp = ri & 1;
        }
        T v[KPL];
#pragma unroll
        for (int t = 0; t < KPL; ++t) {
          const int k = kidx<M>(c, grp, t);
          v[t] = (jj < Nfp && k < Np) ? opg[base + (comp * Nfp + jj) * K2 + s * Np + k] : T(0);
        }
        a[mt] = M::make(v);
      }
#pragma unroll
      for (int sb = 0; sb < 4; ++sb) {
        T v[KPL];
#pragma unroll
        for (int t = 0; t < KPL; ++t) {
          const int k = kidx<M>(c, grp, t);
          v[t] = (k < Np) ? cb[k * kEdgeTile + 16 * sb + col] : T(0);
        }
        const frag_t bb = M::make(v);
#pragma unroll
        for (int mt = 0; mt < MG; ++mt) g[sb][mt] = M::mma(a[mt], bb, g[sb][mt]);
      }
    }
    __syncthreads();   // cb is refilled by the other side
  }

  // flux at the diagonal nodes; lane group grp holds nodes of edge 16 sb + col
  const T Dc = (T)field_D(m, field);
#pragma unroll
  for (int sb = 0; sb < 4; ++sb) {
    const int el = 16 * sb + col;
    const bool ok = el < nval;
    const T gR = (T)__shfl(gam.x, el), gS = (T)__shfl(gam.y, el);
    const T d1 = (T)__shfl(D1, el), d2 = (T)__shfl(D2, el);
#pragma unroll
    for (int mt = 0; mt < MG; ++mt) {
      if (FORM == QUAD) {
        const int jj = 4 * mt + grp;
        if (ok && jj < Nfp) {
          T F = d1 * (gR * g[sb][mt][0] + gS * g[sb][mt][1]) - d2 * (gR * g[sb][mt][2] + gS * g[sb][mt][3]);
          if (CONV) F -= fl[el * Nfp + jj];
          fl[el * Nfp + jj] = F;
        }
      } else {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int jj = 8 * mt + 2 * grp + h;
          if (ok && jj < Nfp) {
            const T D = DM == DM_ALG2 ? d1 * opg[L.w1 + jj] + d2 * opg[L.w2 + jj] : (FORM == PAIR_K ? Dc : d1);
            T F = D * (gR * g[sb][mt][2 * h] + gS * g[sb][mt][2 * h + 1]);
            if (CONV) F -= fl[el * Nfp + jj];
            fl[el * Nfp + jj] = F;
          }
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < Nfp; ++q) {
    const int i = l + q * kEdgeTile;
    if (i < nval * Nfp) out[i] = fl[i];
  }
}

template <int N, typename P, int DM, bool CONV>
__global__ __launch_bounds__(kEdgeTile) void edge_mfma_kernel(DevMesh m,
                                                              const typename Mma<P>::T* __restrict__ u,
                                                              typename Mma<P>::T* __restrict__ flux,
                                                              int nb_bdy, int nf) {
  using T = typename Mma<P>::T;
  constexpr OpLayout L(N);
  constexpr int Np = L.Np, Nfp = L.Nfp;
  __shared__ T cb[Np * kEdgeTile];
  __shared__ T fl[kEdgeTile * Nfp];
  __shared__ int rot[2 * Np];
  const int l = threadIdx.x;
  const int64_t E = m.E_int + m.E_bdy;
  const int64_t b = blockIdx.x;
  const int64_t nbt = (int64_t)nb_bdy * nf;
  if (b < nbt) {
    // boundary faces: mirror-ghost operator on the vector unit, one lane per
    // face, in the first blocks so that their long serial chain runs beside
    // the interior tiles (with exterior data the faces take a launch of
    // their own, launch_boundary_faces, and nb_bdy is 0: the prescribed-state
    // path would set this kernel's register allocation)
    const int field = (int)(b % nf);
    const int64_t e = m.E_int + (b / nf) * kEdgeTile + l;
    if (e < E) boundary_body<N, T, DM, false>(m, opbase<T>(m), e, field, u, flux);
    return;
  }
  int64_t tile;
  int field;
  tile_and_field(b - nbt, (int64_t)gridDim.x - nbt, nf, tile, field);   // nbt % 8 == 0
  const int64_t e0 = tile * kEdgeTile;
  const int nval = (int)((m.E_int - e0) < kEdgeTile ? (m.E_int - e0) : kEdgeTile);
  // rotated lattice node -> element node for faces 0 and 2 (face 1: identity)
  for (int n = l; n < Np; n += kEdgeTile) {
    int j = 0;
    while (lat(N, 0, j + 1) <= n) ++j;
    const int i = n - lat(N, 0, j);
    rot[n] = lat(N, j, N - i - j);
    rot[Np + n] = lat(N, N - i - j, i);
  }
  const bool valid = l < nval;
  const int64_t e = e0 + (valid ? l : 0);
  const int2 ef = m.ef[e];
  const int k1 = ef.x & 0x3fffffff, fa = (int)((unsigned)ef.x >> 30);
  const int k2 = ef.y & 0x3fffffff, fb = (int)((unsigned)ef.y >> 30);
  const double2 mu1 = m.mu1[e], mu2 = m.mu2[e], gam = m.gam[e];
  const double D1 = DM != DM_CONST ? m.Delem[k1] : 0.0, D2 = DM != DM_CONST ? m.Delem[k2] : 0.0;
  const T* uf = u + (int64_t)field * m.K * Np;
  const T* opg = (const T*)(const void*)opbase<T>(m);
  if (CONV && valid) {
    // upwind flux f* = max(n.v,0) u- + min(n.v,0) u+ at the face nodes,
    // subtracted from the diffusive flux; n.v is linear along the edge
    const double2 vn = m.vn[e];
#pragma unroll
    for (int j = 0; j < Nfp; ++j) {
      const T tau = opg[L.tau + j];
      const T vnj = (T)vn.x + tau * (T)(vn.y - vn.x);
      const T um = uf[(int64_t)k1 * Np + fnode(N, fa, j)];
      const T up = uf[(int64_t)k2 * Np + fnode(N, fb, N - j)];
      fl[l * Nfp + j] = (vnj > (T)0) ? vnj * um : vnj * up;
    }
  }
  __syncthreads();
  T* out = flux + ((int64_t)field * E + e0) * Nfp;
  if (DM != DM_ALG1) {
    edge_tile_mfma<N, P, PAIR_K, DM, CONV>(m, opg, field, uf, out, nval, k1, fa, k2, fb, mu1, mu2, gam,
                                           D1, D2, cb, fl, rot);
  } else if (__ballot(valid && D1 != D2) == 0) {
    edge_tile_mfma<N, P, PAIR_UD, DM, CONV>(m, opg, field, uf, out, nval, k1, fa, k2, fb, mu1, mu2, gam,
                                            D1, D2, cb, fl, rot);
  } else {
    edge_tile_mfma<N, P, QUAD, DM, CONV>(m, opg, field, uf, out, nval, k1, fa, k2, fb, mu1, mu2, gam,
                                         D1, D2, cb, fl, rot);
  }
}

// Side-split tile with the conversion on the matrix cores.  A block of two
// waves takes 64 interior edges, wave s side s + 1.  The wave gathers its
// side's element values straight into B fragments (16 edges per fragment,
// rotated by the index remap), converts them to Bernstein coefficients with
// one (Np x Np) x (Np x 16) product per 16 edges, and hands the coefficients
// through its own LDS rows to one lane per edge for the subdivision and its
// side's columns of the reconstruction operator (vector unit, scalar operands,
// as in the vector-unit split kernel).  The conversion runs on the matrix pipe
// beside the other waves' vector work.  The boundary blocks carry only the
// mirror-ghost path (with exterior data the faces take a launch of their own,
// launch_boundary_faces): in FP64 at N = 6 with Algorithm 1 the tiles need
// about 100 registers, the mirror-ghost path about 150 and the
// prescribed-state path about 250.  At least three waves per SIMD: the
// compiler then keeps the accumulators out of the matrix registers and fits
// 154 registers without spilling.
template <int N, typename P, int DM, bool CONV>
__global__ __launch_bounds__(2 * kEdgeTile) __attribute__((amdgpu_waves_per_eu(3))) void edge_smfma_kernel(DevMesh m,
                                                                   const typename Mma<P>::T* __restrict__ u,
                                                                   typename Mma<P>::T* __restrict__ flux,
                                                                   int nb_bdy, int nf) {
  using M = Mma<P>;
  using T = typename M::T;
  typedef typename M::acc acc_t;
  typedef typename M::frag frag_t;
  constexpr int KPL = M::KPL, KS = M::KSTEP;
  constexpr OpLayout L(N);
  constexpr int Np = L.Np, Nfp = L.Nfp, K2 = 2 * Np;
  constexpr int MT = (Np + 15) / 16;
  constexpr int KC = (Np + KS - 1) / KS;
  __shared__ T cbuf[2][Np * kEdgeTile];   // per wave: [coefficient][edge]; wave 1's rows then hold the flux shares
  __shared__ int rot[2 * Np];
  const int64_t E = m.E_int + m.E_bdy;
  const int64_t b = blockIdx.x;
  const int64_t nbt = (int64_t)nb_bdy * nf;
  if (b < nbt) {
    // boundary faces first (mirror-ghost operator, one lane per face)
    const int field = (int)(b % nf);
    const int64_t e = m.E_int + (b / nf) * (2 * kEdgeTile) + threadIdx.x;
    if (e < E) boundary_body<N, T, DM, false>(m, opbase<T>(m), e, field, u, flux);
    return;
  }
  int64_t tile;
  int field;
  tile_and_field(b - nbt, (int64_t)gridDim.x - nbt, nf, tile, field);   // nbt % 8 == 0
  const int64_t e0 = tile * kEdgeTile;
  // rotated lattice node -> element node for faces 0 and 2 (face 1: identity)
  for (int n = threadIdx.x; n < Np; n += 2 * kEdgeTile) {
    int j = 0;
    while (lat(N, 0, j + 1) <= n) ++j;
    const int i = n - lat(N, 0, j);
    rot[n] = lat(N, j, N - i - j);
    rot[Np + n] = lat(N, N - i - j, i);
  }
  const int s = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // this wave's side
  const int l = threadIdx.x & 63, col = l & 15, grp = l >> 4;
  const bool valid = e0 + l < m.E_int;
  const int64_t e = valid ? e0 + l : e0;
  const int2 ef = m.ef[e];
  const double2 mu = s ? m.mu2[e] : m.mu1[e];
  const double2 g = m.gam[e];
  double2 vn = make_double2(0.0, 0.0);
  if (CONV) vn = m.vn[e];
  const int k1 = ef.x & 0x3fffffff, fa = (int)((unsigned)ef.x >> 30);
  const int k2 = ef.y & 0x3fffffff, fb = (int)((unsigned)ef.y >> 30);
  const int k = s ? k2 : k1, f = s ? fb : fa;
  double D1d = 0.0, D2d = 0.0;
  if (DM != DM_CONST) {
    D1d = m.Delem[k1];
    D2d = m.Delem[k2];
  }
  const T* uf = u + (int64_t)field * m.K * Np;
  const cptr<T> op = opbase<T>(m);
  const T* opg = (const T*)(const void*)opbase<T>(m);
  // conversion matrix as A fragments: row 16 mt + col, columns kidx(c, grp, .)
  frag_t aN[MT][KC];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      T v[KPL];
#pragma unroll
      for (int t = 0; t < KPL; ++t) {
        const int i = 16 * mt + col, kk = kidx<M>(c, grp, t);
        v[t] = (i < Np && kk < Np) ? opg[L.n2b + i * Np + kk] : T(0);
      }
      aN[mt][c] = M::make(v);
    }
  __syncthreads();   // rot

  // gather + rotate + convert, 16 edges at a time; coefficients to LDS rows
  T* cb = cbuf[s];
#pragma unroll
  for (int sb = 0; sb < 4; ++sb) {
    const int el = 16 * sb + col;
    const int kk = __shfl(k, el), ff = __shfl(f, el);
    const T* ue = uf + (int64_t)kk * Np;
    frag_t bu[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      T v[KPL];
#pragma unroll
      for (int t = 0; t < KPL; ++t) {
        const int n = kidx<M>(c, grp, t);
        const int nc = n < Np ? n : 0;
        const T x = ue[ff == 1 ? nc : rot[(ff >> 1) * Np + nc]];
        v[t] = n < Np ? x : T(0);
      }
      bu[c] = M::make(v);
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      acc_t cm = M::zero();
#pragma unroll
      for (int c = 0; c < KC; ++c) cm = M::mma(aN[mt][c], bu[c], cm);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * mt + M::row(grp, r);
        if (row < Np) cb[row * kEdgeTile + el] = cm[r];
      }
    }
  }
  // the rows were written by this wave's own lanes: a wave-level fence
  // orders the LDS writes before the reads
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

  // one lane per edge: subdivision, reconstruction columns of this side
  T c[Np], tr[Nfp];
#pragma unroll
  for (int n = 0; n < Np; ++n) c[n] = cb[n * kEdgeTile + l];
  if (CONV) {
    // nodal trace on the face (the hypotenuse of the rotated triangle)
#pragma unroll
    for (int j = 0; j <= N; ++j) tr[j] = c[lat(N, N - j, j)];
    face_bernstein_to_nodal<N, T>(op, tr);
  }
  decasteljau<N, T>(c, mu);
  const bool quad = DM == DM_ALG1 && __ballot(valid && D1d != D2d) != 0;
  const T gR = (T)g.x, gS = (T)g.y;
  T F[Nfp];
  if (DM == DM_ALG2) {
    const T D1 = (T)D1d, D2 = (T)D2d;
    auto emit = [&](int j, const T* a) { F[j] = alg2_coef<N, T>(op, j, D1, D2) * (gR * a[0] + gS * a[1]); };
    matvec_groups<2, Nfp, Nfp, Np, K2, T, decltype(emit), 16>(op + L.kr + s * Np, c, emit);
  } else if (quad) {
    const T D1 = (T)D1d, D2 = (T)D2d;
    const T a1 = D1 * gR, b1 = D1 * gS, a2 = -D2 * gR, b2 = -D2 * gS;
    matvec_groups<4, Nfp, Nfp, Np, K2, T>(op + L.u1r + s * Np, c, [&](int j, const T* a) {
      F[j] = a1 * a[0] + b1 * a[1] + a2 * a[2] + b2 * a[3];
    });
  } else {
    const T D = DM == DM_ALG1 ? (T)D1d : (T)field_D(m, field);
    const T a1 = D * gR, b1 = D * gS;
    auto emit = [&](int j, const T* a) { F[j] = a1 * a[0] + b1 * a[1]; };
    matvec_groups<2, Nfp, Nfp, Np, K2, T, decltype(emit), 16>(op + (DM == DM_ALG1 ? L.udr : L.kr) + s * Np, c, emit);
  }
  if (CONV) {
    // upwind: node j of side 1 meets node N - j of side 2
#pragma unroll
    for (int j = 0; j < Nfp; ++j) {
      const T tau = op[L.tau + j];
      const T vnj = (T)vn.x + tau * (T)(vn.y - vn.x);
      const bool up = s ? !(vnj > (T)0) : (vnj > (T)0);
      F[j] -= up ? vnj * tr[s ? N - j : j] : T(0);
    }
  }
  // side 2's share into its own (already read) LDS rows
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  T* part = cbuf[1];
  if (s == 1) {
#pragma unroll
    for (int j = 0; j < Nfp; ++j) part[j * kEdgeTile + l] = F[j];
  }
  __syncthreads();
  if (s == 0 && valid) {
    T* out = flux + ((int64_t)field * E + e) * Nfp;
#pragma unroll
    for (int j = 0; j < Nfp; ++j) out[j] = F[j] + part[j * kEdgeTile + l];
  }
}

template <int N, typename P>
hipError_t edge_smfma_t(const DevMesh& m, int nfields, const void* u, void* flux, hipStream_t st) {
  using T = typename Mma<P>::T;
  if (m.E_int + m.E_bdy == 0) return hipSuccess;
  const int64_t nbi = (m.E_int + kEdgeTile - 1) / kEdgeTile;
  int64_t nbb = ((m.E_bdy + 2 * kEdgeTile - 1) / (2 * kEdgeTile) + 7) / 8 * 8;
  if (m.ghost) {
    const hipError_t eb = launch_boundary_faces(m, sizeof(T) == 8, nfields, u, flux, st);
    if (eb != hipSuccess) return eb;
    nbb = 0;
  }
  if (nbi + nbb == 0) return hipSuccess;
  dim3 grid((unsigned)((nbi + nbb) * nfields));
  const T* uu = (const T*)u;
  T* ff = (T*)flux;
  const int nbd = (int)nbb;
#define ARDG_SMFMA(A, C) \
  hipLaunchKernelGGL((edge_smfma_kernel<N, P, A, C>), grid, dim3(2 * kEdgeTile), 0, st, m, uu, ff, nbd, nfields)
  switch (m.dmode * 2 + (m.conv ? 1 : 0)) {
    case 0: ARDG_SMFMA(DM_CONST, false); break;
    case 1: ARDG_SMFMA(DM_CONST, true); break;
    case 2: ARDG_SMFMA(DM_ALG1, false); break;
    case 3: ARDG_SMFMA(DM_ALG1, true); break;
    case 4: ARDG_SMFMA(DM_ALG2, false); break;
    case 5: ARDG_SMFMA(DM_ALG2, true); break;
    default: return hipErrorInvalidValue;
  }
#undef ARDG_SMFMA
  return hipGetLastError();
}

template <typename P>
hipError_t edge_smfma_dispatch(const DevMesh& m, int nf, const void* u, void* flux, hipStream_t st) {
  switch (m.N) {
    case 1: return edge_smfma_t<1, P>(m, nf, u, flux, st);
    case 2: return edge_smfma_t<2, P>(m, nf, u, flux, st);
    case 3: return edge_smfma_t<3, P>(m, nf, u, flux, st);
    case 4: return edge_smfma_t<4, P>(m, nf, u, flux, st);
    case 5: return edge_smfma_t<5, P>(m, nf, u, flux, st);
    case 6: return edge_smfma_t<6, P>(m, nf, u, flux, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_edge_split_mfma(const DevMesh& m, int prec, int nfields, const void* u, void* flux,
                                  hipStream_t st) {
  switch (prec) {
    case PREC_FP64: return edge_smfma_dispatch<double>(m, nfields, u, flux, st);
    case PREC_FP32: return edge_smfma_dispatch<float>(m, nfields, u, flux, st);
    case PREC_BF16X3: return edge_smfma_dispatch<Bf16x3>(m, nfields, u, flux, st);
    default: return hipErrorInvalidValue;
  }
}

template <int N, typename P>
hipError_t edge_mfma_t(const DevMesh& m, int nfields, const void* u, void* flux, hipStream_t st) {
  using T = typename Mma<P>::T;
  const int64_t nbi = (m.E_int + kEdgeTile - 1) / kEdgeTile;
  int64_t nbb = ((m.E_bdy + kEdgeTile - 1) / kEdgeTile + 7) / 8 * 8;
  if (m.E_int + m.E_bdy == 0) return hipSuccess;
  if (m.ghost) {
    const hipError_t eb = launch_boundary_faces(m, sizeof(T) == 8, nfields, u, flux, st);
    if (eb != hipSuccess) return eb;
    nbb = 0;
  }
  if (nbi + nbb == 0) return hipSuccess;
  dim3 grid((unsigned)((nbi + nbb) * nfields));
  const T* uu = (const T*)u;
  T* ff = (T*)flux;
  const int nbd = (int)nbb;
#define ARDG_EMFMA(A, C) \
  hipLaunchKernelGGL((edge_mfma_kernel<N, P, A, C>), grid, dim3(kEdgeTile), 0, st, m, uu, ff, nbd, nfields)
  switch (m.dmode * 2 + (m.conv ? 1 : 0)) {
    case 0: ARDG_EMFMA(DM_CONST, false); break;
    case 1: ARDG_EMFMA(DM_CONST, true); break;
    case 2: ARDG_EMFMA(DM_ALG1, false); break;
    case 3: ARDG_EMFMA(DM_ALG1, true); break;
    case 4: ARDG_EMFMA(DM_ALG2, false); break;
    case 5: ARDG_EMFMA(DM_ALG2, true); break;
    default: return hipErrorInvalidValue;
  }
#undef ARDG_EMFMA
  return hipGetLastError();
}

template <typename P>
hipError_t edge_mfma_dispatch(const DevMesh& m, int nf, const void* u, void* flux, hipStream_t st) {
  switch (m.N) {
    case 1: return edge_mfma_t<1, P>(m, nf, u, flux, st);
    case 2: return edge_mfma_t<2, P>(m, nf, u, flux, st);
    case 3: return edge_mfma_t<3, P>(m, nf, u, flux, st);
    case 4: return edge_mfma_t<4, P>(m, nf, u, flux, st);
    case 5: return edge_mfma_t<5, P>(m, nf, u, flux, st);
    case 6: return edge_mfma_t<6, P>(m, nf, u, flux, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_edge_mfma(const DevMesh& m, int prec, int nfields, const void* u, void* flux,
                            hipStream_t st) {
  switch (prec) {
    case PREC_FP64: return edge_mfma_dispatch<double>(m, nfields, u, flux, st);
    case PREC_FP32: return edge_mfma_dispatch<float>(m, nfields, u, flux, st);
    case PREC_BF16X3: return edge_mfma_dispatch<Bf16x3>(m, nfields, u, flux, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ardg
