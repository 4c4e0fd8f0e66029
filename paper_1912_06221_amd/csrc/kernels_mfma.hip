// Element kernel on the matrix cores (gfx950 MFMA, 16x16 tiles).
//
// The per-element operators of the volume term and of the surface term --
// Dr, Ds (Np x Np) and LIFT (Np x 3 Nfp) -- act on every element's vector, so
// for 16 elements at a time they are dense products (Np x Np) x (Np x 16) on
// the matrix cores.  The operators stay resident in registers as MFMA A
// fragments (no per-entry operand loads); the element data enters as B
// fragments and comes out in the accumulator layout, and the conversions
// between the two layouts go through LDS.
//
// A block takes 64 elements; each of its four waves one 16-element sub-tile
// (columns = elements, rows = nodes):
//   (ur; us) = (Dr; Ds) u,  q = (r_x ur + s_x us, r_y ur + s_y us)
//   w_r = D (r_x q_x + r_y q_y) - v_r u,  w_s = D (s_x q_x + s_y q_y) - v_s u
//   rhs = Dr w_r + Ds w_s + LIFT [ (1/J) (G_f - D (sJ n)_f.q_f + (sJ n)_f.v u) ]_f
// with the contravariant velocity v_r = r_x v_x + r_y v_y, v_s = s_x v_x +
// s_y v_y (convection only): because the metric terms are constant on an
// affine element, the strong-form diffusion divergence and the convective
// volume term -(d/dx (v_x u) + d/dy (v_y u)) share one [Dr Ds] product.  G_f
// is the edge kernel's flux, already multiplied by the face's sJ.
// Every global load of a tile (stage input, update operands, vertices, face
// map and the gathered fluxes) is issued before the compute, so a wave waits
// for memory twice (the face map, then the fluxes) instead of once per step.
// The tile's stage input, the Runge-Kutta update and the output use the same
// LDS-staged, coalesced passes as the thread-per-element kernel.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device.hpp"
#include "kernel_common.hpp"
#include "mfma.hpp"

namespace ardg {

constexpr int kMfmaTile = 64;     // elements per block
constexpr int kMfmaThreads = 256; // four waves, one 16-element sub-tile each

// LDS of one 64-element tile: the tile's stage input (then its du/dt), each
// wave's transpose rows, and (FP32 data) the operators.
template <int N, typename P>
struct ElemShared {
  using M = Mma<P>;
  using T = typename M::T;
  static constexpr int Np = (N + 1) * (N + 2) / 2;
  static constexpr int MT = (Np + 15) / 16;
  static constexpr int KC = (Np + M::KSTEP - 1) / M::KSTEP;
  static constexpr int RW = 16 * MT, KW = M::KSTEP * KC;
  static constexpr int SQ = (RW > KW ? RW : KW) * 16;
  T sh[TileShape<N, kMfmaTile, kMfmaThreads>::LDS];
  T sqa[4][2][SQ];            // per wave: w_r, w_s, then q_x, q_y of its sub-tile, [node][column]
  // Dr, Ds, LIFT read once per block with coalesced loads, fragments built
  // from here (all but FP64 above N = 4, which gathers its fragments from the
  // cache with the tile's loads)
  static constexpr bool kOpLds = sizeof(T) == 4 || N <= 4;
  static constexpr int NO = 2 * Np * Np + Np * 3 * (N + 1);
  static constexpr int QO = (NO + 255) / 256;      // entries per thread of the copy
  T opl[kOpLds ? QO * 256 : 1];
  T rs1[2][64];               // reference coordinates + 1 of the nodes (convection)
};

// One 64-element tile starting at element k0 of field `field`; all 256
// threads of the block take part (wave w: sub-tile w).  TENS: the diffusion
// coefficient is a nodal tensor (or the tensor D0 times the solution):
// q = D grad u is formed node by node and the scalar D is 1.
template <int N, typename P, bool CONV, bool TENS = false>
__device__ inline void element_mfma_tile(const DevMesh& m, int64_t k0, int field,
                                         const typename Mma<P>::T* __restrict__ vin,
                                         const typename Mma<P>::T* __restrict__ flux, const Epilogue& epi,
                                         ElemShared<N, P>& S) {
  using M = Mma<P>;
  using T = typename M::T;
  typedef typename M::acc acc_t;
  typedef typename M::frag frag_t;
  constexpr int KPL = M::KPL, KS = M::KSTEP;
  constexpr OpLayout L(N);
  constexpr int Np = L.Np, Nfp = L.Nfp;
  constexpr int MT = (Np + 15) / 16;     // row tiles of nodes
  constexpr int KC = (Np + KS - 1) / KS; // K steps over nodes
  constexpr int NJ = 3 * Nfp;            // face values lifted
  constexpr int KL = (NJ + KS - 1) / KS; // K steps over face values
  constexpr int RW = 16 * MT;            // padded node rows
  constexpr int SQ = ElemShared<N, P>::SQ;
  constexpr bool kPre = N <= 4;
  T* sh = S.sh;
  const int l = threadIdx.x & 63, col = l & 15, grp = l >> 4;
  const int st = threadIdx.x >> 6;       // this wave's sub-tile
  T (*sq)[SQ] = S.sqa[st];
  const int64_t E = m.E_int + m.E_bdy;
  const T* opg = (const T*)(sizeof(T) == 8 ? (const void*)m.ops64 : (const void*)m.ops32);

  // ---- loads: element data, face map, stage input, update operands ----
  // Every global load of the tile is issued before the first wait, and the
  // LDS stores that follow are unconditional, so the only dependent round
  // trip is face map -> fluxes.
  const int el = st * 16 + col;
  const bool valid = k0 + el < m.K;
  const int64_t k = valid ? k0 + el : k0;
  int code[3];
#pragma unroll
  for (int f = 0; f < 3; ++f) code[f] = m.elem_face[f * m.K + k];
  const double2 p1 = m.vert[3 * k], p2 = m.vert[3 * k + 1], p3 = m.vert[3 * k + 2];
  // D: element-wise, or the field's constant (one load from either table,
  // no branch)
  const bool Dk = m.dmode != DM_CONST;
  const double Dd = TENS ? 1.0 : (Dk ? m.Delem : m.Dfield_dev)[Dk ? k : (int64_t)field];

  // Dr and Ds (adjacent in the operator buffer) and LIFT into LDS with
  // coalesced loads; each wave builds its fragments from there after the
  // barrier instead of gathering them from the cache once per lane.  FP32,
  // and FP64 up to N = 4, build the fragments where each product uses them,
  // so they are not live across the tile's loads (one more wave per SIMD);
  // the split-BF16 fragments, whose splitting costs arithmetic, are built
  // once.
  constexpr bool kOpLds = ElemShared<N, P>::kOpLds;
  constexpr bool kLazy = kOpLds && !std::is_same<P, Bf16x3>::value;
  constexpr int NO1 = 2 * Np * Np, NO = NO1 + Np * NJ, QO = ElemShared<N, P>::QO;
  T* opl = S.opl;
  T ov[kOpLds ? QO : 1];
  if (kOpLds) {
#pragma unroll
    for (int q = 0; q < QO; ++q) {
      const int i = threadIdx.x + q * kMfmaThreads;
      const int ic = i < NO ? i : 0;
      ov[q] = opg[ic < NO1 ? L.dr + ic : L.lift + (ic - NO1)];
    }
  }
  T rsv[2] = {T(0), T(0)};
  if (CONV) {
    const int nd = (threadIdx.x & 63) < Np ? (threadIdx.x & 63) : 0;
    rsv[0] = opg[L.nr + nd] + T(1);
    rsv[1] = opg[L.ns + nd] + T(1);
  }
  TileIO<TileShape<N, kMfmaTile, kMfmaThreads>::Q, T> io;
  tile_load<N, T, kMfmaTile, kMfmaThreads>(m, k0, field, vin, epi, io, kPre);

  // face fluxes in the B layout of the lift: value q = kidx(c, grp, t) is node
  // q % Nfp of face q / Nfp, read from its edge (reversed and negated on side
  // 2).  Loads are unconditional from clamped indices; the mask multiplies
  // instead of selecting, so no load is sunk into a branch of its own.
  T G[KL][KPL];
#pragma unroll
  for (int c = 0; c < KL; ++c)
#pragma unroll
    for (int t = 0; t < KPL; ++t) {
      const int q = kidx<M>(c, grp, t);
      const int qc = q < NJ ? q : 0;
      const int f = qc / Nfp, jj = qc - f * Nfp;
      const int cd = (f == 0) ? code[0] : (f == 1 ? code[1] : code[2]);
      const bool side2 = cd & 1;
      const T x = flux[((int64_t)field * E + (cd >> 1)) * Nfp + (side2 ? Nfp - 1 - jj : jj)];
      const T sgn = (valid && q < NJ) ? (side2 ? T(-1) : T(1)) : T(0);
      G[c][t] = sgn * x;
    }

  // LDS stores of the loaded operators, node coordinates and stage input
  if (kOpLds) {
#pragma unroll
    for (int q = 0; q < QO; ++q) opl[threadIdx.x + q * kMfmaThreads] = ov[q];
  }
  if (CONV) {
    // every wave stores the same 64 values (no branch on the thread index)
    S.rs1[0][threadIdx.x & 63] = rsv[0];
    S.rs1[1][threadIdx.x & 63] = rsv[1];
  }
  tile_stage<N, T, kMfmaTile, kMfmaThreads>(sh, io);

  // operator fragments (from LDS, or gathered from the operator buffer):
  // row 16 mt + col, columns kidx(c, grp, .)
  const T* odr = kOpLds ? opl : opg + L.dr;
  const T* olift = kOpLds ? opl + NO1 : opg + L.lift;
  auto build_d = [&](frag_t (&aDr)[MT][KC], frag_t (&aDs)[MT][KC]) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int row = 16 * mt + col;
#pragma unroll
      for (int c = 0; c < KC; ++c) {
        T vr[KPL], vs[KPL];
#pragma unroll
        for (int t = 0; t < KPL; ++t) {
          const int kk = kidx<M>(c, grp, t);
          const bool ok = row < Np && kk < Np;
          vr[t] = ok ? odr[row * Np + kk] : T(0);
          vs[t] = ok ? odr[Np * Np + row * Np + kk] : T(0);
        }
        aDr[mt][c] = M::make(vr);
        aDs[mt][c] = M::make(vs);
      }
    }
  };
  auto build_l = [&](frag_t (&aL)[MT][KL]) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int row = 16 * mt + col;
#pragma unroll
      for (int c = 0; c < KL; ++c) {
        T vl[KPL];
#pragma unroll
        for (int t = 0; t < KPL; ++t) {
          const int kk = kidx<M>(c, grp, t);
          vl[t] = (row < Np && kk < NJ) ? olift[row * NJ + kk] : T(0);
        }
        aL[mt][c] = M::make(vl);
      }
    }
  };
  frag_t aDr[MT][KC], aDs[MT][KC], aL[MT][KL];
  if (!kOpLds) {
    build_d(aDr, aDs);
    build_l(aL);
  }
  __syncthreads();
  if (kOpLds && !kLazy) {
    build_d(aDr, aDs);
    build_l(aL);
  }

  // ---- compute ----
  const ElemGeom gm = elem_geom(p1, p2, p3);
  const T rx = (T)gm.rx, ry = (T)gm.ry, sx = (T)gm.sx, sy = (T)gm.sy;
  const T D = (T)Dd;
  ElemVel ev = {};
  if (CONV) ev = elem_vel(m.vel, p1, gm);

  // u as B fragments: nodes kidx(c, grp, .) of element `col`
  frag_t bu[KC];
#pragma unroll
  for (int c = 0; c < KC; ++c) {
    T v[KPL];
#pragma unroll
    for (int t = 0; t < KPL; ++t) {
      const int n = kidx<M>(c, grp, t);
      v[t] = (valid && n < Np) ? sh[el * Np + n] : T(0);
    }
    bu[c] = M::make(v);
  }
  acc_t ur[MT], us[MT];
  if (kLazy) build_d(aDr, aDs);
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    ur[mt] = M::zero();
    us[mt] = M::zero();
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      ur[mt] = M::mma(aDr[mt][c], bu[c], ur[mt]);
      us[mt] = M::mma(aDs[mt][c], bu[c], us[mt]);
    }
  }
  // accumulator layout: node 16 mt + M::row(grp, r) of element `col`.  w_r and
  // w_s go through LDS to become B fragments; q stays in registers until the
  // same LDS rows are free for the face terms
  T qxa[MT][4], qya[MT][4];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int node = 16 * mt + M::row(grp, r);
      T qx = rx * ur[mt][r] + sx * us[mt][r];
      T qy = ry * ur[mt][r] + sy * us[mt][r];
      if (TENS) {
        const int nc = node < Np ? node : 0;
        T dxx, dxy, dyy;
        if (m.dmode == DM_SOLUTION) {
          const T un = (valid && node < Np) ? sh[el * Np + nc] : T(0);
          dxx = (T)m.D0[0] * un;
          dxy = (T)m.D0[1] * un;
          dyy = (T)m.D0[2] * un;
        } else {
          const double* dn = m.Dnodal + ((int64_t)k * Np + nc) * 3;
          dxx = (T)dn[0];
          dxy = (T)dn[1];
          dyy = (T)dn[2];
        }
        const T tx = dxx * qx + dxy * qy, ty = dxy * qx + dyy * qy;
        qx = tx;
        qy = ty;
      }
      qxa[mt][r] = qx;
      qya[mt][r] = qy;
      T wr = D * (rx * qx + ry * qy);
      T ws = D * (sx * qx + sy * qy);
      if (CONV) {
        const T r1 = S.rs1[0][node], s1 = S.rs1[1][node];
        const T vx = (T)ev.x1 + r1 * (T)ev.xr + s1 * (T)ev.xs;
        const T vy = (T)ev.y1 + r1 * (T)ev.yr + s1 * (T)ev.ys;
        const T un = (valid && node < Np) ? sh[el * Np + (node < Np ? node : 0)] : T(0);
        wr -= (rx * vx + ry * vy) * un;
        ws -= (sx * vx + sy * vy) * un;
      }
      sq[0][node * 16 + col] = wr;
      sq[1][node * 16 + col] = ws;
    }
  __syncthreads();

  acc_t rhs[MT];
  {
    frag_t bw[KC], bs[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      T vw[KPL], vs[KPL];
#pragma unroll
      for (int t = 0; t < KPL; ++t) {
        const int n = kidx<M>(c, grp, t);
        vw[t] = n < RW ? sq[0][n * 16 + col] : T(0);
        vs[t] = n < RW ? sq[1][n * 16 + col] : T(0);
      }
      bw[c] = M::make(vw);
      bs[c] = M::make(vs);
    }
    // two independent accumulator chains (Dr and Ds), summed afterwards
    if (kLazy) build_d(aDr, aDs);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      acc_t rr = M::zero(), rs = M::zero();
#pragma unroll
      for (int c = 0; c < KC; ++c) {
        rr = M::mma(aDr[mt][c], bw[c], rr);
        rs = M::mma(aDs[mt][c], bs[c], rs);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) rhs[mt][r] = rr[r] + rs[r];
    }
  }
  __syncthreads();   // the B fragments are read: the rows take q now
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int node = 16 * mt + M::row(grp, r);
      sq[0][node * 16 + col] = qxa[mt][r];
      sq[1][node * 16 + col] = qya[mt][r];
    }
  __syncthreads();

  // face values (1/J) (G - D (sJ n).q (+ (sJ n).v u)) as B fragments
  frag_t bj[KL];
  const T iJ = (T)gm.iJ;
#pragma unroll
  for (int c = 0; c < KL; ++c) {
    T vj[KPL];
#pragma unroll
    for (int t = 0; t < KPL; ++t) {
      const int q = kidx<M>(c, grp, t);
      const int qc = q < NJ ? q : 0;
      const int f = qc / Nfp;
      const int nd = fnode(N, f, qc - f * Nfp);
      const double2 sn = face_sjn(gm, f);
      const T nx = (T)sn.x, ny = (T)sn.y;
      T jv = G[c][t] - D * (nx * sq[0][nd * 16 + col] + ny * sq[1][nd * 16 + col]);
      if (CONV) {
        const T r1 = S.rs1[0][nd], s1 = S.rs1[1][nd];
        const T vx = (T)ev.x1 + r1 * (T)ev.xr + s1 * (T)ev.xs;
        const T vy = (T)ev.y1 + r1 * (T)ev.yr + s1 * (T)ev.ys;
        jv += (nx * vx + ny * vy) * sh[el * Np + nd];
      }
      vj[t] = (valid && q < NJ) ? iJ * jv : T(0);
    }
    bj[c] = M::make(vj);
  }
  if (kLazy) build_l(aL);
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    acc_t rl = M::zero();
#pragma unroll
    for (int c = 0; c < KL; ++c) rl = M::mma(aL[mt][c], bj[c], rl);
#pragma unroll
    for (int r = 0; r < 4; ++r) rhs[mt][r] += rl[r];
  }

  __syncthreads();   // every read of sq and of this sub-tile's u is done
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int node = 16 * mt + M::row(grp, r);
      if (valid && node < Np) sh[el * Np + node] = rhs[mt][r];
    }
  __syncthreads();
  tile_end<N, T, kMfmaTile, kMfmaThreads>(epi, sh, io, kPre);
}

template <int N, typename P, bool CONV, bool TENS>
__global__ __launch_bounds__(kMfmaThreads) void element_mfma_kernel(DevMesh m,
                                                                    const typename Mma<P>::T* __restrict__ vin,
                                                                    const typename Mma<P>::T* __restrict__ flux,
                                                                    Epilogue epi, int nf) {
  __shared__ ElemShared<N, P> S;
  int64_t tile;
  int field;
  tile_and_field(blockIdx.x, gridDim.x, nf, tile, field);
  element_mfma_tile<N, P, CONV, TENS>(m, tile * kMfmaTile, field, vin, flux, epi, S);
}

// Batched form: persistent blocks over (problem, 64-element tile) items of
// many meshes (constant D, no convection, nodal stage vectors); each item
// reads its problem's descriptor (tables, buffers, dt).
template <int N, typename T>
__global__ __launch_bounds__(kMfmaThreads) void batch_element_mfma_kernel(const BatchProb* __restrict__ probs,
                                                                          const int2* __restrict__ items,
                                                                          int nitems, Epilogue epi0, int in_u,
                                                                          int write_v) {
  __shared__ ElemShared<N, T> S;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 w = items[it];
    const BatchProb* Pb = probs + __builtin_amdgcn_readfirstlane(w.x);
    Epilogue epi = epi0;
    epi.u = Pb->u;
    epi.acc = Pb->acc;
    epi.vnext = write_v ? Pb->v : nullptr;
    epi.dt = Pb->dt;
    const T* vin = in_u ? (const T*)(const void*)Pb->u : (const T*)Pb->v;
    const int64_t k0 = (int64_t)__builtin_amdgcn_readfirstlane(w.y) * kMfmaTile;
    element_mfma_tile<N, T, false>(Pb->m, k0, 0, vin, (const T*)Pb->flux, epi, S);
    __syncthreads();
  }
}

template <int N, typename T>
hipError_t batch_elem_mfma_t(int grid, const BatchProb* probs, const int2* items, int nitems,
                             const Epilogue& epi, int in_u, int write_v, hipStream_t st) {
  hipLaunchKernelGGL((batch_element_mfma_kernel<N, T>), dim3(grid), dim3(kMfmaThreads), 0, st, probs, items,
                     nitems, epi, in_u, write_v);
  return hipGetLastError();
}

hipError_t launch_batch_element_mfma(int N, bool fp64, int grid, const BatchProb* probs, const int2* items,
                                     int nitems, const Epilogue& epi, int in_u, int write_v, hipStream_t st) {
  if (nitems == 0) return hipSuccess;
#define ARDG_BEM(NN)                                                                                    \
  case NN:                                                                                              \
    return fp64 ? batch_elem_mfma_t<NN, double>(grid, probs, items, nitems, epi, in_u, write_v, st)     \
                : batch_elem_mfma_t<NN, float>(grid, probs, items, nitems, epi, in_u, write_v, st);
  switch (N) {
    ARDG_BEM(1) ARDG_BEM(2) ARDG_BEM(3) ARDG_BEM(4) ARDG_BEM(5) ARDG_BEM(6)
    default: return hipErrorInvalidValue;
  }
#undef ARDG_BEM
}

template <int N, typename P>
hipError_t elem_mfma_t(const DevMesh& m, int nfields, const void* vin, const void* flux,
                       const Epilogue& epi, hipStream_t st) {
  using T = typename Mma<P>::T;
  dim3 grid((unsigned)((m.K + kMfmaTile - 1) / kMfmaTile * nfields));
  if (m.dmode == DM_NODAL || m.dmode == DM_SOLUTION) {
    // tensor coefficients: FP64 and FP32 (no split-BF16 form)
    if constexpr (std::is_same<P, Bf16x3>::value) {
      return hipErrorInvalidValue;
    } else {
      if (m.conv)
        hipLaunchKernelGGL((element_mfma_kernel<N, P, true, true>), grid, dim3(kMfmaThreads), 0, st, m,
                           (const T*)vin, (const T*)flux, epi, nfields);
      else
        hipLaunchKernelGGL((element_mfma_kernel<N, P, false, true>), grid, dim3(kMfmaThreads), 0, st, m,
                           (const T*)vin, (const T*)flux, epi, nfields);
      return hipGetLastError();
    }
  }
  if (m.conv)
    hipLaunchKernelGGL((element_mfma_kernel<N, P, true, false>), grid, dim3(kMfmaThreads), 0, st, m,
                       (const T*)vin, (const T*)flux, epi, nfields);
  else
    hipLaunchKernelGGL((element_mfma_kernel<N, P, false, false>), grid, dim3(kMfmaThreads), 0, st, m,
                       (const T*)vin, (const T*)flux, epi, nfields);
  return hipGetLastError();
}

template <typename P>
hipError_t elem_mfma_dispatch(const DevMesh& m, int nf, const void* vin, const void* flux,
                              const Epilogue& epi, hipStream_t st) {
  switch (m.N) {
    case 1: return elem_mfma_t<1, P>(m, nf, vin, flux, epi, st);
    case 2: return elem_mfma_t<2, P>(m, nf, vin, flux, epi, st);
    case 3: return elem_mfma_t<3, P>(m, nf, vin, flux, epi, st);
    case 4: return elem_mfma_t<4, P>(m, nf, vin, flux, epi, st);
    case 5: return elem_mfma_t<5, P>(m, nf, vin, flux, epi, st);
    case 6: return elem_mfma_t<6, P>(m, nf, vin, flux, epi, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_element_mfma(const DevMesh& m, int prec, int nfields, const void* vin, const void* flux,
                               const Epilogue& epi, hipStream_t st) {
  switch (prec) {
    case PREC_FP64: return elem_mfma_dispatch<double>(m, nfields, vin, flux, epi, st);
    case PREC_FP32: return elem_mfma_dispatch<float>(m, nfields, vin, flux, epi, st);
    case PREC_BF16X3: return elem_mfma_dispatch<Bf16x3>(m, nfields, vin, flux, epi, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ardg
