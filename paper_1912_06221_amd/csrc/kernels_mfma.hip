// Element kernel on the matrix cores (gfx950 MFMA, 16x16 tiles).
//
// The per-element operators of the volume term and of the surface term --
// Dr, Ds (Np x Np) and LIFT (Np x 3 Nfp) -- act on every element's vector, so
// for 16 elements at a time they are dense products (Np x Np) x (Np x 16) on
// the matrix cores.  The operators stay resident in registers as MFMA A
// fragments for the whole kernel (no per-entry operand loads); the element
// data enters as B fragments and comes out in the accumulator layout, and the
// conversions between the two layouts go through LDS.
//
// Fragment layouts of the 16x16xK instructions used here (K per instruction
// = 4, one value per lane): lane l supplies A[row = l % 16][k = l / 16] and
// B[k = l / 16][col = l % 16].  The 16x16 result sits in four registers per
// lane with column l % 16; the row of register r differs by instruction:
// 4 (l / 16) + r for the FP32 one and 4 r + l / 16 for the FP64 one.
//
// Per 16-element sub-tile (columns = elements, rows = nodes):
//   (ur; us) = (Dr; Ds) u                    -> q = geometric combination
//   div      = Dr (r_x q_x + r_y q_y) + Ds (s_x q_x + s_y q_y)
//   rhs      = D div + LIFT [ (J_f/J) (F_f - D n_f.q_f (+ n_f.v u)) ]_f
//   (convection: rhs -= r_x Dr(v_x u) + s_x Ds(v_x u) + r_y Dr(v_y u) + s_y Ds(v_y u))
// The tile's stage input, the Runge-Kutta update and the output use the same
// LDS-staged, coalesced passes as the thread-per-element kernel.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "kernel_common.hpp"

namespace ardg {

typedef double mf_d4 __attribute__((ext_vector_type(4)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mma;
template <> struct Mma<double> {
  typedef mf_d4 acc;
  __device__ static acc zero() {
    acc z = {0.0, 0.0, 0.0, 0.0};
    return z;
  }
  __device__ static acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static constexpr int row(int grp, int r) { return 4 * r + grp; }
};
template <> struct Mma<float> {
  typedef mf_f4 acc;
  __device__ static acc zero() {
    acc z = {0.f, 0.f, 0.f, 0.f};
    return z;
  }
  __device__ static acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static constexpr int row(int grp, int r) { return 4 * grp + r; }
};

constexpr int kMfmaTile = 64;   // elements per block (one wave)

template <int N, typename T, bool CONV>
__global__ __launch_bounds__(kMfmaTile) void element_mfma_kernel(DevMesh m, const T* __restrict__ vin,
                                                                 const T* __restrict__ flux,
                                                                 Epilogue epi) {
  constexpr OpLayout L(N);
  constexpr int Np = L.Np, Nfp = L.Nfp;
  constexpr int MT = (Np + 15) / 16;     // row tiles of nodes
  constexpr int KC = (Np + 3) / 4;       // K steps over nodes
  constexpr int NJ = 3 * Nfp;            // face values lifted
  constexpr int KL = (NJ + 3) / 4;       // K steps over face values
  constexpr int RW = 16 * MT;            // padded node rows
  constexpr bool kPre = N <= 4;
  using M = Mma<T>;
  typedef typename M::acc acc_t;
  __shared__ T sh[kMfmaTile * Np];
  __shared__ T sq[4][RW * 16];           // q_x, q_y, w_r, w_s of one sub-tile, [node][column]
  const int l = threadIdx.x, col = l & 15, grp = l >> 4;
  const int64_t k0 = xcd_block(blockIdx.x, gridDim.x) * kMfmaTile;
  const int field = blockIdx.y;
  const int64_t E = m.E_int + m.E_bdy;
  const T* opg = (const T*)(sizeof(T) == 8 ? (const void*)m.ops64 : (const void*)m.ops32);

  // operator fragments, resident for the whole kernel
  T aDr[MT][KC], aDs[MT][KC], aL[MT][KL];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    const int row = 16 * mt + col;
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      const int kk = 4 * c + grp;
      const bool ok = row < Np && kk < Np;
      aDr[mt][c] = ok ? opg[L.dr + row * Np + kk] : T(0);
      aDs[mt][c] = ok ? opg[L.ds + row * Np + kk] : T(0);
    }
#pragma unroll
    for (int c = 0; c < KL; ++c) {
      const int kk = 4 * c + grp;
      aL[mt][c] = (row < Np && kk < NJ) ? opg[L.lift + row * NJ + kk] : T(0);
    }
  }

  TileIO<Np> io;
  tile_begin<N, T, kMfmaTile>(m, k0, field, vin, epi, sh, io, kPre);
  __syncthreads();

  for (int st = 0; st < kMfmaTile / 16; ++st) {
    const int el = st * 16 + col;
    const bool valid = el < io.nel;
    const int64_t k = k0 + (valid ? el : 0);
    const double2 p1 = m.vert[3 * k], p2 = m.vert[3 * k + 1], p3 = m.vert[3 * k + 2];
    const double xr = 0.5 * (p2.x - p1.x), yr = 0.5 * (p2.y - p1.y);
    const double xs = 0.5 * (p3.x - p1.x), ys = 0.5 * (p3.y - p1.y);
    const double J = xr * ys - xs * yr;
    const T rx = (T)(ys / J), ry = (T)(-xs / J), sx = (T)(-yr / J), sy = (T)(xr / J);
    const T D = (T)(m.alg1 ? m.Delem[k] : m.Dfield[field]);

    // u as B fragments: node 4c + grp of element `col`
    T bu[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      const int n = 4 * c + grp;
      bu[c] = (valid && n < Np) ? sh[el * Np + n] : T(0);
    }
    acc_t ur[MT], us[MT];
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
    // accumulator layout: node 16 mt + M::row(grp, r) of element `col`
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int node = 16 * mt + M::row(grp, r);
        const T qx = rx * ur[mt][r] + sx * us[mt][r];
        const T qy = ry * ur[mt][r] + sy * us[mt][r];
        sq[0][node * 16 + col] = qx;
        sq[1][node * 16 + col] = qy;
        sq[2][node * 16 + col] = rx * qx + ry * qy;
        sq[3][node * 16 + col] = sx * qx + sy * qy;
      }
    __syncthreads();

    acc_t rhs[MT];
    {
      T bw[KC], bs[KC];
#pragma unroll
      for (int c = 0; c < KC; ++c) {
        const int n = 4 * c + grp;
        bw[c] = sq[2][n * 16 + col];
        bs[c] = sq[3][n * 16 + col];
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        acc_t dv = M::zero();
#pragma unroll
        for (int c = 0; c < KC; ++c) {
          dv = M::mma(aDr[mt][c], bw[c], dv);
          dv = M::mma(aDs[mt][c], bs[c], dv);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) rhs[mt][r] = D * dv[r];
      }
    }

    // face values as B fragments over q = 4c + grp (face q / Nfp, node q % Nfp)
    T bj[KL];
#pragma unroll
    for (int c = 0; c < KL; ++c) {
      const int q = 4 * c + grp;
      T v = T(0);
      if (valid && q < NJ) {
        const int f = q / Nfp, jj = q - f * Nfp;
        const int nd = (f == 0) ? lat(N, jj, 0) : (f == 1 ? lat(N, N - jj, jj) : lat(N, 0, N - jj));
        const double2 a = (f == 0) ? p1 : (f == 1 ? p2 : p3);
        const double2 b = (f == 0) ? p2 : (f == 1 ? p3 : p1);
        const double tx = b.x - a.x, ty = b.y - a.y;
        const double len = sqrt(tx * tx + ty * ty);
        const T nx = (T)(ty / len), ny = (T)(-tx / len);
        const int code = m.elem_face[f * m.K + k];
        const T* fe = flux + ((int64_t)field * E + (code >> 1)) * Nfp;
        const T G = (code & 1) ? -fe[Nfp - 1 - jj] : fe[jj];
        T jv = G - D * (nx * sq[0][nd * 16 + col] + ny * sq[1][nd * 16 + col]);
        if (CONV) {
          const double rr = (double)opg[L.nr + nd], ss = (double)opg[L.ns + nd];
          const double x = 0.5 * (-(rr + ss) * p1.x + (rr + 1.0) * p2.x + (ss + 1.0) * p3.x);
          const double y = 0.5 * (-(rr + ss) * p1.y + (rr + 1.0) * p2.y + (ss + 1.0) * p3.y);
          const T vx = (T)(m.vel[0] + m.vel[2] * x + m.vel[3] * y);
          const T vy = (T)(m.vel[1] + m.vel[4] * x + m.vel[5] * y);
          jv += (nx * vx + ny * vy) * sh[el * Np + nd];
        }
        v = (T)(0.5 * len / J) * jv;
      }
      bj[c] = v;
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      acc_t lf = M::zero();
#pragma unroll
      for (int c = 0; c < KL; ++c) lf = M::mma(aL[mt][c], bj[c], lf);
#pragma unroll
      for (int r = 0; r < 4; ++r) rhs[mt][r] += lf[r];
    }

    if (CONV) {
      // nodal collocation of v u; -(d/dx (v_x u) + d/dy (v_y u))
      T bfx[KC], bfy[KC];
#pragma unroll
      for (int c = 0; c < KC; ++c) {
        const int n = 4 * c + grp;
        T fx = T(0), fy = T(0);
        if (valid && n < Np) {
          const double rr = (double)opg[L.nr + n], ss = (double)opg[L.ns + n];
          const double x = 0.5 * (-(rr + ss) * p1.x + (rr + 1.0) * p2.x + (ss + 1.0) * p3.x);
          const double y = 0.5 * (-(rr + ss) * p1.y + (rr + 1.0) * p2.y + (ss + 1.0) * p3.y);
          const T uu = sh[el * Np + n];
          fx = (T)(m.vel[0] + m.vel[2] * x + m.vel[3] * y) * uu;
          fy = (T)(m.vel[1] + m.vel[4] * x + m.vel[5] * y) * uu;
        }
        bfx[c] = fx;
        bfy[c] = fy;
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        acc_t xr_ = M::zero(), xs_ = M::zero(), yr_ = M::zero(), ys_ = M::zero();
#pragma unroll
        for (int c = 0; c < KC; ++c) {
          xr_ = M::mma(aDr[mt][c], bfx[c], xr_);
          xs_ = M::mma(aDs[mt][c], bfx[c], xs_);
          yr_ = M::mma(aDr[mt][c], bfy[c], yr_);
          ys_ = M::mma(aDs[mt][c], bfy[c], ys_);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) rhs[mt][r] -= rx * xr_[r] + sx * xs_[r] + ry * yr_[r] + sy * ys_[r];
      }
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
  }
  tile_end<N, T, kMfmaTile>(epi, sh, io, kPre);
}

template <int N, typename T>
hipError_t elem_mfma_t(const DevMesh& m, int nfields, const void* vin, const void* flux,
                       const Epilogue& epi, hipStream_t st) {
  dim3 grid((unsigned)((m.K + kMfmaTile - 1) / kMfmaTile), (unsigned)nfields);
  if (m.conv)
    hipLaunchKernelGGL((element_mfma_kernel<N, T, true>), grid, dim3(kMfmaTile), 0, st, m,
                       (const T*)vin, (const T*)flux, epi);
  else
    hipLaunchKernelGGL((element_mfma_kernel<N, T, false>), grid, dim3(kMfmaTile), 0, st, m,
                       (const T*)vin, (const T*)flux, epi);
  return hipGetLastError();
}

template <typename T>
hipError_t elem_mfma_dispatch(const DevMesh& m, int nf, const void* vin, const void* flux,
                              const Epilogue& epi, hipStream_t st) {
  switch (m.N) {
    case 1: return elem_mfma_t<1, T>(m, nf, vin, flux, epi, st);
    case 2: return elem_mfma_t<2, T>(m, nf, vin, flux, epi, st);
    case 3: return elem_mfma_t<3, T>(m, nf, vin, flux, epi, st);
    case 4: return elem_mfma_t<4, T>(m, nf, vin, flux, epi, st);
    case 5: return elem_mfma_t<5, T>(m, nf, vin, flux, epi, st);
    case 6: return elem_mfma_t<6, T>(m, nf, vin, flux, epi, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_element_mfma(const DevMesh& m, bool fp64, int nfields, const void* vin,
                               const void* flux, const Epilogue& epi, hipStream_t st) {
  return fp64 ? elem_mfma_dispatch<double>(m, nfields, vin, flux, epi, st)
              : elem_mfma_dispatch<float>(m, nfields, vin, flux, epi, st);
}

}  // namespace ardg
