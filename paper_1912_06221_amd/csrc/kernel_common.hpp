// Device helpers shared by the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "device.hpp"

namespace ardg {

// Operator tables live in the constant address space: wave-uniform reads of
// them go through the scalar unit.
template <typename T>
using cptr = const T __attribute__((address_space(4)))*;

__host__ __device__ constexpr int lat(int N, int i, int j) { return j * (N + 1) - (j * (j - 1)) / 2 + i; }

// node index of face f's j-th node (counter-clockwise)
__host__ __device__ constexpr int fnode(int N, int f, int j) {
  return f == 0 ? lat(N, j, 0) : (f == 1 ? lat(N, N - j, j) : lat(N, 0, N - j));
}

// Keeps the scalar loads of one operator row next to the FMAs that use them:
// without it the scheduler hoists whole matrices into SGPRs and spills.
__device__ inline void row_fence() { __builtin_amdgcn_sched_barrier(0); }

// readfirstlane returns a signed int: both halves are widened through uint32_t
// so that the low word is zero-extended.
__device__ inline uint64_t uniform_u64(uint64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | (uint64_t)lo;
}

// Passes an operator pointer through an empty asm so that repeated uses of one
// matrix are loaded again instead of being kept live in SGPRs.
template <typename T>
__device__ inline cptr<T> fresh(cptr<T> p) {
  uint64_t w = uniform_u64((uint64_t)p);
  asm volatile("" : "+s"(w));
  return (cptr<T>)w;
}

// Blocks are dispatched round-robin over the 8 XCDs, each with its own L2.
// Renumbering so that every XCD works on one contiguous range of blocks keeps
// the neighbour data that adjacent blocks share inside one L2.
__device__ inline int64_t xcd_block(int64_t bid, int64_t nb) {
  constexpr int kXcd = 8;
  const int64_t xcd = bid % kXcd, idx = bid / kXcd;
  const int64_t per = nb / kXcd, rem = nb % kXcd;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

// Blocks of a launch over (tile, field) pairs, nb in all: each XCD takes a
// contiguous range of pairs, fields fastest, so that the blocks of one
// tile's fields run together under one L2 and read the tile's edge or element
// tables from HBM once.
__device__ inline void tile_and_field(int64_t bid, int64_t nb, int nf, int64_t& tile, int& field) {
  const int64_t L = xcd_block(bid, nb);
  tile = L / nf;
  field = (int)(L - tile * nf);
}

// The operator pointer is wave-uniform; readfirstlane states that to the
// compiler also when the descriptor was read from memory (batched kernels).
template <typename P>
__device__ inline P* uniform_ptr(P* p) {
  return (P*)uniform_u64((uint64_t)p);
}

template <typename T> __device__ inline cptr<T> opbase(const DevMesh& m);
template <> __device__ inline cptr<double> opbase<double>(const DevMesh& m) {
  return (cptr<double>)uniform_ptr(m.ops64);
}
template <> __device__ inline cptr<float> opbase<float>(const DevMesh& m) {
  return (cptr<float>)uniform_ptr(m.ops32);
}

// The constant D of a field, for a wave-uniform field index: a scalar load
// of the device copy (the kernel-argument array, indexed at run time, would
// be read through a generic address, whose wait also holds every scalar load
// before it).
__device__ inline double field_D(const DevMesh& m, int field) {
  return ((cptr<double>)uniform_ptr(m.Dfield_dev))[__builtin_amdgcn_readfirstlane(field)];
}

// Affine map of a triangle (v1, v2, v3) onto the reference triangle: x_r =
// (v2 - v1) / 2, x_s = (v3 - v1) / 2, J = x_r y_s - x_s y_r, and the inverse
// metric r_x = y_s / J, r_y = -x_s / J, s_x = -y_r / J, s_y = x_r / J
// (section on the mapping of a triangle to the reference element).
struct ElemGeom {
  double xr, yr, xs, ys, iJ, rx, ry, sx, sy;
};

__device__ inline ElemGeom elem_geom(double2 p1, double2 p2, double2 p3) {
  ElemGeom g;
  g.xr = 0.5 * (p2.x - p1.x);
  g.yr = 0.5 * (p2.y - p1.y);
  g.xs = 0.5 * (p3.x - p1.x);
  g.ys = 0.5 * (p3.y - p1.y);
  g.iJ = 1.0 / (g.xr * g.ys - g.xs * g.yr);
  g.rx = g.ys * g.iJ;
  g.ry = -g.xs * g.iJ;
  g.sx = -g.yr * g.iJ;
  g.sy = g.xr * g.iJ;
  return g;
}

// Outward normal of face f times its surface factor sJ_f = |edge| / 2:
// (t_y, -t_x) / 2 for the counter-clockwise edge vector t (no square root).
__device__ inline double2 face_sjn(const ElemGeom& g, int f) {
  if (f == 0) return make_double2(g.yr, -g.xr);                   // t = v2 - v1 = 2 x_r
  if (f == 1) return make_double2(g.ys - g.yr, g.xr - g.xs);      // t = v3 - v2
  return make_double2(-g.ys, g.xs);                               // t = v1 - v3 = -2 x_s
}

// Affine velocity v = (c0 + c2 x + c3 y, c1 + c4 x + c5 y) on one element as
// a function of the reference coordinates: v = v1 + (r + 1) v_r + (s + 1) v_s.
struct ElemVel {
  double x1, y1, xr, yr, xs, ys;
};

__device__ inline ElemVel elem_vel(const double* c, double2 p1, const ElemGeom& g) {
  ElemVel v;
  v.x1 = c[0] + c[2] * p1.x + c[3] * p1.y;
  v.y1 = c[1] + c[4] * p1.x + c[5] * p1.y;
  v.xr = c[2] * g.xr + c[3] * g.yr;
  v.yr = c[4] * g.xr + c[5] * g.yr;
  v.xs = c[2] * g.xs + c[3] * g.ys;
  v.ys = c[4] * g.xs + c[5] * g.ys;
  return v;
}

// For N <= 4 the update operands are prefetched into registers before the
// compute, asking for two waves per SIMD; higher orders keep the registers
// for the element compute and load the operands in the update.
template <int N> struct ElemTune {
  static constexpr bool prefetch = N <= 4;
  static constexpr int waves = N <= 4 ? 2 : 1;
};

// The last stage of classic RK4, which reads the accumulator but not the
// state.
__device__ inline bool last_rk4(const Epilogue& epi) { return epi.kind == EPI_RK4 && epi.stage == 3; }

// One tile = TILE consecutive elements handled by NT threads.  Their nodal
// values form one contiguous chunk of the [F][K][Np] array: tile_begin stages
// it through LDS (sh, TileShape::LDS entries) with coalesced loads and fetches the
// operands of the Runge-Kutta update with the same coalesced pattern; the
// element compute replaces sh's values by du/dt; tile_end runs the update over
// the chunk's degrees of freedom with coalesced global traffic.  Each thread
// owns Q = ceil(TILE*Np/NT) of the chunk's entries, i = thread + q*NT.
template <int Q, typename T>
struct TileIO {
  T x[Q];                // the tile's stage input, in flight to LDS
  double Up[Q], Ap[Q];
  int nel, ndof;
  int64_t base;
  bool rk, need_acc;
};

template <int N, int TILE, int NT>
struct TileShape {
  static constexpr int Np = (N + 1) * (N + 2) / 2;
  static constexpr int Q = (TILE * Np + NT - 1) / NT;
  static constexpr int LDS = Q * NT;   // entries of the tile's LDS buffer (padded)
};

// Issues the global loads of a tile (stage input, and the update operands
// when prefetch is set) into registers.  Loads are issued unconditionally
// from clamped (in-tile) indices and masked afterwards: a load under a
// branch is followed by a wait at the branch's end, which would serialise
// the round trips.
template <int N, typename T, int TILE, int NT = TILE>
__device__ inline void tile_load(const DevMesh& m, int64_t k0, int field, const T* __restrict__ vin,
                                 const Epilogue& epi, TileIO<TileShape<N, TILE, NT>::Q, T>& io, bool prefetch) {
  constexpr int Np = TileShape<N, TILE, NT>::Np, Q = TileShape<N, TILE, NT>::Q;
  const int t = threadIdx.x;
  io.nel = (int)((m.K - k0) < TILE ? (m.K - k0) : TILE);
  io.ndof = io.nel * Np;
  io.base = ((int64_t)field * m.K + k0) * Np;
  io.rk = epi.kind != EPI_RHS;
  io.need_acc = io.rk && epi.stage != 0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int i = t + q * NT;
    io.x[q] = vin[io.base + (i < io.ndof ? i : 0)];
  }
  if (prefetch) {
    // without an update (right-hand side only) the operand loads read the
    // stage input's first value: no branch around them; the accumulator is
    // read (and used) from stage 1 on
    // (the last classic RK4 stage needs only the accumulator: its state
    // loads read the accumulator's addresses again, no second stream)
    const double* U = io.rk ? (last_rk4(epi) ? epi.acc : epi.u) + io.base : (const double*)vin;
    const double* A = io.need_acc ? epi.acc + io.base : U;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int i = t + q * NT;
      const int ic = (io.rk && i < io.ndof) ? i : 0;
      io.Up[q] = U[ic];
      io.Ap[q] = A[ic];
    }
  }
}

// Stores the loaded stage input into the tile's LDS buffer (TileShape::LDS
// entries): unconditionally, so that no branch asks for the loads' wait
// early; entries past the tile's degrees of freedom hold copies of its first
// value and are never read back as results.
template <int N, typename T, int TILE, int NT = TILE>
__device__ inline void tile_stage(T* sh, const TileIO<TileShape<N, TILE, NT>::Q, T>& io) {
  constexpr int Q = TileShape<N, TILE, NT>::Q;
#pragma unroll
  for (int q = 0; q < Q; ++q) sh[threadIdx.x + q * NT] = io.x[q];
}

// tile_load + tile_stage (sh: TileShape::LDS entries).
template <int N, typename T, int TILE, int NT = TILE>
__device__ inline void tile_begin(const DevMesh& m, int64_t k0, int field, const T* __restrict__ vin,
                                  const Epilogue& epi, T* sh, TileIO<TileShape<N, TILE, NT>::Q, T>& io,
                                  bool prefetch) {
  tile_load<N, T, TILE, NT>(m, k0, field, vin, epi, io, prefetch);
  tile_stage<N, T, TILE, NT>(sh, io);
}

template <int N, typename T, int TILE, int NT = TILE>
__device__ inline void tile_end(const Epilogue& epi, T* sh, TileIO<TileShape<N, TILE, NT>::Q, T>& io,
                                bool prefetched) {
  constexpr int Q = TileShape<N, TILE, NT>::Q;
  const int t = threadIdx.x;
  const int ndof = io.ndof;
  if (!io.rk) {
    T* o = (T*)epi.rhs_out + io.base;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int i = t + q * NT;
      if (i < ndof) o[i] = sh[i];
    }
    return;
  }
  double* U = epi.u + io.base;
  double* A = epi.acc + io.base;
  T* vn = epi.vnext ? (T*)epi.vnext + io.base : nullptr;
  const double dt = epi.dt;
  if (!prefetched) {
    const double* Usrc = last_rk4(epi) ? A : U;
    const double* Asrc = io.need_acc ? A : Usrc;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int i = t + q * NT;
      const int ic = i < ndof ? i : 0;
      io.Up[q] = Usrc[ic];
      io.Ap[q] = Asrc[ic];
    }
  }
  if (epi.kind == EPI_RK4) {
    // classic RK4 with the accumulator holding the new state as it forms:
    // A = u + dt/6 k1, A += dt/3 k2, A += dt/3 k3, u = A + dt/6 k4, and the
    // next stage input u + dt/2 k1, u + dt/2 k2, u + dt k3
    const int s = epi.stage;
    if (s < 3) {
      const double c = (s < 2) ? 0.5 * dt : dt;
      const double w = dt * ((s == 0) ? (1.0 / 6.0) : (1.0 / 3.0));
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int i = t + q * NT;
        if (i < ndof) {
          const double r = (double)sh[i];
          A[i] = ((s == 0) ? io.Up[q] : io.Ap[q]) + w * r;
          if (vn) vn[i] = (T)(io.Up[q] + c * r);
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int i = t + q * NT;
        if (i < ndof) {
          const double un = io.Ap[q] + dt * (1.0 / 6.0) * (double)sh[i];
          U[i] = un;
          if (vn) vn[i] = (T)un;
        }
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int i = t + q * NT;
      if (i < ndof) {
        const double r = dt * (double)sh[i];
        const double res = (epi.stage == 0) ? r : epi.a * io.Ap[q] + r;
        A[i] = res;
        const double un = io.Up[q] + epi.b * res;
        U[i] = un;
        if (vn) vn[i] = (T)un;
      }
    }
  }
}

}  // namespace ardg
