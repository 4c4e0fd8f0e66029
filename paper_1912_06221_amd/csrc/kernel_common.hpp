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

// For N <= 4 the update operands are prefetched into registers before the
// compute, asking for two waves per SIMD; higher orders keep the registers
// for the element compute and load the operands in the update.
template <int N> struct ElemTune {
  static constexpr bool prefetch = N <= 4;
  static constexpr int waves = N <= 4 ? 2 : 1;
};

// One tile = TILE consecutive elements handled by TILE threads.  Their nodal
// values form one contiguous chunk of the [F][K][Np] array: tile_begin stages
// it through LDS (sh, TILE*Np entries) with coalesced loads and fetches the
// operands of the Runge-Kutta update with the same coalesced pattern; the
// element compute replaces sh's values by du/dt; tile_end runs the update over
// the chunk's degrees of freedom with coalesced global traffic.
template <int Np>
struct TileIO {
  double Up[Np], Ap[Np];
  int nel, ndof;
  int64_t base;
  bool rk, need_acc;
};

template <int N, typename T, int TILE>
__device__ inline void tile_begin(const DevMesh& m, int64_t k0, int field, const T* __restrict__ vin,
                                  const Epilogue& epi, T* sh, TileIO<(N + 1) * (N + 2) / 2>& io,
                                  bool prefetch) {
  constexpr int Np = (N + 1) * (N + 2) / 2;
  const int t = threadIdx.x;
  io.nel = (int)((m.K - k0) < TILE ? (m.K - k0) : TILE);
  io.ndof = io.nel * Np;
  io.base = ((int64_t)field * m.K + k0) * Np;
#pragma unroll
  for (int q = 0; q < Np; ++q) {
    const int i = t + q * TILE;
    if (i < io.ndof) sh[i] = vin[io.base + i];
  }
  io.rk = epi.kind != EPI_RHS;
  io.need_acc = io.rk && epi.stage != 0;
  if (prefetch && io.rk) {
    const double* U = epi.u + io.base;
    const double* A = epi.acc + io.base;
#pragma unroll
    for (int q = 0; q < Np; ++q) {
      const int i = t + q * TILE;
      io.Up[q] = (i < io.ndof) ? U[i] : 0.0;
      io.Ap[q] = (io.need_acc && i < io.ndof) ? A[i] : 0.0;
    }
  }
}

template <int N, typename T, int TILE>
__device__ inline void tile_end(const Epilogue& epi, const T* sh, TileIO<(N + 1) * (N + 2) / 2>& io,
                                bool prefetched) {
  constexpr int Np = (N + 1) * (N + 2) / 2;
  const int t = threadIdx.x;
  const int ndof = io.ndof;
  if (!io.rk) {
    T* o = (T*)epi.rhs_out + io.base;
#pragma unroll
    for (int q = 0; q < Np; ++q) {
      const int i = t + q * TILE;
      if (i < ndof) o[i] = sh[i];
    }
    return;
  }
  double* U = epi.u + io.base;
  double* A = epi.acc + io.base;
  T* vn = epi.vnext ? (T*)epi.vnext + io.base : nullptr;
  const double dt = epi.dt;
  if (!prefetched) {
#pragma unroll
    for (int q = 0; q < Np; ++q) {
      const int i = t + q * TILE;
      io.Up[q] = (i < ndof) ? U[i] : 0.0;
      io.Ap[q] = (io.need_acc && i < ndof) ? A[i] : 0.0;
    }
  }
  if (epi.kind == EPI_RK4) {
    const int s = epi.stage;
    if (s < 3) {
      const double c = (s < 2) ? 0.5 * dt : dt;
#pragma unroll
      for (int q = 0; q < Np; ++q) {
        const int i = t + q * TILE;
        if (i < ndof) {
          const double r = (double)sh[i];
          A[i] = (s == 0) ? r : io.Ap[q] + 2.0 * r;
          vn[i] = (T)(io.Up[q] + c * r);
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < Np; ++q) {
        const int i = t + q * TILE;
        if (i < ndof) {
          const double un = io.Up[q] + dt / 6.0 * (io.Ap[q] + (double)sh[i]);
          U[i] = un;
          if (vn) vn[i] = (T)un;
        }
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < Np; ++q) {
      const int i = t + q * TILE;
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
