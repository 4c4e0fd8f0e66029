// Matrix-core (MFMA) wrappers for the 16x16x4 FP64 and FP32 instructions of
// gfx950.
//
// Fragment layouts of the 16x16xK instructions used here (K per instruction
// = 4, one value per lane): lane l supplies A[row = l % 16][k = l / 16] and
// B[k = l / 16][col = l % 16].  The 16x16 result sits in four registers per
// lane with column l % 16; the row of register r differs by instruction:
// 4 (l / 16) + r for the FP32 one and 4 r + l / 16 for the FP64 one.  row()
// gives that row; grp_of() and reg_of() invert it (lane group l / 16 and
// register that receive a given row).
#pragma once

#include <hip/hip_runtime.h>

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
  __device__ static constexpr int grp_of(int row) { return row & 3; }
  __device__ static constexpr int reg_of(int row) { return row >> 2; }
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
  __device__ static constexpr int grp_of(int row) { return row >> 2; }
  __device__ static constexpr int reg_of(int row) { return row & 3; }
};

}  // namespace ardg
