// Matrix-core (MFMA) wrappers of gfx950 for the three precisions of the
// library, behind one interface so that the kernels are written once:
//   Mma<double>  v_mfma_f64_16x16x4_f64   (FP64 data, FP64 accumulation)
//   Mma<float>   v_mfma_f32_16x16x4_f32   (FP32 data, FP32 accumulation)
//   Mma<Bf16x3>  v_mfma_f32_16x16x16_bf16 (FP32 data, each operand split into
//                hi = bf16(x) and lo = bf16(x - hi); a product is the sum
//                hi*hi + hi*lo + lo*hi accumulated in FP32, which keeps about
//                16 significant bits of every operand)
//
// Fragment layouts (16 x 16 result, K = KSTEP per instruction, KPL = KSTEP / 4
// values per lane): lane l supplies A[row = l % 16][k] and B[k][col = l % 16]
// for k = KPL (l / 16) + t, t < KPL.  The result sits in four registers per
// lane with column l % 16; the row of register r is 4 (l / 16) + r for the
// FP32-accumulating instructions and 4 r + l / 16 for the FP64 one.  row()
// gives that row; grp_of() and reg_of() invert it (lane group l / 16 and
// register that receive a given row).  kidx(c, grp, t) is the k index that
// lane group grp supplies as its t-th value in K step c.
#pragma once

#include <hip/hip_runtime.h>

namespace ardg {

typedef double mf_d4 __attribute__((ext_vector_type(4)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));
typedef short mf_s4 __attribute__((ext_vector_type(4)));

struct Bf16x3 {};   // precision tag: FP32 data, split-BF16 products

template <typename P> struct Mma;

template <> struct Mma<double> {
  typedef double T;              // data type
  typedef double frag;
  typedef mf_d4 acc;
  static constexpr int KPL = 1, KSTEP = 4;
  __device__ static acc zero() {
    acc z = {0.0, 0.0, 0.0, 0.0};
    return z;
  }
  __device__ static frag make(const T* v) { return v[0]; }
  __device__ static acc mma(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static constexpr int row(int grp, int r) { return 4 * r + grp; }
  __device__ static constexpr int grp_of(int row) { return row & 3; }
  __device__ static constexpr int reg_of(int row) { return row >> 2; }
};

template <> struct Mma<float> {
  typedef float T;
  typedef float frag;
  typedef mf_f4 acc;
  static constexpr int KPL = 1, KSTEP = 4;
  __device__ static acc zero() {
    acc z = {0.f, 0.f, 0.f, 0.f};
    return z;
  }
  __device__ static frag make(const T* v) { return v[0]; }
  __device__ static acc mma(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static constexpr int row(int grp, int r) { return 4 * grp + r; }
  __device__ static constexpr int grp_of(int row) { return row >> 2; }
  __device__ static constexpr int reg_of(int row) { return row & 3; }
};

// bfloat16 bits of x, rounded to nearest even (finite x)
__device__ inline short bf16_bits(float x) {
  const __bf16 h = (__bf16)x;
  return __builtin_bit_cast(short, h);
}
__device__ inline float bf16_value(short b) {
  return __builtin_bit_cast(float, (unsigned)(unsigned short)b << 16);
}

template <> struct Mma<Bf16x3> {
  typedef float T;
  struct frag {
    mf_s4 hi, lo;
  };
  typedef mf_f4 acc;
  static constexpr int KPL = 4, KSTEP = 16;
  __device__ static acc zero() {
    acc z = {0.f, 0.f, 0.f, 0.f};
    return z;
  }
  __device__ static frag make(const T* v) {
    frag f;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const short h = bf16_bits(v[t]);
      f.hi[t] = h;
      f.lo[t] = bf16_bits(v[t] - bf16_value(h));
    }
    return f;
  }
  __device__ static acc mma(const frag& a, const frag& b, acc c) {
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.lo, b.hi, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.hi, b.lo, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.hi, b.hi, c, 0, 0, 0);
  }
  __device__ static constexpr int row(int grp, int r) { return 4 * grp + r; }
  __device__ static constexpr int grp_of(int row) { return row >> 2; }
  __device__ static constexpr int reg_of(int row) { return row & 3; }
};

template <typename M>
__device__ constexpr int kidx(int c, int grp, int t) {
  return M::KSTEP * c + M::KPL * grp + t;
}

}  // namespace ardg
