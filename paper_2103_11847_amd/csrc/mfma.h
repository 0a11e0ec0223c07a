// MFMA 16x16 instruction traits for gfx950 (shared by the GEMM kernels).
#pragma once

#include "internal.h"

namespace dctk {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// MFMA per input type: KSTEP = contraction length of one instruction,
// EPL = elements of A (and of B) each lane supplies.
template <typename TI> struct Mfma;
// ROWS_STRIDED: output register r of lane l holds row (l/16) + 4 r (FP64)
// instead of 4 (l/16) + r (FP32 / BF16 / FP16), column l % 16 in both.
template <> struct Mfma<double> {
  static constexpr int KSTEP = 4, EPL = 1;
  static constexpr bool ROWS_STRIDED = true;
  typedef double acc_t;
  typedef f64x4 frag_t;
  __device__ static frag_t mac(const double* a, const double* b, frag_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], b[0], c, 0, 0, 0);
  }
};
template <> struct Mfma<float> {
  static constexpr bool ROWS_STRIDED = false;
  static constexpr int KSTEP = 4, EPL = 1;
  typedef float acc_t;
  typedef f32x4 frag_t;
  __device__ static frag_t mac(const float* a, const float* b, frag_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], c, 0, 0, 0);
  }
};
template <> struct Mfma<bf16_t> {
  static constexpr bool ROWS_STRIDED = false;
  static constexpr int KSTEP = 32, EPL = 8;
  typedef float acc_t;
  typedef f32x4 frag_t;
  __device__ static frag_t mac(const bf16_t* a, const bf16_t* b, frag_t c) {
    bf16x8 av = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(a));
    bf16x8 bv = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(b));
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
  }
};
template <> struct Mfma<f16_t> {
  static constexpr bool ROWS_STRIDED = false;
  static constexpr int KSTEP = 32, EPL = 8;
  typedef float acc_t;
  typedef f32x4 frag_t;
  __device__ static frag_t mac(const f16_t* a, const f16_t* b, frag_t c) {
    f16x8 av = __builtin_bit_cast(f16x8, *reinterpret_cast<const uint4*>(a));
    f16x8 bv = __builtin_bit_cast(f16x8, *reinterpret_cast<const uint4*>(b));
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(av, bv, c, 0, 0, 0);
  }
};

// 16-byte (or scalar) global/LDS accesses of VW consecutive elements
template <typename T, int VW> struct VecIO;
template <typename T> struct VecIO<T, 1> {
  __device__ static void ld(const T* p, T* v) { v[0] = p[0]; }
  __device__ static void st(T* p, const T* v) { p[0] = v[0]; }
};
template <> struct VecIO<float, 4> {
  __device__ static void ld(const float* p, float* v) {
    const float4 q = *reinterpret_cast<const float4*>(p);
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
  }
  __device__ static void st(float* p, const float* v) {
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
  }
};
template <> struct VecIO<double, 2> {
  __device__ static void ld(const double* p, double* v) {
    const double2 q = *reinterpret_cast<const double2*>(p);
    v[0] = q.x; v[1] = q.y;
  }
  __device__ static void st(double* p, const double* v) {
    *reinterpret_cast<double2*>(p) = make_double2(v[0], v[1]);
  }
};

template <typename TO, typename TA> __device__ inline TO out_cvt(TA v) { return (TO)v; }
template <> __device__ inline bf16_t out_cvt<bf16_t, float>(float v) { return float_to_bf16(v); }

}  // namespace dctk
