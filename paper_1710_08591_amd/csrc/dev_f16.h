// FP16 and FP8 (e4m3) operand helpers for the matrix-core kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fftbf {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half2 __attribute__((ext_vector_type(2)));

// Signed 4-bit dot product of eight nibble pairs, added to the integer c.
__device__ __forceinline__ int sdot8_acc(int a, int b, int c) {
  int r;
  asm("v_dot8_i32_i4 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

// Two floats into FP16 high and low terms: hi = fp16(v) (round to nearest
// even), lo = fp16(v - hi); the residual v - hi is exact in FP32 and comes
// from one mixed-precision fused multiply-add per value.
__device__ __forceinline__ void split2(float v0, float v1, uint32_t& hi, uint32_t& lo) {
  uint32_t h;
  float r0, r1;
  asm("v_cvt_pk_f16_f32 %0, %1, %2" : "=v"(h) : "v"(v0), "v"(v1));
  asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(r0) : "v"(h), "v"(v0));
  asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r1) : "v"(h), "v"(v1));
  asm("v_cvt_pk_f16_f32 %0, %1, %2" : "=v"(lo) : "v"(r0), "v"(r1));
  hi = h;
}

// FP8 coefficient terms: W = hi + 2^-5 lo1 + 2^-9 lo2, each term stored
// times 2^+s so it sits in the normal range of e4m3; the matching data
// operand carries 2^-s (exact for the int4 voltages, |x| <= 8).
__host__ __device__ constexpr int fp8_shift(int p) { return p == 0 ? 0 : (p == 1 ? 5 : 9); }

__device__ __forceinline__ float fp8_to_f32(int byte) { return __builtin_amdgcn_cvt_f32_fp8(byte, 0); }
__device__ __forceinline__ int f32_to_fp8(float v) { return __builtin_amdgcn_cvt_pk_fp8_f32(v, 0.f, 0, false) & 0xFF; }

// dot8 weights (Re, Im) of the first-stage E-W sums: column 0 x0 + x2,
// 1 x1 + x3, 2 x0 - x2, 3 x1 - x3
__device__ __forceinline__ void ew_half_weights(int col, int& wre, int& wim) {
  const int sgn = col < 2 ? 1 : 0xF;
  const int q0 = col & 1, q1 = q0 + 2;
  wre = (1 << (8 * q0 + 4)) | (sgn << (8 * q1 + 4));
  wim = (1 << (8 * q0)) | (sgn << (8 * q1));
}

typedef short short2v __attribute__((ext_vector_type(2)));

// eight small integers times a power-of-two scale as e4m3 bytes (exact for
// the int4 voltages, their first-stage E-W sums and the scales of fp8_shift),
// byte j = v[j].  gfx950's scaled conversion takes two values per
// instruction and applies the scale itself: it divides by the power of two
// in its scale operand, so 1/scale is passed.  The integer-to-float
// conversions are shared by every term of the same values.
__device__ __forceinline__ long to_fp8(const int* v, float scale) {
  const float div = 1.0f / scale;
  short2v w0 = {0, 0}, w1 = {0, 0};
  w0 = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(w0, (float)v[0], (float)v[1], div, false);
  w0 = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(w0, (float)v[2], (float)v[3], div, true);
  w1 = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(w1, (float)v[4], (float)v[5], div, false);
  w1 = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(w1, (float)v[6], (float)v[7], div, true);
  return (long)(unsigned)__builtin_bit_cast(int, w0) | ((long)(unsigned)__builtin_bit_cast(int, w1) << 32);
}

}  // namespace fftbf
