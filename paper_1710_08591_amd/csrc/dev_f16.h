// FP16 operand helpers for the matrix-core kernels (gfx950).
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

}  // namespace fftbf
