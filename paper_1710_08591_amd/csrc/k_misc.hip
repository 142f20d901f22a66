// Table generation in FP64 on the device, and the standalone intensity
// accumulator.
#include "dev_common.h"
#include "kernels.h"

namespace fftbf {

namespace {

// tw[a1][k2] = W_M^{a1 k2} = exp(-i 2 pi (a1 k2 mod M) / M): the index is
// reduced in integers, the phase evaluated in FP64, then rounded to FP32.
__global__ void k_twiddle(float2* tw, int g, int l2, int m) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g * l2) return;
  const int a1 = i / l2, k2 = i % l2;
  const long r = ((long)a1 * k2) % m;
  double s, c;
  sincospi(-2.0 * (double)r / (double)m, &s, &c);
  tw[i] = make_float2((float)c, (float)s);
}

// out[b][s] (+)= sum_{t in block b} |z[t][s]|^2 -- the block sum of the
// squared voltage beams (eq. e:bf).  One thread per output, consecutive
// threads on consecutive series so every load instruction is coalesced.
__global__ __launch_bounds__(256) void k_accumulate(const float2* __restrict__ z, int64_t n_series,
                                                   int64_t n_out, int block, int add,
                                                   float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_out) return;
  const int64_t b = i / n_series, s = i - b * n_series;
  typedef float v2f __attribute__((ext_vector_type(2)));
  const v2f* p = reinterpret_cast<const v2f*>(z) + b * block * n_series + s;
  float acc0 = 0.f, acc1 = 0.f;
  int t = 0;
  for (; t + 1 < block; t += 2) {
    const v2f u = __builtin_nontemporal_load(p + (int64_t)t * n_series);
    const v2f v = __builtin_nontemporal_load(p + (int64_t)(t + 1) * n_series);
    acc0 = fmaf(u.x, u.x, fmaf(u.y, u.y, acc0));
    acc1 = fmaf(v.x, v.x, fmaf(v.y, v.y, acc1));
  }
  if (t < block) {
    const v2f u = p[(int64_t)t * n_series];
    acc0 = fmaf(u.x, u.x, fmaf(u.y, u.y, acc0));
  }
  const float r = acc0 + acc1;
  out[i] = add ? out[i] + r : r;
}

}  // namespace

hipError_t launch_twiddle_table(float2* tw, int g, int l2, int m, hipStream_t s) {
  const int n = g * l2;
  hipLaunchKernelGGL(k_twiddle, dim3((n + 255) / 256), dim3(256), 0, s, tw, g, l2, m);
  return hipGetLastError();
}

hipError_t launch_accumulate(const float2* z, int64_t n_time, int64_t n_series, int block,
                             int add, float* out, hipStream_t s) {
  const int64_t n_out = (n_time / block) * n_series;
  if (n_out == 0) return hipSuccess;
  const int64_t n_wg = (n_out + 255) / 256;
  hipLaunchKernelGGL(k_accumulate, dim3((unsigned)n_wg), dim3(256), 0, s, z, n_series, n_out,
                     block, add, out);
  return hipGetLastError();
}

}  // namespace fftbf
