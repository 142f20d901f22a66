// Table generation in FP64 on the device, and the standalone intensity
// accumulator.
#include "dev_common.h"
#include "kernels.h"

namespace fftbf {

namespace {

// W_M^{a1 k2} = exp(-i 2 pi (a1 k2 mod M) / M): the index is reduced in
// integers, the phase evaluated in FP64.
__device__ void twiddle64(int a1, int k2, int m, double& c, double& s) {
  const long r = ((long)a1 * k2) % m;
  sincospi(-2.0 * (double)r / (double)m, &s, &c);
}

// The factor that the tangent form of pass-1 twiddle (a1, k2) leaves on its
// value: Re W, or 1 where the column keeps whole twiddles (and for k2 = 0).
__device__ double pass1_scale(int a1, int k2, int g, int m) {
  if (k2 == 0 || cmul_col(k2, g, m)) return 1.0;
  double c, s;
  twiddle64(a1, k2, m, c, s);
  return c;
}

// Pass-1 table tw[a1][k2]: (t, 0) with W = Re W (1 + i t), or the whole
// twiddle (Re W, Im W) in the columns that keep it.  Pass-2 table
// mult[k2][slot]: the multipliers of the scaled G-point DIT over a1 whose
// input a1 carries pass1_scale(a1, k2).  FP64 throughout, rounded to FP32.
__global__ void k_twiddle(float2* tw, float* mult, int g, int l2, int m) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < g * l2) {
    const int a1 = i / l2, k2 = i % l2;
    double c, s;
    twiddle64(a1, k2, m, c, s);
    tw[i] = cmul_col(k2, g, m) ? make_float2((float)c, (float)s) : make_float2((float)(s / c), 0.f);
  }
  const int ns = dit_slots(g);
  if (i < l2 * ns) {
    const int k2 = i / ns, slot = i % ns;
    for (int size = 2; size <= g; size *= 2)
      for (int s0 = 0; s0 < g; s0 += size)
        for (int j = 0; j < size / 2; ++j) {
          if (dit_slot(g, size, s0, j) != slot) continue;
          double mu = pass1_scale(bitrev(s0 + size / 2, g), k2, g, m) / pass1_scale(bitrev(s0, g), k2, g, m);
          // the butterfly's own twiddle factor, from the same definition as its tangent
          if (!dit_trivial(j, size)) mu *= tan_outer(j, size);
          mult[i] = (float)mu;
        }
  }
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
  // eight samples' loads in flight at once; even samples go to acc0, odd to
  // acc1, in the same order as the pairwise loop below
  for (; t + 8 <= block; t += 8) {
    v2f u[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) u[q] = __builtin_nontemporal_load(p + (int64_t)(t + q) * n_series);
#pragma unroll
    for (int q = 0; q < 8; q += 2) {
      acc0 = fmaf(u[q].x, u[q].x, fmaf(u[q].y, u[q].y, acc0));
      acc1 = fmaf(u[q + 1].x, u[q + 1].x, fmaf(u[q + 1].y, u[q + 1].y, acc1));
    }
  }
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

int twiddle_mult_count(int g, int l2) { return l2 * dit_slots(g); }

hipError_t launch_twiddle_table(float2* tw, float* mult, int g, int l2, int m, hipStream_t s) {
  const int n = g * l2 > l2 * dit_slots(g) ? g * l2 : l2 * dit_slots(g);
  hipLaunchKernelGGL(k_twiddle, dim3((n + 255) / 256), dim3(256), 0, s, tw, mult, g, l2, m);
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
