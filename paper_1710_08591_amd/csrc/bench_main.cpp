// fftbf_bench: the FP32 FFT beamformer through the C ABI alone (no Python),
// for timing and hardware-counter runs on a chosen lattice.
//
//   fftbf_bench [--n-ns N] [--n-chan C] [--n-pol P] [--n-time T] [--keep K]
//               [--precision 0|1|2] [--steps S] [--warmup W] [--random 0|1]
//   fftbf_bench --copy 1 [--steps S]
//   fftbf_bench --issue 1
//   fftbf_bench --mfma K      (K = 0, 1, 2: one MFMA form; 3: all three)
//   fftbf_bench --n-ns 16 --n-pol 1 --tied P   (tied beams from voltages, P pointings)
//
// Voltages are device-resident, filled with a fixed byte pattern (0x5A) or,
// with --random 1, with hashed bytes: the memory traffic and the instruction
// stream do not depend on the values, but the chip's power draw, and with it
// the clock it holds, does.  The N-S clamp keeps K beams per channel (every
// other beam, 0 = no clamp).
// Prints the average time per launch from HIP events on the launch stream.
// With --copy 1 it only copies 1 GiB between two device buffers with a plain
// streaming kernel (k_copy_calib), S times: the known byte count against
// which memory-traffic counters are calibrated.  With --issue 1 it measures
// the vector issue rate: 16 independent chains of one FP32 instruction form
// (v_fmac_f32, v_fma_f32 with three vector operands, v_add_f32) per lane, at
// 1, 2, 4 and 8 wavefronts per SIMD.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../include/fftbf.h"

namespace {

int arg_int(int argc, char** argv, const char* name, int dflt) {
  for (int i = 1; i + 1 < argc; ++i)
    if (!std::strcmp(argv[i], name)) return std::atoi(argv[i + 1]);
  return dflt;
}

bool ok_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return true;
  std::fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
  return false;
}

// bytes from a 32-bit integer hash of the dword index (deterministic)
__global__ void k_fill_hash(uint32_t* v, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    uint32_t x = (uint32_t)i * 0x9E3779B1u + 0x7F4A7C15u;
    x ^= x >> 16;
    x *= 0x85EBCA6Bu;
    x ^= x >> 13;
    x *= 0xC2B2AE35u;
    x ^= x >> 16;
    v[i] = x;
  }
}

// dst[i] = src[i], grid-stride over n 16-byte elements
__global__ void k_copy_calib(const float4* __restrict__ src, float4* __restrict__ dst, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

int copy_calibration(int steps) {
  const size_t bytes = (size_t)1 << 30;
  void *src = nullptr, *dst = nullptr;
  int rc = 1;
  if (!ok_hip(hipMalloc(&src, bytes), "hipMalloc src") || !ok_hip(hipMalloc(&dst, bytes), "hipMalloc dst")) goto done;
  if (!ok_hip(hipMemset(src, 0x3C, bytes), "hipMemset") || !ok_hip(hipDeviceSynchronize(), "hipMemset")) goto done;
  for (int i = 0; i < steps; ++i) {
    hipLaunchKernelGGL(k_copy_calib, dim3(8192), dim3(256), 0, 0, static_cast<const float4*>(src),
                       static_cast<float4*>(dst), bytes / sizeof(float4));
    if (!ok_hip(hipGetLastError(), "k_copy_calib")) goto done;
  }
  if (!ok_hip(hipDeviceSynchronize(), "k_copy_calib")) goto done;
  std::printf("fftbf_bench: copied %zu bytes per launch, %d launches\n", bytes, steps);
  rc = 0;
done:
  if (src) (void)hipFree(src);
  if (dst) (void)hipFree(dst);
  return rc;
}

constexpr int kIssueChains = 16;

// kind 0: a += x * y (v_fmac_f32); 1: a = a * y + z (v_fma_f32, three vector
// operands); 2: a = a + b (v_add_f32).  One store per thread.
template <int KIND>
__global__ __launch_bounds__(256) void k_issue(float* out, int iters) {
  float u[kIssueChains], v[kIssueChains], a[kIssueChains];
#pragma unroll
  for (int i = 0; i < kIssueChains; ++i) {
    u[i] = KIND == 1 ? 0.999f - threadIdx.x * 1e-7f : threadIdx.x * 1e-6f + i * 1e-3f;
    v[i] = KIND == 1 ? 1e-3f * i + threadIdx.x * 1e-7f : 0.5f + i * 1e-4f;
    a[i] = (float)i;
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < kIssueChains; ++i) {
      if constexpr (KIND == 0) a[i] = fmaf(u[i], v[i], a[i]);
      else if constexpr (KIND == 1) a[i] = fmaf(a[i], u[i], v[i]);
      else a[i] = a[i] + u[i];
    }
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < kIssueChains; ++i) s += a[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

int issue_probe() {
  const int threads = 256, iters = 20000, cus = 256;
  float* out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = 1;
  const char* names[3] = {"v_fmac_f32 (a += x y)", "v_fma_f32 (a = a y + z)", "v_add_f32 (a = a + b)"};
  if (!ok_hip(hipMalloc(&out, sizeof(float) * cus * 8 * threads), "hipMalloc out")) goto done;
  if (!ok_hip(hipEventCreate(&e0), "hipEventCreate") || !ok_hip(hipEventCreate(&e1), "hipEventCreate")) goto done;
  for (int kind = 0; kind < 3; ++kind)
    for (int wps = 1; wps <= 8; wps *= 2) {
      const int blocks = cus * wps;            // a block is 4 wavefronts, one per SIMD of a compute unit
      float best = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {
        if (!ok_hip(hipEventRecord(e0, 0), "hipEventRecord")) goto done;
        if (kind == 0) hipLaunchKernelGGL(k_issue<0>, dim3(blocks), dim3(threads), 0, 0, out, iters);
        if (kind == 1) hipLaunchKernelGGL(k_issue<1>, dim3(blocks), dim3(threads), 0, 0, out, iters);
        if (kind == 2) hipLaunchKernelGGL(k_issue<2>, dim3(blocks), dim3(threads), 0, 0, out, iters);
        if (!ok_hip(hipGetLastError(), "k_issue") || !ok_hip(hipEventRecord(e1, 0), "hipEventRecord") ||
            !ok_hip(hipEventSynchronize(e1), "hipEventSynchronize"))
          goto done;
        float ms = 0.f;
        if (!ok_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime")) goto done;
        if (ms < best) best = ms;
      }
      const double wave_instr = (double)blocks * (threads / 64) * iters * kIssueChains;
      std::printf("fftbf_bench: %-26s %d wavefronts per SIMD: %.3f ms, %.3f wavefront-instructions per SIMD "
                  "and cycle at 2.4 GHz\n", names[kind], wps, best, wave_instr / (best * 1e-3) / (cus * 4) / 2.4e9);
    }
  rc = 0;
done:
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (out) (void)hipFree(out);
  return rc;
}

// Matrix-core issue probe: each wavefront runs kMfmaChains independent
// accumulator chains of one MFMA form, `iters` times, so a launch issues a
// known number of MFMA instructions (blocks x 4 wavefronts x iters x chains):
// the rate per SIMD and the reading of SQ_INSTS_MFMA can both be checked
// against it.  kind 0: v_mfma_f32_16x16x32_f16; 1: v_mfma_f32_16x16x32_fp8_fp8;
// 2: v_mfma_scale_f32_16x16x128_f8f6f4 (FP8 e4m3 operands, unit block scales).
constexpr int kMfmaChains = 4;
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef int i32x8_t __attribute__((ext_vector_type(8)));

template <int KIND>
__global__ __launch_bounds__(256) void k_mfma_issue(float* out, int iters) {
  f32x4_t c[kMfmaChains];
#pragma unroll
  for (int i = 0; i < kMfmaChains; ++i) c[i] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  const int t = (int)threadIdx.x;
  half8_t ha, hb;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    ha[j] = (_Float16)(1e-3f * (float)((t + j) & 7));
    hb[j] = (_Float16)(1e-3f * (float)((t * 3 + j) & 7));
  }
  const long la = 0x3830282018100800L + t, lb = 0x0810182028303840L - t;   // small e4m3 values
  i32x8_t wa, wb;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    wa[j] = (int)(la >> (4 * (j & 1))) & 0x3F3F3F3F;
    wb[j] = (int)(lb >> (4 * (j & 1))) & 0x3F3F3F3F;
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < kMfmaChains; ++i) {
      if constexpr (KIND == 0) c[i] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ha, hb, c[i], 0, 0, 0);
      else if constexpr (KIND == 1) c[i] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(la, lb, c[i], 0, 0, 0);
      else c[i] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(wa, wb, c[i], 0, 0, 0, 0x7F7F7F7F, 0, 0x7F7F7F7F);
    }
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < kMfmaChains; ++i) s += c[i][0] + c[i][1] + c[i][2] + c[i][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

int mfma_probe(int only_kind) {
  const int threads = 256, iters = 4000, cus = 256;
  float* out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = 1;
  const char* names[3] = {"v_mfma_f32_16x16x32_f16", "v_mfma_f32_16x16x32_fp8_fp8",
                          "v_mfma_scale_f32_16x16x128_f8f6f4"};
  const double flop[3] = {16.0 * 16 * 32 * 2, 16.0 * 16 * 32 * 2, 16.0 * 16 * 128 * 2};
  if (!ok_hip(hipMalloc(&out, sizeof(float) * cus * 8 * threads), "hipMalloc out")) goto done;
  if (!ok_hip(hipEventCreate(&e0), "hipEventCreate") || !ok_hip(hipEventCreate(&e1), "hipEventCreate")) goto done;
  for (int kind = 0; kind < 3; ++kind) {
    if (only_kind >= 0 && kind != only_kind) continue;
    for (int wps = 1; wps <= 4; wps *= 2) {
      const int blocks = cus * wps;            // a block is 4 wavefronts, one per SIMD of a compute unit
      float best = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {
        if (!ok_hip(hipEventRecord(e0, 0), "hipEventRecord")) goto done;
        if (kind == 0) hipLaunchKernelGGL(k_mfma_issue<0>, dim3(blocks), dim3(threads), 0, 0, out, iters);
        if (kind == 1) hipLaunchKernelGGL(k_mfma_issue<1>, dim3(blocks), dim3(threads), 0, 0, out, iters);
        if (kind == 2) hipLaunchKernelGGL(k_mfma_issue<2>, dim3(blocks), dim3(threads), 0, 0, out, iters);
        if (!ok_hip(hipGetLastError(), "k_mfma_issue") || !ok_hip(hipEventRecord(e1, 0), "hipEventRecord") ||
            !ok_hip(hipEventSynchronize(e1), "hipEventSynchronize"))
          goto done;
        float ms = 0.f;
        if (!ok_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime")) goto done;
        if (ms < best) best = ms;
      }
      const double instr = (double)blocks * (threads / 64) * iters * kMfmaChains;
      const double per_simd_cycle = instr / (best * 1e-3) / (cus * 4) / 2.4e9;
      std::printf("fftbf_bench: %-34s %d wavefronts per SIMD: %.3f ms, %.0f MFMA per launch, %.4f per SIMD and "
                  "cycle at 2.4 GHz (%.1f cycles each), %.1f TFLOP/s\n", names[kind], wps, best, instr,
                  per_simd_cycle, 1.0 / per_simd_cycle, instr * flop[kind] / (best * 1e-3) / 1e12);
    }
  }
  rc = 0;
done:
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (out) (void)hipFree(out);
  return rc;
}

bool ok_bf(bf_status s, const char* what) {
  if (s == BF_OK) return true;
  std::fprintf(stderr, "%s: %s: %s\n", what, bf_status_string(s), bf_last_error());
  return false;
}

}  // namespace

int main(int argc, char** argv) {
  const int n_ns = arg_int(argc, argv, "--n-ns", 256);
  const int n_chan = arg_int(argc, argv, "--n-chan", 256);
  const int n_pol = arg_int(argc, argv, "--n-pol", 2);
  const int n_time = arg_int(argc, argv, "--n-time", 16384);
  const int keep = arg_int(argc, argv, "--keep", n_ns);
  const int steps = arg_int(argc, argv, "--steps", 10);
  const int warmup = arg_int(argc, argv, "--warmup", 2);
  const int precision = arg_int(argc, argv, "--precision", BF_PREC_FP32);
  const int random = arg_int(argc, argv, "--random", 0);
  const int copy = arg_int(argc, argv, "--copy", 0);
  const int issue = arg_int(argc, argv, "--issue", 0);
  const int mfma = arg_int(argc, argv, "--mfma", -1);
  const int tied = arg_int(argc, argv, "--tied", 0);
  if (n_ns <= 0 || n_chan <= 0 || n_pol <= 0 || n_time <= 0 || keep < 0 || keep > 2 * n_ns || steps <= 0 ||
      warmup < 0 || (random != 0 && random != 1) || (copy != 0 && copy != 1) ||
      (issue != 0 && issue != 1) || tied < 0 || tied > 4096) {
    std::fprintf(stderr, "invalid arguments\n");
    return 2;
  }
  if (copy) return copy_calibration(steps);
  if (issue) return issue_probe();
  if (mfma >= 0) return mfma_probe(mfma <= 2 ? mfma : -1);

  std::vector<int32_t> sel;
  bf_plan_desc d{};
  d.n_ew = 4;
  d.n_ns = n_ns;
  d.m_ew = 4;
  d.m_ns = 2 * n_ns;
  d.n_pol = n_pol;
  d.n_chan = n_chan;
  d.block = 16;
  d.precision = (bf_precision)precision;
  if (keep && keep < 2 * n_ns) {
    sel.resize((size_t)n_chan * keep);
    for (size_t i = 0; i < sel.size(); ++i) sel[i] = (int32_t)(2 * (i % keep));
    d.n_ns_keep = keep;
    d.ns_select = sel.data();
  }
  bf_plan* plan = nullptr;
  if (!ok_bf(bf_plan_create(&d, &plan), "bf_plan_create")) return 1;
  const int kept = d.n_ns_keep ? d.n_ns_keep : d.m_ns;

  const size_t in_bytes = (size_t)n_time * n_chan * n_pol * n_ns * 4;
  const size_t out_bytes = tied ? (size_t)(n_time / 16) * n_chan * n_pol * tied * sizeof(float)
                                : (size_t)(n_time / 16) * n_chan * n_pol * 4 * kept * sizeof(float);
  std::vector<double> dirs((size_t)2 * (tied ? tied : 1));
  for (int p = 0; p < tied; ++p) {          // a spread of directions inside the field of view
    dirs[2 * p] = -0.8 + 1.6 * ((p * 37) % 97) / 96.0;
    dirs[2 * p + 1] = -0.8 + 1.6 * ((p * 61) % 89) / 88.0;
  }
  void *volts = nullptr, *out = nullptr, *dircos = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = 1;
  float ms = 0.f;
  if (!ok_hip(hipMalloc(&volts, in_bytes), "hipMalloc volts")) goto done;
  if (!ok_hip(hipMalloc(&out, out_bytes), "hipMalloc out")) goto done;
  if (random) {
    hipLaunchKernelGGL(k_fill_hash, dim3(4096), dim3(256), 0, 0, static_cast<uint32_t*>(volts), in_bytes / 4);
    if (!ok_hip(hipGetLastError(), "k_fill_hash") || !ok_hip(hipDeviceSynchronize(), "k_fill_hash")) goto done;
  } else if (!ok_hip(hipMemset(volts, 0x5A, in_bytes), "hipMemset")) {
    goto done;
  }
  if (!ok_hip(hipStreamCreate(&s), "hipStreamCreate")) goto done;
  if (!ok_hip(hipEventCreate(&e0), "hipEventCreate") || !ok_hip(hipEventCreate(&e1), "hipEventCreate")) goto done;
  if (tied) {
    if (!ok_hip(hipMalloc(&dircos, dirs.size() * sizeof(double)), "hipMalloc dircos") ||
        !ok_hip(hipMemcpy(dircos, dirs.data(), dirs.size() * sizeof(double), hipMemcpyHostToDevice), "hipMemcpy"))
      goto done;
    for (int i = 0; i < warmup + steps; ++i) {
      if (i == warmup && !ok_hip(hipEventRecord(e0, s), "hipEventRecord")) goto done;
      if (!ok_bf(bf_form_tied_beams_v(plan, static_cast<uint8_t*>(volts), n_time, nullptr, 0, n_chan,
                                      static_cast<double*>(dircos), tied, out, s),
                 "bf_form_tied_beams_v"))
        goto done;
    }
    if (!ok_hip(hipEventRecord(e1, s), "hipEventRecord") || !ok_hip(hipEventSynchronize(e1), "hipEventSynchronize") ||
        !ok_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime"))
      goto done;
    std::printf("fftbf_bench: tied beams from voltages, 4x%d lattice, %d chan, %d pol, %d samples, %d pointings: "
                "%.4f ms per launch, %.4g beam-samples/s (%s voltages)\n",
                n_ns, n_chan, n_pol, n_time, tied, ms / steps,
                (double)n_time * n_chan * n_pol * tied / (ms / steps * 1e-3), random ? "hashed" : "constant");
    rc = 0;
    goto done;
  }
  for (int i = 0; i < warmup; ++i)
    if (!ok_bf(bf_beamform_fft(plan, static_cast<uint8_t*>(volts), n_time, nullptr, BF_OUT_INTENSITY, out, s),
               "bf_beamform_fft"))
      goto done;
  if (!ok_hip(hipEventRecord(e0, s), "hipEventRecord")) goto done;
  for (int i = 0; i < steps; ++i)
    if (!ok_bf(bf_beamform_fft(plan, static_cast<uint8_t*>(volts), n_time, nullptr, BF_OUT_INTENSITY, out, s),
               "bf_beamform_fft"))
      goto done;
  if (!ok_hip(hipEventRecord(e1, s), "hipEventRecord") || !ok_hip(hipEventSynchronize(e1), "hipEventSynchronize"))
    goto done;
  if (!ok_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime")) goto done;
  std::printf("fftbf_bench: 4x%d lattice, %d chan, %d pol, %d samples, %d N-S beams kept, precision %d: "
              "%.4f ms per launch, %.4g antenna-samples/s (%s voltages)\n",
              n_ns, n_chan, n_pol, n_time, kept, precision, ms / steps,
              (double)n_time * n_chan * n_pol * 4 * n_ns / (ms / steps * 1e-3), random ? "hashed" : "constant");
  rc = 0;
done:
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  if (out) (void)hipFree(out);
  if (dircos) (void)hipFree(dircos);
  if (volts) (void)hipFree(volts);
  bf_plan_destroy(plan);
  return rc;
}
