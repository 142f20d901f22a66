// Intensity-domain regridding of FFT beams to arbitrary steering angles
// (eq. e:bp_max_arbitrary, Sec. "Redundancy-stacked visibilities"):
//
//   b_p(theta) = sum_A w^A_p b_A,  w^A_p = (1/M) sin((2n-1) pi y) / sin(pi y),
//   y = (d/lambda) sin(theta) - A/M,
//
// exact whenever M >= 2n - 1, which the zero-padded N-S axis (M = 2n)
// satisfies.  Applied per channel along N-S for every E-W FFT beam, so the
// targets can be the same sin(theta) in every channel (achromatic beams from
// the chromatic FFT grid of eq. e:theta_A).
//
// The weights are generated once in FP64 on the device (the removable
// singularity at integer y takes its limit (2n-1)/M) and stored in FP32.
// The contraction Out[row][target] = sum_A I[row][A] W[target][A] (rows =
// (block, polarisation, E-W beam) of one channel) runs on FP32 MFMA
// (v_mfma_f32_16x16x4_f32).  A 256-thread workgroup owns 64 rows x TT
// targets (TT = 64 or 256); wave w owns rows 16w..16w+15 against all TT
// targets.  The K axis (beams A) is walked in chunks of KC:
//   * the intensity operand goes straight from HBM to registers: lane
//     (m, g) of a wave feeds row m and, at MFMA step s, beam g*KC/4 + s of
//     the chunk (a permutation of K that both operands share), so its KC/4
//     values are contiguous and arrive as float4 loads;
//   * the weight chunk [TT][KC] is staged once per workgroup in LDS and read
//     back as ds_read_b128 in the same permuted order;
//   * the next chunk's global loads are issued before the current chunk's
//     MFMAs, so their latency hides under the matrix work.
#include "dev_common.h"
#include "kernels.h"

namespace fftbf {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Weight w^A of FFT beam A for the steering y (FP64).  coef == nullptr: the
// pointed kernel of eq. e:bp_max_arbitrary in closed form.  Otherwise the
// optimally windowed kernel (eq. e:w_opt mapped by eq. e:wA_from_wdelta):
// w^A = (1/M) [c_0 + 2 sum_{d=1}^{n-1} c_d cos(2 pi d (A/M - y))] with the
// window's lag coefficients c_d = R_d / ((n - d) N), summed with a
// unit-modulus recurrence.
__device__ double regrid_weight(int A, double y, int n, int m, const double* coef) {
  const double ya = y - (double)A / (double)m;
  if (!coef) {
    const double den = sinpi(ya);
    if (fabs(den) < 1e-12) return (double)(2 * n - 1) / m;
    return sinpi((double)(2 * n - 1) * ya) / den / m;
  }
  double s1, c1;
  sincospi(2.0 * ya, &s1, &c1);
  double er = c1, ei = s1, acc = coef[0];
  for (int d = 1; d < n; ++d) {
    acc += 2.0 * coef[d] * er;
    const double nr = er * c1 - ei * s1;
    ei = er * s1 + ei * c1;
    er = nr;
  }
  return acc / m;
}

__global__ void k_regrid_weights(float* w, const double* dl, const double* sin_t, const double* coef, int n_chan,
                                 int n_target, int n_target_pad, int n, int m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)n_chan * n_target_pad * m;
  if (i >= total) return;
  const int A = (int)(i % m);
  const int j = (int)((i / m) % n_target_pad);
  const int c = (int)(i / ((int64_t)m * n_target_pad));
  if (j >= n_target) {
    w[i] = 0.f;
    return;
  }
  w[i] = (float)regrid_weight(A, dl[2 * c + 1] * sin_t[j], n, m, coef);
}

// E-W weights of 2-D pointings: w[chan][target][e], e < m (= 8), zero rows
// for padded targets; the pointed kernel of eq. e:bp_max_arbitrary on the
// (padded) E-W axis.
__global__ void k_regrid_ew_weights(float* w, const double* dl, const double* dircos_ew, int n_chan, int n_target,
                                    int n_target_pad, int n, int m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)n_chan * n_target_pad * m;
  if (i >= total) return;
  const int e = (int)(i % m);
  const int j = (int)((i / m) % n_target_pad);
  const int c = (int)(i / ((int64_t)m * n_target_pad));
  w[i] = j < n_target ? (float)regrid_weight(e, dl[2 * c] * dircos_ew[j], n, m, nullptr) : 0.f;
}

// Compact kernels: the k FFT beams nearest the steering on the circular beam
// grid, first = rint(y M) - (k-1)/2 (mod M), with their full-kernel weights.
// Layout: first[chan][target], tw[chan][tap][target].
__global__ void k_regrid_tap_table(int* first, float* tw, const double* dl, const double* sin_t, const double* coef,
                                   int n_chan, int n_target, int k, int n, int m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)n_chan * k * n_target;
  if (i >= total) return;
  const int t = (int)(i % n_target);
  const int j = (int)((i / n_target) % k);
  const int c = (int)(i / ((int64_t)n_target * k));
  const double y = dl[2 * c + 1] * sin_t[t];
  const int64_t f0 = (int64_t)rint(y * (double)m) - (k - 1) / 2;
  const int f = (int)(((f0 % m) + m) % m);
  if (j == 0) first[(int64_t)c * n_target + t] = f;
  tw[i] = (float)regrid_weight((f + j) % m, y, n, m, coef);
}

// KC: beams per chunk (32 when M = 32, else 64).  NT: 16-target MFMA tiles
// per wave (TT = 16 NT targets per workgroup).  EW2D: 2-D pointings on an
// E-W axis padded to 8 beams -- the 8 E-W rows of each (block, pol group)
// are combined with the E-W weights in the epilogue.
template <int KC, int NT, bool EW2D>
__global__ __launch_bounds__(256, 2) void k_regrid(RegridArgs a) {
  constexpr int TT = 16 * NT;
  constexpr int KS = KC / 4;              // MFMA steps per chunk = beams per lane per chunk
  constexpr int KV = KS / 4;              // float4 per lane per row per chunk
  constexpr int LDW = KC + 4;             // LDS row stride (floats) of the weight chunk
  constexpr int WV = TT * KC / 4 / 256;   // weight float4 staged per thread per chunk
  __shared__ __attribute__((aligned(16))) float lds_w[TT * LDW];

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int m = lane & 15, g = lane >> 4;
  const int chan = blockIdx.z;
  const int rows = a.rows_per_chan;
  const int t0 = blockIdx.y * TT;
  const float* wbase = a.w + ((int64_t)chan * a.n_target_pad + t0) * a.m_ns;

  // this lane's intensity row (channel-local r -> global row through the
  // R = n_pg * m_ew rows of one block, R a power of two)
  const int r = blockIdx.x * 64 + wave * 16 + m;
  const bool row_ok = r < rows;
  const int64_t grow = ((int64_t)(r >> a.log2_r) * a.n_chan + chan) * (1 << a.log2_r) + (r & ((1 << a.log2_r) - 1));
  const float* arow = a.in + (row_ok ? grow : 0) * a.m_ns + g * KS;

  f32x4 acc[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};

  f32x4 av_next[KV], wv_next[WV];
  auto load_chunk = [&](int k0) {
#pragma unroll
    for (int v = 0; v < KV; ++v)
      av_next[v] = row_ok ? *reinterpret_cast<const f32x4*>(arow + k0 + 4 * v) : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int it = 0; it < WV; ++it) {
      const int idx = tid + 256 * it;
      const int tr = idx / (KC / 4), c4 = idx % (KC / 4);
      wv_next[it] = *reinterpret_cast<const f32x4*>(wbase + (int64_t)tr * a.m_ns + k0 + 4 * c4);
    }
  };

  load_chunk(0);
  for (int k0 = 0; k0 < a.m_ns; k0 += KC) {
    f32x4 av[KV];
#pragma unroll
    for (int v = 0; v < KV; ++v) av[v] = av_next[v];
#pragma unroll
    for (int it = 0; it < WV; ++it) {
      const int idx = tid + 256 * it;
      const int tr = idx / (KC / 4), c4 = idx % (KC / 4);
      *reinterpret_cast<f32x4*>(&lds_w[tr * LDW + 4 * c4]) = wv_next[it];
    }
    if (k0 + KC < a.m_ns) load_chunk(k0 + KC);
    __syncthreads();
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const float* wrow = &lds_w[(16 * nt + m) * LDW + g * KS];
#pragma unroll
      for (int v = 0; v < KV; ++v) {
        const f32x4 bv = *reinterpret_cast<const f32x4*>(wrow + 4 * v);
#pragma unroll
        for (int q = 0; q < 4; ++q)
          acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[v][q], bv[q], acc[nt], 0, 0, 0);
      }
    }
    __syncthreads();
  }

  // acc[nt][i]: row 16 wave + 4 g + i, target t0 + 16 nt + lane % 16
  if constexpr (EW2D) {
    // rows 16 wave + [0, 8) and + [8, 16) are two (block, pol group) groups of
    // 8 E-W beams: lane group g holds E-W beams 4 (g & 1) .. +3 of group g >> 1
    const int grp_row = blockIdx.x * 64 + wave * 16 + 8 * (g >> 1);
    const bool ok = grp_row < rows && (g & 1) == 0;
    const int gi = grp_row >> 3;
    const int blk = gi / a.n_pg, pg = gi - blk * a.n_pg;
    float* o = a.out + (((int64_t)blk * a.n_chan + chan) * a.n_pg + pg) * a.n_target;
    const float* wew = a.wew + ((int64_t)chan * a.n_target_pad + t0) * 8 + 4 * (g & 1);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int t = t0 + 16 * nt + m;
      const f32x4 we = *reinterpret_cast<const f32x4*>(wew + (16 * nt + m) * 8);
      float part = we[0] * acc[nt][0];
      part = fmaf(we[1], acc[nt][1], part);
      part = fmaf(we[2], acc[nt][2], part);
      part = fmaf(we[3], acc[nt][3], part);
      part += __shfl_xor(part, 16);
      if (ok && t < a.n_target) o[t] = part;
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int ro = blockIdx.x * 64 + wave * 16 + 4 * g + i;
    if (ro >= rows) continue;
    const int64_t go = ((int64_t)(ro >> a.log2_r) * a.n_chan + chan) * (1 << a.log2_r) + (ro & ((1 << a.log2_r) - 1));
    float* o = a.out + go * a.n_target;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int t = t0 + 16 * nt + m;
      if (t < a.n_target) o[t] = acc[nt][i];
    }
  }
}

// Compact-kernel regridding (K taps per target): an HBM-bound gather.  A
// 256-thread workgroup stages kTapRows rows (all M beams) of one channel in LDS with
// float4 loads; each thread then takes targets t = tid, tid + 256, ... and
// forms sum_j tw[j][t] I[row][(first[t] + j) mod M] for those rows, writing
// each row's targets contiguously.
// rows per workgroup of the compact-tap kernel: 8 rows (16 KB of LDS at
// M = 512) let ten workgroups share a compute unit; 16 rows (32 KB, five
// workgroups) left the loads of one workgroup less to overlap with and
// were 10% slower at the CHIME shape, 4 rows no faster
constexpr int kTapRows = 8;

template <int K>
__global__ __launch_bounds__(256) void k_regrid_taps(RegridArgs a) {
  constexpr int RT = kTapRows;
  __shared__ __attribute__((aligned(16))) float lds[RT * 512];
  const int tid = threadIdx.x, chan = blockIdx.y;
  const int m = a.m_ns, mv = m >> 2;
  const int r0 = blockIdx.x * RT;
  const int nr = min(RT, a.rows_per_chan - r0);
  const int lr = a.log2_r, rmask = (1 << lr) - 1;
  auto grow = [&](int r) -> int64_t { return ((int64_t)(r >> lr) * a.n_chan + chan) * (1 << lr) + (r & rmask); };
  for (int idx = tid; idx < nr * mv; idx += 256) {
    const int rr = idx / mv, c4 = idx - rr * mv;
    *reinterpret_cast<f32x4*>(&lds[rr * m + 4 * c4]) =
        *reinterpret_cast<const f32x4*>(a.in + grow(r0 + rr) * m + 4 * c4);
  }
  __syncthreads();
  const int T = a.n_target;
  for (int t = tid; t < T; t += 256) {
    const int f = a.first[(int64_t)chan * T + t];
    float w[K];
    int ix[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      w[j] = a.tw[((int64_t)chan * K + j) * T + t];
      ix[j] = (f + j) & (m - 1);
    }
    for (int rr = 0; rr < nr; ++rr) {
      const float* row = &lds[rr * m];
      float acc = 0.f;
#pragma unroll
      for (int j = 0; j < K; ++j) acc = fmaf(w[j], row[ix[j]], acc);
      a.out[grow(r0 + rr) * T + t] = acc;
    }
  }
}

template <int KC, bool EW2D>
hipError_t launch_kc(const RegridArgs& a, dim3 grid, bool wide, hipStream_t s) {
  if (wide)
    hipLaunchKernelGGL((k_regrid<KC, 16, EW2D>), grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_regrid<KC, 4, EW2D>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace

// Targets are padded to the workgroup's target tile: 64 for up to 64
// targets, else a multiple of 256.
int regrid_target_pad(int n_target) {
  return n_target <= 64 ? 64 : (n_target + 255) / 256 * 256;
}

hipError_t launch_regrid_weights(float* w, const double* dl, const double* sin_t, const double* coef, int n_chan,
                                 int n_target, int n, int m, hipStream_t s) {
  const int pad = regrid_target_pad(n_target);
  const int64_t total = (int64_t)n_chan * pad * m;
  hipLaunchKernelGGL(k_regrid_weights, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, w, dl, sin_t, coef,
                     n_chan, n_target, pad, n, m);
  return hipGetLastError();
}

hipError_t launch_regrid_ew_weights(float* w, const double* dl, const double* dircos_ew, int n_chan, int n_target,
                                    int n, int m, hipStream_t s) {
  const int pad = regrid_target_pad(n_target);
  const int64_t total = (int64_t)n_chan * pad * m;
  hipLaunchKernelGGL(k_regrid_ew_weights, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, w, dl, dircos_ew,
                     n_chan, n_target, pad, n, m);
  return hipGetLastError();
}

hipError_t launch_regrid_tap_table(int* first, float* tw, const double* dl, const double* sin_t, const double* coef,
                                   int n_chan, int n_target, int k, int n, int m, hipStream_t s) {
  const int64_t total = (int64_t)n_chan * k * n_target;
  hipLaunchKernelGGL(k_regrid_tap_table, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, first, tw, dl, sin_t,
                     coef, n_chan, n_target, k, n, m);
  return hipGetLastError();
}

hipError_t launch_regrid(const RegridArgs& a_in, hipStream_t s) {
  RegridArgs a = a_in;
  if (a.m_ns < 32 || (a.m_ns & (a.m_ns - 1))) return hipErrorNotSupported;
  const int r_blk = a.n_pg * a.m_ew;
  if (r_blk <= 0 || (r_blk & (r_blk - 1))) return hipErrorNotSupported;
  a.log2_r = 0;
  while ((1 << a.log2_r) < r_blk) ++a.log2_r;
  const int64_t rows = a.n_blk * r_blk;
  if (rows == 0) return hipSuccess;
  if (rows > 0x7FFFFF00LL || a.n_chan > 65535) return hipErrorInvalidConfiguration;
  a.rows_per_chan = (int)rows;
  if (a.n_taps > 0) {
    if (a.n_taps > kRegridMaxTaps || a.m_ns > 512) return hipErrorNotSupported;
    const dim3 g((unsigned)((rows + kTapRows - 1) / kTapRows), (unsigned)a.n_chan);
    switch (a.n_taps) {
      case 1: hipLaunchKernelGGL(k_regrid_taps<1>, g, dim3(256), 0, s, a); break;
      case 2: hipLaunchKernelGGL(k_regrid_taps<2>, g, dim3(256), 0, s, a); break;
      case 3: hipLaunchKernelGGL(k_regrid_taps<3>, g, dim3(256), 0, s, a); break;
      case 4: hipLaunchKernelGGL(k_regrid_taps<4>, g, dim3(256), 0, s, a); break;
      case 5: hipLaunchKernelGGL(k_regrid_taps<5>, g, dim3(256), 0, s, a); break;
      case 6: hipLaunchKernelGGL(k_regrid_taps<6>, g, dim3(256), 0, s, a); break;
      case 7: hipLaunchKernelGGL(k_regrid_taps<7>, g, dim3(256), 0, s, a); break;
      default: hipLaunchKernelGGL(k_regrid_taps<8>, g, dim3(256), 0, s, a); break;
    }
    return hipGetLastError();
  }
  const bool wide = a.n_target_pad > 64;
  const int tt = wide ? a.n_target_pad / 256 : 1;
  const dim3 grid((unsigned)((rows + 63) / 64), (unsigned)tt, (unsigned)a.n_chan);
  if (a.wew) {
    if (a.m_ew != 8) return hipErrorNotSupported;
    return a.m_ns == 32 ? launch_kc<32, true>(a, grid, wide, s) : launch_kc<64, true>(a, grid, wide, s);
  }
  return a.m_ns == 32 ? launch_kc<32, false>(a, grid, wide, s) : launch_kc<64, false>(a, grid, wide, s);
}

}  // namespace fftbf
