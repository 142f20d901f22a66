// Matrix-core FFT beamformer for the 4 x 256 lattice (gfx950).
//
// The N-S transform is zero-padded to M = 512 (eq. e:fftbeamform, weights
// of eq. e:w_A^a) and split as 512 = 32 x 16:
//   a = a1 + 16 a2,  A = k2 + 32 k1      (a1, a2, k1 in [0, 16), k2 in [0, 32))
//   stage 1: Y[a1][k2] = sum_{a2} x[a1 + 16 a2] W_32^{a2 k2}   (padded 16 -> 32 DFT)
//   twiddle: Z[a1][k2] = Y[a1][k2] W_512^{a1 k2}
//   stage 2: B[k2 + 32 k1] = sum_{a1} Z[a1][k2] W_16^{a1 k1}
//
// Stage 1 is a dense product on the matrix cores, per sample and E-W beam:
//   C[a1][k2] = A[a1][(a2, re|im)] * B[(a2, re|im)][k2]
// A holds the E-W sums of the E-W beam at N-S position a1 + 16 a2: the
// 4-point E-W DFT has twiddles +-1, +-i, so they are integers of magnitude
// at most 32, formed by signed 4-bit dot products on the packed bytes, and
// FP16 holds them exactly.  B holds the realified coefficients as two FP16
// terms (hi + lo, about 22 significant bits) that accumulate into the same
// FP32 accumulators, so stage 1 is accurate to FP32 rounding.
//
// The twiddle is a whole complex product in FP32 (four operations per
// value).  Its tangent form (two operations, the factor Re W carried into
// per-column stage-2 multipliers, as in the FP32 kernel) issues fewer vector
// instructions, but the 25 multipliers per lane took the kernel past the 168
// registers of three wavefronts per SIMD, and it measured no faster.
//
// Stage 2 is the FP32 16-point DFT over a1 in registers (compile-time
// coefficients), one (E-W beam, k2) per lane.  The data go from the stage-1 layout (lane = (a1 group, k2)) to
// the stage-2 layout (lane = (E-W beam, k2), all a1) through an LDS tile of
// one E-W beam pair at a time (9 KB per wavefront), so three wavefronts per
// SIMD fit.  |B|^2 accumulates in registers over the block; at its end the
// sums pass once more through LDS so the kept beams of the channel's clamp
// table can be stored with coalesced writes.
//
// FP8 variant: e4m3 does not hold every E-W sum (17, for one), so the data
// operand holds only the first radix-2 stage of the E-W DFT (x0 +- x2,
// x1 +- x3: at most 16 in magnitude, exact), and the second stage runs in
// FP32 on the stage-1 outputs, before the twiddle.  The
// coefficients are split into three e4m3 terms, W = hi + 2^-5 lo1 + 2^-9 lo2,
// stacked along K of one v_mfma_scale_f32_16x16x128_f8f6f4 (unit block
// scales): lane group g holds in its 32 K values the (a2, re|im) of a2 in
// [4g, 4g + 4) once per term (8 values each) and 8 zeros, and the power of
// two of each term sits on the exact data bytes (x, 2^-5 x, 2^-9 x).  One
// pair of first-stage columns is formed at a time ((S02, S13) gives E-W
// beams 0 and 2, (D02, D13) beams 1 and 3), and the LDS tile holds that
// E-W beam pair over both beam tiles, as in the FP16 kernel.
#include "dev_common.h"
#include "dev_f16.h"
#include "kernels.h"

namespace fftbf {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));


constexpr int kPrecFp16 = 1;
constexpr int kPrecFp8 = 2;

typedef int i32x8 __attribute__((ext_vector_type(8)));

// plan table layout (bytes)
constexpr size_t kH256B1Off = 0;      // FP16: [term 2][kt 2][part 2][lane 64][8] halves
                                      // FP8:  [kt 2][part 2][lane 64][32] bytes
constexpr size_t kH256TwOff = 8192;   // [lane 64][kt 2][q 4] float2
constexpr size_t kH256Bytes = 8192 + 4096;

// realified coefficient of stage 1: output part `part` (0 Re, 1 Im) of k2
// from input component comp (0 Re, 1 Im) of position a2, W = W_32^{a2 k2} = c + i s,
//   Re(W x) = c xr - s xi,  Im(W x) = s xr + c xi
__device__ double h256_coef(int a2, int comp, int k2, int part) {
  double s, c;
  sincospi(-2.0 * (double)((a2 * k2) & 31) / 32.0, &s, &c);
  return part == 0 ? (comp == 0 ? c : -s) : (comp == 0 ? s : c);
}

// FP64 on the device, rounded once into the operand layouts.
template <int PREC>
__global__ void k_mix256_tables(void* tab) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  char* base = static_cast<char*>(tab);
  if constexpr (PREC == kPrecFp16) {
    // stage-1 operand B[k = 8 g + j][n] of part `part` of k2 = 16 kt + n,
    // input (a2, comp) = (4 g + j / 2, j % 2), as hi + lo FP16 terms
    if (i < 2 * 2 * 64 * 8) {
      const int j = i & 7, lane = (i >> 3) & 63, part = (i >> 9) & 1, kt = (i >> 10) & 1;
      const double v = h256_coef(4 * (lane >> 4) + (j >> 1), j & 1, 16 * kt + (lane & 15), part);
      _Float16* t = reinterpret_cast<_Float16*>(base + kH256B1Off);
      const _Float16 hi = (_Float16)(float)v;
      t[i] = hi;
      t[2048 + i] = (_Float16)(float)(v - (double)(float)hi);
    }
  } else {
    // byte j of lane (g, n): term j / 8 (j >= 24: zero) of (a2, comp) =
    // (4 g + (j % 8) / 2, j % 2), stored times 2^fp8_shift(term)
    if (i < 2 * 2 * 64 * 8) {
      const int jj = i & 7, lane = (i >> 3) & 63, part = (i >> 9) & 1, kt = (i >> 10) & 1;
      double r = h256_coef(4 * (lane >> 4) + (jj >> 1), jj & 1, 16 * kt + (lane & 15), part);
      uint8_t* t = reinterpret_cast<uint8_t*>(base + kH256B1Off) + (((kt * 2 + part) * 64 + lane) * 32) + jj;
      for (int p = 0; p < 3; ++p) {
        const double sc = (double)(1 << fp8_shift(p));
        const int byte = f32_to_fp8((float)(r * sc));
        t[8 * p] = (uint8_t)byte;
        r -= (double)fp8_to_f32(byte) / sc;
      }
      t[24] = 0;
    }
  }
  // twiddles W_512^{a1 k2} of lane (g, n), slot (kt, q): a1 = 4 g + q, k2 = 16 kt + n
  if (i < 64 * 8) {
    const int kt = (i >> 2) & 1, q = i & 3, lane = i >> 3;
    const int a1 = 4 * (lane >> 4) + q, k2 = 16 * kt + (lane & 15);
    double s, c;
    sincospi(-2.0 * (double)((a1 * k2) & 511) / 512.0, &s, &c);
    reinterpret_cast<float2*>(base + kH256TwOff)[i] = make_float2((float)c, (float)s);
  }
}

// dot8 weights of component comp (0 Re, 1 Im) of E-W beam e, sum_q x_q (-i)^{e q}
// (nibble 2q + 1 is Re x_q, nibble 2q is Im x_q)
__device__ __forceinline__ int ew_weights_comp(int e, int comp) {
  int wre = 0, wim = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int k = (e * q) & 3;
    const int sr = 4 * (2 * q + 1), si = 4 * (2 * q);
    if (k == 0) { wre |= 1 << sr;   wim |= 1 << si; }
    if (k == 1) { wre |= 1 << si;   wim |= 0xF << sr; }
    if (k == 2) { wre |= 0xF << sr; wim |= 0xF << si; }
    if (k == 3) { wre |= 0xF << si; wim |= 1 << sr; }
  }
  return comp ? wim : wre;
}

// Stage-1 data operand: (Re, Im) of the E-W beam at the lane's four N-S
// positions, as FP16 without conversion instructions: each dot product
// starts from 0x6600, the FP16 pattern of 1536 (unit step 1), so its low
// half is FP16(1536 + x) for |x| <= 32; Re and Im are packed by one byte
// permute and 1536 comes off in one packed FP16 subtraction (exact).
__device__ __forceinline__ half8 ew_pairs_f16(const uint32_t* dw, int wre, int wim) {
  half8 A;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t re = (uint32_t)sdot8_acc((int)dw[i], wre, 0x6600);
    const uint32_t im = (uint32_t)sdot8_acc((int)dw[i], wim, 0x6600);
    const half2 v = __builtin_bit_cast(half2, __builtin_amdgcn_perm(im, re, 0x05040100u)) -
                    half2{(_Float16)1536.0f, (_Float16)1536.0f};
    A[2 * i] = v[0];
    A[2 * i + 1] = v[1];
  }
  return A;
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Windowed E-W sums (per-antenna real weights h, Sec. "Controlling beam shape
// with windowing") of the lane's four N-S positions for all four E-W beams:
// x[e][2 i], x[e][2 i + 1] = Re, Im of sum_q h_q z_q (-i)^{e q} at position i.
__device__ __forceinline__ void ew_windowed(const uint32_t* dw, const float (&h)[4][4], float (&x)[4][8]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    cf w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      w[q] = cf{h[i][q] * (float)(int)__builtin_amdgcn_sbfe((int)dw[i], 8 * q + 4, 4),
                h[i][q] * (float)(int)__builtin_amdgcn_sbfe((int)dw[i], 8 * q, 4)};
    const cf s02 = cadd(w[0], w[2]), d02 = csub(w[0], w[2]), s13 = cadd(w[1], w[3]), d13 = csub(w[1], w[3]);
    const cf b[4] = {cadd(s02, s13), cf{d02.r + d13.i, d02.i - d13.r}, csub(s02, s13), cf{d02.r - d13.i, d02.i + d13.r}};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      x[e][2 * i] = b[e].r;
      x[e][2 * i + 1] = b[e].i;
    }
  }
}

// One wavefront per (block, channel, polarisation group).  Lane l = 16 g + n:
// stage 1 holds a1 = 4 g + q (q < 4) and k2 = 16 kt + n (kt < 2); stage 2
// takes E-W beam 2 p + (l >> 5) of pair p and k2 = l & 31.
// WIN: per-antenna real weights.  The windowed E-W sums are no longer
// integers, so each is split into FP16 hi + lo and stage 1 takes three
// products (hi x hi, hi x lo, lo x hi of data and coefficients).  The
// window is scaled by a power of two per wavefront so that its largest
// weight lies in [1/2, 1) and the low terms stay in FP16's normal range;
// the block sums are scaled back exactly.
template <bool WIN>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void k_mix256(MixArgs a) {
  constexpr int N = 256, M = 512;
  constexpr int ROW = 18;                     // complex values per (E-W beam, k2) row: 16 a1 + 2 pad
  __shared__ float4 lds_raw[2 * 32 * ROW / 2];
  cf* const tile = reinterpret_cast<cf*>(lds_raw);

  const int lane = threadIdx.x;
  const int n = lane & 15, g = lane >> 4;
  int wg = blockIdx.x;
  const int pg = wg % a.n_pg;
  wg /= a.n_pg;
  const int chan = wg % a.n_chan;
  const int blk = wg / a.n_chan;

  const char* tab = static_cast<const char*>(a.mat);
  half8 B1[2][2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int kt = 0; kt < 2; ++kt)
#pragma unroll
      for (int part = 0; part < 2; ++part)
        B1[p][kt][part] = *reinterpret_cast<const half8*>(
            tab + kH256B1Off + 2 * (p * 2048 + ((kt * 2 + part) * 64 + lane) * 8));
  cf tw[2][4];
  {
    const float2* w = reinterpret_cast<const float2*>(tab + kH256TwOff) + lane * 8;
#pragma unroll
    for (int k = 0; k < 8; ++k) tw[k >> 2][k & 3] = cf{w[k].x, w[k].y};
  }
  const int k2s = lane & 31, es = lane >> 5;  // stage-2 column and E-W beam within the pair
  int wre[4], wim[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    wre[e] = ew_weights_comp(e, 0);
    wim[e] = ew_weights_comp(e, 1);
  }

  float acc[2][16];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[p][k] = 0.f;

  // the window at the lane's N-S positions n + 64 g + 16 i, scaled by 2^-E
  // with 2^E the power of two just above the wavefront's largest |h|
  float hw[4][4];
  float unscale = 1.f;       // 2^{2E}: undoes the scale on |B|^2
  if constexpr (WIN) {
    float m = 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float4 v = *reinterpret_cast<const float4*>(a.taper + 4 * (n + 64 * g + 16 * i));
      hw[i][0] = v.x;
      hw[i][1] = v.y;
      hw[i][2] = v.z;
      hw[i][3] = v.w;
      m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
    }
#pragma unroll
    for (int d = 1; d < 64; d *= 2) m = fmaxf(m, __shfl_xor(m, d));
    const int ex = m > 0.f ? ilogbf(m) + 1 : 0;      // m * 2^-ex in [1/2, 1)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) hw[i][q] = ldexpf(hw[i][q], -ex);
    unscale = ldexpf(1.f, 2 * ex);
  }

  const int pol_lo = (a.pol_iter == 1) ? pg : 0;
  const int pol_hi = (a.pol_iter == 1) ? pg + 1 : a.n_pol;
  const int64_t frame_stride = (int64_t)a.n_chan * a.n_pol * N;   // dwords per sample
  const int64_t t0 = (int64_t)blk * a.block;

  auto frame = [&](const uint32_t (&dw)[4]) {
    float xw[WIN ? 4 : 1][8];
    if constexpr (WIN) ew_windowed(dw, hw, xw);
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      // ---- stage 1 and twiddle for E-W beams 2p, 2p + 1, into the tile ----
#pragma unroll
      for (int ep = 0; ep < 2; ++ep) {
        const int e = 2 * p + ep;
        f32x4 y[2][2];
        if constexpr (WIN) {
          uint32_t hi[4], lo[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) split2(xw[e][2 * i], xw[e][2 * i + 1], hi[i], lo[i]);
          const half8 Ah = __builtin_bit_cast(half8, hi), Al = __builtin_bit_cast(half8, lo);
#pragma unroll
          for (int kt = 0; kt < 2; ++kt)
#pragma unroll
            for (int part = 0; part < 2; ++part) {
              y[kt][part] = __builtin_amdgcn_mfma_f32_16x16x32_f16(Ah, B1[0][kt][part], f32x4{0.f, 0.f, 0.f, 0.f},
                                                                   0, 0, 0);
              y[kt][part] = __builtin_amdgcn_mfma_f32_16x16x32_f16(Ah, B1[1][kt][part], y[kt][part], 0, 0, 0);
              y[kt][part] = __builtin_amdgcn_mfma_f32_16x16x32_f16(Al, B1[0][kt][part], y[kt][part], 0, 0, 0);
            }
        } else {
          const half8 A = ew_pairs_f16(dw, wre[e], wim[e]);
#pragma unroll
          for (int kt = 0; kt < 2; ++kt)
#pragma unroll
            for (int part = 0; part < 2; ++part) {
              y[kt][part] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A, B1[0][kt][part], f32x4{0.f, 0.f, 0.f, 0.f},
                                                                   0, 0, 0);
              y[kt][part] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A, B1[1][kt][part], y[kt][part], 0, 0, 0);
            }
        }
#pragma unroll
        for (int kt = 0; kt < 2; ++kt) {
          cf z[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) z[q] = cmul(cf{y[kt][0][q], y[kt][1][q]}, tw[kt][q]);
          float4* dst = reinterpret_cast<float4*>(&tile[(ep * 32 + 16 * kt + n) * ROW + 4 * g]);
          dst[0] = make_float4(z[0].r, z[0].i, z[1].r, z[1].i);
          dst[1] = make_float4(z[2].r, z[2].i, z[3].r, z[3].i);
        }
      }
      wave_lds_sync();
      // ---- stage 2: 16-point DFT over a1 for (E-W beam 2p + es, k2s) ----
      cf x[16];
      {
        const float4* src = reinterpret_cast<const float4*>(&tile[(es * 32 + k2s) * ROW]);
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          const float4 v = src[m];
          x[2 * m] = cf{v.x, v.y};
          x[2 * m + 1] = cf{v.z, v.w};
        }
      }
      wave_lds_sync();
      dit<16>(x);
#pragma unroll
      for (int k1 = 0; k1 < 16; ++k1) acc[p][k1] = cnorm_acc(x[k1], acc[p][k1]);
    }
  };

  for (int pol = pol_lo; pol < pol_hi; ++pol) {
    // the lane's N-S positions a1 + 16 a2 = n + 64 g + 16 i, i < 4
    const uint32_t* src = a.volts + ((int64_t)chan * a.n_pol + pol) * N + n + 64 * g;
    const uint32_t* last = src + (t0 + a.block - 1) * frame_stride;
    uint32_t b0[4], b1[4];
    const uint32_t* q0 = src + t0 * frame_stride;
#pragma unroll
    for (int i = 0; i < 4; ++i) b0[i] = __builtin_nontemporal_load(q0 + 16 * i);
    // two frame buffers in turn; the load past the block's last frame
    // re-reads that frame (cached), so no load is conditional
    for (int s = 0; s < a.block; s += 2) {
      const uint32_t* q1 = (s + 1 < a.block) ? q0 + frame_stride : last;
#pragma unroll
      for (int i = 0; i < 4; ++i) b1[i] = __builtin_nontemporal_load(q1 + 16 * i);
      frame(b0);
      if (s + 1 >= a.block) break;
      q0 = (s + 2 < a.block) ? q1 + frame_stride : last;
#pragma unroll
      for (int i = 0; i < 4; ++i) b0[i] = __builtin_nontemporal_load(q0 + 16 * i);
      frame(b1);
    }
  }

  // ---- block end: beams A = k2 + 32 k1 of E-W beam 2p + es, clamp, store ----
  float* lds_i = reinterpret_cast<float*>(lds_raw);
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) lds_i[(2 * p + es) * M + k2s + 32 * k1] = acc[p][k1];
  wave_lds_sync();
  const int keep = a.n_keep;
  const int32_t* sel = a.sel ? a.sel + (int64_t)chan * keep : nullptr;
  float* o = a.out + (((int64_t)blk * a.n_chan + chan) * a.n_pg + pg) * 4 * keep;
#pragma unroll
  for (int e = 0; e < 4; ++e)
    for (int j = lane; j < keep; j += 64) o[e * keep + j] = lds_i[e * M + (sel ? sel[j] : j)] * (a.norm * unscale);
}

// FP8: one wavefront per (block, channel, polarisation group).  Lane
// l = 16 g + n: stage 1 holds a1 = 4 g + q and k2 = 16 kt + n for the beam
// tile kt of the round; stage 2 takes E-W beam l >> 4 and k2 = 16 kt + (l & 15).
__global__ __launch_bounds__(64) void k_mix256_fp8(MixArgs a) {
  constexpr int N = 256, M = 512;
  constexpr int ROW = 18;                     // complex values per (E-W beam, k2) row: 16 a1 + 2 pad
  constexpr int kUnitScale = 0x7F7F7F7F;      // E8M0 block scale 2^0
  __shared__ float4 lds_raw[4 * 16 * ROW / 2];
  cf* const tile = reinterpret_cast<cf*>(lds_raw);

  const int lane = threadIdx.x;
  const int n = lane & 15, g = lane >> 4;
  int wg = blockIdx.x;
  const int pg = wg % a.n_pg;
  wg /= a.n_pg;
  const int chan = wg % a.n_chan;
  const int blk = wg / a.n_chan;

  const char* tab = static_cast<const char*>(a.mat);
  i32x8 B[2][2];
#pragma unroll
  for (int kt = 0; kt < 2; ++kt)
#pragma unroll
    for (int part = 0; part < 2; ++part)
      B[kt][part] = *reinterpret_cast<const i32x8*>(tab + kH256B1Off + ((kt * 2 + part) * 64 + lane) * 32);
  cf tw[2][4];
  {
    const float2* w = reinterpret_cast<const float2*>(tab + kH256TwOff) + lane * 8;
#pragma unroll
    for (int k = 0; k < 8; ++k) tw[k >> 2][k & 3] = cf{w[k].x, w[k].y};
  }
  const int bs = lane >> 5, k2s = lane & 31;   // stage-2 beam of the pair and column k2

  float acc[2][16];
#pragma unroll
  for (int cp = 0; cp < 2; ++cp)
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[cp][k] = 0.f;

  const int pol_lo = (a.pol_iter == 1) ? pg : 0;
  const int pol_hi = (a.pol_iter == 1) ? pg + 1 : a.n_pol;
  const int64_t frame_stride = (int64_t)a.n_chan * a.n_pol * N;   // dwords per sample
  const int64_t t0 = (int64_t)blk * a.block;

  auto frame = [&](const uint32_t (&dw)[4]) {
    // one pair of first-stage E-W columns at a time: (S02, S13) gives E-W
    // beams 0 and 2, (D02, D13) beams 1 and 3, through both beam tiles, so
    // only the pair's operands are live and stage 2 takes one E-W beam pair
#pragma unroll
    for (int cp = 0; cp < 2; ++cp) {
      // data operands of the first E-W radix-2 stage (x0 + x2, x1 + x3,
      // x0 - x2, x1 - x3; exact in e4m3): (Re, Im) at the lane's four N-S
      // positions, once per term (times 2^-shift), then zeros
      i32x8 A[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        int wre, wim;
        ew_half_weights(2 * cp + h, wre, wim);
        int v[8];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          v[2 * i] = sdot8((int)dw[i], wre);
          v[2 * i + 1] = sdot8((int)dw[i], wim);
        }
#pragma unroll
        for (int p = 0; p < 3; ++p) {
          const long w = to_fp8(v, 1.0f / (float)(1 << fp8_shift(p)));
          A[h][2 * p] = (int)w;
          A[h][2 * p + 1] = (int)(w >> 32);
        }
        A[h][6] = 0;
        A[h][7] = 0;
      }
#pragma unroll
      for (int kt = 0; kt < 2; ++kt) {
        // ---- stage 1, the second E-W stage and the twiddle, into the tile
        // (row: beam of the pair bs, k2 = 16 kt + n) ----
        f32x4 y[2][2];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int part = 0; part < 2; ++part)
            y[h][part] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                A[h], B[kt][part], f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0, kUnitScale, 0, kUnitScale);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          // X_0 = S02 + S13, X_2 = S02 - S13 (cp = 0); X_1 = D02 - i D13,
          // X_3 = D02 + i D13 (cp = 1)
          const cf u{y[0][0][i], y[0][1][i]}, v{y[1][0][i], y[1][1][i]};
          const cf xa = cp == 0 ? cadd(u, v) : cf{u.r + v.i, u.i - v.r};
          const cf xb = cp == 0 ? csub(u, v) : cf{u.r - v.i, u.i + v.r};
          tile[(16 * kt + n) * ROW + 4 * g + i] = cmul(xa, tw[kt][i]);
          tile[(32 + 16 * kt + n) * ROW + 4 * g + i] = cmul(xb, tw[kt][i]);
        }
      }
      wave_lds_sync();
      // ---- stage 2: 16-point DFT over a1 for (E-W beam cp + 2 bs, k2s) ----
      cf x[16];
      {
        const float4* src = reinterpret_cast<const float4*>(&tile[(bs * 32 + k2s) * ROW]);
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          const float4 v = src[m];
          x[2 * m] = cf{v.x, v.y};
          x[2 * m + 1] = cf{v.z, v.w};
        }
      }
      wave_lds_sync();
      dit<16>(x);
#pragma unroll
      for (int k1 = 0; k1 < 16; ++k1) acc[cp][k1] = cnorm_acc(x[k1], acc[cp][k1]);
    }
  };

  for (int pol = pol_lo; pol < pol_hi; ++pol) {
    const uint32_t* src = a.volts + ((int64_t)chan * a.n_pol + pol) * N + n + 64 * g;
    const uint32_t* last = src + (t0 + a.block - 1) * frame_stride;
    uint32_t b0[4], b1[4];
    const uint32_t* q0 = src + t0 * frame_stride;
#pragma unroll
    for (int i = 0; i < 4; ++i) b0[i] = __builtin_nontemporal_load(q0 + 16 * i);
    for (int s = 0; s < a.block; s += 2) {
      const uint32_t* q1 = (s + 1 < a.block) ? q0 + frame_stride : last;
#pragma unroll
      for (int i = 0; i < 4; ++i) b1[i] = __builtin_nontemporal_load(q1 + 16 * i);
      frame(b0);
      if (s + 1 >= a.block) break;
      q0 = (s + 2 < a.block) ? q1 + frame_stride : last;
#pragma unroll
      for (int i = 0; i < 4; ++i) b0[i] = __builtin_nontemporal_load(q0 + 16 * i);
      frame(b1);
    }
  }

  // ---- block end: beams A = k2s + 32 k1 of E-W beam cp + 2 bs, clamp, store ----
  float* lds_i = reinterpret_cast<float*>(lds_raw);
#pragma unroll
  for (int cp = 0; cp < 2; ++cp)
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) lds_i[(cp + 2 * bs) * M + k2s + 32 * k1] = acc[cp][k1];
  wave_lds_sync();
  const int keep = a.n_keep;
  const int32_t* sel = a.sel ? a.sel + (int64_t)chan * keep : nullptr;
  float* o = a.out + (((int64_t)blk * a.n_chan + chan) * a.n_pg + pg) * 4 * keep;
#pragma unroll
  for (int e = 0; e < 4; ++e)
    for (int j = lane; j < keep; j += 64) o[e * keep + j] = lds_i[e * M + (sel ? sel[j] : j)] * a.norm;
}

}  // namespace

size_t mix256_table_bytes() { return kH256Bytes; }

hipError_t launch_mix256_tables(void* mat, int prec, hipStream_t s) {
  if (prec == kPrecFp16) hipLaunchKernelGGL(k_mix256_tables<kPrecFp16>, dim3(8), dim3(256), 0, s, mat);
  else if (prec == kPrecFp8) hipLaunchKernelGGL(k_mix256_tables<kPrecFp8>, dim3(8), dim3(256), 0, s, mat);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_mix256(const MixArgs& a, int prec, int64_t n_wg, hipStream_t s) {
  if (n_wg == 0) return hipSuccess;
  if (n_wg > 0x7FFFFFFF) return hipErrorInvalidConfiguration;
  if (prec == kPrecFp16 && a.taper) hipLaunchKernelGGL(k_mix256<true>, dim3((unsigned)n_wg), dim3(64), 0, s, a);
  else if (prec == kPrecFp16) hipLaunchKernelGGL(k_mix256<false>, dim3((unsigned)n_wg), dim3(64), 0, s, a);
  else if (prec == kPrecFp8 && a.taper) return hipErrorNotSupported;
  else if (prec == kPrecFp8) hipLaunchKernelGGL(k_mix256_fp8, dim3((unsigned)n_wg), dim3(64), 0, s, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace fftbf
