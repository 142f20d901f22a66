// Mixed-precision FFT beamformer on the MFMA units (gfx950).
//
// On the 4 x 16 lattice the N-S transform is one dense, zero-padded DFT (16
// non-zero inputs -> M = 32 beams; eq. e:fftbeamform with the weights of eq.
// e:w_A^a), so it runs as a matrix product on the matrix cores:
//
//   C[sample][beam] += A[sample][k] * B[k][beam],   k = (re|im, a_ns)
//
// A holds exact integers: in FP16 the E-W sums of one E-W beam (the 4-point
// E-W DFT has twiddles +-1, +-i, so the sums are integers of magnitude at
// most 32, formed by signed 4-bit dot products on the packed bytes); in FP8
// the first radix-2 stage of the E-W DFT only (x0 +- x2, x1 +- x3, at most
// 16 in magnitude), because e4m3 does not hold every full E-W sum (17, for
// one).  B holds the realified DFT coefficients, split into
// terms of the working precision that accumulate into the same FP32
// accumulators:
//   FP16:  W = hi + lo                               (two passes)
//   FP8:   W = hi + 2^-5 lo1 + 2^-9 lo2              (three passes; the
//          power-of-two factor moves onto the exact data operand so that
//          every coefficient term sits in the normal range of e4m3)
// FP16 then needs only |B|^2 and the block sum; FP8 runs the second E-W
// stage in FP32 on the accumulators, in-lane, before them.
//
// v_mfma_f32_16x16x32_f16 operands (lane l): A row = l % 16 (one sample),
// B column = l % 16 (one beam), both holding k in [8 (l/16), 8 (l/16) + 8);
// C holds column l % 16, rows 4 (l/16) + i.  FP8 stacks its three terms
// along K of one v_mfma_scale_f32_16x16x128_f8f6f4 (32 K values per lane).
#include "dev_common.h"
#include "dev_f16.h"
#include "kernels.h"

namespace fftbf {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kPrecFp16 = 1;
constexpr int kPrecFp8 = 2;
constexpr int kMixBlocksPerWave = 4;

template <int PREC> struct Mix;
template <> struct Mix<kPrecFp16> {
  static constexpr int P = 2;
  using op_t = half8;
};
template <> struct Mix<kPrecFp8> {
  static constexpr int P = 3;
  using op_t = long;
};

// realified DFT coefficient B[k][n] of output part `part` (0 re, 1 im) for
// beam k_out = kt*16 + n of the zero-padded 16 -> 32 N-S transform
__device__ double mix_coef(int kt, int part, int k, int n) {
  const int kout = kt * 16 + n;
  const int comp = k >> 4, a = k & 15;
  const int r = (kout * a) & 31;
  double s, c;
  sincospi(-2.0 * (double)r / 32.0, &s, &c);     // W = c + i s = exp(-i 2 pi r / 32)
  if (part == 0) return comp == 0 ? c : -s;        // Re(W x) = c xr - s xi
  return comp == 0 ? s : c;                        // Im(W x) = s xr + c xi
}

// Table layout: [P][kt 2][part 2][lane 64][j 8], entry = term p of
// B[k = 8 (lane/16) + j][n = lane % 16].
template <int PREC>
__global__ void k_mix_tables(void* tab) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * 2 * 64 * 8) return;
  const int j = i & 7, lane = (i >> 3) & 63, part = (i >> 9) & 1, kt = (i >> 10) & 1;
  const int k = 8 * (lane >> 4) + j, n = lane & 15;
  const double v = mix_coef(kt, part, k, n);
  constexpr int P = Mix<PREC>::P;
  const int stride = 2 * 2 * 64 * 8;   // entries per term
  if constexpr (PREC == kPrecFp16) {
    _Float16* t = static_cast<_Float16*>(tab);
    const _Float16 hi = (_Float16)(float)v;
    const _Float16 lo = (_Float16)(float)(v - (double)(float)hi);
    t[0 * stride + i] = hi;
    t[1 * stride + i] = lo;
  } else {
    // K = 128 operand of v_mfma_scale_f32_16x16x128_f8f6f4: lane (g, n), byte
    // j = 8 t + 2 q + comp holds term t (t = 3: zero) of the coefficient of
    // (a_ns = 4 g + q, comp), stored times 2^fp8_shift(t)
    (void)v;
    (void)stride;
    const int q = (j >> 1) & 3, comp = j & 1, g = lane >> 4;
    double r = mix_coef(kt, part, comp * 16 + 4 * g + q, n);
    uint8_t* t = static_cast<uint8_t*>(tab) + ((kt * 2 + part) * 64 + lane) * 32 + (j & 7);
    // this thread fills bytes (j & 7) + 8 t of the lane; j < 8 covers all
    if (j < 8) {
      for (int p = 0; p < P; ++p) {
        const double sc = (double)(1 << fp8_shift(p));
        const int b = f32_to_fp8((float)(r * sc));
        t[8 * p] = (uint8_t)b;
        r -= (double)fp8_to_f32(b) / sc;
      }
      t[24] = 0;
    }
  }
}

typedef int i32x8 __attribute__((ext_vector_type(8)));

template <int PREC>
__device__ __forceinline__ typename Mix<PREC>::op_t load_b(const void* tab, int p, int kt, int part, int lane) {
  const int off = (((p * 2 + kt) * 2 + part) * 64 + lane) * 8;
  if constexpr (PREC == kPrecFp16) {
    return *reinterpret_cast<const half8*>(static_cast<const _Float16*>(tab) + off);
  } else {
    return *reinterpret_cast<const long*>(static_cast<const uint8_t*>(tab) + off);
  }
}

template <int PREC>
__device__ __forceinline__ f32x4 mfma(typename Mix<PREC>::op_t a, typename Mix<PREC>::op_t b, f32x4 c) {
  if constexpr (PREC == kPrecFp16) return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  else return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
}

// dot8 weights for component comp (0 Re, 1 Im) of E-W beam e:
// sum_q x_q (-i)^{e q}; nibble 2q+1 is Re(x_q), nibble 2q is Im(x_q)
__device__ __forceinline__ int ew_dot_weights(int e, int comp) {
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

// The E-W sums x (|x| <= 32) of eight dwords as FP16, without conversion
// instructions: the dot product starts from 0x6600, the FP16 pattern of
// 1536, whose unit step is 1, so the low half of 0x6600 + x is exactly
// FP16(1536 + x); two are packed and 1536 comes off in one packed FP16
// subtraction (exact).
__device__ __forceinline__ half8 ew_sums_f16(const uint32_t* dw, int w) {
  half8 A;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t lo = (uint32_t)sdot8_acc((int)dw[2 * j], w, 0x6600);
    const uint32_t hi = (uint32_t)sdot8_acc((int)dw[2 * j + 1], w, 0x6600);
    const half2 v = __builtin_bit_cast(half2, __builtin_amdgcn_perm(hi, lo, 0x05040100u)) -
                    half2{(_Float16)1536.0f, (_Float16)1536.0f};
    A[2 * j] = v[0];
    A[2 * j + 1] = v[1];
  }
  return A;
}

// WIN (FP16 only): per-antenna real weights h[a_ns][a_ew] (Sec. "Controlling
// beam shape with windowing").  The windowed E-W sums are no longer
// integers, so each is split into FP16 hi + lo and the N-S products take
// three terms (hi x hi, hi x lo, lo x hi of data and coefficients); the
// window is scaled per wavefront by a power of two so that its largest
// weight lies in [1/2, 1), and the block sums are scaled back exactly.
template <int PREC, bool WIN = false>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WIN ? 4 : PREC == kPrecFp16 ? 6 : 4)))
void k_mix16(MixArgs a) {
  static_assert(!WIN || PREC == kPrecFp16, "windows run on the FP16 path");
  constexpr int P = Mix<PREC>::P;
  using op_t = typename Mix<PREC>::op_t;
  __shared__ float lds_i[4 * 32];

  const int lane = threadIdx.x;
  const int n = lane & 15, g = lane >> 4;
  int pg;
  const int wg = pol_pair_task((int)blockIdx.x, (int)gridDim.x, a.n_pg, pg);
  const int chan = wg % a.n_chan;
  const int run = wg / a.n_chan;
  const int64_t n_blk = a.n_time / a.block;
  const int64_t blk0 = (int64_t)run * kMixBlocksPerWave;
  const int64_t blk1 = blk0 + kMixBlocksPerWave < n_blk ? blk0 + kMixBlocksPerWave : n_blk;

  // FP16: B[term][kt][part]; FP8: the three terms stacked along K = 128 in B8[kt][part]
  op_t B[PREC == kPrecFp16 ? P : 1][2][2];
  i32x8 B8[PREC == kPrecFp8 ? 2 : 1][2];
  if constexpr (PREC == kPrecFp16) {
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
      for (int kt = 0; kt < 2; ++kt)
#pragma unroll
        for (int part = 0; part < 2; ++part) B[p][kt][part] = load_b<PREC>(a.mat, p, kt, part, lane);
  } else {
#pragma unroll
    for (int kt = 0; kt < 2; ++kt)
#pragma unroll
      for (int part = 0; part < 2; ++part)
        B8[kt][part] = *reinterpret_cast<const i32x8*>(static_cast<const uint8_t*>(a.mat) +
                                                        ((kt * 2 + part) * 64 + lane) * 32);
  }

  int wts[4];                                 // FP16: E-W dot8 weights of this lane's component
#pragma unroll
  for (int e = 0; e < 4; ++e) wts[e] = ew_dot_weights(e, g >> 1);
  const int pol_lo = (a.pol_iter == 1) ? pg : 0;
  const int pol_hi = (a.pol_iter == 1) ? pg + 1 : a.n_pol;
  const int keep = a.n_keep;
  // the block-end gather: output idx = e keep + j (idx = lane, lane + 64; at
  // most 4 x 32) reads the block sum of E-W beam e at N-S beam sel[j] (or j);
  // the channel is the wavefront's, so the sources are fixed per lane
  int gsrc[2];
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const int idx = lane + 64 * it;
    const int e = idx / keep, j = idx - e * keep;
    gsrc[it] = idx < 4 * keep ? e * 32 + (a.sel ? a.sel[(int64_t)chan * keep + j] : j) : 0;
  }

  // the window at the lane's N-S positions 8 (g & 1) + j, scaled by 2^-E with
  // 2^E the power of two just above the wavefront's largest |h|
  float hw[WIN ? 8 : 1][4];
  float unscale = 1.f;       // 2^{2E}: undoes the scale on |B|^2
  if constexpr (WIN) {
    float m = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float4 v = *reinterpret_cast<const float4*>(a.taper + 4 * (8 * (g & 1) + j));
      hw[j][0] = v.x;
      hw[j][1] = v.y;
      hw[j][2] = v.z;
      hw[j][3] = v.w;
      m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
    }
#pragma unroll
    for (int d = 1; d < 64; d *= 2) m = fmaxf(m, __shfl_xor(m, d));
    const int ex = m > 0.f ? ilogbf(m) + 1 : 0;      // m * 2^-ex in [1/2, 1)
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) hw[j][q] = ldexpf(hw[j][q], -ex);
    unscale = ldexpf(1.f, 2 * ex);
  }
  const bool im_lane = (g >> 1) != 0;         // this lane's component of the data operand

#pragma unroll 1
  for (int64_t blk = blk0; blk < blk1; ++blk) {
    float ia[4][2];
#pragma unroll
    for (int e = 0; e < 4; ++e) ia[e][0] = ia[e][1] = 0.f;

    for (int pol = pol_lo; pol < pol_hi; ++pol) {
      for (int sub = 0; sub < a.block; sub += 16) {
        const int64_t t = blk * a.block + sub + n;
        const uint4* fr = reinterpret_cast<const uint4*>(a.volts + ((t * a.n_chan + chan) * a.n_pol + pol) * 16);
        // FP16: positions 8 (g & 1) to + 8; FP8: positions 4 g to + 4
        const uint4 d0 = fr[PREC == kPrecFp8 && !WIN ? g : 2 * (g & 1)];
        const uint4 d1 = PREC == kPrecFp8 && !WIN ? uint4{0, 0, 0, 0} : fr[2 * (g & 1) + 1];
        const uint32_t dw[8] = {d0.x, d0.y, d0.z, d0.w, d1.x, d1.y, d1.z, d1.w};

        if constexpr (WIN) {
          // windowed E-W sums of every E-W beam at the lane's eight positions,
          // the lane's component of each, split into FP16 hi + lo
          float xw[4][8];
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            cf w[4];
#pragma unroll
            for (int q = 0; q < 4; ++q)
              w[q] = cf{hw[j][q] * (float)(int)__builtin_amdgcn_sbfe((int)dw[j], 8 * q + 4, 4),
                        hw[j][q] * (float)(int)__builtin_amdgcn_sbfe((int)dw[j], 8 * q, 4)};
            const cf s02 = cadd(w[0], w[2]), d02 = csub(w[0], w[2]), s13 = cadd(w[1], w[3]), d13 = csub(w[1], w[3]);
            const cf be[4] = {cadd(s02, s13), cf{d02.r + d13.i, d02.i - d13.r}, csub(s02, s13),
                              cf{d02.r - d13.i, d02.i + d13.r}};
#pragma unroll
            for (int e = 0; e < 4; ++e) xw[e][j] = im_lane ? be[e].i : be[e].r;
          }
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            uint32_t hi[4], lo[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) split2(xw[e][2 * j], xw[e][2 * j + 1], hi[j], lo[j]);
            const half8 Ah = __builtin_bit_cast(half8, hi), Al = __builtin_bit_cast(half8, lo);
#pragma unroll
            for (int kt = 0; kt < 2; ++kt) {
              f32x4 y[2];
#pragma unroll
              for (int part = 0; part < 2; ++part) {
                y[part] = mfma<PREC>(Ah, B[0][kt][part], f32x4{0.f, 0.f, 0.f, 0.f});
                y[part] = mfma<PREC>(Ah, B[1][kt][part], y[part]);
                y[part] = mfma<PREC>(Al, B[0][kt][part], y[part]);
              }
#pragma unroll
              for (int i = 0; i < 4; ++i) ia[e][kt] = cnorm_acc(cf{y[0][i], y[1][i]}, ia[e][kt]);
            }
          }
        } else if constexpr (PREC == kPrecFp16) {
          // FP16 holds the E-W sums exactly, so the E-W DFT goes first (as
          // signed 4-bit dot products on the packed bytes) and each E-W
          // beam's N-S products land straight in its |B|^2
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const half8 A = ew_sums_f16(dw, wts[e]);
#pragma unroll
            for (int kt = 0; kt < 2; ++kt) {
              f32x4 y[2];
#pragma unroll
              for (int part = 0; part < 2; ++part) {
                y[part] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int p = 0; p < P; ++p) y[part] = mfma<PREC>(A, B[p][kt][part], y[part]);
              }
#pragma unroll
              for (int i = 0; i < 4; ++i) ia[e][kt] = cnorm_acc(cf{y[0][i], y[1][i]}, ia[e][kt]);
            }
          }
        } else {
          // FP8: e4m3 holds every integer up to 16 but not every E-W sum, so
          // the data operand takes the first radix-2 stage of the E-W DFT
          // (x0 + x2, x1 + x3, x0 - x2, x1 - x3: exact, as signed 4-bit dot
          // products) through the N-S products, and the second stage runs in
          // FP32 on the accumulators; one beam tile (kt) at a time, so that
          // only half of the accumulators are live
          // lane (g, n): sample n at N-S positions 4 g + q (the dwords of
          // fr[g]); per column its 8 (position, re|im) values once per term
          // (times 2^-shift), then 8 zeros, along K = 128
          const uint32_t dq[4] = {d0.x, d0.y, d0.z, d0.w};
          // column pair cp: (S02, S13) gives beams 0 and 2, (D02, D13) beams 1
          // and 3, so only one pair's operands and products are live at a time
#pragma unroll
          for (int cp = 0; cp < 2; ++cp) {
            i32x8 A[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              int wre, wim;
              ew_half_weights(2 * cp + h, wre, wim);
              int v[8];
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                v[2 * q] = sdot8((int)dq[q], wre);
                v[2 * q + 1] = sdot8((int)dq[q], wim);
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
              f32x4 acc[2][2];
#pragma unroll
              for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int part = 0; part < 2; ++part)
                  acc[h][part] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                      A[h], B8[kt][part], f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0, 0x7F7F7F7F, 0, 0x7F7F7F7F);
              // second E-W stage: B_0 = S02 + S13, B_2 = S02 - S13 (cp = 0),
              // B_1 = D02 - i D13, B_3 = D02 + i D13 (cp = 1); |B|^2, sum of
              // the lane's 4 samples
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const float ar = acc[0][0][i], ai = acc[0][1][i];
                const float br = acc[1][0][i], bi = acc[1][1][i];
                if (cp == 0) {
                  ia[0][kt] = cnorm_acc(cf{ar + br, ai + bi}, ia[0][kt]);
                  ia[2][kt] = cnorm_acc(cf{ar - br, ai - bi}, ia[2][kt]);
                } else {
                  ia[1][kt] = cnorm_acc(cf{ar + bi, ai - br}, ia[1][kt]);
                  ia[3][kt] = cnorm_acc(cf{ar - bi, ai + br}, ia[3][kt]);
                }
              }
            }
          }
        }
      }
    }

    // sum the four sample groups (lanes l, l^16, l^32, l^48)
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int kt = 0; kt < 2; ++kt) {
        float v = ia[e][kt];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        ia[e][kt] = v;
      }
    if (g == 0) {
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int kt = 0; kt < 2; ++kt) lds_i[e * 32 + kt * 16 + n] = ia[e][kt] * (a.norm * unscale);
    }
    __syncthreads();
    float* o = a.out + ((blk * a.n_chan + chan) * a.n_pg + pg) * 4 * keep;
#pragma unroll
    for (int it = 0; it < 2; ++it)
      if (lane + 64 * it < 4 * keep) o[lane + 64 * it] = lds_i[gsrc[it]];
    __syncthreads();
  }
}

// ---- 4 x 32, 4 x 64, 4 x 128: polyphase split onto the 16 -> 32 products ----
//
// With n = 16 R N-S positions (R = 2, 4, 8) and M = 2 n = 32 R beams:
//   a = R a' + a0   (a' < 16, a0 < R),   A = m + 32 r   (m < 32, r < R)
//   D_a0[m]     = sum_{a'} x[R a' + a0] W_32^{a' m}              (matrix cores)
//   Y[m + 32 r] = sum_{a0} (W_M^{a0 m} D_a0[m]) W_R^{a0 r}        (FP32)
// since W_M^{a A} = W_32^{a' m} W_M^{a0 m} W_R^{a0 r}.  Each D_a0 is the
// zero-padded 16 -> 32 transform above, with the same operand tables, on the
// dwords of one polyphase (stride R); the accumulator layout puts every
// D_a0[m] of one (sample, m) in one lane, so the twiddles W_M^{a0 m} (FP64-
// generated, rounded to FP32) and the R-point DFT over a0 run in that lane.
// |B|^2 is summed over the lane's four samples, then over the four sample
// groups by cross-lane adds, and each sum lands in the LDS in a slot that one
// lane owns.
// FP8: e4m3 holds every integer up to 16 but not every E-W sum, so the data
// operand takes the first radix-2 stage of the E-W DFT only (x0 +- x2 and
// x1 +- x3, exact) and the second stage runs in FP32 on the accumulators:
//   B_0 = S02 + S13,  B_2 = S02 - S13,  B_1 = D02 - i D13,  B_3 = D02 + i D13.
// Below R = 8 one pass makes both E-W beams of a pair from the same four
// products; at R = 8 each pass makes one (fewer live registers).
constexpr size_t kMixTwOff = 8192;   // twiddles after the 16 -> 32 operand table

// W_M^{a0 m} with M = 32 R, as float2 at [m][a0]
__global__ void k_mixp_twiddles(void* tab, int R) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 32 * R) return;
  const int m = i / R, a0 = i % R;
  double s, c;
  sincospi(-2.0 * (double)((a0 * m) % (32 * R)) / (double)(32 * R), &s, &c);
  reinterpret_cast<float2*>(static_cast<char*>(tab) + kMixTwOff)[i] = make_float2((float)c, (float)s);
}

template <int PREC, int R, bool WIN>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(R == 2 ? 4 : R == 4 && PREC == kPrecFp16 ? 3 : 2))) void k_mixp(MixArgs a) {
  static_assert(!WIN || PREC == kPrecFp16, "windows run on the FP16 path");
  constexpr int N = 16 * R, M = 2 * N;
  constexpr bool PAIR = PREC == kPrecFp8 && R <= 4;
  constexpr int NE = PAIR ? 2 : 1;               // E-W beams per pass
  constexpr int NPASS = PAIR ? 2 : 4;
  constexpr int NDW = PREC == kPrecFp16 ? 8 * R : 4 * R;   // dwords per lane per sample
  constexpr int P = Mix<PREC>::P;
  using op_t = typename Mix<PREC>::op_t;
  __shared__ float lds_i[4 * M];

  const int lane = threadIdx.x;
  const int n = lane & 15, g = lane >> 4;
  int wg = blockIdx.x;
  const int pg = wg % a.n_pg;
  wg /= a.n_pg;
  const int chan = wg % a.n_chan;
  const int run = wg / a.n_chan;
  const int64_t n_blk = a.n_time / a.block;
  const int64_t blk0 = (int64_t)run * kMixBlocksPerWave;
  const int64_t blk1 = blk0 + kMixBlocksPerWave < n_blk ? blk0 + kMixBlocksPerWave : n_blk;

  // operand columns of both beam tiles (m = 16 kt + n) in registers, the
  // twiddles W_M^{a0 m} in the LDS
  __shared__ float2 lds_tw[32 * R];
  op_t B[2][PREC == kPrecFp16 ? P : 1][2];
  i32x8 B8[2][2];
  {
    const float2* twt = reinterpret_cast<const float2*>(static_cast<const char*>(a.mat) + kMixTwOff);
    for (int i = lane; i < 32 * R; i += 64) lds_tw[i] = twt[i];
#pragma unroll
    for (int kt = 0; kt < 2; ++kt) {
#pragma unroll
      for (int part = 0; part < 2; ++part) {
        if constexpr (PREC == kPrecFp16) {
#pragma unroll
          for (int p = 0; p < P; ++p) B[kt][p][part] = load_b<PREC>(a.mat, p, kt, part, lane);
        } else {
          B8[kt][part] = *reinterpret_cast<const i32x8*>(static_cast<const uint8_t*>(a.mat) +
                                                          ((kt * 2 + part) * 64 + lane) * 32);
        }
      }
    }
  }

  const int comp = g >> 1;                 // FP16: the lane's component of the data operand

  // WIN: component `comp` of (-i)^k z is s_k * (nibble at offset o_k) with
  // comp 0: (+Re, +Im, -Re, -Im), comp 1: (+Im, -Re, -Im, +Re) for k = 0..3
  float wsg[4];
  int woff[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int kk = (k + comp) & 3;         // comp 1 is comp 0 of (-i) w
    wsg[k] = kk < 2 ? 1.f : -1.f;
    woff[k] = (kk & 1) ? 0 : 4;
  }
  float wscale = 1.f, unscale = 1.f;       // 2^-E on the window, 2^{2E} back on |B|^2
  if constexpr (WIN) {
    float mx = 0.f;
    for (int i = lane; i < 4 * N; i += 64) mx = fmaxf(mx, fabsf(a.taper[i]));
#pragma unroll
    for (int d = 1; d < 64; d *= 2) mx = fmaxf(mx, __shfl_xor(mx, d));
    const int ex = mx > 0.f ? ilogbf(mx) + 1 : 0;
    wscale = ldexpf(1.f, -ex);
    unscale = ldexpf(1.f, 2 * ex);
  }

  const int pol_lo = (a.pol_iter == 1) ? pg : 0;
  const int pol_hi = (a.pol_iter == 1) ? pg + 1 : a.n_pol;
  const int keep = a.n_keep;
  const int32_t* sel = a.sel ? a.sel + (int64_t)chan * keep : nullptr;

  for (int i = lane; i < 4 * M; i += 64) lds_i[i] = 0.f;
  __syncthreads();

  for (int64_t blk = blk0; blk < blk1; ++blk) {
    for (int pol = pol_lo; pol < pol_hi; ++pol) {
      for (int sub = 0; sub < a.block; sub += 16) {
        const int64_t t = blk * a.block + sub + n;
        const uint32_t* frame = a.volts + ((t * a.n_chan + chan) * a.n_pol + pol) * N;
        // FP16: positions R a' + a0 with a' in [8 (g & 1), + 8); FP8: a' in [4 g, + 4)
        const uint4* fr = reinterpret_cast<const uint4*>(frame + (PREC == kPrecFp16 ? 8 * R * (g & 1) : 4 * R * g));
        uint32_t dw[NDW];
#pragma unroll
        for (int k = 0; k < NDW / 4; ++k) {
          const uint4 d = fr[k];
          dw[4 * k] = d.x;
          dw[4 * k + 1] = d.y;
          dw[4 * k + 2] = d.z;
          dw[4 * k + 3] = d.w;
        }

        // one pass per E-W beam (FP8 below R = 8: per pair), not unrolled:
        // the passes share no values, and one at a time bounds the registers
#pragma unroll 1
        for (int ps = 0; ps < NPASS; ++ps) {
          const int wt = ew_dot_weights(ps, comp);           // FP16: E-W dot8 weights
          int cwr[2], cwi[2];                                 // FP8: the pair's first-stage sums
          ew_half_weights(2 * (ps & 1), cwr[0], cwi[0]);
          ew_half_weights(2 * (ps & 1) + 1, cwr[1], cwi[1]);
          // the beam tiles m < 16 and m >= 16 in turn (not unrolled either; the
          // tile's operands are picked from the registers by a uniform select)
#pragma unroll 1
          for (int kt = 0; kt < 2; ++kt) {
            if constexpr (WIN) {
              // the windowed sums are formed per tile: without this the compiler
              // converts every nibble of the frame ahead of the loops and holds them
#pragma unroll
              for (int k = 0; k < NDW; ++k) asm volatile("" : "+v"(dw[k]));
            }
            const auto& Bt = kt ? B[1] : B[0];
            const auto& B8t = kt ? B8[1] : B8[0];
            cf twk[R];
#pragma unroll
            for (int a0 = 1; a0 < R; ++a0) {
              const float2 v = lds_tw[(16 * kt + n) * R + a0];
              twk[a0] = cf{v.x, v.y};
            }
            cf y[NE][R][4];
#pragma unroll
            for (int a0 = 0; a0 < R; ++a0) {
              if constexpr (WIN) __builtin_amdgcn_sched_barrier(0);   // one polyphase's loads at a time
              if constexpr (PREC == kPrecFp16 && !WIN) {
                uint32_t sdw[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) sdw[j] = dw[R * j + a0];
                const half8 A = ew_sums_f16(sdw, wt);
                f32x4 c[2];
#pragma unroll
                for (int part = 0; part < 2; ++part) {
                  c[part] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                  for (int p = 0; p < P; ++p) c[part] = mfma<PREC>(A, Bt[p][part], c[part]);
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) y[0][a0][i] = cf{c[0][i], c[1][i]};
              } else if constexpr (WIN) {
                // windowed E-W sum of beam ps, component comp, at the lane's
                // eight positions of polyphase a0, scaled by 2^-E
                float xv[8];
                // the window is loop-invariant: reading it here again (through a
                // pointer the compiler cannot follow) keeps it out of registers
                const float* tp = a.taper;
                asm volatile("" : "+s"(tp));
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                  const int pos = R * (8 * (g & 1) + j) + a0;
                  const float4 h = *reinterpret_cast<const float4*>(tp + 4 * pos);
                  const float hq[4] = {h.x, h.y, h.z, h.w};
                  float s = 0.f;
#pragma unroll
                  for (int q = 0; q < 4; ++q) {
                    const int k = (ps * q) & 3;
                    const float v = (float)(int)__builtin_amdgcn_sbfe((int)dw[R * j + a0], 8 * q + woff[k], 4);
                    s = fmaf(hq[q] * wsg[k], v, s);
                  }
                  xv[j] = s * wscale;
                }
                uint32_t hi[4], lo[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) split2(xv[2 * j], xv[2 * j + 1], hi[j], lo[j]);
                const half8 Ah = __builtin_bit_cast(half8, hi), Al = __builtin_bit_cast(half8, lo);
                f32x4 c[2];
#pragma unroll
                for (int part = 0; part < 2; ++part) {
                  c[part] = mfma<PREC>(Ah, Bt[0][part], f32x4{0.f, 0.f, 0.f, 0.f});
                  c[part] = mfma<PREC>(Ah, Bt[1][part], c[part]);
                  c[part] = mfma<PREC>(Al, Bt[0][part], c[part]);
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) y[0][a0][i] = cf{c[0][i], c[1][i]};
              } else {
                // FP8: the two first-stage columns of pair ep at the lane's
                // four positions R (4 g + q) + a0, three scaled terms along K
                const int ep = ps & 1;
                f32x4 c[2][2];
#pragma unroll
                for (int cc = 0; cc < 2; ++cc) {
                  int v[8];
#pragma unroll
                  for (int q = 0; q < 4; ++q) {
                    v[2 * q] = sdot8((int)dw[R * q + a0], cwr[cc]);
                    v[2 * q + 1] = sdot8((int)dw[R * q + a0], cwi[cc]);
                  }
                  i32x8 A;
#pragma unroll
                  for (int p = 0; p < 3; ++p) {
                    const long w = to_fp8(v, 1.0f / (float)(1 << fp8_shift(p)));
                    A[2 * p] = (int)w;
                    A[2 * p + 1] = (int)(w >> 32);
                  }
                  A[6] = 0;
                  A[7] = 0;
#pragma unroll
                  for (int part = 0; part < 2; ++part)
                    c[cc][part] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                        A, B8t[part], f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0, 0x7F7F7F7F, 0, 0x7F7F7F7F);
                }
                // second E-W stage: pair 0 gives beams 0 (sum) and 2 (difference),
                // pair 1 beams 1 (D02 - i D13) and 3 (D02 + i D13)
#pragma unroll
                for (int w = 0; w < NE; ++w) {
                  const int up = PAIR ? w : (ps >> 1);     // 0: beam ep, 1: beam ep + 2
#pragma unroll
                  for (int i = 0; i < 4; ++i) {
                    const float ar = c[0][0][i], ai = c[0][1][i], br = c[1][0][i], bi = c[1][1][i];
                    if (ep == 0) y[w][a0][i] = up ? cf{ar - br, ai - bi} : cf{ar + br, ai + bi};
                    else y[w][a0][i] = up ? cf{ar - bi, ai + br} : cf{ar + bi, ai - br};
                  }
                }
              }
            }
            // twiddle, R-point DFT over a0, |B|^2 over the lane's four samples
#pragma unroll
            for (int w = 0; w < NE; ++w) {
              const int e = PAIR ? (ps & 1) + 2 * w : ps;
              float v[R];
#pragma unroll
              for (int r = 0; r < R; ++r) v[r] = 0.f;
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                cf z[R];
                z[0] = y[w][0][i];
#pragma unroll
                for (int a0 = 1; a0 < R; ++a0) z[a0] = cmul(y[w][a0][i], twk[a0]);
                dit<R>(z);
#pragma unroll
                for (int r = 0; r < R; ++r) v[r] = cnorm_acc(z[r], v[r]);
              }
              // sum the four sample groups; lane group g adds r = g, g + 4, ... to
              // the LDS (masked per r, so that no register array is indexed at
              // run time; one lane per slot, so the adds need no ordering)
#pragma unroll
              for (int r = 0; r < R; ++r) {
                v[r] += __shfl_xor(v[r], 16);
                v[r] += __shfl_xor(v[r], 32);
                if ((r & 3) == g) atomicAdd(&lds_i[e * M + 16 * kt + n + 32 * r], v[r]);   // no return value
              }
            }
          }
        }
      }
    }
    __syncthreads();
    float* o = a.out + ((blk * a.n_chan + chan) * a.n_pg + pg) * 4 * keep;
    for (int idx = lane; idx < 4 * keep; idx += 64) {
      const int e = idx / keep, j = idx - e * keep;
      o[idx] = lds_i[e * M + (sel ? sel[j] : j)] * (a.norm * unscale);
    }
    __syncthreads();
    for (int i = lane; i < 4 * M; i += 64) lds_i[i] = 0.f;
    __syncthreads();
  }
}

}  // namespace

// polyphase factor R of the 4 x 16 R lattices (0: not one of them)
static int mixp_r(int n_ns) { return n_ns == 32 ? 2 : n_ns == 64 ? 4 : n_ns == 128 ? 8 : 0; }

bool mix_window_supported(int n_ns, int prec) {
  return (n_ns == 16 || mixp_r(n_ns) || n_ns == 256) && prec == kPrecFp16;
}

bool mix_supported(int n_ns, int prec, int block) {
  if (n_ns == 16 || mixp_r(n_ns)) return (prec == kPrecFp16 || prec == kPrecFp8) && block % 16 == 0;
  if (n_ns == 256) return (prec == kPrecFp16 || prec == kPrecFp8) && block >= 1;
  return false;
}

size_t mix_table_bytes(int n_ns, int prec) {
  if (n_ns == 256) return mix256_table_bytes();
  const size_t base = prec == kPrecFp16 ? (size_t)Mix<kPrecFp16>::P * 2048 * 2 : (size_t)2 * 2 * 64 * 32;
  static_assert(kMixTwOff == 8192, "twiddles follow the operand table of either precision");
  return mixp_r(n_ns) ? kMixTwOff + sizeof(float2) * 32 * mixp_r(n_ns) : base;
}

hipError_t launch_mix_tables(void* mat, int n_ns, int prec, hipStream_t s) {
  if (!mix_supported(n_ns, prec, 16)) return hipErrorNotSupported;
  if (n_ns == 256) return launch_mix256_tables(mat, prec, s);
  if (prec == kPrecFp16) hipLaunchKernelGGL(k_mix_tables<kPrecFp16>, dim3(8), dim3(256), 0, s, mat);
  else hipLaunchKernelGGL(k_mix_tables<kPrecFp8>, dim3(8), dim3(256), 0, s, mat);
  if (const int r = mixp_r(n_ns)) hipLaunchKernelGGL(k_mixp_twiddles, dim3(1), dim3(256), 0, s, mat, r);
  return hipGetLastError();
}

template <int R>
static void launch_mixp(const MixArgs& a, int prec, unsigned n_wg, hipStream_t s) {
  if (prec == kPrecFp16 && a.taper) hipLaunchKernelGGL((k_mixp<kPrecFp16, R, true>), dim3(n_wg), dim3(64), 0, s, a);
  else if (prec == kPrecFp16) hipLaunchKernelGGL((k_mixp<kPrecFp16, R, false>), dim3(n_wg), dim3(64), 0, s, a);
  else hipLaunchKernelGGL((k_mixp<kPrecFp8, R, false>), dim3(n_wg), dim3(64), 0, s, a);
}

hipError_t launch_mix(const MixArgs& a, int n_ns, int prec, int64_t n_wg_blocks, hipStream_t s) {
  if (!mix_supported(n_ns, prec, a.block) || (a.taper && !mix_window_supported(n_ns, prec)))
    return hipErrorNotSupported;
  if (n_ns == 256) return launch_mix256(a, prec, n_wg_blocks, s);
  const int64_t n_blk = a.n_time / a.block;
  const int64_t n_run = (n_blk + kMixBlocksPerWave - 1) / kMixBlocksPerWave;
  const int64_t n_wg = n_run * a.n_chan * a.n_pg;
  if (n_wg == 0) return hipSuccess;
  if (n_wg > 0x7FFFFFFF) return hipErrorInvalidConfiguration;
  switch (n_ns) {
    case 32: launch_mixp<2>(a, prec, (unsigned)n_wg, s); return hipGetLastError();
    case 64: launch_mixp<4>(a, prec, (unsigned)n_wg, s); return hipGetLastError();
    case 128: launch_mixp<8>(a, prec, (unsigned)n_wg, s); return hipGetLastError();
    default: break;
  }
  if (prec == kPrecFp16 && a.taper) hipLaunchKernelGGL((k_mix16<kPrecFp16, true>), dim3((unsigned)n_wg), dim3(64), 0, s, a);
  else if (prec == kPrecFp16) hipLaunchKernelGGL(k_mix16<kPrecFp16>, dim3((unsigned)n_wg), dim3(64), 0, s, a);
  else hipLaunchKernelGGL(k_mix16<kPrecFp8>, dim3((unsigned)n_wg), dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace fftbf
