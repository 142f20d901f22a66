// Tied-array (pointed) beams at arbitrary directions by interpolating the
// complex FFT beams.
//
// Substituting the zero-padded inverse transform
//   eta_a = (sqrt(n)/M) sum_A B_A exp(+i 2 pi A a / M),   a < n,
// into the pointed weights of eq. e:c_pointed gives, per axis,
//   B_p = sum_A c_A(y) B_A,   c_A(y) = (1/M) sum_{a<n} exp(+i 2 pi a (A/M - y)),
// exact whenever M >= n -- the voltage-domain counterpart of the intensity
// regridding of eq. e:bp_max_arbitrary, which needs M >= 2n - 1.  The
// weights are generated in FP64 on the device (the series is summed term by
// term with a unit-modulus recurrence, so on-grid pointings need no 0/0
// limit) and applied in FP32.
//
// One 64-lane wavefront per (pointing tile, channel, polarisation group,
// run of time blocks); lane = pointing.  Every lane of a wave reads the same
// FFT beam at the same time, so beam reads are wave-uniform (scalar loads
// from the complex-beam array, LDS broadcasts in the voltage variant).
#include "dev_common.h"
#include "dev_f16.h"
#include "kernels.h"

namespace fftbf {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kTiedBlocksPerWg = 16;

template <int M>
__device__ __forceinline__ void interp_weights(double y, int n, cf* c) {
#pragma unroll
  for (int A = 0; A < M; ++A) {
    const double u = (double)A / (double)M - y;
    double s, co;
    sincospi(2.0 * u, &s, &co);
    double wr = 1.0, wi = 0.0, ar = 0.0, ai = 0.0;
    for (int a = 0; a < n; ++a) {
      ar += wr;
      ai += wi;
      const double t = wr * co - wi * s;
      wi = wr * s + wi * co;
      wr = t;
    }
    c[A] = cf{(float)(ar / M), (float)(ai / M)};
  }
}

template <int MNS>
__device__ __forceinline__ cf interp_one(const cf* __restrict__ b /* [4][MNS] */, const cf* cew, const cf* cns) {
  cf bp{0.f, 0.f};
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    float zr = 0.f, zi = 0.f;
#pragma unroll
    for (int A = 0; A < MNS; ++A) {
      const cf v = b[e * MNS + A];
      zr = fmaf(cns[A].r, v.r, zr);
      zr = fmaf(-cns[A].i, v.i, zr);
      zi = fmaf(cns[A].r, v.i, zi);
      zi = fmaf(cns[A].i, v.r, zi);
    }
    bp.r = fmaf(cew[e].r, zr, fmaf(-cew[e].i, zi, bp.r));
    bp.i = fmaf(cew[e].r, zi, fmaf(cew[e].i, zr, bp.i));
  }
  return bp;
}

template <int MNS>
__global__ __launch_bounds__(64) void k_tied(TiedArgs a) {
  const int lane = threadIdx.x;
  const int n_ptile = (a.n_point + 63) / 64;
  const int n_pg = a.pol_sum ? 1 : a.n_pol;
  int wg = blockIdx.x;
  const int ptile = wg % n_ptile;
  wg /= n_ptile;
  const int trun = wg;                     // run of kTiedBlocksPerWg blocks
  const int cs = blockIdx.y, pg = blockIdx.z;
  const int chan = a.chan_lo + cs;
  const int p = ptile * 64 + lane;
  const bool live = p < a.n_point;
  const int pp = live ? p : a.n_point - 1;

  cf cew[4], cns[MNS];
  {
    const double dl_ew = a.dl[2 * chan], dl_ns = a.dl[2 * chan + 1];
    interp_weights<4>(dl_ew * a.dircos[2 * pp], a.n_ew, cew);
    interp_weights<MNS>(dl_ns * a.dircos[2 * pp + 1], a.n_ns, cns);
  }
  const int pol_lo = a.pol_sum ? 0 : pg, pol_hi = a.pol_sum ? a.n_pol : pg + 1;
  const int64_t span = (int64_t)(a.complex_out ? 16 : a.block) * kTiedBlocksPerWg;
  const int64_t t0 = (int64_t)trun * span;
  const int64_t t1 = t0 + span < a.n_time ? t0 + span : a.n_time;

  if (a.complex_out) {
    for (int64_t t = t0; t < t1; ++t) {
      const cf* b = reinterpret_cast<const cf*>(a.beams) + ((t * a.n_chan + chan) * a.n_pol + pg) * 4 * MNS;
      const cf bp = interp_one<MNS>(b, cew, cns);
      if (live) {
        float2* o = static_cast<float2*>(a.out) + ((t * a.n_chan_sub + cs) * a.n_pol + pg) * (int64_t)a.n_point + p;
        *o = make_float2(bp.r, bp.i);
      }
    }
    return;
  }
  for (int64_t tb = t0; tb < t1; tb += a.block) {
    float acc = 0.f;
    for (int t = 0; t < a.block; ++t) {
      for (int pol = pol_lo; pol < pol_hi; ++pol) {
        const cf* b = reinterpret_cast<const cf*>(a.beams) +
                      (((tb + t) * a.n_chan + chan) * a.n_pol + pol) * 4 * MNS;
        acc += cnorm(interp_one<MNS>(b, cew, cns));
      }
    }
    if (live) {
      const int64_t blk = tb / a.block;
      float* o = static_cast<float*>(a.out) + ((blk * a.n_chan_sub + cs) * n_pg + pg) * (int64_t)a.n_point + p;
      *o = acc;
    }
  }
}

// Voltage variant for the 4 x 16 lattice (M_ns = 32): per group of 16
// samples the wave forms the 4 x 32 FFT beams of each sample in LDS (lane =
// (sample, E-W beam): two signed 4-bit dot products per N-S position for the
// E-W DFT, then the zero-padded 32-point N-S DFT in registers), then every
// lane interpolates its own pointing from LDS broadcasts.
constexpr int kV16N = 16, kV16M = 32, kV16TS = 16;

struct V16Lane {
  int ts, e, wre, wim;
};

__device__ __forceinline__ V16Lane v16_lane(int lane) {
  V16Lane l;
  l.ts = lane >> 2;
  l.e = lane & 3;
  l.wre = 0;
  l.wim = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int k = (l.e * q) & 3;
    const int sr = 4 * (2 * q + 1), si = 4 * (2 * q);
    if (k == 0) { l.wre |= 1 << sr;   l.wim |= 1 << si; }
    if (k == 1) { l.wre |= 1 << si;   l.wim |= 0xF << sr; }
    if (k == 2) { l.wre |= 0xF << sr; l.wim |= 0xF << si; }
    if (k == 3) { l.wre |= 0xF << si; l.wim |= 1 << sr; }
  }
  return l;
}

// The interpolation of a group of 16 samples runs on the FP16 matrix cores
// (v_mfma_f32_16x16x32_f16) with two-term operands:
//   Out[s][p] = sum_k A[s][k] W[k][p] ~ sum_k (A_hi W_hi + A_lo W_hi + A_hi W_lo),
// A = hi + lo and W = hi + lo split in FP16, so each term carries ~22
// significant bits and only the lo x lo product (~2^-22 relative) is
// dropped; products are exact and accumulate in FP32.  k = 2 beam + (re|im)
// over the 128 FFT beams (beam = 32 e + A_ns); the Re and Im parts of Out
// are two products with the same A operand:
//   W_re[2b][p] = Re c_b, W_re[2b+1][p] = -Im c_b,  W_im[2b][p] = Im c_b,
//   W_im[2b+1][p] = Re c_b.
// The FFT beams are scaled by 2^ds and the weights by 2^10 before the split
// (powers of two, exact), so that the low terms stay in FP16's normal range;
// the block sum of |Out|^2 is scaled back by 2^-2(ds+10).
//
// LDS operand layout of one group (FP16, 16 KB): [hi|lo][kb 8][g 4][s 16][j 8]
// with k = 32 kb + 8 g + j, so lane (s, g) of the A operand reads its eight
// values of k-block kb as one 16-byte load.
constexpr int kV16Wscale = 10;

// |FFT beam| <= (1/8) * 64 antennas * |h|max * 8 sqrt(2) on the 4 x 16 lattice;
// the largest power of two keeping the scaled beams below 2^15.
__device__ __forceinline__ int v16_data_scale(float hmax) {
  if (!(hmax > 0.f)) return 8;
  int e;
  frexpf(32768.f / (90.51f * hmax), &e);
  return e - 1;
}

// This lane's frame of one group: the kV16N dwords of sample l.ts (the
// voltages need only 4-byte alignment).
__device__ __forceinline__ void v16_load(const uint32_t* __restrict__ src, uint32_t (&dw)[kV16N]) {
#pragma unroll
  for (int j = 0; j < kV16N; ++j) dw[j] = src[j];
}

// FFT beams of the 16 samples whose frames the lanes hold (lane = sample
// l.ts, E-W beam l.e), normalised by 1/sqrt(64), scaled by 2^ds and split
// into the FP16 operand layout above.
// LDS position (16-byte chunk) of the operand vector (term, kb, g, sample s)
// of one group.  For the FFT beams formed on chip the sample index is
// XOR-swizzled so that the 16 lanes of one LDS pass land on 16 different bank
// groups, for the readers (16 consecutive s, fixed (kb, g)) and for the
// writers (the lanes of a pass differ in E-W beam, kb = 2 e + c / 4, which
// s ^ 4 (kb >> 1) spreads).  The stored-beam layout stays plain: its
// swizzle (s ^ ((4 kb + g) mod 16), lane-dependent) took the kernel past 256
// registers, to one wavefront per SIMD, and ran 1.9 against 1.5 ms.
__device__ __forceinline__ int v16_chunk(int term, int kb, int g, int s) {
  return ((term * 8 + kb) * 4 + g) * 16 + (s ^ ((kb >> 1) << 2));
}
__device__ __forceinline__ int b16_chunk(int term, int kb, int g, int s) {
  return ((term * 8 + kb) * 4 + g) * 16 + s;
}

template <bool TAPER>
__device__ __forceinline__ void v16_fft_to_lds(const uint32_t (&dw)[kV16N], const V16Lane& l,
                                               const float* lds_h, _Float16* lds_g, int ds) {
  constexpr int N = kV16N, MNS = kV16M;
  cf x[N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const uint32_t d = dw[j];
    if constexpr (TAPER) {
      float re = 0.f, im = 0.f;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = (l.e * q) & 3;
        const float h = lds_h[j * 4 + q];
        const float xr = (float)(int)__builtin_amdgcn_sbfe((int)d, 8 * q + 4, 4) * h;
        const float xi = (float)(int)__builtin_amdgcn_sbfe((int)d, 8 * q, 4) * h;
        // x * (-i)^k
        const float ur = (k == 0) ? xr : (k == 1) ? xi : (k == 2) ? -xr : -xi;
        const float ui = (k == 0) ? xi : (k == 1) ? -xr : (k == 2) ? -xi : xr;
        re += ur;
        im += ui;
      }
      x[j] = cf{re, im};
    } else {
      x[j] = cf{(float)sdot8((int)d, l.wre), (float)sdot8((int)d, l.wim)};
    }
  }
  cf y[MNS];
  padded_dft<N>(x, y);
  const float nrm = ldexpf(0.125f, ds);   // 2^ds / sqrt(4 * 16)
#pragma unroll
  for (int c = 0; c < MNS / 4; ++c) {     // four beams A = 4c .. 4c+3 per 16-byte vector
    uint32_t hw[4], lw[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) split2(y[4 * c + q].r * nrm, y[4 * c + q].i * nrm, hw[q], lw[q]);
    const int kb = 2 * l.e + c / 4, g = c % 4;
    *reinterpret_cast<half8*>(lds_g + v16_chunk(0, kb, g, l.ts) * 8) = __builtin_bit_cast(half8, hw);
    *reinterpret_cast<half8*>(lds_g + v16_chunk(1, kb, g, l.ts) * 8) = __builtin_bit_cast(half8, lw);
  }
}

// (1/m) sum_{a<n} z^a for |z| = 1 and n a power of two, as the product
// (1 + z)(1 + z^2)(1 + z^4)... of log2 n factors (z^2k by squaring): no
// singular point, log2 n complex products instead of n terms.
__device__ __forceinline__ void geom_pow2(double zr, double zi, int n, int m, double* wr_out, double* wi_out) {
  double ar = 1.0 + zr, ai = zi;
  for (int k = 2; k < n; k <<= 1) {
    const double t = zr * zr - zi * zi;
    zi = 2.0 * zr * zi;
    zr = t;
    const double fr = 1.0 + zr;
    const double q = ar * fr - ai * zi;
    ai = ar * zi + ai * fr;
    ar = q;
  }
  *wr_out = ar / m;
  *wi_out = ai / m;
}

// Interpolation weight c_A(y) = (1/m) sum_{a<n} z^a, z = e^{2 pi i (A/m - y)},
// of one FFT beam, in FP64: the product above for n a power of two, else the
// series summed term by term with a unit-modulus recurrence.
__device__ __forceinline__ void interp_weight_d(int A, int m, int n, double y, double* wr_out, double* wi_out) {
  const double u = (double)A / (double)m - y;
  double s, co;
  sincospi(2.0 * u, &s, &co);
  if (n >= 2 && (n & (n - 1)) == 0) {
    geom_pow2(co, s, n, m, wr_out, wi_out);
    return;
  }
  double wr = 1.0, wi = 0.0, ar = 0.0, ai = 0.0;
  for (int a = 0; a < n; ++a) {
    ar += wr;
    ai += wi;
    const double t = wr * co - wi * s;
    wi = wr * s + wi * co;
    wr = t;
  }
  *wr_out = ar / m;
  *wi_out = ai / m;
}

// B operands of one pointing (lane column p = l % 16, k rows 8 g .. 8 g + 7 of
// every k-block, g = l / 16): Re and Im parts, high and low FP16 terms.
struct TiedW {
  half8 rh[8], rl[8], ih[8], il[8];
};

// e^{i pi j / 16}, j < 4, and e^{i pi g / 4}, g < 4, as the nearest doubles
__device__ __constant__ double kRot16[4][2] = {{1.0, 0.0},
                                               {0.9807852804032304, 0.19509032201612825},
                                               {0.9238795325112867, 0.3826834323650898},
                                               {0.8314696123025452, 0.5555702330196022}};
__device__ __constant__ double kRot4[4][2] = {{1.0, 0.0},
                                              {0.7071067811865476, 0.7071067811865476},
                                              {0.0, 1.0},
                                              {-0.7071067811865476, 0.7071067811865476}};

__device__ __forceinline__ void tied_weights(double y_ew, double y_ns, int g, TiedW& w) {
  static_assert(kV16M == 32 && kV16N == 16, "the 4 x 16 lattice's beams");
  // E-W: z_e = e^{2 pi i (e/4 - y)} = i^e b with b = e^{-2 pi i y} (one
  // sine and cosine per pointing)
  double ewr[4], ewi[4];
  {
    double bs, bc;
    sincospi(-2.0 * y_ew, &bs, &bc);
    geom_pow2(bc, bs, 4, 4, &ewr[0], &ewi[0]);
    geom_pow2(-bs, bc, 4, 4, &ewr[1], &ewi[1]);
    geom_pow2(-bc, -bs, 4, 4, &ewr[2], &ewi[2]);
    geom_pow2(bs, -bc, 4, 4, &ewr[3], &ewi[3]);
  }
  // N-S: this lane's k rows hold beams 16 kb + 4 g + jj (jj < 4), N-S beams
  // A = 16 h + 4 g + jj, and z_A = e^{2 pi i (A/32 - y)} =
  // (-1)^h e^{i pi g/4} e^{i pi jj/16} c with c = e^{-2 pi i y}
  double nsr[2][4], nsi[2][4];
  {
    double cs, cc;
    sincospi(-2.0 * y_ns, &cs, &cc);
    const double gr = kRot4[g][0], gi = kRot4[g][1];
    const double dr = gr * cc - gi * cs, di = gr * cs + gi * cc;
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const double rr = kRot16[jj][0], ri = kRot16[jj][1];
      const double zr = rr * dr - ri * di, zi = rr * di + ri * dr;
      geom_pow2(zr, zi, kV16N, kV16M, &nsr[0][jj], &nsi[0][jj]);
      geom_pow2(-zr, -zi, kV16N, kV16M, &nsr[1][jj], &nsi[1][jj]);
    }
  }
  const double sc = (double)(1 << kV16Wscale);
#pragma unroll
  for (int kb = 0; kb < 8; ++kb) {
    const int e = kb >> 1, h = kb & 1;
    uint32_t rh[4], rl[4], ih[4], il[4];
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const double cr = (ewr[e] * nsr[h][jj] - ewi[e] * nsi[h][jj]) * sc;
      const double ci = (ewr[e] * nsi[h][jj] + ewi[e] * nsr[h][jj]) * sc;
      split2((float)cr, (float)(-ci), rh[jj], rl[jj]);     // W_re rows 2b, 2b+1
      split2((float)ci, (float)cr, ih[jj], il[jj]);        // W_im rows 2b, 2b+1
    }
    w.rh[kb] = __builtin_bit_cast(half8, rh);
    w.rl[kb] = __builtin_bit_cast(half8, rl);
    w.ih[kb] = __builtin_bit_cast(half8, ih);
    w.il[kb] = __builtin_bit_cast(half8, il);
  }
}

// sum over the group's 16 samples of |Out|^2 for this lane's pointing,
// scaled by 2^2(ds+10) (the same value in every lane of a column)
__device__ __forceinline__ float tied_block_mfma(const _Float16* lds_g, const TiedW& w, int lane) {
  const int s = lane & 15, g = lane >> 4;
  f32x4 cre = {0.f, 0.f, 0.f, 0.f}, cim = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kb = 0; kb < 8; ++kb) {
    const half8 ah = *reinterpret_cast<const half8*>(lds_g + v16_chunk(0, kb, g, s) * 8);
    const half8 al = *reinterpret_cast<const half8*>(lds_g + v16_chunk(1, kb, g, s) * 8);
    cre = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, w.rh[kb], cre, 0, 0, 0);
    cim = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, w.ih[kb], cim, 0, 0, 0);
    cre = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, w.rh[kb], cre, 0, 0, 0);
    cim = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, w.ih[kb], cim, 0, 0, 0);
    cre = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, w.rl[kb], cre, 0, 0, 0);
    cim = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, w.il[kb], cim, 0, 0, 0);
  }
  float v = 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i) v = fmaf(cre[i], cre[i], fmaf(cim[i], cim[i], v));
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}

// As tied_block_mfma, with a power-of-two scale 2^ds[row] per sample row
// (stored FFT beams have no fixed bound): the row's |Out|^2 is scaled back
// by 2^-2(ds + 10) before the sum over the group's samples.
__device__ __forceinline__ float tied_block_mfma_rows(const _Float16* lds_g, const TiedW& w, int lane,
                                                      const int* ds) {
  const int s = lane & 15, g = lane >> 4;
  f32x4 cre = {0.f, 0.f, 0.f, 0.f}, cim = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kb = 0; kb < 8; ++kb) {
    const half8 ah = *reinterpret_cast<const half8*>(lds_g + b16_chunk(0, kb, g, s) * 8);
    const half8 al = *reinterpret_cast<const half8*>(lds_g + b16_chunk(1, kb, g, s) * 8);
    cre = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, w.rh[kb], cre, 0, 0, 0);
    cim = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, w.ih[kb], cim, 0, 0, 0);
    cre = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, w.rh[kb], cre, 0, 0, 0);
    cim = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, w.ih[kb], cim, 0, 0, 0);
    cre = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, w.rl[kb], cre, 0, 0, 0);
    cim = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, w.il[kb], cim, 0, 0, 0);
  }
  float v = 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    v = fmaf(fmaf(cre[i], cre[i], cim[i] * cim[i]), ldexpf(1.f, -2 * (ds[4 * g + i] + kV16Wscale)), v);
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}

// Tied beams from stored complex FFT beams of the 4 x 16 lattice (M_ns = 32)
// on the matrix cores: the k_tied_v16 tile structure, with each wavefront
// loading one group of 16 samples' beams instead of forming them.  A
// sample's 128 complex beams (beam 32 e + A_ns, re|im) are exactly its k
// vector; each lane loads 8 consecutive floats (k = 8 c .. 8 c + 7) with two
// 16-byte loads, consecutive lanes consecutive chunks.  Each sample gets the
// largest power-of-two scale keeping its beams below 2^15 (a max over the 32
// lanes holding it).
__global__ __launch_bounds__(256) void k_tied_b16(TiedArgs a) {
  __shared__ __attribute__((aligned(16))) _Float16 lds_b[4 * 2 * 8 * 4 * 16 * 8];
  __shared__ int lds_ds[4][16];
  constexpr int kBuf = 2 * 8 * 4 * 16 * 8;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int n_ptile = (a.n_point + 63) / 64;
  const int n_pg = a.pol_sum ? 1 : a.n_pol;
  int wg = blockIdx.x;
  const int ptile = wg % n_ptile;
  const int trun = wg / n_ptile;
  const int cs = blockIdx.y, pg = blockIdx.z;
  const int chan = a.chan_lo + cs;
  const int p = ptile * 64 + wave * 16 + (lane & 15);
  const bool live = p < a.n_point;
  const bool wave_live = ptile * 64 + wave * 16 < a.n_point;
  const int pp = live ? p : a.n_point - 1;

  TiedW w;
  if (wave_live) tied_weights(a.dl[2 * chan] * a.dircos[2 * pp], a.dl[2 * chan + 1] * a.dircos[2 * pp + 1], lane >> 4, w);

  const int pol_lo = a.pol_sum ? 0 : pg, pol_hi = a.pol_sum ? a.n_pol : pg + 1;
  const int64_t span = (int64_t)a.block * kTiedBlocksPerWg;
  const int64_t t0 = (int64_t)trun * span;
  const int64_t t1 = t0 + span < a.n_time ? t0 + span : a.n_time;
  const float* beams = reinterpret_cast<const float*>(a.beams);
  const int kbg = lane & 31, kb = kbg >> 2, gq = kbg & 3;

  // this wavefront's group of 16 samples (pol) starting at tw: lane (kbg,
  // half) holds 8 consecutive floats of samples 2 it + half, it < 8
  auto load_group = [&](int64_t tw, int pol, f32x4 (&v)[8][2]) {
#pragma unroll
    for (int it = 0; it < 8; ++it) {
      const int s = 2 * it + (lane >> 5);
      const float* src = beams + (((tw + s) * a.n_chan + chan) * a.n_pol + pol) * 256 + 8 * kbg;
      v[it][0] = *reinterpret_cast<const f32x4*>(src);
      v[it][1] = *reinterpret_cast<const f32x4*>(src + 4);
    }
  };
  // The next group's beams are loaded into registers while the matrix
  // cores interpolate the current quad, so the loads overlap that work.
  f32x4 nv[8][2];
  {
    const int64_t tw = t0 + kV16TS * wave;
    if (tw < t1) {
      load_group(tw, pol_lo, nv);
    } else {
#pragma unroll
      for (int it = 0; it < 8; ++it) nv[it][0] = nv[it][1] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  }

  // groups of kV16TS samples per block, and the block being summed (a
  // workgroup's span starts at a block boundary)
  const int gpb = a.block / kV16TS;
  int gcnt = 0;
  int64_t blk = (int64_t)trun * kTiedBlocksPerWg;
  float acc = 0.f;
  for (int64_t tq = t0; tq < t1; tq += 4 * kV16TS) {
    float accg[4] = {0.f, 0.f, 0.f, 0.f};
    for (int pol = pol_lo; pol < pol_hi; ++pol) {
      const int64_t tw = tq + kV16TS * wave;
      if (tw < t1) {
        _Float16* lds_g = lds_b + wave * kBuf;
#pragma unroll
        for (int it = 0; it < 8; ++it) {
          const int s = 2 * it + (lane >> 5);
          const f32x4 v0 = nv[it][0];
          const f32x4 v1 = nv[it][1];
          float m = fmaxf(fmaxf(fmaxf(fabsf(v0[0]), fabsf(v0[1])), fmaxf(fabsf(v0[2]), fabsf(v0[3]))),
                          fmaxf(fmaxf(fabsf(v1[0]), fabsf(v1[1])), fmaxf(fabsf(v1[2]), fabsf(v1[3]))));
#pragma unroll
          for (int off = 1; off < 32; off <<= 1) m = fmaxf(m, __shfl_xor(m, off));
          int e = 0;
          if (m > 0.f) frexpf(32768.f / m, &e);
          const int ds = m > 0.f ? e - 1 : 0;
          if (kbg == 0) lds_ds[wave][s] = ds;
          const float sc = ldexpf(1.f, ds);
          uint32_t hw[4], lw[4];
          split2(v0[0] * sc, v0[1] * sc, hw[0], lw[0]);
          split2(v0[2] * sc, v0[3] * sc, hw[1], lw[1]);
          split2(v1[0] * sc, v1[1] * sc, hw[2], lw[2]);
          split2(v1[2] * sc, v1[3] * sc, hw[3], lw[3]);
          *reinterpret_cast<half8*>(lds_g + b16_chunk(0, kb, gq, s) * 8) = __builtin_bit_cast(half8, hw);
          *reinterpret_cast<half8*>(lds_g + b16_chunk(1, kb, gq, s) * 8) = __builtin_bit_cast(half8, lw);
        }
      }
      __syncthreads();
      {
        // the next (quad, pol) of this wavefront, if any
        int64_t tn = tq;
        int pn = pol + 1;
        if (pn >= pol_hi) {
          pn = pol_lo;
          tn = tq + 4 * kV16TS;
        }
        const int64_t twn = tn + kV16TS * wave;
        if (tn < t1 && twn < t1) {
          load_group(twn, pn, nv);
        } else {
#pragma unroll
          for (int it = 0; it < 8; ++it) nv[it][0] = nv[it][1] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
      }
      if (wave_live) {
#pragma unroll
        for (int g = 0; g < 4; ++g)
          if (tq + kV16TS * g < t1) accg[g] += tied_block_mfma_rows(lds_b + g * kBuf, w, lane, lds_ds[g]);
      }
      __syncthreads();
    }
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      if (tq + kV16TS * g >= t1) break;
      acc += accg[g];
      if (++gcnt == gpb) {                         // the block's last group
        if (live && lane < 16) {
          float* o = static_cast<float*>(a.out) + ((blk * a.n_chan_sub + cs) * n_pg + pg) * (int64_t)a.n_point + p;
          *o = acc;
        }
        acc = 0.f;
        gcnt = 0;
        ++blk;
      }
    }
  }
}

// Voltage variant on the matrix cores: workgroup = 4 wavefronts = 64
// pointings.  Samples go in quads of 16-sample groups: wavefront w forms the
// FFT beams of group w of the quad in its own LDS buffer, then every
// wavefront interpolates its 16 pointings over all four groups, so no
// wavefront waits while another forms beams.
constexpr int kV16Buf = 2 * 8 * 4 * 16 * 8;          // FP16 values per group buffer (16 KB)

template <bool TAPER>
__global__ __launch_bounds__(256) void k_tied_v16(TiedArgs a) {
  __shared__ __attribute__((aligned(16))) _Float16 lds_b[4 * kV16Buf];
  __shared__ float lds_h[TAPER ? kV16N * 4 : 1];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int n_ptile = (a.n_point + 63) / 64;
  const int n_pg = a.pol_sum ? 1 : a.n_pol;
  int wg = blockIdx.x;
  const int ptile = wg % n_ptile;
  const int trun = wg / n_ptile;
  const int cs = blockIdx.y, pg = blockIdx.z;
  const int chan = a.chan_lo + cs;
  const int p = ptile * 64 + wave * 16 + (lane & 15);
  const bool live = p < a.n_point;
  const bool wave_live = ptile * 64 + wave * 16 < a.n_point;
  const int pp = live ? p : a.n_point - 1;

  if constexpr (TAPER) {
    for (int i = tid; i < kV16N * 4; i += 256) lds_h[i] = a.taper[i];
  }
  TiedW w;
  if (wave_live) tied_weights(a.dl[2 * chan] * a.dircos[2 * pp], a.dl[2 * chan + 1] * a.dircos[2 * pp + 1], lane >> 4, w);
  const V16Lane l = v16_lane(lane);
  __syncthreads();
  int ds = 8;
  if constexpr (TAPER) {
    float hmax = 0.f;
    for (int i = 0; i < kV16N * 4; ++i) hmax = fmaxf(hmax, fabsf(lds_h[i]));
    ds = v16_data_scale(hmax);
  }
  const float out_scale = ldexpf(1.f, -2 * (ds + kV16Wscale));

  const int pol_lo = a.pol_sum ? 0 : pg, pol_hi = a.pol_sum ? a.n_pol : pg + 1;
  const int64_t span = (int64_t)a.block * kTiedBlocksPerWg;
  const int64_t t0 = (int64_t)trun * span;
  const int64_t t1 = t0 + span < a.n_time ? t0 + span : a.n_time;
  const int64_t frame_dw = (int64_t)a.n_chan * a.n_pol * kV16N;   // dwords per sample

  // groups of kV16TS samples per block, and the block being summed (a
  // workgroup's span starts at a block boundary)
  const int gpb = a.block / kV16TS;
  int gcnt = 0;
  int64_t blk = (int64_t)trun * kTiedBlocksPerWg;
  // The next group's frames are loaded into registers while the matrix
  // cores interpolate the current quad.
  auto frames = [&](int64_t tw, int pol) {
    return a.volts + (tw + l.ts) * frame_dw + ((int64_t)chan * a.n_pol + pol) * kV16N;
  };
  uint32_t nd[kV16N];
  if (t0 + kV16TS * wave < t1) {
    v16_load(frames(t0 + kV16TS * wave, pol_lo), nd);
  } else {
#pragma unroll
    for (int j = 0; j < kV16N; ++j) nd[j] = 0u;
  }
  float acc = 0.f;
  for (int64_t tq = t0; tq < t1; tq += 4 * kV16TS) {
    float accg[4] = {0.f, 0.f, 0.f, 0.f};
    for (int pol = pol_lo; pol < pol_hi; ++pol) {
      const int64_t tw = tq + kV16TS * wave;
      if (tw < t1) v16_fft_to_lds<TAPER>(nd, l, lds_h, lds_b + wave * kV16Buf, ds);
      __syncthreads();
      {
        // the next (quad, pol) of this wavefront, if any
        int64_t tn = tq;
        int pn = pol + 1;
        if (pn >= pol_hi) {
          pn = pol_lo;
          tn = tq + 4 * kV16TS;
        }
        const int64_t twn = tn + kV16TS * wave;
        if (twn < t1) {
          v16_load(frames(twn, pn), nd);
        } else {
#pragma unroll
          for (int j = 0; j < kV16N; ++j) nd[j] = 0u;
        }
      }
      if (wave_live) {
#pragma unroll
        for (int g = 0; g < 4; ++g)
          if (tq + kV16TS * g < t1) accg[g] += tied_block_mfma(lds_b + g * kV16Buf, w, lane) * out_scale;
      }
      __syncthreads();
    }
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      if (tq + kV16TS * g >= t1) break;
      acc += accg[g];
      if (++gcnt == gpb) {                         // the block's last group
        if (live && lane < 16) {
          float* o = static_cast<float*>(a.out) + ((blk * a.n_chan_sub + cs) * n_pg + pg) * (int64_t)a.n_point + p;
          *o = acc;
        }
        acc = 0.f;
        gcnt = 0;
        ++blk;
      }
    }
  }
}

// Persistent tile worker of the tied-beam server: each workgroup takes tiles
// (request, channel, 64 pointings, run of 16-sample blocks) from the batch,
// reading voltages from the device ring (absolute sample s lives in slot
// s mod ring_samples).  A tile's arithmetic is the same as k_tied_v16's (the
// same quads of 16-sample groups) and does not depend on which other tiles
// share the launch.
__global__ __launch_bounds__(256) void k_serve(const ServeTile* __restrict__ tiles, int n_tiles,
                                               const uint32_t* __restrict__ ring, int64_t ring_samples,
                                               int n_chan, int n_pol, const double* __restrict__ dl) {
  __shared__ __attribute__((aligned(16))) _Float16 lds_b[4 * kV16Buf];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const V16Lane l = v16_lane(lane);
  const float out_scale = ldexpf(1.f, -2 * (8 + kV16Wscale));
  const int64_t frame_dw = (int64_t)n_chan * n_pol * kV16N;
  for (int ti = blockIdx.x; ti < n_tiles; ti += gridDim.x) {
    const ServeTile t = tiles[ti];
    const int p = t.ptile * 64 + wave * 16 + (lane & 15);
    const bool live = p < t.n_point;
    const bool wave_live = t.ptile * 64 + wave * 16 < t.n_point;
    const int pp = live ? p : t.n_point - 1;
    TiedW w;
    if (wave_live)
      tied_weights(dl[2 * t.chan] * t.dircos[2 * pp], dl[2 * t.chan + 1] * t.dircos[2 * pp + 1], lane >> 4, w);
    // ring slot of this wavefront's first sample (the same for every pol),
    // advanced by a quad of groups per pass (the ring holds at least 16
    // samples, so a lane's sample l.ts < 16 past it wraps at most once)
    const int64_t sl0 = (t.t_start + (int64_t)(t.blk0 + wave) * kV16TS) % ring_samples;
    auto frames = [&](int64_t sl, int pol) {
      int64_t slot = sl + l.ts;
      if (slot >= ring_samples) slot -= ring_samples;
      return ring + slot * frame_dw + ((int64_t)t.chan * n_pol + pol) * kV16N;
    };
    // the next group's frames are loaded while the current quad is interpolated
    uint32_t nd[kV16N];
    if (wave < t.n_blk) {
      v16_load(frames(sl0, 0), nd);
    } else {
#pragma unroll
      for (int j = 0; j < kV16N; ++j) nd[j] = 0u;
    }
    for (int pol = 0; pol < n_pol; ++pol) {
      int64_t sl = sl0;
      for (int b0 = 0; b0 < t.n_blk; b0 += 4) {
        if (b0 + wave < t.n_blk) v16_fft_to_lds<false>(nd, l, nullptr, lds_b + wave * kV16Buf, 8);
        __syncthreads();
        {
          int64_t sn = sl + 4 * kV16TS;
          while (sn >= ring_samples) sn -= ring_samples;
          int bn = b0 + 4, pn = pol;
          if (bn >= t.n_blk) {
            bn = 0;
            ++pn;
            sn = sl0;
          }
          if (pn < n_pol && bn + wave < t.n_blk) {
            v16_load(frames(sn, pn), nd);
          } else {
#pragma unroll
            for (int j = 0; j < kV16N; ++j) nd[j] = 0u;
          }
        }
        float accg[4] = {0.f, 0.f, 0.f, 0.f};
        if (wave_live) {
#pragma unroll
          for (int g = 0; g < 4; ++g)
            if (b0 + g < t.n_blk) accg[g] = tied_block_mfma(lds_b + g * kV16Buf, w, lane) * out_scale;
        }
        __syncthreads();
        if (live && lane < 16) {
#pragma unroll
          for (int g = 0; g < 4; ++g) {
            if (b0 + g >= t.n_blk) break;
            const int64_t ob = t.blk0 + b0 + g;
            t.out[((ob * t.n_chan_req + (t.chan - t.chan_lo)) * n_pol + pol) * (int64_t)t.n_point + p] = accg[g];
          }
        }
        sl += 4 * kV16TS;
        while (sl >= ring_samples) sl -= ring_samples;
      }
    }
  }
}

// ---- larger lattices (m_ns = 128, 256, 512): FP32 matrix cores ----
//
// Per (16-pointing tile, channel, pol) the interpolation is a complex product
//   Z[p][(t, e)] = sum_A c_A(y_ns,p) B[t][e][A],   B_p[t] = sum_e c_e(y_ew,p) Z[p][(t, e)]
// run on v_mfma_f32_16x16x4_f32 (FP32 operands and accumulation, so the
// result is FP32-grade without split terms): rows = the 16 pointings, columns
// = 4 samples x 4 E-W beams, K = 4 beams A per instruction, the complex
// product as four real products (Re c Re B, Im c Im B, Re c Im B, Im c Re B
// into three accumulators).  Lane (g, n) takes A = g (M/4) + kb at step kb,
// so its beam reads walk contiguous memory (16-byte loads, two steps each)
// and its weights sit in one LDS row.  The N-S weights of the tile's
// pointings are generated once per workgroup in FP64 (the product form of
// interp_weight_d) and held in LDS as FP32; the E-W weights of the lane's four pointings (rows
// 4 g + i) and E-W beam (n mod 4) in registers.  The E-W sum is a sum over
// the four lanes of a column quad; |B_p|^2 is summed over the quad's samples
// by two more cross-lane adds.  Each wavefront owns whole output units
// (blocks of the intensity, or quads of samples for complex output).
constexpr int kTmfP = 16;                  // pointings per workgroup

template <int M>
__global__ __launch_bounds__(256) void k_tied_mf(TiedArgs a) {
  constexpr int KS = M / 4;                  // MFMA steps; A = g KS + kb
  constexpr int ROW = 2 * KS + 4;            // floats per (pointing, g) row; 16-byte pad against bank conflicts
  __shared__ __attribute__((aligned(16))) float lds_w[kTmfP * 4 * ROW];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int n = lane & 15, g = lane >> 4;
  const int e = n & 3, s = n >> 2;           // the lane's column: sample s of the quad, E-W beam e
  const int n_ptile = (a.n_point + kTmfP - 1) / kTmfP;
  const int ptile = blockIdx.x % n_ptile, run = blockIdx.x / n_ptile;
  const int cs = blockIdx.y, pg = blockIdx.z;
  const int chan = a.chan_lo + cs;
  const double dl_ew = a.dl[2 * chan], dl_ns = a.dl[2 * chan + 1];

  for (int i = tid; i < kTmfP * M; i += 256) {
    const int pl = i / M, A = i - pl * M;
    const int p = min(ptile * kTmfP + pl, a.n_point - 1);
    double wr, wi;
    interp_weight_d(A, M, a.n_ns, dl_ns * a.dircos[2 * p + 1], &wr, &wi);
    const int gg = A / KS, kb = A - gg * KS;
    float* row = lds_w + (pl * 4 + gg) * ROW;
    row[2 * kb] = (float)wr;
    row[2 * kb + 1] = (float)wi;
  }
  cf cew[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int p = min(ptile * kTmfP + 4 * g + i, a.n_point - 1);
    double wr, wi;
    interp_weight_d(e, 4, a.n_ew, dl_ew * a.dircos[2 * p], &wr, &wi);
    cew[i] = cf{(float)wr, (float)wi};
  }
  __syncthreads();

  // output units: intensity blocks, or quads of samples for complex output
  const int unit = a.complex_out ? 4 : a.block;
  const int64_t n_unit = (a.n_time + unit - 1) / unit;
  const int64_t u0 = (int64_t)run * a.run_units;
  const int64_t u1 = u0 + a.run_units < n_unit ? u0 + a.run_units : n_unit;
  const int n_pg = a.pol_sum ? 1 : a.n_pol;
  const int pol_lo = a.pol_sum ? 0 : pg, pol_hi = a.pol_sum ? a.n_pol : pg + 1;
  const float* wrow = lds_w + (n * 4 + g) * ROW;
  const float* beams = reinterpret_cast<const float*>(a.beams);

  for (int64_t u = u0 + wave; u < u1; u += 4) {
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    for (int pol = pol_lo; pol < pol_hi; ++pol) {
      for (int q = 0; q < unit; q += 4) {
        const int64_t t = u * unit + q + s;
        const int64_t tc = t < a.n_time ? t : a.n_time - 1;
        const float* bp = beams + ((((tc * a.n_chan + chan) * a.n_pol + pol) * 4 + e) * M + (int64_t)g * KS) * 2;
        f32x4 p1 = {0.f, 0.f, 0.f, 0.f}, p2 = p1, zi = p1;
#pragma unroll 4
        for (int kb = 0; kb < KS; kb += 2) {
          const float4 b = *reinterpret_cast<const float4*>(bp + 2 * kb);
          const float4 w = *reinterpret_cast<const float4*>(wrow + 2 * kb);
          p1 = __builtin_amdgcn_mfma_f32_16x16x4f32(w.x, b.x, p1, 0, 0, 0);
          p2 = __builtin_amdgcn_mfma_f32_16x16x4f32(w.y, b.y, p2, 0, 0, 0);
          zi = __builtin_amdgcn_mfma_f32_16x16x4f32(w.x, b.y, zi, 0, 0, 0);
          zi = __builtin_amdgcn_mfma_f32_16x16x4f32(w.y, b.x, zi, 0, 0, 0);
          p1 = __builtin_amdgcn_mfma_f32_16x16x4f32(w.z, b.z, p1, 0, 0, 0);
          p2 = __builtin_amdgcn_mfma_f32_16x16x4f32(w.w, b.w, p2, 0, 0, 0);
          zi = __builtin_amdgcn_mfma_f32_16x16x4f32(w.z, b.w, zi, 0, 0, 0);
          zi = __builtin_amdgcn_mfma_f32_16x16x4f32(w.w, b.z, zi, 0, 0, 0);
        }
        // E-W weights, then the sum over the column quad's four E-W beams
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          cf b = cmul(cf{p1[i] - p2[i], zi[i]}, cew[i]);
          b.r += __shfl_xor(b.r, 1);
          b.i += __shfl_xor(b.i, 1);
          b.r += __shfl_xor(b.r, 2);
          b.i += __shfl_xor(b.i, 2);
          if (a.complex_out) {
            const int p = ptile * kTmfP + 4 * g + i;
            if (e == 0 && t < a.n_time && p < a.n_point)
              static_cast<float2*>(a.out)[((t * a.n_chan_sub + cs) * a.n_pol + pol) * (int64_t)a.n_point + p] =
                  make_float2(b.r, b.i);
          } else {
            float v = cnorm(b);
            v += __shfl_xor(v, 4);
            v += __shfl_xor(v, 8);
            acc[i] += v;
          }
        }
      }
    }
    if (!a.complex_out && n == 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int p = ptile * kTmfP + 4 * g + i;
        if (p < a.n_point) static_cast<float*>(a.out)[((u * a.n_chan_sub + cs) * n_pg + pg) * (int64_t)a.n_point + p] = acc[i];
      }
    }
  }
}

}  // namespace

// m_ns = 128, 256, 512 (16-byte aligned beams): enough runs of output units
// per (pointing tile, channel, pol group) that the grid holds about 8192
// workgroups, each run a multiple of the four wavefronts' units
static hipError_t launch_tied_mf(TiedArgs a, hipStream_t s) {
  if ((a.m_ns != 128 && a.m_ns != 256 && a.m_ns != 512) || a.m_ew != 4 ||
      (reinterpret_cast<uintptr_t>(a.beams) & 15) != 0)
    return hipErrorNotSupported;
  const int n_ptile = (a.n_point + kTmfP - 1) / kTmfP;
  const int n_pg = (a.pol_sum && !a.complex_out) ? 1 : a.n_pol;
  const int unit = a.complex_out ? 4 : a.block;
  const int64_t n_unit = (a.n_time + unit - 1) / unit;
  const int64_t base = (int64_t)n_ptile * a.n_chan_sub * n_pg;
  int64_t runs = (8192 + base - 1) / base;
  const int64_t max_runs = (n_unit + 3) / 4;
  if (runs > max_runs) runs = max_runs;
  if (runs < 1) runs = 1;
  int64_t per = (n_unit + runs - 1) / runs;
  per = (per + 3) / 4 * 4;
  runs = (n_unit + per - 1) / per;
  if (per > 0x7FFFFFFF || (int64_t)n_ptile * runs > 0x7FFFFFFF || a.n_chan_sub > 65535)
    return hipErrorInvalidConfiguration;
  a.run_units = (int)per;
  dim3 grid((unsigned)(n_ptile * runs), (unsigned)a.n_chan_sub, (unsigned)n_pg);
  if (a.m_ns == 128) hipLaunchKernelGGL(k_tied_mf<128>, grid, dim3(256), 0, s, a);
  else if (a.m_ns == 256) hipLaunchKernelGGL(k_tied_mf<256>, grid, dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_tied_mf<512>, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_tied(const TiedArgs& a, hipStream_t s) {
  const int n_ptile = (a.n_point + 63) / 64;
  // the 4 x 16 lattice, intensities in blocks of 16k samples, 16-byte aligned beams: matrix cores
  if (a.m_ns == 32 && a.n_ns == 16 && !a.complex_out && a.block % 16 == 0 &&
      (reinterpret_cast<uintptr_t>(a.beams) & 15) == 0) {
    const int64_t span_m = (int64_t)a.block * kTiedBlocksPerWg;
    const int64_t n_run_m = (a.n_time + span_m - 1) / span_m;
    const int n_pg_m = a.pol_sum ? 1 : a.n_pol;
    if ((int64_t)n_ptile * n_run_m > 0x7FFFFFFF || a.n_chan_sub > 65535) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(k_tied_b16, dim3((unsigned)(n_ptile * n_run_m), (unsigned)a.n_chan_sub, (unsigned)n_pg_m),
                       dim3(256), 0, s, a);
    return hipGetLastError();
  }
  const int64_t span = (int64_t)(a.complex_out ? 16 : a.block) * kTiedBlocksPerWg;
  const int64_t n_run = (a.n_time + span - 1) / span;
  const int n_pg = (a.pol_sum && !a.complex_out) ? 1 : a.n_pol;
  if ((int64_t)n_ptile * n_run > 0x7FFFFFFF || a.n_chan_sub > 65535) return hipErrorInvalidConfiguration;
  dim3 grid((unsigned)(n_ptile * n_run), (unsigned)a.n_chan_sub, (unsigned)n_pg);
  if (a.m_ns == 32) hipLaunchKernelGGL(k_tied<32>, grid, dim3(64), 0, s, a);
  else if (a.m_ns == 64) hipLaunchKernelGGL(k_tied<64>, grid, dim3(64), 0, s, a);
  else return launch_tied_mf(a, s);
  return hipGetLastError();
}

hipError_t launch_serve(const ServeTile* tiles, int n_tiles, const uint32_t* ring, int64_t ring_samples,
                        int n_chan, int n_pol, const double* dl, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  const int grid = n_tiles < 8192 ? n_tiles : 8192;
  hipLaunchKernelGGL(k_serve, dim3(grid), dim3(256), 0, s, tiles, n_tiles, ring, ring_samples, n_chan, n_pol, dl);
  return hipGetLastError();
}

hipError_t launch_tied_v(const TiedArgs& a, hipStream_t s) {
  if (a.n_ns != 16 || a.m_ns != 32 || a.block % 16) return hipErrorNotSupported;
  const int n_ptile = (a.n_point + 63) / 64;
  const int64_t span = (int64_t)a.block * kTiedBlocksPerWg;
  const int64_t n_run = (a.n_time + span - 1) / span;
  const int n_pg = a.pol_sum ? 1 : a.n_pol;
  if ((int64_t)n_ptile * n_run > 0x7FFFFFFF || a.n_chan_sub > 65535) return hipErrorInvalidConfiguration;
  dim3 grid((unsigned)(n_ptile * n_run), (unsigned)a.n_chan_sub, (unsigned)n_pg);
  if (a.taper) hipLaunchKernelGGL(k_tied_v16<true>, grid, dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_tied_v16<false>, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace fftbf
