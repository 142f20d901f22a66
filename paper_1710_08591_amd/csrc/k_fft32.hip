// FP32 FFT beamformer for gfx950 (the voltage-rate hot path).
//
// Computes, per (channel, polarisation, sample), the 2-D FFT beams of the
// 4 x n_ns lattice -- inner sum of eq. e:fftbeamform with the voltage
// weights of eq. e:w_A^a, E-W unpadded (M_ew = 4), N-S zero-padded to
// M = 2 n_ns -- then |B|^2 summed over blocks of samples (the time sum of
// eq. e:bf), clamped to the kept N-S beams of each channel.
//
// Work split (one 64-lane wavefront per (block, channel, polarisation
// group), each with its own LDS tile; one wave per workgroup, or a few that
// share the table of per-antenna factors):
//   * the N-S transform M = (2L) x G, with n_ns = L G:
//       a = a1 + G a2,  A = k2 + 2L k1
//       pass 1 (one lane per (frame, E-W beam e, a1)): zero-padded 2L-point
//         DFT over a2, in registers, then the twiddle W_M^{a1 k2};
//       LDS transpose (rows padded by one element against bank conflicts);
//       pass 2 (lanes over (frame, e, k2)): G-point DFT over a1, in registers.
//     The in-register DFTs are radix-2 decimation in time with each
//     compile-time twiddle factored into a tangent form (6 operations per
//     twiddled butterfly instead of 8).  The pass-1 twiddle and the
//     zero-padding pre-twiddles take the same form (2 operations instead of
//     4): their real factors stay on the values and are absorbed by the
//     multipliers of the following butterflies, so no output carries one.
//   * the E-W 4-point DFT has twiddles in {1, -i, -1, +i}: without a window
//     it is two signed 4-bit dot products per N-S position (v_dot8_i32_i4
//     straight on the packed voltage bytes, exact integers); with a window
//     the nibbles are sign-extended, converted and weighted in FP32.
//   * |B|^2 accumulates in registers across the block; at the block end the
//     sums go through LDS once more so the kept beams can be gathered in
//     the channel's clamp-table order and stored with coalesced writes.
//   * the two axes' transforms commute: on the 4 x 256 lattice, with complex
//     gains or with the E-W axis zero-padded to 8 beams, the N-S transform
//     runs first on the four E-W antenna columns and the E-W transform runs
//     per N-S beam after pass 2 (fft32_nsf_run below).
#include "dev_common.h"
#include "kernels.h"

namespace fftbf {

namespace {

// Per-lane dot8 weights for the E-W beam e: real and imaginary part of
// sum_q x_q (-i)^{e q}.  Nibble 2q is Im(x_q), nibble 2q+1 is Re(x_q).
__device__ __forceinline__ void ew_weights(int e, int& wre, int& wim) {
  wre = 0;
  wim = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int k = (e * q) & 3;
    const int sr = 4 * (2 * q + 1), si = 4 * (2 * q);
    // Re: k0 +r, k1 +i, k2 -r, k3 -i ; Im: k0 +i, k1 -r, k2 -i, k3 +r
    if (k == 0) { wre |= 1 << sr;   wim |= 1 << si; }
    if (k == 1) { wre |= 1 << si;   wim |= 0xF << sr; }
    if (k == 2) { wre |= 0xF << sr; wim |= 0xF << si; }
    if (k == 3) { wre |= 0xF << si; wim |= 1 << sr; }
  }
}

// dot8 weight words for sum_q c_q x_q over the four E-W samples of a dword,
// c_q = cr[q] + i ci[q] with components in {-1, 0, 1}: Re = cr xr - ci xi,
// Im = ci xr + cr xi, one signed nibble per term.
__device__ __forceinline__ void cweights(const int* cr, const int* ci, int& wre, int& wim) {
  wre = 0;
  wim = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int sr = 4 * (2 * q + 1), si = 4 * (2 * q);
    wre |= ((cr[q] & 0xF) << sr) | (((-ci[q]) & 0xF) << si);
    wim |= ((ci[q] & 0xF) << sr) | ((cr[q] & 0xF) << si);
  }
}

// Odd beam 2e+1 of the zero-padded 8-point E-W transform of x_0..x_3:
//   sum_q x_q W_8^{q (2e+1)} = P + Q / sqrt(2),
//   P = x_0 + (-1)^e (-i) x_2,   Q = (-i)^e (1 - i) x_1 + i^e (-1 - i) x_3,
// both integer combinations with coefficients in {-1, 0, 1}.
__device__ __forceinline__ void ew8_odd_weights(int e, int& wpr, int& wpi, int& wqr, int& wqi) {
  const int mr[4] = {1, 0, -1, 0}, mi[4] = {0, -1, 0, 1};          // (-i)^e
  int pcr[4] = {1, 0, 0, 0}, pci[4] = {0, 0, (e & 1) ? 1 : -1, 0};
  int qcr[4] = {0, 0, 0, 0}, qci[4] = {0, 0, 0, 0};
  qcr[1] = mr[e] + mi[e];                  // (-i)^e (1 - i)
  qci[1] = mi[e] - mr[e];
  qcr[3] = -mr[e] - mi[e];                 // i^e (-1 - i), i^e = conj((-i)^e)
  qci[3] = mi[e] - mr[e];
  cweights(pcr, pci, wpr, wpi);
  cweights(qcr, qci, wqr, wqi);
}

// sign-extended 4-bit field (the builtin's result type is unsigned)
__device__ __forceinline__ float nib(uint32_t d, int shift) {
  return (float)(int)__builtin_amdgcn_sbfe((int)d, shift, 4);
}

// Real weights h_q on the four E-W antennas of a byte-packed N-S position
// (antenna q: real part in bits 8q+4..8q+7, imaginary in 8q..8q+3).  Beam e
// of sum_q h_q z_q (-i)^{eq}, with s = (-1)^e, splits into
//   Re = (h0 x0 + s h2 x2) + tr (h1 u1 + s h3 u3),
//   Im = (h0 y0 + s h2 y2) + ti (h1 v1 + s h3 v3),
// x, y the real and imaginary parts, (u, v) = (x, y) for even e and (y, x)
// for odd e, tr = +1 for e < 2, ti = +1 for e in {0, 3} (-1 otherwise).
// The lane picks u and v by the bit offset of its field, so its beam costs
// no selects, and its signs two multiplies per position.  With complex
// gains the same split holds for w_q = g_q z_q, and the lane's choice of
// component folds into the product: with r = +1 for odd e, -1 for even,
//   w1u = g1r u1 + r g1i v1,   w1v = g1r v1 - r g1i u1
// (u, v the nibbles above), and s r = -1 for every e.
struct WindowLane {
  float s, r, tr, ti;
  int ou, ov;      // bit offsets of u1 and v1 (u3, v3: 16 higher)
};

__device__ __forceinline__ WindowLane window_lane(int e) {
  WindowLane w;
  w.s = (e & 1) ? -1.f : 1.f;
  w.r = (e & 1) ? 1.f : -1.f;
  w.tr = e < 2 ? 1.f : -1.f;
  w.ti = (e == 0 || e == 3) ? 1.f : -1.f;
  w.ou = (e & 1) ? 8 : 12;
  w.ov = (e & 1) ? 12 : 8;
  return w;
}

// Each wavefront works in an LDS tile of its own, and a wavefront's LDS
// operations execute in the order it issues them: between the transpose's
// writes and reads only the compiler's order has to be kept, with no wait
// for the writes to land.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// row[k] = y[k] W_M^{a1 k} / Re W (tangent form, two fused multiply-adds), or
// y[k] W_M^{a1 k} in the columns that keep whole twiddles
template <int G, int M, int L2, int K>
struct Pass1Tw {
  static __device__ __forceinline__ void run(const cf* y, const float* t1, const cf* c1, cf* row) {
    if constexpr (cmul_col(K, G, M)) row[K] = cmul(y[K], c1[K]);
    else row[K] = cf{fmaf(-t1[K], y[K].i, y[K].r), fmaf(t1[K], y[K].r, y[K].i)};
    if constexpr (K + 1 < L2) Pass1Tw<G, M, L2, K + 1>::run(y, t1, c1, row);
  }
};

// the same for the even columns k = 2 m only, from the unpadded L-point DFT
// x[m], stored at row[m] (cyclic co-adding keeps only the even outputs)
template <int G, int M, int L, int MI>
struct Pass1TwEven {
  static __device__ __forceinline__ void run(const cf* x, const float* t1, const cf* c1, cf* row) {
    constexpr int K = 2 * MI;
    if constexpr (cmul_col(K, G, M)) row[MI] = cmul(x[MI], c1[K]);
    else row[MI] = cf{fmaf(-t1[K], x[MI].i, x[MI].r), fmaf(t1[K], x[MI].r, x[MI].i)};
    if constexpr (MI + 1 < L) Pass1TwEven<G, M, L, MI + 1>::run(x, t1, c1, row);
  }
};

// Waves per workgroup.  Every wave transforms its own (block, channel,
// polarisation group) in its own LDS tile; the variants with per-antenna
// factors keep one table of them per workgroup, shared by its waves.  With
// one wave per workgroup that table would let the LDS, not the registers,
// bound the waves per CU (7 instead of 8 with real weights on 256 N-S
// positions, 6 with complex gains); enough waves share it that the LDS
// allows the occupancy the registers do (8 waves per CU at N x FOLD = 256,
// 16 below).
template <int N, int G, int TAPER, int FOLD>
constexpr int fft32_wpg() {
  constexpr int kLds = 160 * 1024;
  constexpr int tile = 64 * ((FOLD > 1 ? 1 : 2) * (N / G) + 1) * 8;   // F * 4 * G = 64 rows
  constexpr int table = TAPER == 2 ? N * FOLD * 32 : TAPER == 1 ? N * FOLD * 16 : 0;
  if (table == 0) return 1;
  constexpr int want = (N * FOLD >= 256 ? 8 : 16) < kLds / tile ? (N * FOLD >= 256 ? 8 : 16) : kLds / tile;
  for (int w = 1; w < 4; w *= 2)
    if (kLds / (w * tile + table) * w >= want) return w;
  return 4;
}

// TAPER: 0 none (E-W DFT as signed 4-bit dot products), 1 real per-antenna
// weights h_a, 2 complex per-antenna gains g_a (float2), applied before the
// E-W DFT, 3 none and the odd beams of the zero-padded 8-point E-W transform
// (signed 4-bit dot products again).
// FOLD > 1: cyclic co-adding (fewer beams than antennas, e:fftbeamform with
// M < n): the N * FOLD antennas along N-S are summed onto N positions by
// a mod N before an N-point transform, whose outputs are the even outputs
// of the zero-padded 2N-point transform (only those are computed).
// The complex-gain intensity variant below 256 N-S positions is held to 128
// registers (four wavefronts per SIMD, the occupancy its shared table is
// sized for; it fits without spilling, the complex-output variant does not).
template <int N, int G, int TAPER, bool CPLX, int FOLD>
constexpr int fft32_min_waves() {
  // co-adding 256 N-S antennas (folds 2 to 8; with a window from fold 4 on,
  // the windowed 2-fold kernel does not fit 128 registers)
  return (TAPER == 2 && !CPLX && N * FOLD < 256) ||
                 (N * FOLD == 256 && FOLD > 1 && FOLD < 16 && !CPLX && (TAPER == 0 || (TAPER == 1 && FOLD >= 4)))
             ? 4
             : 1;
}

template <int N, int G, int TAPER, bool CPLX, int FOLD = 1>
__global__ __launch_bounds__((64 * fft32_wpg<N, G, TAPER, FOLD>()))
__attribute__((amdgpu_waves_per_eu(fft32_min_waves<N, G, TAPER, CPLX, FOLD>()))) void k_fft32(Fft32Args p) {
  constexpr int L = N / G, L2 = 2 * L, M = 2 * N;
  constexpr int NA = N * FOLD, LA = L * FOLD;   // antennas along N-S; dwords per lane per frame
  constexpr int F = 64 / (4 * G);      // frames handled side by side
  // With cyclic co-adding only the outputs A = k2 + L2 k1 with k2 even are
  // beams: pass 1 then runs the unpadded L-point DFT (the even columns), and
  // where the even columns' tasks tile the wavefront pass 2 takes only those
  // (elsewhere the odd columns' tasks run on unused data and are never read).
  constexpr bool EVEN = FOLD > 1;
  constexpr bool REMAP = EVEN && (F * 4 * L) % 64 == 0;
  constexpr int NCOL = REMAP ? L : L2;  // pass-2 columns per (frame, E-W beam)
  constexpr int R2 = (F * 4 * NCOL) / 64; // pass-2 tasks per lane
  constexpr int YS = (EVEN ? L : L2) + 1;   // padded LDS row (only the even columns with co-adding)
  static_assert(F >= 1 && F * 4 * G == 64, "pass-1 lanes must fill the wavefront");
  static_assert(R2 >= 1 && R2 * 64 == F * 4 * NCOL, "pass-2 tasks must tile the wavefront");
  static_assert(F * 4 * M * 4 <= F * 4 * G * YS * 8, "block-end sums must fit the LDS");

  constexpr int WPG = fft32_wpg<N, G, TAPER, FOLD>();
  constexpr int TILE = F * 4 * G * YS;
  __shared__ cf lds_tiles[WPG * TILE];
  __shared__ float lds_h[TAPER == 2 ? NA * 8 : TAPER == 1 ? NA * 4 : 1];

  const int lane = WPG == 1 ? (int)threadIdx.x : (int)(threadIdx.x & 63);
  const int wave = WPG == 1 ? 0 : __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  cf* const lds_y = lds_tiles + wave * TILE;
  const int f1 = lane / (4 * G), e1 = (lane / G) & 3, a1 = lane % G;

  int pg, wg;
  if constexpr (WPG == 1 && N * FOLD == 16) {
    wg = pol_pair_task((int)blockIdx.x, (int)p.n_wg, p.n_pg, pg);
  } else {
    wg = (int)((int64_t)blockIdx.x * WPG + wave);
    pg = wg % p.n_pg;
    wg /= p.n_pg;
  }
  const int chan = wg % p.n_chan;
  const int blk = wg / p.n_chan;

  if constexpr (TAPER == 1) {
    for (int i = threadIdx.x; i < NA * 4; i += 64 * WPG) lds_h[i] = p.taper[i];
    __syncthreads();
  } else if constexpr (TAPER == 2) {
    // per antenna (a_ns, q): g = 1, h or the complex gain, times W_8^q when twisting
    constexpr float kS = 0.70710678118654752f;
    for (int i = threadIdx.x; i < NA * 4; i += 64 * WPG) {
      float gr = 1.f, gi = 0.f;
      if (p.gain_src == 2) {
        gr = p.taper[2 * i];
        gi = p.taper[2 * i + 1];
      } else if (p.gain_src == 1) {
        gr = p.taper[i];
      }
      if (p.twist) {
        const int q = i & 3;
        const float wr = q == 0 ? 1.f : q == 1 ? kS : q == 2 ? 0.f : -kS;
        const float wi = q == 0 ? 0.f : q == 1 ? -kS : q == 2 ? -1.f : -kS;
        const float tr = gr * wr - gi * wi;
        gi = gr * wi + gi * wr;
        gr = tr;
      }
      lds_h[2 * i] = gr;
      lds_h[2 * i + 1] = gi;
    }
    __syncthreads();
  }
  // the last workgroup's spare waves (task count not a multiple of WPG)
  // leave after the workgroup's only barrier
  if (WPG > 1 && (int64_t)blockIdx.x * WPG + wave >= p.n_wg) return;

  // pass-1 twiddles W_M^{a1 k2}, generated in FP64 at plan creation, in
  // tangent form W = Re W (1 + i t): only t is applied here, the factor
  // Re W travels into pass 2's multipliers (columns where some lane has
  // Re W = 0 keep whole twiddles)
  constexpr int NSL = dit_slots(G);
  float t1[L2];
  cf c1[L2];
#pragma unroll
  for (int k = 0; k < L2; ++k) {
    const float2 w = p.tw[a1 * L2 + k];
    t1[k] = w.x;
    c1[k] = cf{w.x, w.y};
  }
  // pass-2 multipliers of this lane's column k2 (the same for all its tasks)
  float mu[NSL];
#pragma unroll
  for (int i = 0; i < NSL; ++i) mu[i] = p.mult[(REMAP ? 2 * (lane % L) : lane % L2) * NSL + i];

  int wre = 0, wim = 0, wqr = 0, wqi = 0;
  WindowLane wl{};
  if constexpr (TAPER == 3) ew8_odd_weights(e1, wre, wim, wqr, wqi);
  else if constexpr (TAPER == 1 || TAPER == 2) wl = window_lane(e1);
  else ew_weights(e1, wre, wim);

  float acc[R2][G];
#pragma unroll
  for (int r = 0; r < R2; ++r)
#pragma unroll
    for (int k = 0; k < G; ++k) acc[r][k] = 0.f;

  const int64_t t_base = (int64_t)blk * p.block;
  const int n_it = p.block / F;
  const int64_t frame_stride = (int64_t)(p.chan_stride ? p.chan_stride : p.n_chan) * p.n_pol * NA;  // dwords per sample

  // Frames of this block that hold data: all of them, except in a short
  // final block (complex output with n_time not a multiple of the block).
  // Every load is unconditional (a lane whose frame lies past the data
  // re-reads its last valid one; its results are never stored), so no load
  // sits under an execution mask and the next frames stay in flight while
  // the current ones are transformed.
  const int n_valid = (int)((p.n_time - t_base) < p.block ? (p.n_time - t_base) : p.block);
  const int64_t f_step = (int64_t)F * frame_stride;

  for (int pi = 0; pi < p.pol_iter; ++pi) {
    const int pol = (p.pol_iter == 1) ? pg : pi;
    const uint32_t* src = p.volts + ((int64_t)chan * p.n_pol + pol) * NA + a1;

    // two frame buffers in turn: while one group of frames is transformed,
    // the next one is in flight in the other
    uint32_t b0[LA], b1[LA];
    const uint32_t* p0 = src + (t_base + (f1 < n_valid ? f1 : n_valid - 1)) * frame_stride;
    const uint32_t* p1 = p0;
#pragma unroll
    for (int j = 0; j < LA; ++j) b0[j] = __builtin_nontemporal_load(p0 + G * j);
    // this lane's frame in pass k follows its frame in pass k - 1, unless
    // that is past the data (then the lane re-reads its last valid frame);
    // the prefetch past the block's last pass reads the first frame of the
    // voltage buffer instead, which every wavefront shares, so it stays in
    // the L2 cache and costs no memory traffic
    auto next = [&](const uint32_t* q, int k) {
      if (k >= n_it) return p.volts + a1;
      return (k * F + f1 < n_valid) ? q + f_step : q;
    };

    auto frame_pass = [&](const uint32_t (&cur)[LA], int it) {
        // ---- E-W DFT for this lane's beam e1 at N-S positions a1 + G j ----
        // (with FOLD > 1, summed over the antennas a1 + G j + N f, f < FOLD)
        cf x[L];
#pragma unroll
        for (int j = 0; j < L; ++j) {
          if constexpr (TAPER == 0) {
            int sr = 0, si = 0;
#pragma unroll
            for (int f = 0; f < FOLD; ++f) {
              sr += sdot8((int)cur[j + L * f], wre);
              si += sdot8((int)cur[j + L * f], wim);
            }
            x[j] = cf{(float)sr, (float)si};
          } else if constexpr (TAPER == 3) {
            constexpr float kS = 0.70710678118654752f;
            const uint32_t d = cur[j];
            const float pr = (float)sdot8((int)d, wre), pi = (float)sdot8((int)d, wim);
            const float qr = (float)sdot8((int)d, wqr), qi = (float)sdot8((int)d, wqi);
            x[j] = cf{fmaf(kS, qr, pr), fmaf(kS, qi, pi)};
          } else if constexpr (TAPER == 2) {
            // w_q = g_q z_q, split as for real weights (WindowLane)
            const uint32_t d = cur[j];
            const float4 g01 = *reinterpret_cast<const float4*>(&lds_h[(a1 + G * j) * 8]);
            const float4 g23 = *reinterpret_cast<const float4*>(&lds_h[(a1 + G * j) * 8 + 4]);
            const float s2r = wl.s * g23.x, s2i = wl.s * g23.y;     // s g2
            const float r1i = wl.r * g01.w;                          // r g1i
            const float s3r = wl.s * g23.z;                          // s g3r (s r g3i = -g3i)
            const float xr0 = nib(d, 4), xi0 = nib(d, 0), xr2 = nib(d, 20), xi2 = nib(d, 16);
            const float u1 = nib(d, wl.ou), v1 = nib(d, wl.ov);
            const float u3 = nib(d, wl.ou + 16), v3 = nib(d, wl.ov + 16);
            const float pr = fmaf(-s2i, xi2, fmaf(s2r, xr2, fmaf(-g01.y, xi0, g01.x * xr0)));
            const float pi = fmaf(s2i, xr2, fmaf(s2r, xi2, fmaf(g01.y, xr0, g01.x * xi0)));
            const float qr = fmaf(-g23.w, v3, fmaf(s3r, u3, fmaf(r1i, v1, g01.z * u1)));
            const float qi = fmaf(g23.w, u3, fmaf(s3r, v3, fmaf(-r1i, u1, g01.z * v1)));
            x[j] = cf{fmaf(wl.tr, qr, pr), fmaf(wl.ti, qi, pi)};
          } else {
            float pr = 0.f, pi = 0.f, qr = 0.f, qi = 0.f;
#pragma unroll
            for (int f = 0; f < FOLD; ++f) {
              const uint32_t d = cur[j + L * f];
              const float4 h = *reinterpret_cast<const float4*>(&lds_h[(a1 + G * (j + L * f)) * 4]);
              const float h2 = wl.s * h.z, h3 = wl.s * h.w;
              pr = fmaf(h2, nib(d, 20), fmaf(h.x, nib(d, 4), pr));
              pi = fmaf(h2, nib(d, 16), fmaf(h.x, nib(d, 0), pi));
              qr = fmaf(h3, nib(d, wl.ou + 16), fmaf(h.y, nib(d, wl.ou), qr));
              qi = fmaf(h3, nib(d, wl.ov + 16), fmaf(h.y, nib(d, wl.ov), qi));
            }
            const float re = fmaf(wl.tr, qr, pr), im = fmaf(wl.ti, qi, pi);
            x[j] = cf{re, im};
          }
        }

        // ---- pass 1: zero-padded 2L-point DFT over a2, twiddle, to LDS ----
        cf* row = &lds_y[((f1 * 4 + e1) * G + a1) * YS];
        if constexpr (EVEN) {
          dit<L>(x);
          row[0] = x[0];
          if constexpr (L > 1) Pass1TwEven<G, M, L, 1>::run(x, t1, c1, row);
        } else {
          cf y[L2];
          padded_dft_t<L>(x, y);
          row[0] = y[0];
          Pass1Tw<G, M, L2, 1>::run(y, t1, c1, row);
        }
        wave_lds_sync();

        // ---- pass 2: G-point DFT over a1 ----
        // every task's column is read before any is transformed, so the later
        // tasks' reads overlap the first task's arithmetic
        cf zz[R2][G];
#pragma unroll
        for (int r = 0; r < R2; ++r) {
          const int q = lane + 64 * r;
          const int k2 = REMAP ? 2 * (q % NCOL) : q % NCOL, e = (q / NCOL) & 3, f = q / (4 * NCOL);
          const cf* col = &lds_y[(f * 4 + e) * G * YS + (EVEN ? k2 / 2 : k2)];
#pragma unroll
          for (int j = 0; j < G; ++j) zz[r][j] = col[j * YS];
        }
        __builtin_amdgcn_sched_barrier(0);     // keep every read ahead of the transforms
#pragma unroll
        for (int r = 0; r < R2; ++r) {
          const int q = lane + 64 * r;
          const int k2 = REMAP ? 2 * (q % NCOL) : q % NCOL, e = (q / NCOL) & 3, f = q / (4 * NCOL);
          cf* z = zz[r];
          dit_rs<G>(z, mu);
          if constexpr (CPLX) {
            // with FOLD > 1 only the even padded outputs 2A are beams (A < N)
            constexpr int MO = FOLD > 1 ? N : M, SO = FOLD > 1 ? 2 : 1;
            const int64_t tt = t_base + (int64_t)it * F + f;
            if (tt < p.n_time && (k2 % SO) == 0) {
              float2* o = static_cast<float2*>(p.out) +
                          (((tt * p.n_chan + chan) * p.n_pol + pg) * p.ew_rows + e * p.ew_mul + p.ew_off) * MO + k2 / SO;
#pragma unroll
              for (int k1 = 0; k1 < G; ++k1) {
                const cf b = z[k1];
                o[(L2 / SO) * k1] = make_float2(b.r * p.norm, b.i * p.norm);
              }
            }
          } else {
#pragma unroll
            for (int k1 = 0; k1 < G; ++k1) acc[r][k1] = cnorm_acc(z[k1], acc[r][k1]);
          }
        }
        wave_lds_sync();
    };

    for (int it = 0; it < n_it; it += 2) {
      p1 = next(p0, it + 1);
#pragma unroll
      for (int j = 0; j < LA; ++j) b1[j] = __builtin_nontemporal_load(p1 + G * j);
      frame_pass(b0, it);
      if (it + 1 == n_it) break;
      p0 = next(p1, it + 2);
#pragma unroll
      for (int j = 0; j < LA; ++j) b0[j] = __builtin_nontemporal_load(p0 + G * j);
      frame_pass(b1, it + 1);
    }
  }

  if constexpr (!CPLX) {
    // ---- block end: gather the kept beams, sum frame groups, store ----
    float* lds_i = reinterpret_cast<float*>(lds_y);
#pragma unroll
    for (int r = 0; r < R2; ++r) {
      const int q = lane + 64 * r;
      const int k2 = REMAP ? 2 * (q % NCOL) : q % NCOL, e = (q / NCOL) & 3, f = q / (4 * NCOL);
#pragma unroll
      for (int k1 = 0; k1 < G; ++k1) lds_i[(f * 4 + e) * M + k2 + L2 * k1] = acc[r][k1];
    }
    wave_lds_sync();
    const int keep = p.n_keep;
    const int32_t* sel = p.sel ? p.sel + (int64_t)chan * keep : nullptr;
    float* o = static_cast<float*>(p.out) + (((int64_t)blk * p.n_chan + chan) * p.n_pg + pg) * p.ew_rows * keep;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      for (int j = lane; j < keep; j += 64) {
        const int A = sel ? sel[j] : j;
        float v = 0.f;
#pragma unroll
        for (int f = 0; f < F; ++f) v += lds_i[(f * 4 + e) * M + A];
        o[(e * p.ew_mul + p.ew_off) * keep + j] = v * p.norm;
      }
    }
  }
}

// ---- the 4 x 256 lattice: the pass-1 output in two halves ----
// The zero-padded 32-point DFT over a2 splits into its even outputs (the
// 16-point DFT of x) and its odd outputs (the 16-point DFT of x_j W_32^j,
// pre-twiddles in tangent form with their factors carried through the DIT).
// Each half is twiddled, transposed through an LDS tile of half the size and
// transformed by pass 2 before the other half is formed: 8.7 KB of tile per
// wavefront.  Lane (e, a1) of pass 1 is lane (e, m = a1) of pass 2, which
// takes column k2 = 2 m + h of half h.  The pass-1 tangent values and the
// pass-2 multipliers live in one LDS copy per workgroup (its four waves
// share it), not in registers, and the next frame's voltages are loaded
// during the second half only: about 125 registers and 10 KB of LDS per
// wavefront, so four wavefronts fit per SIMD (two for the kernel above).
// Intensities: k_fft32_h unwindowed and k_fft32_hw with a real window
// (three wavefronts per SIMD); the complex-output variants of this lattice
// take the kernel above.  Complex gains and an E-W axis zero-padded to 8
// beams take the N-S-first kernels below (the N-S transform on the four E-W
// antenna columns, then the E-W transform per N-S beam).
constexpr int kHWpg = 4;                 // wavefronts per workgroup
constexpr int kHRow = 44;                // LDS floats per (half, a1) row: 16 tangents, 25 multipliers, pad

template <int L>
__device__ __forceinline__ void padded_odd_t(const cf* x, cf* xo) {
  PadPreT<L, 0>::run(x, xo);
  cf z[L];
#pragma unroll
  for (int i = 0; i < L; ++i) z[i] = xo[bitrev(i, L)];
  DitPad<L, 2, 0, 0>::run(z);
#pragma unroll
  for (int i = 0; i < L; ++i) xo[i] = z[i];
}

// half h of pass 1's output, twiddled, into the lane's LDS row: k2 = 2 m + h
template <int H, int MI>
struct HalfTw {
  static __device__ __forceinline__ void run(const cf* y, const float* t1, cf c16, cf* row) {
    constexpr int K = 2 * MI + H;
    if constexpr (K == 0) row[MI] = y[MI];
    else if constexpr (cmul_col(K, 16, 512)) row[MI] = cmul(y[MI], c16);
    else row[MI] = cf{fmaf(-t1[MI], y[MI].i, y[MI].r), fmaf(t1[MI], y[MI].r, y[MI].i)};
    if constexpr (MI + 1 < 16) HalfTw<H, MI + 1>::run(y, t1, c16, row);
  }
};

// TAPER 1: real per-antenna weights h (Sec. "Controlling beam shape with
// windowing"), applied to the decoded nibbles before the E-W DFT as in the
// kernel above (WindowLane), from one LDS copy per workgroup.
template <int TAPER = 0>
__device__ __forceinline__ void fft32_h_run(const Fft32Args& p) {
  constexpr int N = 256, G = 16, L = 16, M = 512;
  constexpr int NSL = dit_slots(G);
  constexpr int YS = L + 1;
  static_assert(L + NSL <= kHRow && kHRow % 4 == 0 && (kHRow / 4) % 2 == 1, "table rows");
  static_assert((4 * M + 34) * 4 <= 64 * YS * 8, "block-end sums must fit the tile");
  __shared__ cf lds_tiles[kHWpg * 64 * YS];
  // [h][a1][44]: floats 0-15 the tangents of W_512^{a1 (2m + h)}, 16-40
  // the pass-2 multipliers of column k2 = 2 a1 + h; rows of 11 float4 chunks
  // put the 16 rows a lane group reads on different bank groups
  __shared__ __attribute__((aligned(16))) float lds_tab[2][G][kHRow];
  __shared__ cf lds_c16[G];                                           // whole twiddle of column k2 = 16
  static_assert(TAPER == 0 || TAPER == 1, "unwindowed or a real window");
  // the window [a_ns][a_ew] (TAPER 1)
  __shared__ __attribute__((aligned(16))) float lds_h[TAPER == 1 ? N * 4 : 1];

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  cf* const lds_y = lds_tiles + wave * 64 * YS;
  const int e1 = lane >> 4, a1 = lane & 15;

  for (int i = threadIdx.x; i < 2 * G * L; i += 64 * kHWpg) {
    const int h = i / (G * L), r = i % (G * L), aa = r / L, m = r % L;
    lds_tab[h][aa][m] = p.tw[aa * 32 + 2 * m + h].x;
  }
  for (int i = threadIdx.x; i < 32 * NSL; i += 64 * kHWpg) {
    const int k2 = i / NSL;
    lds_tab[k2 & 1][k2 >> 1][L + i % NSL] = p.mult[i];
  }
  if (threadIdx.x < G) {
    const float2 w = p.tw[threadIdx.x * 32 + 16];
    lds_c16[threadIdx.x] = cf{w.x, w.y};
  }
  if constexpr (TAPER == 1) {
    for (int i = threadIdx.x; i < N * 4; i += 64 * kHWpg) lds_h[i] = p.taper[i];
  }
  __syncthreads();
  const int64_t task = (int64_t)blockIdx.x * kHWpg + wave;
  if (task >= p.n_wg) return;
  int wg = (int)task;
  const int pg = wg % p.n_pg;
  wg /= p.n_pg;
  const int chan = wg % p.n_chan;
  const int blk = wg / p.n_chan;

  const int64_t t_base = (int64_t)blk * p.block;
  const int n_it = p.block;
  const int64_t frame_stride = (int64_t)(p.chan_stride ? p.chan_stride : p.n_chan) * p.n_pol * N;
  const int n_valid = (int)((p.n_time - t_base) < p.block ? (p.n_time - t_base) : p.block);
  cf* const row = &lds_y[lane * YS];

  {
    int wre = 0, wim = 0;
    WindowLane wl{};
    if constexpr (TAPER != 0) wl = window_lane(e1);
    else ew_weights(e1, wre, wim);

    float acc[2][G];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int k = 0; k < G; ++k) acc[h][k] = 0.f;

    for (int pi = 0; pi < p.pol_iter; ++pi) {
      const int pol = (p.pol_iter == 1) ? pg : pi;
      // the frame pointer is the wavefront's (scalar); the lane adds a1
      const uint32_t* q = p.volts + ((int64_t)chan * p.n_pol + pol) * N + t_base * frame_stride;
      uint32_t b[L];
#pragma unroll
      for (int j = 0; j < L; ++j) b[j] = __builtin_nontemporal_load(q + a1 + G * j);
      for (int it = 0; it < n_it; ++it) {
        cf x[L];
        if constexpr (TAPER == 1) {
#pragma unroll
          for (int j = 0; j < L; ++j) {
            const uint32_t d = b[j];
            const float4 h = *reinterpret_cast<const float4*>(&lds_h[(a1 + G * j) * 4]);
            const float h2 = wl.s * h.z, h3 = wl.s * h.w;
            const float pr = fmaf(h2, nib(d, 20), h.x * nib(d, 4));
            const float pim = fmaf(h2, nib(d, 16), h.x * nib(d, 0));
            const float qr = fmaf(h3, nib(d, wl.ou + 16), h.y * nib(d, wl.ou));
            const float qi = fmaf(h3, nib(d, wl.ov + 16), h.y * nib(d, wl.ov));
            x[j] = cf{fmaf(wl.tr, qr, pr), fmaf(wl.ti, qi, pim)};
          }
        } else {
#pragma unroll
          for (int j = 0; j < L; ++j) x[j] = cf{(float)sdot8((int)b[j], wre), (float)sdot8((int)b[j], wim)};
        }
        cf xo[L];
        padded_odd_t<L>(x, xo);
        dit<L>(x);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const cf* y = h ? xo : x;
          if (h == 1) {
            // the next frame's loads, in flight through this half (past the
            // block: the buffer's first frame, cached)
            q = (it + 1 >= n_it) ? p.volts : ((it + 1 < n_valid) ? q + frame_stride : q);
#pragma unroll
            for (int j = 0; j < L; ++j) b[j] = __builtin_nontemporal_load(q + a1 + G * j);
          }
          {
            float t1[L];
            const float4* tp = reinterpret_cast<const float4*>(&lds_tab[h][a1][0]);
#pragma unroll
            for (int k = 0; k < L / 4; ++k) {
              const float4 v = tp[k];
              t1[4 * k] = v.x;
              t1[4 * k + 1] = v.y;
              t1[4 * k + 2] = v.z;
              t1[4 * k + 3] = v.w;
            }
            // (the whole twiddle of column 16 is read per frame: held across
            // the frame loop it would take the last free register)
            if (h == 0) HalfTw<0, 0>::run(y, t1, lds_c16[a1], row);
            else HalfTw<1, 0>::run(y, t1, cf{}, row);
          }
          wave_lds_sync();
          cf z[G];
#pragma unroll
          for (int j = 0; j < G; ++j) z[j] = lds_y[(e1 * 16 + j) * YS + a1];
          wave_lds_sync();
          float mu[28];
          const float4* mp = reinterpret_cast<const float4*>(&lds_tab[h][a1][L]);
#pragma unroll
          for (int k = 0; k < 7; ++k) {
            const float4 v = mp[k];
            mu[4 * k] = v.x;
            mu[4 * k + 1] = v.y;
            mu[4 * k + 2] = v.z;
            mu[4 * k + 3] = v.w;
          }
          dit_rs<G>(z, mu);
#pragma unroll
          for (int k1 = 0; k1 < G; ++k1) acc[h][k1] = cnorm_acc(z[k1], acc[h][k1]);
        }
      }
    }

    // ---- block end: the kept beams of the channel, coalesced stores ----
    // E-W beam e's sums start at 512 e + (e & 1) + 32 (e >> 1): the four lane
    // groups of one store then cover all 64 banks
    float* lds_i = reinterpret_cast<float*>(lds_y);
    auto ebase = [](int e) { return e * M + (e & 1) + 32 * (e >> 1); };
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int k1 = 0; k1 < G; ++k1) lds_i[ebase(e1) + 2 * a1 + h + 32 * k1] = acc[h][k1];
    wave_lds_sync();
    const int keep = p.n_keep;
    const int32_t* sel = p.sel ? p.sel + (int64_t)chan * keep : nullptr;
    float* o = static_cast<float*>(p.out) + (((int64_t)blk * p.n_chan + chan) * p.n_pg + pg) * p.ew_rows * keep;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = e * p.ew_mul + p.ew_off;
      for (int j = lane; j < keep; j += 64) {
        const int A = sel ? sel[j] : j;
        o[r * keep + j] = lds_i[ebase(e) + A] * p.norm;
      }
    }
  }
}

// |B|^2 of the four beams of the unpadded 4-point E-W transform of one N-S
// beam, from its four E-W antenna columns z_q, added to acc[e]
__device__ __forceinline__ void ew4_beams_acc(const cf* z, float* acc) {
  const cf s02 = cadd(z[0], z[2]), d02 = csub(z[0], z[2]), s13 = cadd(z[1], z[3]), d13 = csub(z[1], z[3]);
  acc[0] = cnorm_acc(cadd(s02, s13), acc[0]);
  acc[2] = cnorm_acc(csub(s02, s13), acc[2]);
  acc[1] = cnorm_acc(cf{d02.r + d13.i, d02.i - d13.r}, acc[1]);   // d02 - i d13
  acc[3] = cnorm_acc(cf{d02.r - d13.i, d02.i + d13.r}, acc[3]);   // d02 + i d13
}

// |B|^2 of the eight beams of the zero-padded 8-point E-W transform of one
// N-S beam, from its four E-W antenna columns z_q, added to acc[E]: the even
// beams 2e are the 4-point DFT of z_q, the odd beams 2e + 1 that of
// w_q = z_q W_8^q, with w_0 = z_0, w_2 = -i z_2 and the factor 1/sqrt(2) of
// w_1 and w_3 applied in the last fused multiply-adds.
__device__ __forceinline__ void ew8_beams_acc(const cf* z, float* acc) {
  constexpr float kS = 0.70710678118654752f;
  const cf s02 = cadd(z[0], z[2]), d02 = csub(z[0], z[2]), s13 = cadd(z[1], z[3]), d13 = csub(z[1], z[3]);
  acc[0] = cnorm_acc(cadd(s02, s13), acc[0]);
  acc[4] = cnorm_acc(csub(s02, s13), acc[4]);
  acc[2] = cnorm_acc(cf{d02.r + d13.i, d02.i - d13.r}, acc[2]);   // d02 - i d13
  acc[6] = cnorm_acc(cf{d02.r - d13.i, d02.i + d13.r}, acc[6]);   // d02 + i d13
  const cf S02 = cf{z[0].r + z[2].i, z[0].i - z[2].r};            // w_0 + w_2
  const cf D02 = cf{z[0].r - z[2].i, z[0].i + z[2].r};            // w_0 - w_2
  // sqrt(2) w_1 = z_1 (1 - i), sqrt(2) w_3 = -z_3 (1 + i), so their sum and
  // difference come from s13 and d13
  const cf S13 = cf{d13.r + s13.i, d13.i - s13.r};                 // sqrt(2) (w_1 + w_3)
  const cf D13 = cf{s13.r + d13.i, s13.i - d13.r};                 // sqrt(2) (w_1 - w_3)
  acc[1] = cnorm_acc(cf{fmaf(kS, S13.r, S02.r), fmaf(kS, S13.i, S02.i)}, acc[1]);
  acc[5] = cnorm_acc(cf{fmaf(-kS, S13.r, S02.r), fmaf(-kS, S13.i, S02.i)}, acc[5]);
  acc[3] = cnorm_acc(cf{fmaf(kS, D13.i, D02.r), fmaf(-kS, D13.r, D02.i)}, acc[3]);   // D02 - i D13
  acc[7] = cnorm_acc(cf{fmaf(-kS, D13.i, D02.r), fmaf(kS, D13.r, D02.i)}, acc[7]);   // D02 + i D13
}

// The 4 x 256 intensities with the E-W axis zero-padded to 8 beams, N-S
// transform first.  The transforms along the two axes commute, so the
// zero-padded N-S transform runs on the four E-W antenna columns (lane
// (q, a1) of pass 1 takes the nibbles of antenna q instead of an E-W beam's
// dot products): the same work as the unpadded step.  After pass 2 the four
// columns of each N-S beam meet in one lane through the wavefront's LDS
// tile, which forms all eight E-W beams and their |B|^2: lane (g, m) holds
// the N-S beams A = (2 m + h) + 32 (4 g + r), r < 4, of half h.  The block
// sums leave in two rounds, the even E-W beams and then the odd ones, so
// that each round fits the tile.  TAPER 1 (real per-antenna weights) and 2
// (complex gains, or real weights when gain_src is 1) scale each decoded
// antenna value before the N-S transform, from one LDS copy per workgroup.
template <int TAPER, int MEW>
__device__ __forceinline__ void fft32_nsf_run(const Fft32Args& p) {
  static_assert(MEW == 4 || MEW == 8, "E-W transform of 4 or 8 beams");
  constexpr int N = 256, G = 16, L = 16, M = 512;
  constexpr int NSL = dit_slots(G);
  constexpr int YS = L + 1;
  static_assert(L + NSL <= kHRow && kHRow % 4 == 0 && (kHRow / 4) % 2 == 1, "table rows");
  static_assert((4 * M + 34) * 4 <= 64 * YS * 8, "block-end sums of four E-W rows must fit the tile");
  static_assert(G * 4 * 16 <= 64 * YS, "the E-W transposition must fit the tile");
  __shared__ cf lds_tiles[kHWpg * 64 * YS];
  __shared__ __attribute__((aligned(16))) float lds_tab[2][G][kHRow];
  __shared__ cf lds_c16[G];
  // the factor of antenna (a_ns, q) at [q][a_ns] (TAPER 2: complex, interleaved)
  __shared__ float lds_h[TAPER == 2 ? N * 8 : TAPER == 1 ? N * 4 : 1];

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  cf* const lds_y = lds_tiles + wave * 64 * YS;
  const int e1 = lane >> 4, a1 = lane & 15;      // pass 1 and 2: E-W antenna column e1
  if constexpr (TAPER == 1) {
    for (int i = threadIdx.x; i < N * 4; i += 64 * kHWpg) lds_h[(i & 3) * N + (i >> 2)] = p.taper[i];
  } else if constexpr (TAPER == 2) {
    for (int i = threadIdx.x; i < N * 4; i += 64 * kHWpg) {
      const int o = 2 * ((i & 3) * N + (i >> 2));
      lds_h[o] = p.gain_src == 2 ? p.taper[2 * i] : p.gain_src == 1 ? p.taper[i] : 1.f;
      lds_h[o + 1] = p.gain_src == 2 ? p.taper[2 * i + 1] : 0.f;
    }
  }

  for (int i = threadIdx.x; i < 2 * G * L; i += 64 * kHWpg) {
    const int h = i / (G * L), r = i % (G * L), aa = r / L, m = r % L;
    lds_tab[h][aa][m] = p.tw[aa * 32 + 2 * m + h].x;
  }
  for (int i = threadIdx.x; i < 32 * NSL; i += 64 * kHWpg) {
    const int k2 = i / NSL;
    lds_tab[k2 & 1][k2 >> 1][L + i % NSL] = p.mult[i];
  }
  if (threadIdx.x < G) {
    const float2 w = p.tw[threadIdx.x * 32 + 16];
    lds_c16[threadIdx.x] = cf{w.x, w.y};
  }
  __syncthreads();
  const int64_t task = (int64_t)blockIdx.x * kHWpg + wave;
  if (task >= p.n_wg) return;
  int wg = (int)task;
  const int pg = wg % p.n_pg;
  wg /= p.n_pg;
  const int chan = wg % p.n_chan;
  const int blk = wg / p.n_chan;

  const int64_t t_base = (int64_t)blk * p.block;
  const int n_it = p.block;
  const int64_t frame_stride = (int64_t)(p.chan_stride ? p.chan_stride : p.n_chan) * p.n_pol * N;
  const int n_valid = (int)((p.n_time - t_base) < p.block ? (p.n_time - t_base) : p.block);
  cf* const row = &lds_y[lane * YS];
  const int sh_re = 8 * e1 + 4, sh_im = 8 * e1;    // antenna e1: real part high nibble, imaginary low

  float acc[2][4][MEW];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int e = 0; e < MEW; ++e) acc[h][r][e] = 0.f;

  for (int pi = 0; pi < p.pol_iter; ++pi) {
    const int pol = (p.pol_iter == 1) ? pg : pi;
    const uint32_t* q = p.volts + ((int64_t)chan * p.n_pol + pol) * N + t_base * frame_stride;
    uint32_t b[L];
#pragma unroll
    for (int j = 0; j < L; ++j) b[j] = __builtin_nontemporal_load(q + a1 + G * j);
    for (int it = 0; it < n_it; ++it) {
      cf x[L];
#pragma unroll
      for (int j = 0; j < L; ++j) {
        const float xr = nib(b[j], sh_re), xi = nib(b[j], sh_im);
        if constexpr (TAPER == 1) {
          const float hh = lds_h[e1 * N + a1 + G * j];
          x[j] = cf{hh * xr, hh * xi};
        } else if constexpr (TAPER == 2) {
          const float2 gg = *reinterpret_cast<const float2*>(&lds_h[2 * (e1 * N + a1 + G * j)]);
          x[j] = cf{fmaf(-gg.y, xi, gg.x * xr), fmaf(gg.y, xr, gg.x * xi)};
        } else {
          x[j] = cf{xr, xi};
        }
      }
      cf xo[L];
      padded_odd_t<L>(x, xo);
      dit<L>(x);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const cf* y = h ? xo : x;
        if (h == 1) {
          q = (it + 1 >= n_it) ? p.volts : ((it + 1 < n_valid) ? q + frame_stride : q);
#pragma unroll
          for (int j = 0; j < L; ++j) b[j] = __builtin_nontemporal_load(q + a1 + G * j);
        }
        {
          float t1[L];
          const float4* tp = reinterpret_cast<const float4*>(&lds_tab[h][a1][0]);
#pragma unroll
          for (int k = 0; k < L / 4; ++k) {
            const float4 v = tp[k];
            t1[4 * k] = v.x;
            t1[4 * k + 1] = v.y;
            t1[4 * k + 2] = v.z;
            t1[4 * k + 3] = v.w;
          }
          if (h == 0) HalfTw<0, 0>::run(y, t1, lds_c16[a1], row);
          else HalfTw<1, 0>::run(y, t1, cf{}, row);
        }
        wave_lds_sync();
        cf z[G];
#pragma unroll
        for (int j = 0; j < G; ++j) z[j] = lds_y[(e1 * 16 + j) * YS + a1];
        wave_lds_sync();
        {
          float mu[28];
          const float4* mp = reinterpret_cast<const float4*>(&lds_tab[h][a1][L]);
#pragma unroll
          for (int k = 0; k < 7; ++k) {
            const float4 v = mp[k];
            mu[4 * k] = v.x;
            mu[4 * k + 1] = v.y;
            mu[4 * k + 2] = v.z;
            mu[4 * k + 3] = v.w;
          }
          dit_rs<G>(z, mu);
        }
        // z[k1]: N-S beam (2 a1 + h) + 32 k1 of column e1, to slot (k1, e1, a1)
#pragma unroll
        for (int k1 = 0; k1 < G; ++k1) lds_y[k1 * 64 + lane] = z[k1];
        wave_lds_sync();
        // lane (g, m) = (e1, a1) takes k1 = 4 g + r of every column
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          cf zq[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) zq[c] = lds_y[(4 * e1 + r) * 64 + c * 16 + a1];
          if constexpr (MEW == 8) ew8_beams_acc(zq, acc[h][r]);
          else ew4_beams_acc(zq, acc[h][r]);
        }
        wave_lds_sync();
      }
    }
  }

  // ---- block end: the kept beams of the channel, even E-W rows, then odd ----
  float* lds_i = reinterpret_cast<float*>(lds_y);
  auto ebase = [](int e) { return e * M + (e & 1) + 32 * (e >> 1); };
  const int keep = p.n_keep;
  const int32_t* sel = p.sel ? p.sel + (int64_t)chan * keep : nullptr;
  float* o = static_cast<float*>(p.out) + (((int64_t)blk * p.n_chan + chan) * p.n_pg + pg) * p.ew_rows * keep;
#pragma unroll
  for (int odd = 0; odd < MEW / 4; ++odd) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          lds_i[ebase(e) + 2 * a1 + h + 32 * (4 * e1 + r)] = acc[h][r][MEW == 8 ? 2 * e + odd : e];
    wave_lds_sync();
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      for (int j = lane; j < keep; j += 64) {
        const int A = sel ? sel[j] : j;
        o[(MEW == 8 ? 2 * e + odd : e * p.ew_mul + p.ew_off) * keep + j] = lds_i[ebase(e) + A] * p.norm;
      }
    }
    wave_lds_sync();
  }
}

__global__ __launch_bounds__(64 * kHWpg) __attribute__((amdgpu_waves_per_eu(3))) void k_fft32_ew8(Fft32Args p) {
  fft32_nsf_run<0, 8>(p);
}

__global__ __launch_bounds__(64 * kHWpg) __attribute__((amdgpu_waves_per_eu(3))) void k_fft32_ew8w(Fft32Args p) {
  fft32_nsf_run<1, 8>(p);
}

__global__ __launch_bounds__(64 * kHWpg) __attribute__((amdgpu_waves_per_eu(3))) void k_fft32_ew8g(Fft32Args p) {
  fft32_nsf_run<2, 8>(p);
}

__global__ __launch_bounds__(64 * kHWpg) __attribute__((amdgpu_waves_per_eu(3))) void k_fft32_ng(Fft32Args p) {
  fft32_nsf_run<2, 4>(p);
}

__global__ __launch_bounds__(64 * kHWpg) __attribute__((amdgpu_waves_per_eu(4))) void k_fft32_h(Fft32Args p) {
  fft32_h_run<0>(p);
}

// the window's LDS copy (4 KB) leaves room for three workgroups of four
// wavefronts per CU, so the registers may take three wavefronts per SIMD
__global__ __launch_bounds__(64 * kHWpg) __attribute__((amdgpu_waves_per_eu(3))) void k_fft32_hw(Fft32Args p) {
  fft32_h_run<1>(p);
}


template <int N, int G, int T, int FOLD = 1>
void launch_nt(const Fft32Args& a, bool cplx, hipStream_t s) {
  constexpr int W = fft32_wpg<N, G, T, FOLD>();
  const dim3 grid((unsigned)((a.n_wg + W - 1) / W)), threads(64 * W);
  if (cplx) hipLaunchKernelGGL((k_fft32<N, G, T, true, FOLD>), grid, threads, 0, s, a);
  else hipLaunchKernelGGL((k_fft32<N, G, T, false, FOLD>), grid, threads, 0, s, a);
}

// The one choice of the group size G for each transform length N (and fold):
// the launches below take it as a template argument and the plan sizes its
// pass-1 twiddle and pass-2 multiplier tables with it (fft32_group).
// Co-adding at N = 128 uses G = 8, two frames per pass, so that the even
// columns' pass-2 tasks tile the wavefront.
constexpr int fft32_g(int n, int fold) {
  return n == 16 ? 4 : n == 32 ? 8 : n == 64 ? 8 : n == 128 ? (fold > 1 ? 8 : 16) : n == 256 ? 16 : 0;
}

// cyclic co-adding: no window, or a real window for folds up to 8 (the
// 16-fold windowed variant would not fit its registers)
template <int N, int FOLD>
hipError_t launch_fold(const Fft32Args& a, int taper, bool cplx, hipStream_t s) {
  constexpr int G = fft32_g(N, FOLD);
  if (taper == 0) {
    launch_nt<N, G, 0, FOLD>(a, cplx, s);
  } else if (taper == 1) {
    if constexpr (FOLD <= 8) launch_nt<N, G, 1, FOLD>(a, cplx, s);
    else return hipErrorNotSupported;
  } else {
    return hipErrorNotSupported;
  }
  return hipGetLastError();
}

template <int N>
hipError_t launch_n(const Fft32Args& a, int taper, bool cplx, hipStream_t s) {
  constexpr int G = fft32_g(N, 1);
  if constexpr (N == 256) {
    if (taper == 0 && !cplx) {       // the 4 x 256 intensities: half-size tiles, four waves per SIMD
      const dim3 grid((unsigned)((a.n_wg + kHWpg - 1) / kHWpg)), threads(64 * kHWpg);
      if (a.ew_rows == 8) hipLaunchKernelGGL(k_fft32_ew8, grid, threads, 0, s, a);   // even and odd E-W beams
      else hipLaunchKernelGGL(k_fft32_h, grid, threads, 0, s, a);
      return hipGetLastError();
    }
    if ((taper == 1 || taper == 2) && !cplx) {   // windowed or gain-weighted 4 x 256 intensities
      const dim3 grid((unsigned)((a.n_wg + kHWpg - 1) / kHWpg)), threads(64 * kHWpg);
      if (a.ew_rows == 8) {                      // with the E-W axis padded: all eight E-W beams
        if (taper == 1) hipLaunchKernelGGL(k_fft32_ew8w, grid, threads, 0, s, a);
        else hipLaunchKernelGGL(k_fft32_ew8g, grid, threads, 0, s, a);
      } else if (taper == 1) {
        hipLaunchKernelGGL(k_fft32_hw, grid, threads, 0, s, a);
      } else {
        hipLaunchKernelGGL(k_fft32_ng, grid, threads, 0, s, a);
      }
      return hipGetLastError();
    }
  }
  if (taper == 3) launch_nt<N, G, 3>(a, cplx, s);
  else if (taper == 2) launch_nt<N, G, 2>(a, cplx, s);
  else if (taper == 1) launch_nt<N, G, 1>(a, cplx, s);
  else launch_nt<N, G, 0>(a, cplx, s);
  return hipGetLastError();
}

}  // namespace

int fft32_group(int n_ns, int fold) { return fft32_g(n_ns, fold); }

bool fft32_fuses_ew8(int n_ns, int taper, bool cplx, int fold) {
  return n_ns == 256 && taper >= 0 && taper <= 2 && !cplx && fold == 1;
}

hipError_t launch_fft32(const Fft32Args& a, int n_ns, int taper, bool cplx, int64_t n_wg,
                        hipStream_t s) {
  Fft32Args b = a;
  b.n_wg = n_wg;
  if (b.fold > 1) {
    const int key = n_ns * 1000 + b.fold;
    switch (key) {
      case 16002: return launch_fold<16, 2>(b, taper, cplx, s);
      case 16004: return launch_fold<16, 4>(b, taper, cplx, s);
      case 16008: return launch_fold<16, 8>(b, taper, cplx, s);
      case 16016: return launch_fold<16, 16>(b, taper, cplx, s);
      case 32002: return launch_fold<32, 2>(b, taper, cplx, s);
      case 32004: return launch_fold<32, 4>(b, taper, cplx, s);
      case 32008: return launch_fold<32, 8>(b, taper, cplx, s);
      case 64002: return launch_fold<64, 2>(b, taper, cplx, s);
      case 64004: return launch_fold<64, 4>(b, taper, cplx, s);
      case 128002: return launch_fold<128, 2>(b, taper, cplx, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (n_ns) {
    case 16: return launch_n<16>(b, taper, cplx, s);
    case 32: return launch_n<32>(b, taper, cplx, s);
    case 64: return launch_n<64>(b, taper, cplx, s);
    case 128: return launch_n<128>(b, taper, cplx, s);
    case 256: return launch_n<256>(b, taper, cplx, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fftbf
