// Device-side helpers for the gfx950 beamforming kernels: complex FP32
// arithmetic, compile-time DFT coefficients (evaluated in double precision
// by the compiler) and fully unrolled in-register radix-2 transforms.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fftbf {

struct cf {
  float r, i;
};

__device__ __forceinline__ cf cadd(cf a, cf b) { return {a.r + b.r, a.i + b.i}; }
__device__ __forceinline__ cf csub(cf a, cf b) { return {a.r - b.r, a.i - b.i}; }
// a * w, two multiplies and two fused multiply-adds
__device__ __forceinline__ cf cmul(cf a, cf w) {
  return {fmaf(a.r, w.r, -(a.i * w.i)), fmaf(a.r, w.i, a.i * w.r)};
}
__device__ __forceinline__ float cnorm(cf a) { return fmaf(a.r, a.r, a.i * a.i); }
// acc + |a|^2 as two fused multiply-adds
__device__ __forceinline__ float cnorm_acc(cf a, float acc) { return fmaf(a.r, a.r, fmaf(a.i, a.i, acc)); }

// ---- compile-time exp(-i 2 pi k / M) in double --------------------------
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double cx_sin(double x) {
  double term = x, sum = x;
  for (int n = 1; n < 24; ++n) {
    term *= -x * x / double((2 * n) * (2 * n + 1));
    sum += term;
  }
  return sum;
}
constexpr double cx_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int n = 1; n < 24; ++n) {
    term *= -x * x / double((2 * n - 1) * (2 * n));
    sum += term;
  }
  return sum;
}
// angle reduced to [-pi, pi] through the integer index before the series
constexpr double tw_re(int k, int m) {
  k = ((k % m) + m) % m;
  int s = (2 * k > m) ? k - m : k;
  return cx_cos(-2.0 * kPi * double(s) / double(m));
}
constexpr double tw_im(int k, int m) {
  k = ((k % m) + m) % m;
  int s = (2 * k > m) ? k - m : k;
  return cx_sin(-2.0 * kPi * double(s) / double(m));
}

// x * W_M^k for a compile-time (k, M); the four axis-aligned twiddles are
// exact sign/swap operations.
template <int K, int M>
__device__ __forceinline__ cf twiddle(cf x) {
  constexpr int k = ((K % M) + M) % M;
  if constexpr (k == 0) {
    return x;
  } else if constexpr (4 * k == M) {          // -i
    return {x.i, -x.r};
  } else if constexpr (2 * k == M) {          // -1
    return {-x.r, -x.i};
  } else if constexpr (4 * k == 3 * M) {      // +i
    return {-x.i, x.r};
  } else {
    constexpr float wr = float(tw_re(k, M));
    constexpr float wi = float(tw_im(k, M));
    return cmul(x, cf{wr, wi});
  }
}

// ---- in-register radix-2 decimation-in-frequency ------------------------
// Natural-order input, bit-reversed output: after dif<L>(x), x[bitrev(k)]
// holds sum_j x_in[j] W_L^{jk}.
template <int L, int SPAN, int S, int J>
struct DifBfly {
  static __device__ __forceinline__ void run(cf* x) {
    cf a = x[S + J], b = x[S + J + SPAN];
    x[S + J] = cadd(a, b);
    x[S + J + SPAN] = twiddle<J, 2 * SPAN>(csub(a, b));
    if constexpr (J + 1 < SPAN) DifBfly<L, SPAN, S, J + 1>::run(x);
  }
};
template <int L, int SPAN, int S>
struct DifGroup {
  static __device__ __forceinline__ void run(cf* x) {
    DifBfly<L, SPAN, S, 0>::run(x);
    if constexpr (S + 2 * SPAN < L) DifGroup<L, SPAN, S + 2 * SPAN>::run(x);
  }
};
template <int L, int SPAN>
struct DifStage {
  static __device__ __forceinline__ void run(cf* x) {
    DifGroup<L, SPAN, 0>::run(x);
    if constexpr (SPAN > 1) DifStage<L, SPAN / 2>::run(x);
  }
};
template <int L>
__device__ __forceinline__ void dif(cf* x) {
  if constexpr (L > 1) DifStage<L, L / 2>::run(x);
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }
constexpr int bitrev(int k, int n) {
  int r = 0;
  for (int b = 0; b < ilog2(n); ++b) r |= ((k >> b) & 1) << (ilog2(n) - 1 - b);
  return r;
}

// ---- in-register radix-2 decimation-in-time ------------------------------
// Butterfly a' = a + W b, b' = a - W b with W = W_M^K fixed at compile time.
// A general twiddle is factored as W = c (1 + i t), t = s/c (|c| >= |s|), or
// W = s (u + i), u = c/s (otherwise), so that W b costs two fused
// multiply-adds and the outer factor folds into the butterfly's own four
// fused multiply-adds: 6 operations instead of 8.
constexpr double cx_abs(double v) { return v < 0 ? -v : v; }

template <int K, int M>
__device__ __forceinline__ void bfly(cf& a, cf& b) {
  constexpr int k = ((K % M) + M) % M;
  if constexpr (k == 0) {
    const cf t = a;
    a = cadd(t, b);
    b = csub(t, b);
  } else if constexpr (4 * k == M) {          // W = -i
    const cf wb{b.i, -b.r}, t = a;
    a = cadd(t, wb);
    b = csub(t, wb);
  } else if constexpr (2 * k == M) {          // W = -1
    const cf t = a;
    a = csub(t, b);
    b = cadd(t, b);
  } else if constexpr (4 * k == 3 * M) {      // W = +i
    const cf wb{-b.i, b.r}, t = a;
    a = cadd(t, wb);
    b = csub(t, wb);
  } else {
    constexpr double c = tw_re(k, M), s = tw_im(k, M);
    cf bp;
    float f;
    if constexpr (cx_abs(c) >= cx_abs(s)) {
      constexpr float t = float(s / c);
      f = float(c);
      bp = cf{fmaf(-t, b.i, b.r), fmaf(t, b.r, b.i)};
    } else {
      constexpr float u = float(c / s);
      f = float(s);
      bp = cf{fmaf(u, b.r, -b.i), fmaf(u, b.i, b.r)};
    }
    const cf t0 = a;
    a = cf{fmaf(f, bp.r, t0.r), fmaf(f, bp.i, t0.i)};
    b = cf{fmaf(-f, bp.r, t0.r), fmaf(-f, bp.i, t0.i)};
  }
}

template <int SIZE, int S, int J>
struct DitBfly {
  static __device__ __forceinline__ void run(cf* y) {
    bfly<J, SIZE>(y[S + J], y[S + J + SIZE / 2]);
    if constexpr (J + 1 < SIZE / 2) DitBfly<SIZE, S, J + 1>::run(y);
  }
};
template <int L, int SIZE, int S>
struct DitGroup {
  static __device__ __forceinline__ void run(cf* y) {
    DitBfly<SIZE, S, 0>::run(y);
    if constexpr (S + SIZE < L) DitGroup<L, SIZE, S + SIZE>::run(y);
  }
};
template <int L, int SIZE>
struct DitStage {
  static __device__ __forceinline__ void run(cf* y) {
    DitGroup<L, SIZE, 0>::run(y);
    if constexpr (SIZE < L) DitStage<L, SIZE * 2>::run(y);
  }
};

// In-place L-point DFT, natural order in and out: x[k] <- sum_j x[j] W_L^{jk}.
// (The bit-reversal permutation is a compile-time renaming of registers.)
template <int L>
__device__ __forceinline__ void dit(cf* x) {
  if constexpr (L > 1) {
    cf y[L];
#pragma unroll
    for (int i = 0; i < L; ++i) y[i] = x[bitrev(i, L)];
    DitStage<L, 2>::run(y);
#pragma unroll
    for (int i = 0; i < L; ++i) x[i] = y[i];
  }
}

// Zero-padded DFT, L non-zero inputs -> 2L outputs in natural order:
// y[k] = sum_{j<L} x[j] W_{2L}^{jk}.  Even outputs are the L-point DFT of x,
// odd outputs the L-point DFT of x_j W_{2L}^j (the first stage of the 2L-point
// transform with a zero upper half).
template <int L, int J>
struct PadPre {
  static __device__ __forceinline__ void run(const cf* x, cf* xo) {
    xo[J] = twiddle<J, 2 * L>(x[J]);
    if constexpr (J + 1 < L) PadPre<L, J + 1>::run(x, xo);
  }
};
template <int L>
__device__ __forceinline__ void padded_dft(cf* x /* in: [L], */, cf* y /* out: [2L] */) {
  cf xo[L];
  PadPre<L, 0>::run(x, xo);
  dit<L>(x);
  dit<L>(xo);
#pragma unroll
  for (int m = 0; m < L; ++m) {
    y[2 * m] = x[m];
    y[2 * m + 1] = xo[m];
  }
}

// ---- scaled radix-2 decimation in time -----------------------------------
// A twiddle in tangent form, W = f (1 + i t) or W = f (u + i), costs two fused
// multiply-adds when its real factor f is left on the value: the value held
// is then the true value divided by its scale f.  A DIT butterfly whose
// operands carry scales s_top and s_bot costs no more than the plain one
// (4 operations, or 6 with a non-trivial twiddle of its own) when the bottom
// operand is multiplied by mu = f_W s_bot / s_top, f_W being the outer factor
// of the butterfly's own tangent-form twiddle (1 for W = 1 or -i): both
// outputs then carry s_top.  Every value of a group [S, S + SIZE) leaves a
// stage with the scale of the group's first input, so after the last stage
// all outputs carry the scale of input 0, which is 1 for every use here.
constexpr bool tan_re_form(int k, int m) { return cx_abs(tw_re(k, m)) >= cx_abs(tw_im(k, m)); }
constexpr double tan_outer(int k, int m) { return tan_re_form(k, m) ? tw_re(k, m) : tw_im(k, m); }
constexpr bool dit_trivial(int j, int size) { return j == 0 || 4 * j == size; }

// multipliers of a scaled G-point DIT: one per (stage, group) for its
// trivial-twiddle butterflies, one more per non-trivial twiddle
constexpr int dit_group_slots(int size) {
  int n = 1;
  for (int j = 0; j < size / 2; ++j) n += dit_trivial(j, size) ? 0 : 1;
  return n;
}
constexpr int dit_slots(int g) {
  int n = 0;
  for (int z = 2; z <= g; z *= 2) n += (g / z) * dit_group_slots(z);
  return n;
}
constexpr int dit_slot(int g, int size, int s, int j) {
  int base = 0;
  for (int z = 2; z < size; z *= 2) base += (g / z) * dit_group_slots(z);
  base += (s / size) * dit_group_slots(size);
  if (dit_trivial(j, size)) return base;
  int n = 1;
  for (int i = 0; i < j; ++i) n += dit_trivial(i, size) ? 0 : 1;
  return base + n;
}

template <int J, int SIZE>
__device__ __forceinline__ void bfly_mu(cf& a, cf& b, float mu) {
  const cf t0 = a;
  if constexpr (J == 0) {
    a = cf{fmaf(mu, b.r, t0.r), fmaf(mu, b.i, t0.i)};
    b = cf{fmaf(-mu, b.r, t0.r), fmaf(-mu, b.i, t0.i)};
  } else if constexpr (4 * J == SIZE) {       // W = -i: W b = (b.i, -b.r)
    a = cf{fmaf(mu, b.i, t0.r), fmaf(-mu, b.r, t0.i)};
    b = cf{fmaf(-mu, b.i, t0.r), fmaf(mu, b.r, t0.i)};
  } else {
    cf bp;
    if constexpr (tan_re_form(J, SIZE)) {
      constexpr float t = float(tw_im(J, SIZE) / tw_re(J, SIZE));
      bp = cf{fmaf(-t, b.i, b.r), fmaf(t, b.r, b.i)};
    } else {
      constexpr float u = float(tw_re(J, SIZE) / tw_im(J, SIZE));
      bp = cf{fmaf(u, b.r, -b.i), fmaf(u, b.i, b.r)};
    }
    a = cf{fmaf(mu, bp.r, t0.r), fmaf(mu, bp.i, t0.i)};
    b = cf{fmaf(-mu, bp.r, t0.r), fmaf(-mu, bp.i, t0.i)};
  }
}

// scaled G-point DIT with run-time multipliers mu[dit_slot(...)]
template <int G, int SIZE, int S, int J>
struct DitRs {
  static __device__ __forceinline__ void run(cf* y, const float* mu) {
    bfly_mu<J, SIZE>(y[S + J], y[S + J + SIZE / 2], mu[dit_slot(G, SIZE, S, J)]);
    if constexpr (J + 1 < SIZE / 2) DitRs<G, SIZE, S, J + 1>::run(y, mu);
    else if constexpr (S + SIZE < G) DitRs<G, SIZE, S + SIZE, 0>::run(y, mu);
    else if constexpr (SIZE < G) DitRs<G, 2 * SIZE, 0, 0>::run(y, mu);
  }
};
template <int G>
__device__ __forceinline__ void dit_rs(cf* x, const float* mu) {
  cf y[G];
#pragma unroll
  for (int i = 0; i < G; ++i) y[i] = x[bitrev(i, G)];
  DitRs<G, 2, 0, 0>::run(y, mu);
#pragma unroll
  for (int i = 0; i < G; ++i) x[i] = y[i];
}

// Zero-padded DFT as padded_dft, with the pre-twiddles x_j W_{2L}^j in
// tangent form and their factors carried through the odd half's DIT as
// compile-time multipliers (the outputs carry no scale).
constexpr double pad_scale(int j, int l) { return (j == 0 || 2 * j == l) ? 1.0 : tan_outer(j, 2 * l); }
constexpr double pad_mu(int l, int size, int s, int j) {
  const double rho = pad_scale(bitrev(s + size / 2, l), l) / pad_scale(bitrev(s, l), l);
  return dit_trivial(j, size) ? rho : rho * tan_outer(j, size);
}
template <int L, int SIZE, int S, int J>
struct DitPad {
  static __device__ __forceinline__ void run(cf* y) {
    constexpr float mu = float(pad_mu(L, SIZE, S, J));
    bfly_mu<J, SIZE>(y[S + J], y[S + J + SIZE / 2], mu);
    if constexpr (J + 1 < SIZE / 2) DitPad<L, SIZE, S, J + 1>::run(y);
    else if constexpr (S + SIZE < L) DitPad<L, SIZE, S + SIZE, 0>::run(y);
    else if constexpr (SIZE < L) DitPad<L, 2 * SIZE, 0, 0>::run(y);
  }
};
template <int L, int J>
struct PadPreT {
  static __device__ __forceinline__ void run(const cf* x, cf* xo) {
    constexpr int M = 2 * L;
    if constexpr (J == 0) {
      xo[0] = x[0];
    } else if constexpr (4 * J == M) {        // -i
      xo[J] = cf{x[J].i, -x[J].r};
    } else if constexpr (tan_re_form(J, M)) {
      constexpr float t = float(tw_im(J, M) / tw_re(J, M));
      xo[J] = cf{fmaf(-t, x[J].i, x[J].r), fmaf(t, x[J].r, x[J].i)};
    } else {
      constexpr float u = float(tw_re(J, M) / tw_im(J, M));
      xo[J] = cf{fmaf(u, x[J].r, -x[J].i), fmaf(u, x[J].i, x[J].r)};
    }
    if constexpr (J + 1 < L) PadPreT<L, J + 1>::run(x, xo);
  }
};
template <int L>
__device__ __forceinline__ void padded_dft_t(cf* x /* in: [L], */, cf* y /* out: [2L] */) {
  cf xo[L];
  PadPreT<L, 0>::run(x, xo);
  dit<L>(x);
  if constexpr (L > 1) {
    cf z[L];
#pragma unroll
    for (int i = 0; i < L; ++i) z[i] = xo[bitrev(i, L)];
    DitPad<L, 2, 0, 0>::run(z);
#pragma unroll
    for (int i = 0; i < L; ++i) xo[i] = z[i];
  }
#pragma unroll
  for (int m = 0; m < L; ++m) {
    y[2 * m] = x[m];
    y[2 * m + 1] = xo[m];
  }
}

// Pass-1 columns k of the M = 2L x G transform that keep the whole twiddle
// W_M^{a1 k}: those where some a1 < G has Re W = 0, which the tangent form
// cannot hold.
constexpr bool cmul_col(int k, int g, int m) {
  for (int a1 = 0; a1 < g; ++a1) {
    const int r = (a1 * k) % m;
    if (4 * r == m || 4 * r == 3 * m) return true;
  }
  return false;
}

// Task w of n_wg single-wavefront workgroups -> (polarisation group pg,
// rest = the task's other indices).  A 4 x 16 frame is 64 bytes, half a
// 128-byte line whose other half is the other polarisation, and consecutive
// workgroups go to different XCDs (separate L2 caches), so with two
// polarisation groups the pair is placed 8 apart (same XCD, close in time)
// and shares the line; a tail that is not a multiple of 16 keeps the plain
// order.
__device__ __forceinline__ int pol_pair_task(int w, int n_wg, int n_pg, int& pg) {
  if (n_pg == 2 && w < n_wg - n_wg % 16) {
    const int slot = w >> 3;
    pg = slot & 1;
    return ((slot >> 1) << 3) | (w & 7);
  }
  pg = w % n_pg;
  return w / n_pg;
}

// Signed 4-bit dot product of the eight nibbles of a and b, accumulator 0
// (the three-operand VOP3P form, so no register has to be zeroed first).
__device__ __forceinline__ int sdot8(int a, int b) {
  int r;
  asm("v_dot8_i32_i4 %0, %1, %2, 0" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

}  // namespace fftbf
