// Newton's-method localisation of a point source from one row of FFT-beam
// intensities of a linear array (Sec. "Localization"), batched over rows.
//
// With the regridded pointed beam of eq. e:bp_max_arbitrary,
//   b_p(y) = sum_A w^A(y) b_A,   w^A(y) = D(y - A/M) / M,
//   D(u) = sin((2n-1) pi u) / sin(pi u),
// the estimator in y = (d/lambda) sin(theta) replaces the likelihood's
// curvature by its value at the maximum (the baseline moment of inertia,
// eq. e:baseline_MOI) and iterates
//   y <- y + n^2 b_p'(y) / (4 pi^2 MOI b_p(y)),
// starting from the strongest FFT beam and summing over the K beams nearest
// it (the paper keeps ~10).  An update is not taken, and the iteration
// stops, when b_p <= 0 or when it would leave one beam spacing around the
// starting beam.
//
// Each 64-lane wavefront takes the argmax of its rows (lane l holds the PER
// consecutive beams from l PER on, all rows' loads in flight together,
// deterministic lowest-index tie break), then runs the Newton phase for all
// of them at once: with windows of up to 16 beams, four rows per wavefront
// in 16-lane groups (else one row per wavefront).  Lane j < K of a group owns
// beam A_0 - (K-1)/2 + j and evaluates D and D' in FP64 in closed form (with
// a Taylor branch within 0.01 / (pi (2n-1)) of an integer, where the closed
// form of D' cancels); the two sums are segmented shuffle reductions.
#include "dev_common.h"
#include "kernels.h"

namespace fftbf {

namespace {

constexpr double kPiD = 3.14159265358979323846;

// D(u) and dD/du for N = 2n - 1 (odd, so D has period 1 and is even).
__device__ __forceinline__ void dirichlet(double u, int N, double& d, double& dd) {
  const double e = u - rint(u);
  const double Nd = (double)N;
  if (fabs(Nd * e) < 0.01 / kPiD) {
    const double x = kPiD * e, x2 = x * x, N2 = Nd * Nd;
    const double c4 = (3.0 * N2 * N2 - 10.0 * N2 + 7.0);
    d = Nd * (1.0 - (N2 - 1.0) * x2 / 6.0 + c4 * x2 * x2 / 360.0);
    dd = kPiD * Nd * (-(N2 - 1.0) * x / 3.0 + c4 * x2 * x / 90.0);
    return;
  }
  double s, c, S, C;
  sincospi(e, &s, &c);
  sincospi(Nd * e, &S, &C);
  const double inv = 1.0 / s;                     // one division: dD = pi (N C - D c) / s
  d = S * inv;
  dd = kPiD * (Nd * C - d * c) * inv;
}

// sum over the G-lane group of this lane (G a power of two <= 64)
template <int G>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// G lanes per row in the Newton phase: G = 16 packs 4 rows per wavefront
// (windows of up to 16 beams), G = 64 gives a row the whole wavefront.
// PER = max(1, m / 64) beams per lane in the argmax; VEC loads them as
// 16-byte vectors (PER >= 4 and a 16-byte aligned input).
template <int G, int PER, bool VEC>
__global__ __launch_bounds__(256) void k_localize(LocArgs a) {
  constexpr int RW = 64 / G;                       // rows per wavefront
  const int lane = threadIdx.x & 63;
  const int64_t row0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * RW;
  if (row0 >= a.n_rows) return;                    // wave-uniform
  const int m = a.m;

  // every row's loads first, so that the wave waits for memory once
  float v[RW][PER];
#pragma unroll
  for (int r = 0; r < RW; ++r) {
    const bool ok = row0 + r < a.n_rows;           // wave-uniform
    const float* x = a.in + (ok ? row0 + r : row0) * m + lane * PER;
    if constexpr (VEC) {
#pragma unroll
      for (int q = 0; q < PER / 4; ++q) {
        const float4 f = reinterpret_cast<const float4*>(x)[q];
        v[r][4 * q] = f.x;
        v[r][4 * q + 1] = f.y;
        v[r][4 * q + 2] = f.z;
        v[r][4 * q + 3] = f.w;
      }
    } else {
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        v[r][i] = -INFINITY;
        if (lane * PER + i < m) v[r][i] = x[i];     // lanes past a short row load nothing
      }
    }
  }

  // argmax of each of the wave's rows
  int a0v[RW];
#pragma unroll
  for (int r = 0; r < RW; ++r) {
    a0v[r] = 0;
    if (row0 + r >= a.n_rows) continue;            // wave-uniform
    float best = -INFINITY;
    int bi = 0x7FFFFFFF;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      if (lane * PER + i < m && v[r][i] > best) {
        best = v[r][i];
        bi = lane * PER + i;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const float ov = __shfl_xor(best, off);
      const int oi = __shfl_xor(bi, off);
      if (ov > best || (ov == best && oi < bi)) {
        best = ov;
        bi = oi;
      }
    }
    a0v[r] = bi == 0x7FFFFFFF ? 0 : bi;
  }

  // Newton phase: lane = (row r of the wave, window beam j)
  const int r = lane / G, j = lane % G;
  int a0 = a0v[0];
#pragma unroll
  for (int q = 1; q < RW; ++q)
    if (r == q) a0 = a0v[q];
  const int64_t row = row0 + r;
  const bool row_ok = row < a.n_rows;
  const int K = a.n_window;
  const bool active = row_ok && j < K;
  const int Aj = (((a0 - (K - 1) / 2 + j) % m) + m) % m;
  const double bj = active ? (double)a.in[row * m + Aj] : 0.0;
  const double inv_m = 1.0 / (double)m;
  const double y0 = (double)a0 * inv_m;
  const double gain = (double)a.n * (double)a.n / (4.0 * kPiD * kPiD * a.moi);
  const int N = 2 * a.n - 1;

  auto eval = [&](double y, double& p, double& dp) {
    double d = 0.0, dd = 0.0;
    if (active) dirichlet(y - (double)Aj * inv_m, N, d, dd);
    p = group_sum<G>(d * bj) * inv_m;
    dp = group_sum<G>(dd * bj) * inv_m;
  };

  double y = y0, p, dp;
  bool done = false;
  for (int it = 0; it < a.n_iter; ++it) {
    eval(y, p, dp);
    if (!done) {
      const double yn = y + gain * dp / p;
      if (!(p > 0.0) || fabs(yn - y0) > inv_m) done = true;
      else y = yn;
    }
  }
  eval(y, p, dp);
  if (row_ok && j == 0) {
    const double yw = (y + 0.5) - floor(y + 0.5) - 0.5;
    const int chan = (int)((row / a.rows_per_chan_blk) % a.n_chan);
    a.sin_out[row] = yw / a.dl[2 * chan + 1];
    if (a.peak_out) a.peak_out[row] = (float)p;
  }
}

}  // namespace

namespace {

template <int G, int PER>
void launch_loc(const LocArgs& a, bool vec, unsigned nb, hipStream_t s) {
  if constexpr (PER >= 4) {
    if (vec) {
      hipLaunchKernelGGL((k_localize<G, PER, true>), dim3(nb), dim3(256), 0, s, a);
      return;
    }
  }
  hipLaunchKernelGGL((k_localize<G, PER, false>), dim3(nb), dim3(256), 0, s, a);
}

template <int G>
hipError_t launch_loc_g(const LocArgs& a, unsigned nb, hipStream_t s) {
  const bool vec = (reinterpret_cast<uintptr_t>(a.in) % 16) == 0;
  switch (a.m) {
    case 32:
    case 64: launch_loc<G, 1>(a, vec, nb, s); break;
    case 128: launch_loc<G, 2>(a, vec, nb, s); break;
    case 256: launch_loc<G, 4>(a, vec, nb, s); break;
    case 512: launch_loc<G, 8>(a, vec, nb, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_localize(const LocArgs& a, hipStream_t s) {
  if (a.n_rows <= 0) return hipSuccess;
  if (a.n_window < 1 || a.n_window > 64 || a.n_window > a.m) return hipErrorInvalidValue;
  const bool packed = a.n_window <= 16;
  const int64_t waves = packed ? (a.n_rows + 3) / 4 : a.n_rows;
  const int64_t nb = (waves + 3) / 4;
  if (nb > 0x7FFFFFFF) return hipErrorInvalidConfiguration;
  return packed ? launch_loc_g<16>(a, (unsigned)nb, s) : launch_loc_g<64>(a, (unsigned)nb, s);
}

}  // namespace fftbf
