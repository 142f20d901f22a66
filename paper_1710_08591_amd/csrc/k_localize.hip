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
// Each 64-lane wavefront owns 64 rows.  It takes their argmax four rows at
// a time (lane l holds the PER consecutive beams from l PER on, the four
// rows' loads in flight together, deterministic lowest-index tie break;
// DPP rotations within rows of 16 lanes, then two lane permutes) and
// leaves each row's K window beams in LDS; then every lane runs the Newton
// phase for one row.  The window beams A_j = A_0 + j sit at u_j = u_0 - j/M,
// so one sincospi pair of u_0 per evaluation gives every beam's sines and
// cosines by the angle-addition formulas with the FP64 constants of j/M
// (held in LDS); D and D' then follow in closed form (one division), with a
// Taylor branch within 0.01 / (pi (2n-1)) of an integer, where the closed
// form of D' cancels.
#include "dev_common.h"
#include "kernels.h"

namespace fftbf {

namespace {

constexpr double kPiD = 3.14159265358979323846;

// One step of the wavefront argmax: combine with the (value, index) that
// the DPP control CTRL brings in (a rotation within each row of 16 lanes),
// the larger value winning and the lower index on ties.
template <int CTRL>
__device__ __forceinline__ void argmax_dpp(float& best, int& bi) {
  const float ov = __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, best), CTRL, 0xF, 0xF, false));
  const int oi = __builtin_amdgcn_update_dpp(0, bi, CTRL, 0xF, 0xF, false);
  if (ov > best || (ov == best && oi < bi)) {
    best = ov;
    bi = oi;
  }
}

// Window of up to KMAX beams per row (16 or 64); PER = max(1, m / 64) beams
// per lane in the argmax; VEC loads them as 16-byte vectors (PER >= 4 and a
// 16-byte aligned input).
template <int PER, bool VEC, int KMAX>
__global__ __launch_bounds__(256) void k_localize(LocArgs a) {
  constexpr int WS = KMAX + 1;                     // padded LDS row of window beams
  __shared__ float win[4][64 * WS];
  __shared__ double tab[4][KMAX];                  // cos, sin of pi j/M and of pi N j/M
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m = a.m, K = a.n_window, N = 2 * a.n - 1;
  const double inv_m = 1.0 / (double)m;
  if (threadIdx.x < KMAX) {
    const int jj = threadIdx.x;
    sincospi((double)jj * inv_m, &tab[1][jj], &tab[0][jj]);
    sincospi((double)(N * jj) * inv_m, &tab[3][jj], &tab[2][jj]);
  }
  __syncthreads();
  const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * 64;
  if (row0 >= a.n_rows) return;                    // wave-uniform, after the only barrier
  float* w = win[wave];
  const int half = (K - 1) / 2;

  // ---- argmax of the wave's 64 rows, four at a time; window beams to LDS ----
  int my_a0 = 0;
  for (int rb = 0; rb < 64; rb += 4) {
    float v[4][PER];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t rr = row0 + rb + r < a.n_rows ? row0 + rb + r : a.n_rows - 1;   // rows past the end: unused
      const float* x = a.in + rr * m + lane * PER;
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
          if (lane * PER + i < m) v[r][i] = x[i];   // lanes past a short row load nothing
        }
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float best = -INFINITY;
      int bi = 0x7FFFFFFF;
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        if (lane * PER + i < m && v[r][i] > best) {
          best = v[r][i];
          bi = lane * PER + i;
        }
      }
      // within each row of 16 lanes: rotations by 8, 4, 2, 1 (DPP row_ror)
      argmax_dpp<0x128>(best, bi);
      argmax_dpp<0x124>(best, bi);
      argmax_dpp<0x122>(best, bi);
      argmax_dpp<0x121>(best, bi);
      // across the four rows
#pragma unroll
      for (int off = 16; off < 64; off <<= 1) {
        const float ov = __shfl_xor(best, off);
        const int oi = __shfl_xor(bi, off);
        if (ov > best || (ov == best && oi < bi)) {
          best = ov;
          bi = oi;
        }
      }
      const int a0 = bi == 0x7FFFFFFF ? 0 : bi;
      if (lane == rb + r) my_a0 = a0;
      // window slot of each of this lane's beams: A = a0 - half + jj (mod m, a
      // power of two), jj < K
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int A = lane * PER + i;
        const int jj = (A - a0 + half) & (m - 1);
        if (A < m && jj < K) w[(rb + r) * WS + jj] = v[r][i];
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

  // ---- Newton phase: lane = row ----
  const int64_t row = row0 + lane;
  const bool row_ok = row < a.n_rows;
  const double y0 = (double)my_a0 * inv_m;
  const double gain = (double)a.n * (double)a.n / (4.0 * kPiD * kPiD * a.moi);
  const double Nd = (double)N;
  const float* wr = w + lane * WS;

  auto eval = [&](double y, double& p, double& dp) {
    // u_j = y - A_j / M with A_j = a0 - half + j; reduced to [-1/2, 1/2] for j = 0
    double u0 = y - (double)(my_a0 - half) * inv_m;
    u0 -= rint(u0);
    double s0, c0, S0, C0;
    sincospi(u0, &s0, &c0);
    sincospi(Nd * u0, &S0, &C0);
    double sp = 0.0, sdp = 0.0;
    for (int j = 0; j < K; ++j) {
      const double bj = (double)wr[j];
      const double u = u0 - (double)j * inv_m;
      const double e = u - rint(u);
      double d, dd;
      if (fabs(Nd * e) < 0.01 / kPiD) {
        const double x = kPiD * e, x2 = x * x, N2 = Nd * Nd;
        const double c4 = (3.0 * N2 * N2 - 10.0 * N2 + 7.0);
        d = Nd * (1.0 - (N2 - 1.0) * x2 / 6.0 + c4 * x2 * x2 / 360.0);
        dd = kPiD * Nd * (-(N2 - 1.0) * x / 3.0 + c4 * x2 * x / 90.0);
      } else {
        // sin, cos of pi u and of N pi u by angle addition (u = u0 - j/M)
        const double cj = tab[0][j], sj = tab[1][j], Cj = tab[2][j], Sj = tab[3][j];
        const double s = s0 * cj - c0 * sj, c = c0 * cj + s0 * sj;
        const double S = S0 * Cj - C0 * Sj, C = C0 * Cj + S0 * Sj;
        const double inv = 1.0 / s;                 // one division: dD = pi (N C - D c) / s
        d = S * inv;
        dd = kPiD * (Nd * C - d * c) * inv;
      }
      sp = fma(d, bj, sp);
      sdp = fma(dd, bj, sdp);
    }
    p = sp * inv_m;
    dp = sdp * inv_m;
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
  if (row_ok) {
    const double yw = (y + 0.5) - floor(y + 0.5) - 0.5;
    const int chan = (int)((row / a.rows_per_chan_blk) % a.n_chan);
    a.sin_out[row] = yw / a.dl[2 * chan + 1];
    if (a.peak_out) a.peak_out[row] = (float)p;
  }
}

}  // namespace

namespace {

template <int PER, int KMAX>
void launch_loc(const LocArgs& a, bool vec, unsigned nb, hipStream_t s) {
  if constexpr (PER >= 4) {
    if (vec) {
      hipLaunchKernelGGL((k_localize<PER, true, KMAX>), dim3(nb), dim3(256), 0, s, a);
      return;
    }
  }
  hipLaunchKernelGGL((k_localize<PER, false, KMAX>), dim3(nb), dim3(256), 0, s, a);
}

template <int KMAX>
hipError_t launch_loc_k(const LocArgs& a, unsigned nb, hipStream_t s) {
  const bool vec = (reinterpret_cast<uintptr_t>(a.in) % 16) == 0;
  switch (a.m) {
    case 32:
    case 64: launch_loc<1, KMAX>(a, vec, nb, s); break;
    case 128: launch_loc<2, KMAX>(a, vec, nb, s); break;
    case 256: launch_loc<4, KMAX>(a, vec, nb, s); break;
    case 512: launch_loc<8, KMAX>(a, vec, nb, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_localize(const LocArgs& a, hipStream_t s) {
  if (a.n_rows <= 0) return hipSuccess;
  if (a.n_window < 1 || a.n_window > 64 || a.n_window > a.m) return hipErrorInvalidValue;
  const int64_t nb = (a.n_rows + 255) / 256;      // 64 rows per wavefront, 4 wavefronts per workgroup
  if (nb > 0x7FFFFFFF) return hipErrorInvalidConfiguration;
  return a.n_window <= 16 ? launch_loc_k<16>(a, (unsigned)nb, s) : launch_loc_k<64>(a, (unsigned)nb, s);
}

}  // namespace fftbf
