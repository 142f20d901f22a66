// Internal launch interface between the C-ABI host layer and the gfx950
// kernels.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fftbf {

struct Fft32Args {
  const uint32_t* volts;   // frames as dwords: [t][chan][pol][n_ns] (4 E-W bytes each)
  int64_t n_time;
  int n_chan, n_pol;
  int n_pg;                // polarisation groups in the output (n_pol, or 1 when summed)
  int pol_iter;            // polarisations folded into one workgroup (1 or n_pol)
  int block;               // samples per intensity block (chunk for complex output)
  const float2* tw;        // [G][2L] pass-1 twiddles W_M^{a1 k2}: (t, 0) of W = Re W (1 + i t), or whole
  const float* mult;       // [2L][dit_slots(G)] pass-2 multipliers (the factors Re W moved there)
  const float* taper;      // [n_ns][4] real weights, [n_ns][4][2] complex gains, or null
  const int32_t* sel;      // [n_chan][n_keep] or null (identity)
  int n_keep;
  void* out;
  float norm;              // 1/(n_ew n_ns) for intensities, its square root for complex beams
  // E-W rows: the output holds ew_rows E-W beams per (sample or block, chan,
  // pol group); this launch's E-W beam e goes to row e * ew_mul + ew_off.
  int ew_rows, ew_mul, ew_off;
  // complex-gain variant only: where the per-antenna factors come from (0 unit,
  // 1 real weights in `taper`, 2 complex gains in `taper`), and whether they
  // are multiplied by W_8^{a_ew} (the odd E-W beams of an 8-point padded E-W
  // transform are the 4-point DFT of x_a W_8^{a_ew})
  int gain_src, twist;
  // cyclic co-adding: the n_ns = fold * N antennas along N-S are summed by
  // a mod N onto the N positions of the transform (1: none)
  int fold;
  // (block, channel, polarisation group) tasks, one per wave; set by the launch
  int64_t n_wg;
  // channels per sample in the voltage buffer, when the call covers a subset of
  // them (volts then points at the first channel of the subset); 0: n_chan
  int chan_stride;
};

// group size G of the transform of length n_ns (fold: n_ns / m_ns of a
// co-adding plan, 1 for none); 0 for an unsupported length
int fft32_group(int n_ns, int fold = 1);
// n_ns: the transform's N (m_ns / 2, or m_ns when folding); taper: 0 none,
// 1 real weights, 2 complex gains, 3 none with the odd E-W beams of the
// zero-padded 8-point E-W transform.  With a.ew_rows == 8 and
// fft32_fuses_ew8(...) one launch writes the even and the odd E-W beams.
hipError_t launch_fft32(const Fft32Args& a, int n_ns, int taper, bool cplx, int64_t n_wg,
                        hipStream_t s);
bool fft32_fuses_ew8(int n_ns, int taper, bool cplx, int fold);

// FP64 table generation on the device
int twiddle_mult_count(int g, int l2);
hipError_t launch_twiddle_table(float2* tw, float* mult, int g, int l2, int m, hipStream_t s);

// standalone |z|^2 block sums
hipError_t launch_accumulate(const float2* z, int64_t n_time, int64_t n_series, int block,
                             int add, float* out, hipStream_t s);

// tied-array beams from complex FFT beams
struct TiedArgs {
  const float2* beams;     // [t][n_chan][n_pol][m_ew][m_ns]
  const uint32_t* volts;   // voltage variant: [t][n_chan][n_pol][n_ns] dwords
  const float* taper;      // voltage variant: [n_ns][4] or null
  int64_t n_time;
  int n_chan, n_pol, chan_lo, n_chan_sub;
  int n_ew, n_ns, m_ew, m_ns;
  const double* dircos;    // [n_point][2]
  const double* dl;        // [n_chan][2] d/lambda
  int n_point;
  int block;
  int pol_sum;
  int complex_out;
  void* out;
  int run_units;           // output units per workgroup run (set by the launcher)
};
hipError_t launch_tied(const TiedArgs& a, hipStream_t s);

// one tile of the tied-beam server (4 x 16 lattice, 16-sample blocks)
struct ServeTile {
  const double* dircos;    // request pointings [n_point][2]
  float* out;              // request output [n_blk][n_chan_req][n_pol][n_point]
  int64_t t_start;         // absolute sample index of the request window start
  int32_t n_point, n_chan_req, chan_lo, chan;
  int32_t ptile, blk0, n_blk, pad;
};
hipError_t launch_serve(const ServeTile* tiles, int n_tiles, const uint32_t* ring, int64_t ring_samples,
                        int n_chan, int n_pol, const double* dl, hipStream_t s);
hipError_t launch_tied_v(const TiedArgs& a, hipStream_t s);

// intensity-domain regridding of FFT beams (N-S axis)
struct RegridArgs {
  const float* in;         // [n_blk][n_chan][n_pg][m_ew][m_ns]
  const float* w;          // [n_chan][n_target_pad][m_ns]
  float* out;              // [n_blk][n_chan][n_pg][m_ew][n_target]
  const int* first;        // compact kernels: [n_chan][n_target] first tap (mod m_ns)
  const float* tw;         //                  [n_chan][n_taps][n_target] tap weights
  int64_t n_blk;
  int n_chan, n_pg, m_ew, m_ns, n_target, n_target_pad;
  int n_taps;              // 0: dense weights w; 1..kRegridMaxTaps: compact kernels
  const float* wew;        // 2-D pointings: [n_chan][n_target_pad][8] E-W weights, else null;
                           // out is then [n_blk][n_chan][n_pg][n_target]
  int rows_per_chan, log2_r;   // set by launch_regrid
};
constexpr int kRegridMaxTaps = 8;
int regrid_target_pad(int n_target);
// coef: device double [n] window lag coefficients, or nullptr for the pointed kernel
hipError_t launch_regrid_weights(float* w, const double* dl, const double* sin_t, const double* coef, int n_chan,
                                 int n_target, int n, int m, hipStream_t s);
// E-W regridding weights of 2-D pointings, w[chan][target_pad][m_ew = 8]
hipError_t launch_regrid_ew_weights(float* w, const double* dl, const double* dircos_ew, int n_chan, int n_target,
                                    int n, int m, hipStream_t s);
hipError_t launch_regrid_tap_table(int* first, float* tw, const double* dl, const double* sin_t, const double* coef,
                                   int n_chan, int n_target, int k, int n, int m, hipStream_t s);
hipError_t launch_regrid(const RegridArgs& a, hipStream_t s);

// Newton localisation over rows of FFT-beam intensities
struct LocArgs {
  const float* in;         // [n_rows][m] (rows = (blk, chan, pol group, E-W beam))
  const double* dl;        // [n_chan][2] d/lambda (ew, ns)
  double* sin_out;         // [n_rows]
  float* peak_out;         // [n_rows] or nullptr
  int64_t n_rows;
  int64_t rows_per_chan_blk;   // rows per (blk, chan) = n_pg * m_ew
  int n_chan, n, m, n_window, n_iter;
  double moi;              // sum over lags of delta^2 (n - |delta|)
};
hipError_t launch_localize(const LocArgs& a, hipStream_t s);

// mixed-precision (MFMA) beamformer
struct MixArgs {
  const uint32_t* volts;
  int64_t n_time;
  int n_chan, n_pol, n_pg, pol_iter, block;
  const void* mat;         // per-precision DFT operand tables (plan-owned)
  const float* taper;
  const int32_t* sel;
  int n_keep;
  float* out;
  float norm;
};
hipError_t launch_mix(const MixArgs& a, int n_ns, int prec, int64_t n_wg, hipStream_t s);
size_t mix_table_bytes(int n_ns, int prec);
hipError_t launch_mix_tables(void* mat, int n_ns, int prec, hipStream_t s);
bool mix_supported(int n_ns, int prec, int block);
// per-antenna real weights on the matrix cores (windowed data split into FP16 terms)
bool mix_window_supported(int n_ns, int prec);
// the 4 x 256 lattice (k_mix256.hip): stage 1 on the matrix cores (FP16 or
// FP8), stage 2 in FP32
size_t mix256_table_bytes();
hipError_t launch_mix256_tables(void* mat, int prec, hipStream_t s);
hipError_t launch_mix256(const MixArgs& a, int prec, int64_t n_wg, hipStream_t s);

}  // namespace fftbf
