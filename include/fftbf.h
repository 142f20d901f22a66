/*
 * fftbf.h -- C ABI of the MI355X FFT beamformer (libfftbf.so).
 *
 * FFT beamforming of channelised antenna voltages on a regular 2-D lattice,
 * after K. W. Masui et al., "Algorithms for FFT Beamforming Radio
 * Interferometers" (arXiv:1710.08591).
 *
 * Conventions shared by every call:
 *   - Voltages: uint8 volts[t][chan][pol][a_ns][a_ew], E-W index fastest.
 *     Each byte is one complex sample: two's-complement 4-bit real part in
 *     the high nibble, 4-bit imaginary part in the low nibble (the
 *     digitised antenna signal eta_a[t] of eq. e:Vab).
 *   - Beams: FFT beam (A_ew, A_ns) carries the voltage weights of eq.
 *     e:w_A^a per axis, n^-1/2 exp(-i 2 pi A a / M), on the separable 2-D
 *     lattice with n = n_ew * n_ns; the N-S axis is zero-padded from n_ns
 *     to m_ns (Sec. "Redundant arrays and Fourier transform beamforming",
 *     eq. e:fftbeamform).  Beam A points at sin(theta_A) = A lambda / (M d)
 *     (eq. e:theta_A), natural FFT order A in [0, M).
 *   - Intensities: |B|^2 summed (not averaged) over `block` consecutive
 *     samples, blocks aligned to t = 0 of the call (the time sum of eqs.
 *     e:bf and e:fftbeamform without the 1/n_samp and unit factors).
 *   - Every device pointer is caller-owned device memory (the library never
 *     allocates or frees caller memory).  The plan owns its device tables.
 *   - `stream` is a hipStream_t (NULL = the null stream).  The creators and
 *     destroyers (plans, regrid objects, servers) are synchronous; every
 *     other call that takes a stream is asynchronous on it.
 *   - Arguments are validated before any launch; on a validation error
 *     nothing is written and nothing is launched.  No call aborts or throws.
 *     Device faults surface as BF_ERR_DEVICE.  bf_last_error() gives a
 *     thread-local description of the last failing call.
 */
#ifndef FFTBF_H
#define FFTBF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BF_OK = 0,
  BF_ERR_INVALID_ARGUMENT = -1,
  BF_ERR_UNSUPPORTED = -2,
  BF_ERR_OUT_OF_MEMORY = -3,
  BF_ERR_DEVICE = -4,
  BF_ERR_REJECTED = -5,   /* serving: request exceeds the memory budget */
  BF_ERR_EVICTED = -6,    /* serving: requested window left the ring    */
  BF_ERR_NOT_READY = -7   /* serving: result not finished yet           */
} bf_status;

typedef enum {
  BF_PREC_FP32 = 0,       /* FP32 radix FFT on the vector ALUs            */
  BF_PREC_FP16_MFMA = 1,  /* N-S DFT stages on FP16 MFMA, FP32 accumulate */
  BF_PREC_FP8_MFMA = 2    /* N-S DFT stages on FP8 MFMA, FP32 accumulate  */
} bf_precision;

typedef enum {
  BF_OUT_INTENSITY = 0,   /* float intensities, see each call           */
  BF_OUT_COMPLEX = 1      /* float2 complex beams, one per sample        */
} bf_out_kind;

typedef struct bf_plan bf_plan;

/*
 * Plan geometry.  Supported: n_ew = 4 with m_ew = 4 (unpadded E-W axis)
 * or, for FP32 plans, m_ew = 8 (E-W zero-padded to M_ew >= 2 n_ew - 1, so
 * that intensity regridding is exact on both axes; the odd E-W beams are
 * the 4-point DFT of x_a W_8^{a_ew}, formed by a second launch over the
 * voltages, except for 4 x 256 intensities (with or without a window or
 * gains), where one launch transforms the four E-W antenna columns along
 * N-S and forms all eight E-W beams of each N-S beam; tied beams and the
 * server need m_ew = 4);
 * n_ns a power of two in [16, 256] with m_ns = 2 n_ns (zero padding by two,
 * the smallest power of two with M >= 2n - 1, eq. e:b2n-1), or, for FP32
 * plans with m_ew = 4 and no clamp, m_ns a power of two in [16, 128] below
 * n_ns: cyclic co-adding (Sec. "Redundant arrays and Fourier transform
 * beamforming"), the N-S antennas summed by a_ns mod m_ns before an m_ns-point
 * transform, i.e. the weights n^-1/2 e^{-i 2 pi A a / M} of eq. e:w_A^a with
 * M < n (a real window is allowed up to n_ns = 8 m_ns, complex gains are
 * not); block a
 * multiple of 16 (mixed precision) or of 4 (FP32); 1 <= n_pol <= 2.
 * Other shapes return BF_ERR_UNSUPPORTED.
 */
typedef struct {
  int32_t n_ew, n_ns;          /* antennas per axis                          */
  int32_t m_ew, m_ns;          /* transform lengths per axis                 */
  int32_t n_pol, n_chan;       /* polarisations (independent antennas), channels */
  int32_t block;               /* samples summed per intensity (n_samp)      */
  int32_t n_ns_keep;           /* N-S beams kept per channel; 0 -> m_ns      */
  int32_t pol_sum;             /* 1: intensities summed over polarisations   */
  int32_t precision;           /* bf_precision                               */
  const double *d_over_lambda; /* host [n_chan][2] (ew, ns) spacing in wavelengths;
                                  NULL -> 0.5 on both axes.  Used by tied beams. */
  const int32_t *ns_select;    /* host [n_chan][n_ns_keep] kept N-S beam indices
                                  in [0, m_ns); NULL -> identity (needs n_ns_keep
                                  0 or m_ns).  Copied into the plan. */
} bf_plan_desc;

/* Validate the descriptor, build the plan's device tables (twiddles in FP64
 * on the current device, rounded to the working precision; clamp table;
 * d/lambda table).  Synchronous.  On success *plan owns device memory until
 * bf_plan_destroy.  Errors: BF_ERR_INVALID_ARGUMENT (NULL pointers, bad
 * sizes, ns_select entries out of range), BF_ERR_UNSUPPORTED (shape),
 * BF_ERR_OUT_OF_MEMORY, BF_ERR_DEVICE. */
bf_status bf_plan_create(const bf_plan_desc *desc, bf_plan **plan);

/* Free the plan's device tables (synchronises the device first).  NULL is a no-op. */
bf_status bf_plan_destroy(bf_plan *plan);

/* Copy the plan's descriptor (pointers in the copy are NULL). */
bf_status bf_plan_get_desc(const bf_plan *plan, bf_plan_desc *desc);

/*
 * FFT beamforming of a contiguous voltage time series (the hot path).
 * Sec. "Redundant arrays and Fourier transform beamforming", eq.
 * e:fftbeamform, with the per-antenna window of Sec. "Controlling beam
 * shape with windowing" (w_nw^a ~ h^a w_p^a) applied before the transform.
 *
 *   volts  device uint8 [n_time][n_chan][n_pol][n_ns][n_ew]
 *   n_time samples; a multiple of the plan's block for BF_OUT_INTENSITY
 *   taper  device float [n_ns][n_ew] real per-antenna weights h_a, or NULL (h = 1)
 *   kind   BF_OUT_INTENSITY: out is float
 *            [n_time/block][n_chan][n_pol][m_ew][n_ns_keep]   (pol_sum = 0)
 *            [n_time/block][n_chan][m_ew][n_ns_keep]          (pol_sum = 1)
 *          holding sum over each block of |B|^2 for the kept N-S beams
 *          ns_select[chan][j], j < n_ns_keep, in that order.
 *          BF_OUT_COMPLEX (FP32 plans only): out is float2
 *            [n_time][n_chan][n_pol][m_ew][m_ns], every beam, unclamped.
 * The mixed-precision plans take the int4 samples exactly into FP16 / FP8
 * operands and round the DFT coefficients (split into a high and a low
 * part) to the working precision, accumulating in FP32; they produce
 * intensities only.  With a taper, FP16 plans split the windowed E-W sums
 * into FP16 high and low parts (taper 16-byte aligned); FP8 plans return
 * BF_ERR_UNSUPPORTED.  Mixed-precision plans need 16-byte aligned volts.
 */
bf_status bf_beamform_fft(const bf_plan *plan, const uint8_t *volts, int64_t n_time,
                          const float *taper, int32_t kind, void *out, void *stream);

/*
 * bf_beamform_fft with complex per-antenna gains in place of the real
 * window: eta_a -> g_a eta_a before the transform, g_a = e^{gamma_a + i psi_a}
 * the per-antenna amplitude and phase response of eq. e:vis_pert (Sec.
 * "Non-redundancy"), or the inverse of estimated gains (calibration).
 *   gains  device float [n_ns][n_ew][2] (re, im), 16-byte aligned, not NULL.
 * FP32 plans only (BF_ERR_UNSUPPORTED otherwise); every other argument,
 * layout and error as bf_beamform_fft.
 */
bf_status bf_beamform_fft_gains(const bf_plan *plan, const uint8_t *volts, int64_t n_time,
                                const float *gains, int32_t kind, void *out, void *stream);

/*
 * Tied-array (pointed) beams at arbitrary directions, formed by
 * interpolating complex FFT beams.  The weights follow from substituting
 * the zero-padded inverse transform into the pointed-beam weights of eq.
 * e:c_pointed (the voltage-domain analogue of the regridding of eq.
 * e:bp_max_arbitrary): per axis
 *     c_A(y) = (1/M) sum_{a<n} exp(+i 2 pi a (A/M - y)),  y = (d/lambda) n_axis,
 * exact for M >= n.  They are generated in FP64 on the device and applied
 * in FP32: B_p[t] = sum_{A_ew, A_ns} c_{A_ew}(y_ew) c_{A_ns}(y_ns) B_A[t].
 *
 *   fft_beams  device float2 [n_time][n_chan][n_pol][m_ew][m_ns] (as written
 *              by bf_beamform_fft with BF_OUT_COMPLEX)
 *   chan_lo, n_chan_sub   channel range [chan_lo, chan_lo + n_chan_sub)
 *   dircos     device double [n_point][2] direction cosines (ew, ns)
 *   kind       BF_OUT_INTENSITY: out float [n_time/block][n_chan_sub][n_pol][n_point]
 *              (pol_sum: [n_time/block][n_chan_sub][n_point]);
 *              BF_OUT_COMPLEX: out float2 [n_time][n_chan_sub][n_pol][n_point]
 * Per-channel d/lambda comes from the plan.  Plans with m_ew = 4 and
 * 32 <= m_ns <= 512, m_ns >= n_ns (BF_ERR_UNSUPPORTED otherwise); for
 * m_ns >= 128 fft_beams must be 16-byte aligned (BF_ERR_INVALID_ARGUMENT).
 * At most 4096 pointings per call.
 */
bf_status bf_form_tied_beams(const bf_plan *plan, const void *fft_beams, int64_t n_time,
                             int32_t chan_lo, int32_t n_chan_sub, const double *dircos,
                             int32_t n_point, int32_t kind, void *out, void *stream);

/*
 * Tied-array beams straight from voltages: the FFT beams of each sample are
 * formed on chip (FP32, as bf_beamform_fft) and interpolated as in
 * bf_form_tied_beams without leaving the compute unit.
 *
 *   volts     device uint8 [n_time][n_chan][n_pol][n_ns][n_ew] (full channel set)
 *   taper     device float [n_ns][n_ew] or NULL
 *   other arguments as bf_form_tied_beams (intensity output only).
 * The 4 x 16 lattice with block a multiple of 16 (BF_ERR_UNSUPPORTED
 * otherwise: other lattices take bf_form_tied_beams_v_ws).
 */
bf_status bf_form_tied_beams_v(const bf_plan *plan, const uint8_t *volts, int64_t n_time,
                               const float *taper, int32_t chan_lo, int32_t n_chan_sub,
                               const double *dircos, int32_t n_point, void *out, void *stream);

/*
 * Bytes of caller workspace that bf_form_tied_beams_v_ws uses to take
 * chunk_samples samples of n_chan_sub channels at a time: their complex FFT
 * beams, chunk_samples * n_chan_sub * n_pol * m_ew * m_ns * 8.  0 for a
 * NULL plan or negative sizes.
 */
size_t bf_tied_workspace_size(const bf_plan *plan, int32_t n_chan_sub, int64_t chunk_samples);

/*
 * bf_form_tied_beams_v for every lattice a tied-beam plan takes (m_ew = 4,
 * 32 <= m_ns <= 512, m_ns >= n_ns): the samples go in chunks of whole
 * blocks; per chunk the complex FFT beams of the channel range are written to
 * the caller's workspace by the FFT beamformer (FP32, with the taper) and
 * interpolated from there by the bf_form_tied_beams kernels, both on
 * `stream`, so the method is the same as on the 4 x 16 lattice (interpolated
 * FFT beams) with the beams passing through HBM.  The chunk is the largest
 * whole number of blocks whose beams fit in workspace_bytes (at most n_time).
 * On the 4 x 16 lattice with block a multiple of 16 this is
 * bf_form_tied_beams_v and the workspace is not used (it may be NULL).
 *   workspace  device memory, 16-byte aligned, owned by the caller; the call
 *              overwrites it, so calls that share one must not overlap.
 * Errors: as bf_form_tied_beams_v; BF_ERR_INVALID_ARGUMENT when the
 * workspace is NULL, misaligned or smaller than one block's beams.
 */
bf_status bf_form_tied_beams_v_ws(const bf_plan *plan, const uint8_t *volts, int64_t n_time,
                                  const float *taper, int32_t chan_lo, int32_t n_chan_sub,
                                  const double *dircos, int32_t n_point, void *workspace,
                                  size_t workspace_bytes, void *out, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * bf_form_tied_beams_v_ws with the workspace taken from a static device
 * array of the library (64 MiB, one per GPU, held until the process ends)
 * instead of an argument.  The call itself allocates nothing.  Every call on
 * one GPU shares that array and leaves its last contents there; calls that
 * overlap on one GPU (concurrent streams or threads) race on it.
 * Errors: as bf_form_tied_beams_v_ws; BF_ERR_INVALID_ARGUMENT when one block
 * of the channel range needs more than the 64 MiB (n_chan_sub * n_pol *
 * block * m_ew * m_ns * 8 bytes).  On the 4 x 16 lattice with block a
 * multiple of 16 it is bf_form_tied_beams_v (no workspace).
 */
bf_status bf_form_tied_beams_v_noalloc(const bf_plan *plan, const uint8_t *volts, int64_t n_time,
                                       const float *taper, int32_t chan_lo, int32_t n_chan_sub,
                                       const double *dircos, int32_t n_point, void *out, void *stream);

/*
 * Standalone intensity accumulation (the |B|^2 time sum of eq. e:bf):
 *   out[b][s] (+)= sum_{t in block b} |z[t][s]|^2
 *   z    device float2 [n_time][n_series]
 *   out  device float [n_time/block][n_series]
 *   add  0: overwrite out, 1: add to out
 * n_time must be a multiple of block (block >= 1).
 */
bf_status bf_accumulate_intensity(const void *z, int64_t n_time, int64_t n_series,
                                  int32_t block, int32_t add, float *out, void *stream);

/*
 * ---- Regridding FFT-beam intensities to arbitrary steering angles ----
 * Eq. e:bp_max_arbitrary (Sec. "Redundancy-stacked visibilities"): a beam
 * pointed at sin(theta) is formed from the FFT-beam intensities b_A as
 *     b = sum_A w^A b_A,   w^A = (1/M) sin((2n-1) pi y) / sin(pi y),
 *     y = (d/lambda) sin(theta) - A/M,
 * exact for M >= 2n - 1.  Applied along N-S (M = 2n) for each E-W FFT beam,
 * so the same sin(theta) targets give achromatic beams in every channel
 * (the FFT beams' own positions move with wavelength, eq. e:theta_A).
 *
 * With a window h (Sec. "Controlling beam shape with windowing"), the
 * weights are those of the optimally windowed beam, eq. e:w_opt carried to
 * the FFT beams by eq. e:wA_from_wdelta (eq. e:wA_windowed):
 *     w^A = (1/M) [c_0 + 2 sum_{d=1}^{n-1} c_d cos(2 pi d (A/M - (d/lambda) sin(theta)))],
 *     c_d = R_d / ((n - d) N),  R_d = sum_a h[a+d] h[a],
 * N chosen so that the beam's noise equals the unwindowed pointed beam's
 * (N = 1 without a window).  Pass intensities formed without a voltage
 * taper for the beam of eq. e:w_opt.
 *
 * Compact kernels (n_taps = k > 0): only the k FFT beams nearest each
 * target on the circular beam grid, A = rint(y M) - (k-1)/2 + j (mod M),
 * j < k, with their full-kernel weights; an approximation, much cheaper
 * than the dense form.
 *
 * The weights are generated in FP64 on the device at creation and stored in
 * FP32 (owned by the regrid object); the contraction runs in FP32.
 */
typedef struct bf_regrid bf_regrid;

/* plan: the geometry and per-channel d/lambda, without a clamp (n_ns_keep 0
 * or m_ns).  sin_theta: host double [n_target] (copied), n_target in
 * [1, 65536].  window: host double [n_ns] (real, copied) or NULL.  n_taps:
 * 0 (dense, exact) or 1..8 (compact).  Synchronous.  Errors:
 * BF_ERR_INVALID_ARGUMENT (NULLs, clamped plan, non-finite values, window
 * without power, n_taps out of range), BF_ERR_UNSUPPORTED (m_ns < 2 n_ns - 1),
 * BF_ERR_OUT_OF_MEMORY / BF_ERR_DEVICE. */
bf_status bf_regrid_create(const bf_plan *plan, const double *sin_theta, int32_t n_target,
                           const double *window, int32_t n_taps, bf_regrid **rg);
/* 2-D pointings: each pointing (direction cosines ew, ns) is regridded along
 * N-S as above and then along E-W with the same pointed kernel of eq.
 * e:bp_max_arbitrary, w^{A_ew} = (1/M_ew) sin((2n_ew-1) pi y)/sin(pi y),
 * y = (d/lambda)_ew dircos_ew - A_ew/M_ew; exact for a plan with m_ew = 8
 * (>= 2 n_ew - 1) and m_ns = 2 n_ns.  The result is the intensity of the
 * pointed beam at each pointing in every channel.
 *   dircos  host double [n_point][2] (ew, ns), copied; n_point in [1, 65536].
 * Errors as bf_regrid_create; BF_ERR_UNSUPPORTED unless m_ew >= 2 n_ew - 1.
 * bf_regrid_intensity then writes out: device float
 * [n_blk][n_chan][n_pol][n_point] ([n_blk][n_chan][n_point] when the plan sums
 * polarisations). */
bf_status bf_regrid_create_2d(const bf_plan *plan, const double *dircos, int32_t n_point, bf_regrid **rg);
bf_status bf_regrid_destroy(bf_regrid *rg);
/* fft_intensity: device float [n_blk][n_chan][n_pol][m_ew][m_ns] as written by
 * bf_beamform_fft with the plan ([n_blk][n_chan][m_ew][m_ns] when it sums
 * polarisations); out: device float [n_blk][n_chan][n_pol][m_ew][n_target]
 * (or [n_blk][n_chan][m_ew][n_target]).  fft_intensity 16-byte aligned.
 * n_blk = 0 is a no-op.  Asynchronous on stream; the caller owns both
 * buffers. */
bf_status bf_regrid_intensity(const bf_regrid *rg, const float *fft_intensity, int64_t n_blk,
                              float *out, void *stream);

/*
 * ---- Localisation of a point source (Sec. "Localization") ----
 * Newton's-method maximum-likelihood estimate of sin(theta) along N-S, for
 * every row (block, channel, polarisation, E-W beam) of FFT-beam
 * intensities.  In y = (d/lambda) sin(theta), with the regridded pointed
 * beam b_p(y) = sum_A w^A(y) b_A of eq. e:bp_max_arbitrary:
 *     y <- y + n^2 b_p'(y) / (4 pi^2 MOI b_p(y)),
 *     MOI = sum_delta delta^2 (n - |delta|)        (eq. e:baseline_MOI),
 * the likelihood's curvature taken at its maximum, so the source flux
 * cancels.  Start: y_0 = A_0 / M for the strongest beam A_0 (lowest index on
 * ties).  Sums over the n_window beams A_0 - (n_window-1)/2 + j (mod M).
 * n_iter updates; an update is not taken, and the iteration stops, when
 * b_p(y) <= 0 or when it would leave [y_0 - 1/M, y_0 + 1/M].  The estimator
 * is meant for the source's contribution to the intensities (background
 * removed); the arithmetic is applied to whatever is passed.  FP64.
 *
 * plan: without a clamp, m_ns >= 2 n_ns - 1 (d/lambda per channel from the
 * plan).  fft_intensity: device float [n_blk][n_chan][n_pol][m_ew][m_ns]
 * ([n_blk][n_chan][m_ew][m_ns] when the plan sums polarisations), finite.
 * n_window in [1, min(64, m_ns)], n_iter in [0, 64].
 * sin_theta: device double, one per row (y wrapped to [-1/2, 1/2) and divided
 * by d/lambda); peak: device float b_p at the estimate, one per row, or NULL.
 * n_blk = 0 is a no-op.  Asynchronous on stream; the caller owns the buffers.
 */
bf_status bf_localize(const bf_plan *plan, const float *fft_intensity, int64_t n_blk, int32_t n_window,
                      int32_t n_iter, double *sin_theta, float *peak, void *stream);

/*
 * ---- Tied-beam server --------------------------------------------------
 * Serves tied-array beam requests (arbitrary pointings, a contiguous channel
 * range, the most recent n_time samples) from a device-resident voltage ring
 * of the 4 x 16 lattice.  The beams are the interpolated FFT beams of
 * bf_form_tied_beams_v; pointed beams formed from FFT beams are the use the
 * paper gives for the regridding of eq. e:bp_max_arbitrary (Sec. "Discussion
 * and Conclusions": tied-array beams from FFT beams).
 *
 * Requests are admitted against a fixed device-memory budget (outputs and
 * pointing tables live in one pool of hbm_budget bytes), cut into tiles
 * (channel x up to 64 pointings x blocks_per_tile blocks of 16 samples; each
 * tile forms its FP64 interpolation weights once, so longer tiles amortise
 * them: 32 blocks served the benchmark's request mix with the lowest p99) and
 * batched -- round robin over the active requests, at most
 * max_tiles_per_launch tiles and two launches in flight -- into launches of
 * a persistent tile worker on the server's own stream.  Requests that arrive
 * while others run join at the next launch.  A tile's arithmetic does not
 * depend on the batch, so a result is bitwise the same alone and in a mix.
 * The ring holds the last ring_samples samples; a request's window is
 * leased until it finishes and bf_server_advance refuses to overwrite it.
 * Host calls are not thread safe: drive one server from one thread.
 */
typedef struct bf_server bf_server;

typedef struct {
  int64_t submitted, completed, rejected, evicted, in_flight;
  int64_t budget_used;   /* bytes of the pool in use */
  int64_t tiles_done, launches;
} bf_server_stats;

/* plan: FP32, n_ew = 4, n_ns = 16, m_ns = 32, block 16, pol_sum 0.
 * ring_samples: multiple of 16.  Allocates the ring (ring_samples x n_chan x
 * n_pol x 64 bytes, zero filled) and the pool (hbm_budget bytes).  The plan
 * may be destroyed afterwards.  Errors: INVALID_ARGUMENT, UNSUPPORTED,
 * OUT_OF_MEMORY, DEVICE. */
bf_status bf_server_create(const bf_plan *plan, int64_t ring_samples, int64_t hbm_budget,
                           int32_t blocks_per_tile, int32_t max_tiles_per_launch, bf_server **srv);
/* Drain the server's stream and free everything. */
bf_status bf_server_destroy(bf_server *srv);
/* Device ring [ring_samples][n_chan][n_pol][16][4] uint8, its length, and
 * the head (samples written so far; sample s lives in slot s mod ring). */
bf_status bf_server_ring(bf_server *srv, void **ring, int64_t *ring_samples, int64_t *head);
/* The writer appends n_samples: copies them from device src, produced on
 * `stream` (the copy waits for that stream, and that stream waits for the
 * copy), or, if src is NULL, takes the ring contents as already written;
 * then advances the head.  Returns BF_ERR_NOT_READY without change if that
 * would overwrite a leased window, unless force != 0 (then those requests
 * end as BF_ERR_EVICTED). */
bf_status bf_server_advance(bf_server *srv, int64_t n_samples, const uint8_t *src, int32_t force,
                            void *stream);
/* Admit a request for the n_time samples before the head (n_time a multiple
 * of 16, at most ring_samples), channels [chan_lo, chan_lo + n_chan),
 * n_point pointings given as host double [n_point][2] direction cosines
 * (copied).  arrival_s is the request's arrival time on bf_server_now's
 * clock (latency is measured from it).  Errors: INVALID_ARGUMENT,
 * EVICTED (window not in the ring), REJECTED (over the memory budget). */
bf_status bf_server_submit(bf_server *srv, int32_t n_point, int32_t chan_lo, int32_t n_chan,
                           int64_t n_time, const double *dircos, double arrival_s, int64_t *id);
/* Retire finished launches and issue new ones; never blocks. */
bf_status bf_server_pump(bf_server *srv);
/* BF_OK when finished (latency_s = completion - arrival), BF_ERR_NOT_READY
 * while running, BF_ERR_EVICTED, or BF_ERR_INVALID_ARGUMENT (unknown or
 * cancelled). */
bf_status bf_server_poll(bf_server *srv, int64_t id, double *latency_s);
/* Device pointer to a finished request's intensities
 * float [n_time/16][n_chan][n_pol][n_point], valid until released. */
bf_status bf_server_result(bf_server *srv, int64_t id, float **out, int64_t *n_floats);
/* Copy a finished result into caller device memory dst on stream. */
bf_status bf_server_copy_result(bf_server *srv, int64_t id, float *dst, void *stream);
/* Return a finished, cancelled or evicted request's memory to the pool
 * (BF_ERR_NOT_READY while its tiles are still on the device). */
bf_status bf_server_release(bf_server *srv, int64_t id);
/* Stop issuing a request's remaining tiles. */
bf_status bf_server_cancel(bf_server *srv, int64_t id);
bf_status bf_server_stats_get(bf_server *srv, bf_server_stats *st);
/* Seconds on the server's monotonic clock. */
double bf_server_now(bf_server *srv);

/* Static description of a status code. */
const char *bf_status_string(int32_t status);

/* Thread-local detail of the last non-OK status returned on this thread. */
const char *bf_last_error(void);

/* Library version string. */
const char *bf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FFTBF_H */
