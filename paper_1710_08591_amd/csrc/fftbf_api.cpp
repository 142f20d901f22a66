// C-ABI host layer of libfftbf: plan objects, argument validation,
// dispatch of the gfx950 kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/fftbf.h"
#include "kernels.h"
#include "trace.h"

struct bf_plan {
  bf_plan_desc d;          // copy; pointer members are NULL
  int device = 0;
  int g = 0, l2 = 0;       // FP32 N-S split: m_ns = l2 * g
  float2* tw = nullptr;    // [g][l2] FP32 pass-1 twiddles W_M^{a1 k2} (tangent form)
  float* mult = nullptr;   // [l2][slots] pass-2 multipliers
  int32_t* sel = nullptr;  // [n_chan][n_ns_keep] or null (identity)
  int fold = 1;            // cyclic co-adding: n_ns / m_ns when m_ns < n_ns
  int32_t* even = nullptr; // cyclic co-adding: [n_chan][m_ns] = 2 A (the even padded outputs)
  double* dl = nullptr;    // [n_chan][2]
  void* mix = nullptr;     // mixed-precision operand tables
};

namespace {

thread_local std::string g_err;

bf_status fail(bf_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
bf_status fail(bf_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

bf_status dev_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? BF_ERR_OUT_OF_MEMORY : BF_ERR_DEVICE, "%s: %s", what,
              hipGetErrorString(e));
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

void free_plan(bf_plan* p) {
  if (!p) return;
  if (p->tw) (void)hipFree(p->tw);
  if (p->mult) (void)hipFree(p->mult);
  if (p->sel) (void)hipFree(p->sel);
  if (p->even) (void)hipFree(p->even);
  if (p->dl) (void)hipFree(p->dl);
  if (p->mix) (void)hipFree(p->mix);
  delete p;
}

int keep_of(const bf_plan_desc& d) { return d.n_ns_keep ? d.n_ns_keep : d.m_ns; }

// The creators build their device tables on a non-blocking stream of their
// own and wait for that stream only (temporary buffers come from the
// stream-ordered allocator), so creating a plan or a regridder does not wait
// for work that other streams have in flight.
class SetupStream {
 public:
  hipError_t init() { return hipStreamCreateWithFlags(&s_, hipStreamNonBlocking); }
  hipStream_t get() const { return s_; }
  hipError_t finish() { return hipStreamSynchronize(s_); }
  ~SetupStream() {
    if (s_) (void)hipStreamDestroy(s_);
  }

 private:
  hipStream_t s_ = nullptr;
};

}  // namespace

extern "C" {

const char* bf_version(void) { return "fftbf 0.1 (gfx950)"; }

const char* bf_status_string(int32_t s) {
  switch (s) {
    case BF_OK: return "ok";
    case BF_ERR_INVALID_ARGUMENT: return "invalid argument";
    case BF_ERR_UNSUPPORTED: return "unsupported shape or option";
    case BF_ERR_OUT_OF_MEMORY: return "out of device memory";
    case BF_ERR_DEVICE: return "device error";
    case BF_ERR_REJECTED: return "request rejected (over budget)";
    case BF_ERR_EVICTED: return "requested window evicted from the ring";
    case BF_ERR_NOT_READY: return "not ready";
    default: return "unknown status";
  }
}

const char* bf_last_error(void) { return g_err.c_str(); }

__attribute__((visibility("hidden"))) void bf_internal_set_error(const char* msg) { g_err = msg ? msg : ""; }

bf_status bf_plan_create(const bf_plan_desc* desc, bf_plan** plan) {
  FFTBF_TRACE("bf_plan_create");
  if (!desc || !plan) return fail(BF_ERR_INVALID_ARGUMENT, "plan_create: NULL desc or plan");
  *plan = nullptr;
  const bf_plan_desc& d = *desc;
  if (d.n_ew <= 0 || d.n_ns <= 0 || d.m_ew <= 0 || d.m_ns <= 0 || d.n_pol <= 0 || d.n_chan <= 0 ||
      d.block <= 0 || d.n_ns_keep < 0)
    return fail(BF_ERR_INVALID_ARGUMENT, "plan_create: sizes must be positive");
  if (d.m_ew < d.n_ew) return fail(BF_ERR_INVALID_ARGUMENT, "plan_create: E-W transform shorter than the array");
  const bool folded = d.m_ns < d.n_ns;    // cyclic co-adding (e:fftbeamform with M < n)
  if (d.n_ew != 4 || (d.m_ew != 4 && d.m_ew != 8))
    return fail(BF_ERR_UNSUPPORTED, "plan_create: n_ew = 4 with m_ew = 4 or 8 is supported");
  if (d.m_ew == 8 && d.precision != BF_PREC_FP32)
    return fail(BF_ERR_UNSUPPORTED, "plan_create: the padded E-W axis (m_ew = 8) needs an FP32 plan");
  if (!is_pow2(d.n_ns) || d.n_ns < 16 || d.n_ns > 256 ||
      (folded ? (!is_pow2(d.m_ns) || d.m_ns < 16 || d.m_ns > 128) : d.m_ns != 2 * d.n_ns))
    return fail(BF_ERR_UNSUPPORTED,
                "plan_create: n_ns must be a power of two in [16, 256] with m_ns = 2 n_ns, or (cyclic "
                "co-adding) m_ns a power of two in [16, 128] below n_ns");
  if (folded && (d.precision != BF_PREC_FP32 || d.m_ew != 4 || (d.n_ns_keep && d.n_ns_keep != d.m_ns)))
    return fail(BF_ERR_UNSUPPORTED, "plan_create: cyclic co-adding needs an FP32 plan, m_ew = 4 and no clamp");
  if (d.n_pol > 2) return fail(BF_ERR_UNSUPPORTED, "plan_create: at most 2 polarisations");
  if (d.pol_sum != 0 && d.pol_sum != 1) return fail(BF_ERR_INVALID_ARGUMENT, "plan_create: pol_sum is 0 or 1");
  if (d.precision < BF_PREC_FP32 || d.precision > BF_PREC_FP8_MFMA)
    return fail(BF_ERR_INVALID_ARGUMENT, "plan_create: unknown precision %d", d.precision);
  const int keep = keep_of(d);
  if (keep > d.m_ns) return fail(BF_ERR_INVALID_ARGUMENT, "plan_create: n_ns_keep > m_ns");
  if (!d.ns_select && keep != d.m_ns)
    return fail(BF_ERR_INVALID_ARGUMENT, "plan_create: a clamp (n_ns_keep < m_ns) needs ns_select");
  if (d.block % 4 != 0) return fail(BF_ERR_UNSUPPORTED, "plan_create: block must be a multiple of 4");
  if (d.precision != BF_PREC_FP32 && !fftbf::mix_supported(d.n_ns, d.precision, d.block))
    return fail(BF_ERR_UNSUPPORTED, "plan_create: mixed precision not available for n_ns=%d block=%d",
                d.n_ns, d.block);
  if (d.ns_select) {
    for (int64_t i = 0; i < (int64_t)d.n_chan * keep; ++i)
      if (d.ns_select[i] < 0 || d.ns_select[i] >= d.m_ns)
        return fail(BF_ERR_INVALID_ARGUMENT, "plan_create: ns_select[%lld] = %d out of [0, %d)",
                    (long long)i, d.ns_select[i], d.m_ns);
  }
  if (d.d_over_lambda) {
    for (int64_t i = 0; i < (int64_t)d.n_chan * 2; ++i)
      if (!(d.d_over_lambda[i] > 0.0) || d.d_over_lambda[i] > 1e6)
        return fail(BF_ERR_INVALID_ARGUMENT, "plan_create: d_over_lambda must be positive and finite");
  }

  bf_plan* p = new (std::nothrow) bf_plan();
  if (!p) return fail(BF_ERR_OUT_OF_MEMORY, "plan_create: host allocation");
  p->d = d;
  p->d.d_over_lambda = nullptr;
  p->d.ns_select = nullptr;
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) { free_plan(p); return dev_fail(e, "plan_create: hipGetDevice"); }

  // the transform's N: n_ns, or m_ns when folding (its padded outputs 2A are the beams)
  const int kn = folded ? d.m_ns : d.n_ns;
  p->fold = d.n_ns / kn;
  p->g = fftbf::fft32_group(kn, p->fold);
  p->l2 = 2 * kn / p->g;
  SetupStream ss;
  e = ss.init();
  const hipStream_t s = ss.get();
  if (e == hipSuccess) e = hipMalloc(&p->tw, sizeof(float2) * p->g * p->l2);
  if (e == hipSuccess) e = hipMalloc(&p->mult, sizeof(float) * fftbf::twiddle_mult_count(p->g, p->l2));
  if (e == hipSuccess) e = fftbf::launch_twiddle_table(p->tw, p->mult, p->g, p->l2, 2 * kn, s);
  std::vector<int32_t> ev;
  if (e == hipSuccess && folded) {
    ev.resize((size_t)d.n_chan * d.m_ns);
    for (size_t i = 0; i < ev.size(); ++i) ev[i] = 2 * (int32_t)(i % d.m_ns);
    e = hipMalloc(&p->even, sizeof(int32_t) * ev.size());
    if (e == hipSuccess) e = hipMemcpyAsync(p->even, ev.data(), sizeof(int32_t) * ev.size(), hipMemcpyHostToDevice, s);
  }
  if (e == hipSuccess && d.ns_select) {
    e = hipMalloc(&p->sel, sizeof(int32_t) * d.n_chan * keep);
    if (e == hipSuccess)
      e = hipMemcpyAsync(p->sel, d.ns_select, sizeof(int32_t) * d.n_chan * keep, hipMemcpyHostToDevice, s);
  }
  std::vector<double> dl((size_t)d.n_chan * 2, 0.5);
  if (e == hipSuccess) {
    if (d.d_over_lambda) std::memcpy(dl.data(), d.d_over_lambda, sizeof(double) * dl.size());
    e = hipMalloc(&p->dl, sizeof(double) * dl.size());
    if (e == hipSuccess) e = hipMemcpyAsync(p->dl, dl.data(), sizeof(double) * dl.size(), hipMemcpyHostToDevice, s);
  }
  if (e == hipSuccess && d.precision != BF_PREC_FP32) {
    e = hipMalloc(&p->mix, fftbf::mix_table_bytes(d.n_ns, d.precision));
    if (e == hipSuccess) e = fftbf::launch_mix_tables(p->mix, d.n_ns, d.precision, s);
  }
  if (e == hipSuccess) e = ss.finish();
  if (e != hipSuccess) {
    free_plan(p);
    return dev_fail(e, "plan_create: device tables");
  }
  *plan = p;
  return BF_OK;
}

bf_status bf_plan_destroy(bf_plan* plan) {
  FFTBF_TRACE("bf_plan_destroy");
  if (!plan) return BF_OK;
  hipError_t e = hipDeviceSynchronize();
  free_plan(plan);
  if (e != hipSuccess) return dev_fail(e, "plan_destroy: pending device error");
  return BF_OK;
}

__attribute__((visibility("hidden"))) const double* bf_internal_plan_dl(const bf_plan* plan, bf_plan_desc* desc) {
  *desc = plan->d;
  return plan->dl;
}

bf_status bf_plan_get_desc(const bf_plan* plan, bf_plan_desc* desc) {
  if (!plan || !desc) return fail(BF_ERR_INVALID_ARGUMENT, "plan_get_desc: NULL argument");
  *desc = plan->d;
  return BF_OK;
}

}  // extern "C"

// taper_kind: 1 real weights [n_ns][n_ew], 2 complex gains [n_ns][n_ew][2]
static bf_status beamform_fft_impl(const bf_plan* plan, const uint8_t* volts, int64_t n_time, const float* taper,
                                   int taper_kind, int32_t kind, void* out, void* stream) {
  if (!plan) return fail(BF_ERR_INVALID_ARGUMENT, "beamform_fft: NULL plan");
  const bf_plan_desc& d = plan->d;
  if (kind != BF_OUT_INTENSITY && kind != BF_OUT_COMPLEX)
    return fail(BF_ERR_INVALID_ARGUMENT, "beamform_fft: unknown output kind %d", kind);
  if (n_time < 0) return fail(BF_ERR_INVALID_ARGUMENT, "beamform_fft: negative n_time");
  if (n_time == 0) return BF_OK;
  if (!volts || !out) return fail(BF_ERR_INVALID_ARGUMENT, "beamform_fft: NULL volts or out");
  if (!aligned(volts, 4)) return fail(BF_ERR_INVALID_ARGUMENT, "beamform_fft: volts must be 4-byte aligned");
  if (!aligned(out, kind == BF_OUT_COMPLEX ? 8 : 4))
    return fail(BF_ERR_INVALID_ARGUMENT, "beamform_fft: out is misaligned");
  if (taper && !aligned(taper, 16)) return fail(BF_ERR_INVALID_ARGUMENT, "beamform_fft: taper must be 16-byte aligned");
  if (kind == BF_OUT_INTENSITY && n_time % d.block)
    return fail(BF_ERR_INVALID_ARGUMENT, "beamform_fft: n_time %lld is not a multiple of block %d",
                (long long)n_time, d.block);
  if (kind == BF_OUT_COMPLEX && d.precision != BF_PREC_FP32)
    return fail(BF_ERR_UNSUPPORTED, "beamform_fft: complex beams are produced by FP32 plans only");
  if (d.precision != BF_PREC_FP32 && taper && !fftbf::mix_window_supported(d.n_ns, d.precision))
    return fail(BF_ERR_UNSUPPORTED,
                "beamform_fft: a window on the matrix cores needs an FP16 plan (use an FP32 plan)");
  if (d.precision != BF_PREC_FP32 && !aligned(volts, 16))
    return fail(BF_ERR_INVALID_ARGUMENT, "beamform_fft: mixed-precision plans need 16-byte aligned volts");
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t n_blk = (n_time + d.block - 1) / d.block;
  const int n_pg = (kind == BF_OUT_INTENSITY && d.pol_sum) ? 1 : d.n_pol;
  const int64_t n_wg = n_blk * d.n_chan * n_pg;
  if (n_wg > 0x7FFFFFFFLL) return fail(BF_ERR_UNSUPPORTED, "beamform_fft: grid too large, split the call");
  hipError_t e;
  if (d.precision == BF_PREC_FP32) {
    fftbf::Fft32Args a{};
    a.volts = reinterpret_cast<const uint32_t*>(volts);
    a.n_time = n_time;
    a.n_chan = d.n_chan;
    a.n_pol = d.n_pol;
    a.n_pg = n_pg;
    a.pol_iter = (n_pg == 1) ? d.n_pol : 1;
    a.block = d.block;
    a.tw = plan->tw;
    a.mult = plan->mult;
    a.taper = taper;
    a.sel = plan->fold > 1 ? plan->even : plan->sel;
    a.n_keep = keep_of(d);
    a.fold = plan->fold;
    a.out = out;
    const float inv_n = 1.0f / float(d.n_ew * d.n_ns);
    a.norm = (kind == BF_OUT_COMPLEX) ? 1.0f / std::sqrt(float(d.n_ew * d.n_ns)) : inv_n;
    a.ew_rows = d.m_ew;
    a.ew_mul = d.m_ew / 4;
    a.ew_off = 0;
    a.gain_src = taper ? taper_kind : 0;
    a.twist = 0;
    if (plan->fold > 1 && taper && (taper_kind != 1 || plan->fold > 8))
      return fail(BF_ERR_UNSUPPORTED, "beamform_fft: cyclic co-adding takes a real window only, up to 8-fold");
    e = fftbf::launch_fft32(a, d.n_ns / plan->fold, taper ? taper_kind : 0, kind == BF_OUT_COMPLEX, n_wg, s);
    const bool fused = fftbf::fft32_fuses_ew8(d.n_ns / plan->fold, taper ? taper_kind : 0, kind == BF_OUT_COMPLEX,
                                              plan->fold);
    if (e == hipSuccess && d.m_ew == 8 && !fused) {
      // odd E-W beams of the zero-padded 8-point E-W transform: the 4-point
      // DFT of x_a W_8^{a_ew} (with the window or gains, if any)
      a.ew_off = 1;
      a.twist = 1;
      e = fftbf::launch_fft32(a, d.n_ns, taper ? 2 : 3, kind == BF_OUT_COMPLEX, n_wg, s);
    }
  } else {
    fftbf::MixArgs a{};
    a.volts = reinterpret_cast<const uint32_t*>(volts);
    a.n_time = n_time;
    a.n_chan = d.n_chan;
    a.n_pol = d.n_pol;
    a.n_pg = n_pg;
    a.pol_iter = (n_pg == 1) ? d.n_pol : 1;
    a.block = d.block;
    a.mat = plan->mix;
    a.taper = taper;
    a.sel = plan->sel;
    a.n_keep = keep_of(d);
    a.out = static_cast<float*>(out);
    a.norm = 1.0f / float(d.n_ew * d.n_ns);
    e = fftbf::launch_mix(a, d.n_ns, d.precision, n_wg, s);
  }
  if (e != hipSuccess) return dev_fail(e, "beamform_fft: launch");
  return BF_OK;
}

extern "C" {

bf_status bf_beamform_fft(const bf_plan* plan, const uint8_t* volts, int64_t n_time, const float* taper, int32_t kind,
                          void* out, void* stream) {
  FFTBF_TRACE("bf_beamform_fft");
  return beamform_fft_impl(plan, volts, n_time, taper, 1, kind, out, stream);
}

bf_status bf_beamform_fft_gains(const bf_plan* plan, const uint8_t* volts, int64_t n_time, const float* gains,
                                int32_t kind, void* out, void* stream) {
  FFTBF_TRACE("bf_beamform_fft_gains");
  if (!gains) return fail(BF_ERR_INVALID_ARGUMENT, "beamform_fft_gains: NULL gains");
  if (plan && plan->d.precision != BF_PREC_FP32)
    return fail(BF_ERR_UNSUPPORTED, "beamform_fft_gains: complex gains need an FP32 plan");
  return beamform_fft_impl(plan, volts, n_time, gains, 2, kind, out, stream);
}

static bf_status tied_common(const bf_plan* plan, int64_t n_time, int32_t chan_lo, int32_t n_chan_sub,
                             const double* dircos, int32_t n_point, const void* out, const char* who) {
  if (!plan) return fail(BF_ERR_INVALID_ARGUMENT, "%s: NULL plan", who);
  const bf_plan_desc& d = plan->d;
  if (n_time < 0 || n_point < 0 || n_chan_sub < 0)
    return fail(BF_ERR_INVALID_ARGUMENT, "%s: negative size", who);
  if (chan_lo < 0 || (int64_t)chan_lo + n_chan_sub > d.n_chan)
    return fail(BF_ERR_INVALID_ARGUMENT, "%s: channel range [%d, %d) outside [0, %d)", who, chan_lo,
                chan_lo + n_chan_sub, d.n_chan);
  if (n_time && n_point && n_chan_sub && (!dircos || !out))
    return fail(BF_ERR_INVALID_ARGUMENT, "%s: NULL dircos or out", who);
  if (dircos && !aligned(dircos, 8)) return fail(BF_ERR_INVALID_ARGUMENT, "%s: dircos misaligned", who);
  if (out && !aligned(out, 8)) return fail(BF_ERR_INVALID_ARGUMENT, "%s: out must be 8-byte aligned", who);
  if (n_point > 4096) return fail(BF_ERR_UNSUPPORTED, "%s: at most 4096 pointings per call", who);
  return BF_OK;
}

bf_status bf_form_tied_beams(const bf_plan* plan, const void* fft_beams, int64_t n_time, int32_t chan_lo,
                             int32_t n_chan_sub, const double* dircos, int32_t n_point, int32_t kind,
                             void* out, void* stream) {
  FFTBF_TRACE("bf_form_tied_beams");
  bf_status st = tied_common(plan, n_time, chan_lo, n_chan_sub, dircos, n_point, out, "form_tied_beams");
  if (st != BF_OK) return st;
  const bf_plan_desc& d = plan->d;
  if (kind != BF_OUT_INTENSITY && kind != BF_OUT_COMPLEX)
    return fail(BF_ERR_INVALID_ARGUMENT, "form_tied_beams: unknown output kind %d", kind);
  if (n_time == 0 || n_point == 0 || n_chan_sub == 0) return BF_OK;
  if (!fft_beams || !aligned(fft_beams, 8))
    return fail(BF_ERR_INVALID_ARGUMENT, "form_tied_beams: NULL or misaligned fft_beams");
  if (kind == BF_OUT_INTENSITY && n_time % d.block)
    return fail(BF_ERR_INVALID_ARGUMENT, "form_tied_beams: n_time not a multiple of block");
  if (kind == BF_OUT_COMPLEX && d.pol_sum)
    return fail(BF_ERR_INVALID_ARGUMENT, "form_tied_beams: complex output cannot sum polarisations");
  if (d.m_ns < 32 || d.m_ns > 512 || d.m_ew != 4 || d.m_ns < d.n_ns)
    return fail(BF_ERR_UNSUPPORTED, "form_tied_beams: m_ns must be in [32, 512] (and >= n_ns) and m_ew 4");
  if (d.m_ns >= 128 && !aligned(fft_beams, 16))
    return fail(BF_ERR_INVALID_ARGUMENT, "form_tied_beams: fft_beams must be 16-byte aligned for m_ns >= 128");
  fftbf::TiedArgs a{};
  a.beams = static_cast<const float2*>(fft_beams);
  a.n_time = n_time;
  a.n_chan = d.n_chan;
  a.n_pol = d.n_pol;
  a.chan_lo = chan_lo;
  a.n_chan_sub = n_chan_sub;
  a.n_ew = d.n_ew;
  a.n_ns = d.n_ns;
  a.m_ew = d.m_ew;
  a.m_ns = d.m_ns;
  a.dircos = dircos;
  a.dl = plan->dl;
  a.n_point = n_point;
  a.block = d.block;
  a.pol_sum = d.pol_sum;
  a.complex_out = kind == BF_OUT_COMPLEX;
  a.out = out;
  hipError_t e = fftbf::launch_tied(a, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return dev_fail(e, "form_tied_beams: launch");
  return BF_OK;
}

static bf_status tied_v_impl(const bf_plan* plan, const uint8_t* volts, int64_t n_time, const float* taper,
                             int32_t chan_lo, int32_t n_chan_sub, const double* dircos, int32_t n_point, void* out,
                             void* stream) {
  bf_status st = tied_common(plan, n_time, chan_lo, n_chan_sub, dircos, n_point, out, "form_tied_beams_v");
  if (st != BF_OK) return st;
  const bf_plan_desc& d = plan->d;
  if (n_time == 0 || n_point == 0 || n_chan_sub == 0) return BF_OK;
  if (!volts || !aligned(volts, 4)) return fail(BF_ERR_INVALID_ARGUMENT, "form_tied_beams_v: NULL or misaligned volts");
  if (taper && !aligned(taper, 16)) return fail(BF_ERR_INVALID_ARGUMENT, "form_tied_beams_v: taper misaligned");
  if (n_time % d.block) return fail(BF_ERR_INVALID_ARGUMENT, "form_tied_beams_v: n_time not a multiple of block");
  if (d.n_ns != 16 || d.m_ew != 4 || d.block % 16)
    return fail(BF_ERR_UNSUPPORTED, "form_tied_beams_v: needs the 4 x 16 lattice (m_ew 4) and block a multiple of 16");
  fftbf::TiedArgs a{};
  a.volts = reinterpret_cast<const uint32_t*>(volts);
  a.taper = taper;
  a.n_time = n_time;
  a.n_chan = d.n_chan;
  a.n_pol = d.n_pol;
  a.chan_lo = chan_lo;
  a.n_chan_sub = n_chan_sub;
  a.n_ew = d.n_ew;
  a.n_ns = d.n_ns;
  a.m_ew = d.m_ew;
  a.m_ns = d.m_ns;
  a.dircos = dircos;
  a.dl = plan->dl;
  a.n_point = n_point;
  a.block = d.block;
  a.pol_sum = d.pol_sum;
  a.complex_out = 0;
  a.out = out;
  hipError_t e = fftbf::launch_tied_v(a, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return dev_fail(e, e == hipErrorNotSupported ? "form_tied_beams_v: shape" : "form_tied_beams_v: launch");
  return BF_OK;
}

bf_status bf_form_tied_beams_v(const bf_plan* plan, const uint8_t* volts, int64_t n_time, const float* taper,
                               int32_t chan_lo, int32_t n_chan_sub, const double* dircos, int32_t n_point,
                               void* out, void* stream) {
  FFTBF_TRACE("bf_form_tied_beams_v");
  return tied_v_impl(plan, volts, n_time, taper, chan_lo, n_chan_sub, dircos, n_point, out, stream);
}

size_t bf_tied_workspace_size(const bf_plan* plan, int32_t n_chan_sub, int64_t chunk_samples) {
  if (!plan || n_chan_sub < 0 || chunk_samples < 0) return 0;
  const bf_plan_desc& d = plan->d;
  return (size_t)chunk_samples * (size_t)n_chan_sub * (size_t)d.n_pol * (size_t)d.m_ew * (size_t)d.m_ns * 8u;
}

static bf_status tied_v_ws_impl(const bf_plan* plan, const uint8_t* volts, int64_t n_time, const float* taper,
                                int32_t chan_lo, int32_t n_chan_sub, const double* dircos, int32_t n_point,
                                void* workspace, size_t workspace_bytes, void* out, void* stream) {
  bf_status st = tied_common(plan, n_time, chan_lo, n_chan_sub, dircos, n_point, out, "form_tied_beams_v_ws");
  if (st != BF_OK) return st;
  const bf_plan_desc& d = plan->d;
  if (d.n_ns == 16 && d.m_ew == 4 && d.block % 16 == 0)
    return tied_v_impl(plan, volts, n_time, taper, chan_lo, n_chan_sub, dircos, n_point, out, stream);
  if (n_time == 0 || n_point == 0 || n_chan_sub == 0) return BF_OK;
  if (!volts || !aligned(volts, 4)) return fail(BF_ERR_INVALID_ARGUMENT, "form_tied_beams_v_ws: NULL or misaligned volts");
  if (taper && !aligned(taper, 16)) return fail(BF_ERR_INVALID_ARGUMENT, "form_tied_beams_v_ws: taper misaligned");
  if (n_time % d.block) return fail(BF_ERR_INVALID_ARGUMENT, "form_tied_beams_v_ws: n_time not a multiple of block");
  if (d.precision != BF_PREC_FP32 || d.m_ew != 4 || d.m_ns < 32 || d.m_ns > 512 || d.m_ns < d.n_ns)
    return fail(BF_ERR_UNSUPPORTED, "form_tied_beams_v_ws: needs an FP32 plan with m_ew 4 and m_ns in [32, 512], >= n_ns");
  const size_t per_block = bf_tied_workspace_size(plan, n_chan_sub, d.block);
  if (!workspace || !aligned(workspace, 16) || workspace_bytes < per_block)
    return fail(BF_ERR_INVALID_ARGUMENT, "form_tied_beams_v_ws: workspace NULL, misaligned or below %zu bytes (one block)",
                per_block);
  int64_t chunk = (int64_t)(workspace_bytes / per_block) * d.block;
  if (chunk > n_time) chunk = n_time;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const int n_pg = d.pol_sum ? 1 : d.n_pol;
  for (int64_t t0 = 0; t0 < n_time; t0 += chunk) {
    const int64_t len = n_time - t0 < chunk ? n_time - t0 : chunk;
    // complex FFT beams of samples [t0, t0 + len), channels [chan_lo, chan_lo + n_chan_sub)
    fftbf::Fft32Args f{};
    f.volts = reinterpret_cast<const uint32_t*>(volts) + (t0 * d.n_chan + chan_lo) * (int64_t)d.n_pol * d.n_ns;
    f.n_time = len;
    f.n_chan = n_chan_sub;
    f.chan_stride = d.n_chan;
    f.n_pol = d.n_pol;
    f.n_pg = d.n_pol;
    f.pol_iter = 1;
    f.block = d.block;
    f.tw = plan->tw;
    f.mult = plan->mult;
    f.taper = taper;
    f.sel = nullptr;
    f.n_keep = d.m_ns;
    f.fold = 1;
    f.out = workspace;
    f.norm = 1.0f / std::sqrt(float(d.n_ew * d.n_ns));
    f.ew_rows = 4;
    f.ew_mul = 1;
    f.ew_off = 0;
    f.gain_src = taper ? 1 : 0;
    f.twist = 0;
    const int64_t n_wg = (len + d.block - 1) / d.block * n_chan_sub * d.n_pol;
    if (n_wg > 0x7FFFFFFFLL) return fail(BF_ERR_UNSUPPORTED, "form_tied_beams_v_ws: chunk grid too large, split the call");
    hipError_t e = fftbf::launch_fft32(f, d.n_ns, taper ? 1 : 0, true, n_wg, s);
    if (e != hipSuccess) return dev_fail(e, "form_tied_beams_v_ws: FFT launch");
    // tied beams of the chunk from those beams
    fftbf::TiedArgs a{};
    a.beams = static_cast<const float2*>(workspace);
    a.n_time = len;
    a.n_chan = n_chan_sub;
    a.n_pol = d.n_pol;
    a.chan_lo = 0;
    a.n_chan_sub = n_chan_sub;
    a.n_ew = d.n_ew;
    a.n_ns = d.n_ns;
    a.m_ew = d.m_ew;
    a.m_ns = d.m_ns;
    a.dircos = dircos;
    a.dl = plan->dl + 2 * (int64_t)chan_lo;
    a.n_point = n_point;
    a.block = d.block;
    a.pol_sum = d.pol_sum;
    a.complex_out = 0;
    a.out = static_cast<float*>(out) + (t0 / d.block) * (int64_t)n_chan_sub * n_pg * n_point;
    e = fftbf::launch_tied(a, s);
    if (e != hipSuccess) return dev_fail(e, "form_tied_beams_v_ws: interpolation launch");
  }
  return BF_OK;
}

bf_status bf_form_tied_beams_v_ws(const bf_plan* plan, const uint8_t* volts, int64_t n_time, const float* taper,
                                  int32_t chan_lo, int32_t n_chan_sub, const double* dircos, int32_t n_point,
                                  void* workspace, size_t workspace_bytes, void* out, void* stream) {
  FFTBF_TRACE("bf_form_tied_beams_v_ws");
  return tied_v_ws_impl(plan, volts, n_time, taper, chan_lo, n_chan_sub, dircos, n_point, workspace,
                        workspace_bytes, out, stream);
}

}  // extern "C"

// The workspace of bf_form_tied_beams_v_noalloc: a file-scope device array,
// one copy per GPU the library runs on, held until the process ends.  In
// host code `scratch` is a host-side stand-in, not a device address: its
// address on the current device comes from hipGetSymbolAddress (taken once
// per device) and only that address is handed to the kernels.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

static bf_status static_scratch(void** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* ptrs[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return dev_fail(e, "form_tied_beams_v_noalloc: hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(BF_ERR_UNSUPPORTED, "form_tied_beams_v_noalloc: device %d", dev);
  std::lock_guard<std::mutex> lock(mu);
  if (!ptrs[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return dev_fail(e, "form_tied_beams_v_noalloc: hipGetSymbolAddress");
    ptrs[dev] = p;
  }
  *out = ptrs[dev];
  return BF_OK;
}

extern "C" {

bf_status bf_form_tied_beams_v_noalloc(const bf_plan* plan, const uint8_t* volts, int64_t n_time,
                                       const float* taper, int32_t chan_lo, int32_t n_chan_sub,
                                       const double* dircos, int32_t n_point, void* out, void* stream) {
  bf_status st = tied_common(plan, n_time, chan_lo, n_chan_sub, dircos, n_point, out, "form_tied_beams_v_noalloc");
  if (st != BF_OK) return st;
  const bf_plan_desc& d = plan->d;
  if (d.n_ns == 16 && d.m_ew == 4 && d.block % 16 == 0)      // the fused kernel uses no workspace
    return tied_v_impl(plan, volts, n_time, taper, chan_lo, n_chan_sub, dircos, n_point, out, stream);
  const size_t per_block = bf_tied_workspace_size(plan, n_chan_sub, d.block);
  if (per_block > kStaticScratchBytes)
    return fail(BF_ERR_INVALID_ARGUMENT,
                "form_tied_beams_v_noalloc: one block of %d channels needs %zu bytes of workspace, above the "
                "%zu-byte static scratch (fewer channels per call, or bf_form_tied_beams_v_ws)",
                n_chan_sub, per_block, kStaticScratchBytes);
  void* ws = nullptr;
  st = static_scratch(&ws);
  if (st != BF_OK) return st;
  return tied_v_ws_impl(plan, volts, n_time, taper, chan_lo, n_chan_sub, dircos, n_point, ws, kStaticScratchBytes,
                        out, stream);
}

}  // extern "C"

struct bf_regrid {
  int n_chan = 0, n_pg = 0, m_ew = 0, m_ns = 0, n_ns = 0, n_target = 0, pad = 0, n_taps = 0;
  float* w = nullptr;       // dense weights [n_chan][pad][m_ns]
  int* first = nullptr;     // compact kernels [n_chan][n_target]
  float* tw = nullptr;      //                 [n_chan][n_taps][n_target]
  float* wew = nullptr;     // 2-D pointings: E-W weights [n_chan][pad][8]
};

namespace {

// Lag coefficients of the optimally windowed kernel (eq. e:w_opt): with the
// window's auto-convolution R_d = sum_a h[a + d] h[a] (real window, so
// R_-d = R_d), c_d = R_d / ((n - d) N) for d = 0 .. n-1, where N makes the
// beam's noise equal to the unwindowed pointed beam's:
// N = (1/n) sqrt(sum_{d=-(n-1)}^{n-1} R_d^2 / (n - |d|)).  Returns false when
// the window has no power.
bool window_lag_coefficients(const double* h, int n, std::vector<double>& c) {
  std::vector<double> r(n, 0.0);
  for (int d = 0; d < n; ++d)
    for (int a = 0; a + d < n; ++a) r[d] += h[a + d] * h[a];
  double s = r[0] * r[0] / n;
  for (int d = 1; d < n; ++d) s += 2.0 * r[d] * r[d] / (n - d);
  if (!(s > 0.0)) return false;
  const double norm = std::sqrt(s) / n;
  c.resize(n);
  for (int d = 0; d < n; ++d) c[d] = r[d] / ((n - d) * norm);
  return true;
}

void regrid_free(bf_regrid* r) {
  if (r->w) (void)hipFree(r->w);
  if (r->first) (void)hipFree(r->first);
  if (r->tw) (void)hipFree(r->tw);
  if (r->wew) (void)hipFree(r->wew);
  delete r;
}

}  // namespace

extern "C" {

bf_status bf_regrid_create(const bf_plan* plan, const double* sin_theta, int32_t n_target, const double* window,
                           int32_t n_taps, bf_regrid** rg) {
  FFTBF_TRACE("bf_regrid_create");
  if (!rg) return fail(BF_ERR_INVALID_ARGUMENT, "regrid_create: NULL rg");
  *rg = nullptr;
  if (!plan || !sin_theta) return fail(BF_ERR_INVALID_ARGUMENT, "regrid_create: NULL plan or sin_theta");
  const bf_plan_desc& d = plan->d;
  if (plan->sel || keep_of(d) != d.m_ns)
    return fail(BF_ERR_INVALID_ARGUMENT, "regrid_create: needs a plan without a clamp (all m_ns beams)");
  if (d.m_ns < 2 * d.n_ns - 1)
    return fail(BF_ERR_UNSUPPORTED, "regrid_create: exact regridding needs m_ns >= 2 n_ns - 1");
  if (n_target < 1 || n_target > 65536) return fail(BF_ERR_INVALID_ARGUMENT, "regrid_create: n_target out of [1, 65536]");
  if (n_taps < 0 || n_taps > fftbf::kRegridMaxTaps)
    return fail(BF_ERR_INVALID_ARGUMENT, "regrid_create: n_taps out of [0, %d]", fftbf::kRegridMaxTaps);
  for (int j = 0; j < n_target; ++j)
    if (!(sin_theta[j] >= -1e6 && sin_theta[j] <= 1e6))
      return fail(BF_ERR_INVALID_ARGUMENT, "regrid_create: sin_theta[%d] not finite", j);
  std::vector<double> coef;
  if (window) {
    for (int a = 0; a < d.n_ns; ++a)
      if (!(window[a] >= -1e30 && window[a] <= 1e30))
        return fail(BF_ERR_INVALID_ARGUMENT, "regrid_create: window[%d] not finite", a);
    if (!window_lag_coefficients(window, d.n_ns, coef))
      return fail(BF_ERR_INVALID_ARGUMENT, "regrid_create: window has no power");
  }
  bf_regrid* r = new (std::nothrow) bf_regrid();
  if (!r) return fail(BF_ERR_OUT_OF_MEMORY, "regrid_create: host allocation");
  r->n_chan = d.n_chan;
  r->n_pg = d.pol_sum ? 1 : d.n_pol;
  r->m_ew = d.m_ew;
  r->m_ns = d.m_ns;
  r->n_ns = d.n_ns;
  r->n_target = n_target;
  r->n_taps = n_taps;
  r->pad = fftbf::regrid_target_pad(n_target);
  double *st = nullptr, *dcoef = nullptr;
  SetupStream ss;
  hipError_t e = ss.init();
  const hipStream_t s = ss.get();
  if (e == hipSuccess) e = hipMallocAsync(reinterpret_cast<void**>(&st), sizeof(double) * n_target, s);
  if (e == hipSuccess) e = hipMemcpyAsync(st, sin_theta, sizeof(double) * n_target, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && window) {
    e = hipMallocAsync(reinterpret_cast<void**>(&dcoef), sizeof(double) * d.n_ns, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dcoef, coef.data(), sizeof(double) * d.n_ns, hipMemcpyHostToDevice, s);
  }
  if (n_taps == 0) {
    if (e == hipSuccess) e = hipMalloc(&r->w, sizeof(float) * (size_t)r->n_chan * r->pad * r->m_ns);
    if (e == hipSuccess)
      e = fftbf::launch_regrid_weights(r->w, plan->dl, st, dcoef, r->n_chan, n_target, r->n_ns, r->m_ns, s);
  } else {
    if (e == hipSuccess) e = hipMalloc(&r->first, sizeof(int) * (size_t)r->n_chan * n_target);
    if (e == hipSuccess) e = hipMalloc(&r->tw, sizeof(float) * (size_t)r->n_chan * n_taps * n_target);
    if (e == hipSuccess)
      e = fftbf::launch_regrid_tap_table(r->first, r->tw, plan->dl, st, dcoef, r->n_chan, n_target, n_taps, r->n_ns,
                                         r->m_ns, s);
  }
  if (st) (void)hipFreeAsync(st, s);
  if (dcoef) (void)hipFreeAsync(dcoef, s);
  if (e == hipSuccess) e = ss.finish();
  if (e != hipSuccess) {
    regrid_free(r);
    return dev_fail(e, "regrid_create: weights");
  }
  *rg = r;
  return BF_OK;
}

bf_status bf_regrid_create_2d(const bf_plan* plan, const double* dircos, int32_t n_point, bf_regrid** rg) {
  FFTBF_TRACE("bf_regrid_create_2d");
  if (!rg) return fail(BF_ERR_INVALID_ARGUMENT, "regrid_create_2d: NULL rg");
  *rg = nullptr;
  if (!plan || !dircos) return fail(BF_ERR_INVALID_ARGUMENT, "regrid_create_2d: NULL plan or dircos");
  const bf_plan_desc& d = plan->d;
  if (plan->sel || keep_of(d) != d.m_ns)
    return fail(BF_ERR_INVALID_ARGUMENT, "regrid_create_2d: needs a plan without a clamp (all m_ns beams)");
  if (d.m_ns < 2 * d.n_ns - 1 || d.m_ew < 2 * d.n_ew - 1)
    return fail(BF_ERR_UNSUPPORTED, "regrid_create_2d: exact 2-D regridding needs m >= 2 n - 1 on both axes (m_ew = 8)");
  if (n_point < 1 || n_point > 65536) return fail(BF_ERR_INVALID_ARGUMENT, "regrid_create_2d: n_point out of [1, 65536]");
  std::vector<double> dew(n_point), dns(n_point);
  for (int j = 0; j < n_point; ++j) {
    dew[j] = dircos[2 * j];
    dns[j] = dircos[2 * j + 1];
    if (!(dew[j] >= -1e6 && dew[j] <= 1e6 && dns[j] >= -1e6 && dns[j] <= 1e6))
      return fail(BF_ERR_INVALID_ARGUMENT, "regrid_create_2d: dircos[%d] not finite", j);
  }
  bf_regrid* r = new (std::nothrow) bf_regrid();
  if (!r) return fail(BF_ERR_OUT_OF_MEMORY, "regrid_create_2d: host allocation");
  r->n_chan = d.n_chan;
  r->n_pg = d.pol_sum ? 1 : d.n_pol;
  r->m_ew = d.m_ew;
  r->m_ns = d.m_ns;
  r->n_ns = d.n_ns;
  r->n_target = n_point;
  r->pad = fftbf::regrid_target_pad(n_point);
  double *dd = nullptr;
  SetupStream ss;
  hipError_t e = ss.init();
  const hipStream_t s = ss.get();
  if (e == hipSuccess) e = hipMallocAsync(reinterpret_cast<void**>(&dd), sizeof(double) * 2 * n_point, s);
  if (e == hipSuccess) e = hipMemcpyAsync(dd, dns.data(), sizeof(double) * n_point, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(dd + n_point, dew.data(), sizeof(double) * n_point, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMalloc(&r->w, sizeof(float) * (size_t)r->n_chan * r->pad * r->m_ns);
  if (e == hipSuccess) e = hipMalloc(&r->wew, sizeof(float) * (size_t)r->n_chan * r->pad * 8);
  if (e == hipSuccess)
    e = fftbf::launch_regrid_weights(r->w, plan->dl, dd, nullptr, r->n_chan, n_point, r->n_ns, r->m_ns, s);
  if (e == hipSuccess)
    e = fftbf::launch_regrid_ew_weights(r->wew, plan->dl, dd + n_point, r->n_chan, n_point, d.n_ew, d.m_ew, s);
  if (dd) (void)hipFreeAsync(dd, s);
  if (e == hipSuccess) e = ss.finish();
  if (e != hipSuccess) {
    regrid_free(r);
    return dev_fail(e, "regrid_create_2d: weights");
  }
  *rg = r;
  return BF_OK;
}

bf_status bf_regrid_destroy(bf_regrid* rg) {
  FFTBF_TRACE("bf_regrid_destroy");
  if (!rg) return BF_OK;
  hipError_t e = hipDeviceSynchronize();
  regrid_free(rg);
  if (e != hipSuccess) return dev_fail(e, "regrid_destroy: pending device error");
  return BF_OK;
}

bf_status bf_regrid_intensity(const bf_regrid* rg, const float* fft_intensity, int64_t n_blk, float* out,
                              void* stream) {
  FFTBF_TRACE("bf_regrid_intensity");
  if (!rg) return fail(BF_ERR_INVALID_ARGUMENT, "regrid_intensity: NULL regrid");
  if (n_blk < 0) return fail(BF_ERR_INVALID_ARGUMENT, "regrid_intensity: negative n_blk");
  if (n_blk == 0) return BF_OK;
  if (!fft_intensity || !out) return fail(BF_ERR_INVALID_ARGUMENT, "regrid_intensity: NULL in or out");
  if (!aligned(fft_intensity, 16) || !aligned(out, 4))
    return fail(BF_ERR_INVALID_ARGUMENT, "regrid_intensity: fft_intensity must be 16-byte aligned, out 4-byte");
  fftbf::RegridArgs a{};
  a.in = fft_intensity;
  a.w = rg->w;
  a.out = out;
  a.n_blk = n_blk;
  a.n_chan = rg->n_chan;
  a.n_pg = rg->n_pg;
  a.m_ew = rg->m_ew;
  a.m_ns = rg->m_ns;
  a.n_target = rg->n_target;
  a.n_target_pad = rg->pad;
  a.n_taps = rg->n_taps;
  a.first = rg->first;
  a.tw = rg->tw;
  a.wew = rg->wew;
  hipError_t e = fftbf::launch_regrid(a, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return dev_fail(e, "regrid_intensity: launch");
  return BF_OK;
}

bf_status bf_localize(const bf_plan* plan, const float* fft_intensity, int64_t n_blk, int32_t n_window,
                      int32_t n_iter, double* sin_theta, float* peak, void* stream) {
  FFTBF_TRACE("bf_localize");
  if (!plan) return fail(BF_ERR_INVALID_ARGUMENT, "localize: NULL plan");
  const bf_plan_desc& d = plan->d;
  if (plan->sel || keep_of(d) != d.m_ns)
    return fail(BF_ERR_INVALID_ARGUMENT, "localize: needs a plan without a clamp (all m_ns beams)");
  if (d.m_ns < 2 * d.n_ns - 1)
    return fail(BF_ERR_UNSUPPORTED, "localize: the estimator needs m_ns >= 2 n_ns - 1");
  if (n_blk < 0) return fail(BF_ERR_INVALID_ARGUMENT, "localize: negative n_blk");
  if (n_window < 1 || n_window > 64 || n_window > d.m_ns)
    return fail(BF_ERR_INVALID_ARGUMENT, "localize: n_window out of [1, min(64, m_ns)]");
  if (n_iter < 0 || n_iter > 64) return fail(BF_ERR_INVALID_ARGUMENT, "localize: n_iter out of [0, 64]");
  if (n_blk == 0) return BF_OK;
  if (!fft_intensity || !sin_theta) return fail(BF_ERR_INVALID_ARGUMENT, "localize: NULL intensity or sin_theta");
  if (!aligned(fft_intensity, 4) || !aligned(sin_theta, 8) || (peak && !aligned(peak, 4)))
    return fail(BF_ERR_INVALID_ARGUMENT, "localize: misaligned buffer");
  fftbf::LocArgs a{};
  a.in = fft_intensity;
  a.dl = plan->dl;
  a.sin_out = sin_theta;
  a.peak_out = peak;
  a.rows_per_chan_blk = (int64_t)(d.pol_sum ? 1 : d.n_pol) * d.m_ew;
  a.n_rows = n_blk * d.n_chan * a.rows_per_chan_blk;
  a.n_chan = d.n_chan;
  a.n = d.n_ns;
  a.m = d.m_ns;
  a.n_window = n_window;
  a.n_iter = n_iter;
  int64_t moi = 0;
  for (int64_t k = 1; k < d.n_ns; ++k) moi += 2 * k * k * (d.n_ns - k);
  a.moi = (double)moi;
  hipError_t e = fftbf::launch_localize(a, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return dev_fail(e, "localize: launch");
  return BF_OK;
}

bf_status bf_accumulate_intensity(const void* z, int64_t n_time, int64_t n_series, int32_t block, int32_t add,
                                  float* out, void* stream) {
  FFTBF_TRACE("bf_accumulate_intensity");
  if (n_time < 0 || n_series < 0) return fail(BF_ERR_INVALID_ARGUMENT, "accumulate_intensity: negative size");
  if (block <= 0) return fail(BF_ERR_INVALID_ARGUMENT, "accumulate_intensity: block must be positive");
  if (add != 0 && add != 1) return fail(BF_ERR_INVALID_ARGUMENT, "accumulate_intensity: add is 0 or 1");
  if (n_time % block) return fail(BF_ERR_INVALID_ARGUMENT, "accumulate_intensity: n_time %lld not a multiple of block %d",
                                  (long long)n_time, block);
  if (n_time == 0 || n_series == 0) return BF_OK;
  if (!z || !out) return fail(BF_ERR_INVALID_ARGUMENT, "accumulate_intensity: NULL z or out");
  if (!aligned(z, 8) || !aligned(out, 4)) return fail(BF_ERR_INVALID_ARGUMENT, "accumulate_intensity: misaligned buffer");
  if ((n_time / block) * n_series > (int64_t)0x7FFFFFFF * 256)
    return fail(BF_ERR_UNSUPPORTED, "accumulate_intensity: too many outputs for one launch");
  hipError_t e = fftbf::launch_accumulate(static_cast<const float2*>(z), n_time, n_series, block, add, out,
                                          static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return dev_fail(e, "accumulate_intensity: launch");
  return BF_OK;
}

}  // extern "C"
