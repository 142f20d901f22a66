// Tied-beam server: C ABI over the host scheduler (serve_sched.*) with a
// HIP backend -- device voltage ring, one device memory pool for request
// outputs and pointing tables, batched launches of the persistent tile
// worker on the server's own stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/fftbf.h"
#include "kernels.h"
#include "serve_sched.h"
#include "trace.h"

extern "C" __attribute__((visibility("hidden"))) void bf_internal_set_error(const char* msg);

using fftbf::serve::Request;
using fftbf::serve::Tile;

namespace {

bf_status sfail(bf_status s, const std::string& m) {
  bf_internal_set_error(m.c_str());
  return s;
}

bf_status map_status(int s) {
  switch (s) {
    case fftbf::serve::kOk: return BF_OK;
    case fftbf::serve::kInvalid: return BF_ERR_INVALID_ARGUMENT;
    case fftbf::serve::kUnsupported: return BF_ERR_UNSUPPORTED;
    case fftbf::serve::kRejected: return BF_ERR_REJECTED;
    case fftbf::serve::kEvicted: return BF_ERR_EVICTED;
    case fftbf::serve::kNotReady: return BF_ERR_NOT_READY;
    default: return BF_ERR_DEVICE;
  }
}

class HipBackend final : public fftbf::serve::Backend {
 public:
  static constexpr int kSlots = 3;   // > max launches in flight, so a staging slot is never reused early

  ~HipBackend() override {
    if (stream_) (void)hipStreamSynchronize(stream_);
    for (int i = 0; i < kSlots; ++i) {
      if (ev_[i]) (void)hipEventDestroy(ev_[i]);
      if (host_[i]) (void)hipHostFree(host_[i]);
      if (dev_[i]) (void)hipFree(dev_[i]);
    }
    if (ev_in_) (void)hipEventDestroy(ev_in_);
    if (ev_out_) (void)hipEventDestroy(ev_out_);
    if (pool_) (void)hipFree(pool_);
    if (ring_) (void)hipFree(ring_);
    if (dl_) (void)hipFree(dl_);
    if (stream_) (void)hipStreamDestroy(stream_);
  }

  hipError_t init(const bf_plan_desc& d, const double* dl_dev_src, int64_t ring_samples, size_t pool_bytes,
                  int max_tiles) {
    n_chan_ = d.n_chan;
    n_pol_ = d.n_pol;
    ring_samples_ = ring_samples;
    frame_bytes_ = (size_t)d.n_ns * d.n_ew;
    max_tiles_ = max_tiles;
    hipError_t e = hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc(&ring_, sample_bytes() * ring_samples);
    if (e == hipSuccess) e = hipMemsetAsync(ring_, 0, sample_bytes() * ring_samples, stream_);
    if (e == hipSuccess) e = hipMalloc(&pool_, pool_bytes);
    if (e == hipSuccess) e = hipMalloc(&dl_, sizeof(double) * 2 * n_chan_);
    if (e == hipSuccess) e = hipMemcpy(dl_, dl_dev_src, sizeof(double) * 2 * n_chan_, hipMemcpyDeviceToDevice);
    for (int i = 0; i < kSlots && e == hipSuccess; ++i) {
      e = hipHostMalloc(&host_[i], sizeof(fftbf::ServeTile) * max_tiles, hipHostMallocDefault);
      if (e == hipSuccess) e = hipMalloc(&dev_[i], sizeof(fftbf::ServeTile) * max_tiles);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_in_, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_out_, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamSynchronize(stream_);
    t0_ = std::chrono::steady_clock::now();
    return e;
  }

  size_t sample_bytes() const { return frame_bytes_ * n_chan_ * n_pol_; }

  bool upload_pointings(size_t off, const double* dircos, int n_point) override {
    return hipMemcpy(static_cast<char*>(pool_) + off, dircos, sizeof(double) * 2 * n_point,
                     hipMemcpyHostToDevice) == hipSuccess;
  }

  int64_t launch(const std::vector<Tile>& tiles, const std::vector<const Request*>& reqs) override {
    const int slot = (int)(count_ % kSlots);
    const int n = (int)tiles.size();
    if (n > max_tiles_) return -1;
    fftbf::ServeTile* h = host_[slot];
    for (int i = 0; i < n; ++i) {
      const Tile& t = tiles[i];
      const Request& r = *reqs[i];
      fftbf::ServeTile& d = h[i];
      d.dircos = reinterpret_cast<const double*>(static_cast<char*>(pool_) + r.dir_offset);
      d.out = reinterpret_cast<float*>(static_cast<char*>(pool_) + r.out_offset);
      d.t_start = r.t_start;
      d.n_point = r.n_point;
      d.n_chan_req = r.n_chan;
      d.chan_lo = r.chan_lo;
      d.chan = t.chan;
      d.ptile = t.ptile;
      d.blk0 = (int32_t)t.blk0;
      d.n_blk = t.n_blk;
      d.pad = 0;
    }
    FFTBF_TRACE("bf_server batch launch");
    hipError_t e = hipMemcpyAsync(dev_[slot], h, sizeof(fftbf::ServeTile) * n, hipMemcpyHostToDevice, stream_);
    if (e == hipSuccess)
      e = fftbf::launch_serve(dev_[slot], n, static_cast<const uint32_t*>(ring_), ring_samples_, n_chan_, n_pol_, dl_,
                              stream_);
    if (e == hipSuccess) e = hipEventRecord(ev_[slot], stream_);
    if (e != hipSuccess) {
      err_ = e;
      return -1;
    }
    return count_++;
  }

  bool finished(int64_t handle) override {
    const hipError_t e = hipEventQuery(ev_[handle % kSlots]);
    if (e == hipSuccess) return true;
    if (e != hipErrorNotReady) err_ = e;
    return false;
  }

  double now() override {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_).count();
  }

  hipStream_t stream_ = nullptr;
  hipEvent_t ev_in_ = nullptr, ev_out_ = nullptr;   // ordering against a caller's stream
  void* ring_ = nullptr;
  void* pool_ = nullptr;
  double* dl_ = nullptr;
  hipError_t err_ = hipSuccess;

 private:
  int n_chan_ = 0, n_pol_ = 0, max_tiles_ = 0;
  int64_t ring_samples_ = 0, count_ = 0;
  size_t frame_bytes_ = 0;
  fftbf::ServeTile* host_[kSlots] = {};
  fftbf::ServeTile* dev_[kSlots] = {};
  hipEvent_t ev_[kSlots] = {};
  std::chrono::steady_clock::time_point t0_;
};

}  // namespace

struct bf_server {
  HipBackend be;
  fftbf::serve::Scheduler* sched = nullptr;
  int64_t ring_samples = 0;
  ~bf_server() { delete sched; }
};

// the plan's descriptor and device d/lambda table (defined with the plan)
extern "C" __attribute__((visibility("hidden"))) const double* bf_internal_plan_dl(const bf_plan* plan,
                                                                                 bf_plan_desc* desc);

extern "C" {

bf_status bf_server_create(const bf_plan* plan, int64_t ring_samples, int64_t hbm_budget, int32_t blocks_per_tile,
                           int32_t max_tiles_per_launch, bf_server** srv) {
  FFTBF_TRACE("bf_server_create");
  if (!srv) return sfail(BF_ERR_INVALID_ARGUMENT, "server_create: NULL srv");
  *srv = nullptr;
  if (!plan) return sfail(BF_ERR_INVALID_ARGUMENT, "server_create: NULL plan");
  bf_plan_desc d;
  const double* dl = bf_internal_plan_dl(plan, &d);
  if (d.n_ew != 4 || d.m_ew != 4 || d.n_ns != 16 || d.m_ns != 32 || d.block != 16 || d.precision != BF_PREC_FP32 ||
      d.pol_sum)
    return sfail(BF_ERR_UNSUPPORTED, "server_create: needs an FP32 4 x 16 lattice plan, block 16, per-pol output");
  if (ring_samples < 16 || ring_samples % 16)
    return sfail(BF_ERR_INVALID_ARGUMENT, "server_create: ring_samples must be a positive multiple of 16");
  if (hbm_budget < 4096) return sfail(BF_ERR_INVALID_ARGUMENT, "server_create: budget too small");
  if (blocks_per_tile < 1 || blocks_per_tile > 4096)
    return sfail(BF_ERR_INVALID_ARGUMENT, "server_create: blocks_per_tile out of range");
  if (max_tiles_per_launch < 1 || max_tiles_per_launch > (1 << 20))
    return sfail(BF_ERR_INVALID_ARGUMENT, "server_create: max_tiles_per_launch out of range");
  bf_server* s = new (std::nothrow) bf_server();
  if (!s) return sfail(BF_ERR_OUT_OF_MEMORY, "server_create: host allocation");
  hipError_t e = s->be.init(d, dl, ring_samples, (size_t)hbm_budget, max_tiles_per_launch);
  if (e != hipSuccess) {
    delete s;
    return sfail(e == hipErrorOutOfMemory ? BF_ERR_OUT_OF_MEMORY : BF_ERR_DEVICE,
                 std::string("server_create: ") + hipGetErrorString(e));
  }
  fftbf::serve::Config c;
  c.ring_samples = ring_samples;
  c.pool_bytes = (size_t)hbm_budget;
  c.n_chan = d.n_chan;
  c.n_pol = d.n_pol;
  c.block = d.block;
  c.blocks_per_tile = blocks_per_tile;
  c.max_tiles_per_launch = max_tiles_per_launch;
  s->ring_samples = ring_samples;
  s->sched = new (std::nothrow) fftbf::serve::Scheduler(c, &s->be);
  if (!s->sched) {
    delete s;
    return sfail(BF_ERR_OUT_OF_MEMORY, "server_create: host allocation");
  }
  *srv = s;
  return BF_OK;
}

bf_status bf_server_destroy(bf_server* srv) {
  FFTBF_TRACE("bf_server_destroy");
  delete srv;   // the backend drains its stream before freeing device memory
  return BF_OK;
}

bf_status bf_server_ring(bf_server* srv, void** ring, int64_t* ring_samples, int64_t* head) {
  if (!srv || !ring || !ring_samples || !head) return sfail(BF_ERR_INVALID_ARGUMENT, "server_ring: NULL argument");
  *ring = srv->be.ring_;
  *ring_samples = srv->ring_samples;
  *head = srv->sched->head();
  return BF_OK;
}

bf_status bf_server_advance(bf_server* srv, int64_t n_samples, const uint8_t* src, int32_t force, void* stream) {
  FFTBF_TRACE("bf_server_advance");
  if (!srv || n_samples < 0) return sfail(BF_ERR_INVALID_ARGUMENT, "server_advance: bad argument");
  if (src && n_samples > srv->ring_samples)
    return sfail(BF_ERR_INVALID_ARGUMENT, "server_advance: more samples than the ring holds");
  const int64_t head = srv->sched->head();
  const int r = srv->sched->advance(n_samples, force != 0);
  if (r != fftbf::serve::kOk) return sfail(map_status(r), srv->sched->last_error);
  if (src && n_samples) {
    // copy into slots head mod ring .. (wrapping), on the server stream so the
    // data lands before any later batch reads it; the copy waits for the
    // caller's stream (where src was produced) and the caller's stream waits
    // for the copy (so src may be reused after the call on that stream)
    const hipStream_t cs = static_cast<hipStream_t>(stream);
    hipError_t e0 = hipEventRecord(srv->be.ev_in_, cs);
    if (e0 == hipSuccess) e0 = hipStreamWaitEvent(srv->be.stream_, srv->be.ev_in_, 0);
    if (e0 != hipSuccess) return sfail(BF_ERR_DEVICE, std::string("server_advance: ") + hipGetErrorString(e0));
    const size_t sb = srv->be.sample_bytes();
    int64_t done = 0;
    while (done < n_samples) {
      const int64_t slot = (head + done) % srv->ring_samples;
      const int64_t n = std::min<int64_t>(n_samples - done, srv->ring_samples - slot);
      hipError_t e = hipMemcpyAsync(static_cast<char*>(srv->be.ring_) + slot * sb, src + done * sb, n * sb,
                                    hipMemcpyDeviceToDevice, srv->be.stream_);
      if (e != hipSuccess) return sfail(BF_ERR_DEVICE, std::string("server_advance: ") + hipGetErrorString(e));
      done += n;
    }
    e0 = hipEventRecord(srv->be.ev_out_, srv->be.stream_);
    if (e0 == hipSuccess) e0 = hipStreamWaitEvent(cs, srv->be.ev_out_, 0);
    if (e0 != hipSuccess) return sfail(BF_ERR_DEVICE, std::string("server_advance: ") + hipGetErrorString(e0));
  }
  return BF_OK;
}

bf_status bf_server_submit(bf_server* srv, int32_t n_point, int32_t chan_lo, int32_t n_chan, int64_t n_time,
                           const double* dircos, double arrival_s, int64_t* id) {
  FFTBF_TRACE("bf_server_submit");
  if (!srv || !id) return sfail(BF_ERR_INVALID_ARGUMENT, "server_submit: NULL argument");
  const int r = srv->sched->submit(n_point, chan_lo, n_chan, n_time, dircos, arrival_s, id);
  if (r != fftbf::serve::kOk) return sfail(map_status(r), srv->sched->last_error);
  return BF_OK;
}

bf_status bf_server_pump(bf_server* srv) {
  FFTBF_TRACE("bf_server_pump");
  if (!srv) return sfail(BF_ERR_INVALID_ARGUMENT, "server_pump: NULL srv");
  const int r = srv->sched->pump();
  if (srv->be.err_ != hipSuccess)
    return sfail(BF_ERR_DEVICE, std::string("server_pump: ") + hipGetErrorString(srv->be.err_));
  if (r != fftbf::serve::kOk) return sfail(map_status(r), srv->sched->last_error);
  return BF_OK;
}

bf_status bf_server_poll(bf_server* srv, int64_t id, double* latency_s) {
  if (!srv) return sfail(BF_ERR_INVALID_ARGUMENT, "server_poll: NULL srv");
  const int r = srv->sched->poll(id, latency_s);
  if (r == fftbf::serve::kNotReady) return BF_ERR_NOT_READY;
  if (r != fftbf::serve::kOk) return sfail(map_status(r), "server_poll: request failed, was cancelled or is unknown");
  return BF_OK;
}

bf_status bf_server_result(bf_server* srv, int64_t id, float** out, int64_t* n_floats) {
  if (!srv || !out || !n_floats) return sfail(BF_ERR_INVALID_ARGUMENT, "server_result: NULL argument");
  const Request* r = srv->sched->get(id);
  if (!r) return sfail(BF_ERR_INVALID_ARGUMENT, "server_result: unknown request");
  if (r->state != fftbf::serve::ReqState::kDone) return sfail(BF_ERR_NOT_READY, "server_result: not finished");
  *out = reinterpret_cast<float*>(static_cast<char*>(srv->be.pool_) + r->out_offset);
  *n_floats = (int64_t)(r->out_bytes / sizeof(float));
  return BF_OK;
}

bf_status bf_server_release(bf_server* srv, int64_t id) {
  if (!srv) return sfail(BF_ERR_INVALID_ARGUMENT, "server_release: NULL srv");
  const int r = srv->sched->release(id);
  if (r != fftbf::serve::kOk) return sfail(map_status(r), "server_release: request unknown or still running");
  return BF_OK;
}

bf_status bf_server_cancel(bf_server* srv, int64_t id) {
  FFTBF_TRACE("bf_server_cancel");
  if (!srv) return sfail(BF_ERR_INVALID_ARGUMENT, "server_cancel: NULL srv");
  const int r = srv->sched->cancel(id);
  if (r != fftbf::serve::kOk) return sfail(map_status(r), "server_cancel: unknown request");
  return BF_OK;
}

bf_status bf_server_stats_get(bf_server* srv, bf_server_stats* st) {
  if (!srv || !st) return sfail(BF_ERR_INVALID_ARGUMENT, "server_stats_get: NULL argument");
  const fftbf::serve::Stats s = srv->sched->stats();
  st->submitted = s.submitted;
  st->completed = s.completed;
  st->rejected = s.rejected;
  st->evicted = s.evicted;
  st->in_flight = s.in_flight;
  st->budget_used = s.budget_used;
  st->tiles_done = s.tiles_done;
  st->launches = s.launches;
  return BF_OK;
}

double bf_server_now(bf_server* srv) { return srv ? srv->be.now() : 0.0; }

bf_status bf_server_copy_result(bf_server* srv, int64_t id, float* dst, void* stream) {
  FFTBF_TRACE("bf_server_copy_result");
  float* src = nullptr;
  int64_t n = 0;
  const bf_status st = bf_server_result(srv, id, &src, &n);
  if (st != BF_OK) return st;
  if (!dst) return sfail(BF_ERR_INVALID_ARGUMENT, "server_copy_result: NULL dst");
  // the result was written on the server stream; order the copy after it
  hipError_t e = hipStreamSynchronize(srv->be.stream_);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dst, src, sizeof(float) * n, hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return sfail(BF_ERR_DEVICE, std::string("server_copy_result: ") + hipGetErrorString(e));
  return BF_OK;
}

}  // extern "C"
