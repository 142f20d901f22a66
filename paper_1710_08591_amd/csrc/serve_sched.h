// Host-side scheduler of the tied-beam server: admission by memory budget,
// ring-window leases, tiling, fair batching into bounded launches, latency
// accounting.  Pure C++17 (no HIP): the device work goes through Backend,
// so the same scheduler runs against the GPU or against a simulated device.
#pragma once

#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <string>
#include <vector>

namespace fftbf {
namespace serve {

enum class ReqState { kQueued, kRunning, kDone, kCancelled, kEvicted };

// One unit of device work: one channel, one tile of up to 64 pointings, a
// run of consecutive blocks of one request.
struct Tile {
  int64_t req = 0;
  int32_t chan = 0;      // absolute channel
  int32_t ptile = 0;     // pointings [64 ptile, 64 ptile + 64)
  int64_t blk0 = 0;      // first block, counted within the request window
  int32_t n_blk = 0;
};

struct Request {
  int64_t id = 0;
  int32_t n_point = 0, chan_lo = 0, n_chan = 0;
  int64_t n_time = 0;
  int64_t t_start = 0;          // absolute sample index of the window start
  double arrival = 0, admitted = 0, completed = -1;
  size_t out_bytes = 0;
  size_t out_offset = 0;        // offset of the output in the memory pool
  size_t dir_offset = 0;        // offset of the pointing table in the pool
  ReqState state = ReqState::kQueued;
  // tiling cursor
  int64_t n_tiles = 0, issued = 0, finished = 0;
  int32_t cur_ptile = 0, cur_chan = 0;
  int64_t cur_blk = 0;
};

// First-fit allocator over an offset range (the device pool), coalescing on free.
class PoolAllocator {
 public:
  explicit PoolAllocator(size_t bytes = 0, size_t align = 256) : total_(bytes), align_(align) {
    if (bytes) free_[0] = bytes;
  }
  bool alloc(size_t bytes, size_t* off);
  void release(size_t off);
  size_t used() const { return used_; }
  size_t total() const { return total_; }
  size_t largest_free() const;
  bool check_invariants() const;

 private:
  size_t total_, align_, used_ = 0;
  std::map<size_t, size_t> free_;   // offset -> size
  std::map<size_t, size_t> live_;   // offset -> size
};

class Backend {
 public:
  virtual ~Backend() = default;
  // copy a request's pointing table (host [n_point][2] doubles) to pool offset
  virtual bool upload_pointings(size_t off, const double* dircos, int n_point) = 0;
  // start device work on a batch; returns a handle
  virtual int64_t launch(const std::vector<Tile>& tiles, const std::vector<const Request*>& reqs) = 0;
  virtual bool finished(int64_t handle) = 0;
  virtual double now() = 0;   // seconds, monotonic
};

struct Config {
  int64_t ring_samples = 65536;
  size_t pool_bytes = size_t(16) << 30;   // memory budget for outputs + pointing tables
  int32_t n_chan = 256, n_pol = 1, block = 16;
  int32_t blocks_per_tile = 32;
  int32_t max_tiles_per_launch = 8192;
  int32_t tiles_per_turn = 256;          // round-robin quantum per request per batch
  int32_t max_in_flight = 2;
};

struct Stats {
  int64_t submitted = 0, completed = 0, rejected = 0, evicted = 0, in_flight = 0;
  int64_t budget_used = 0, tiles_done = 0, launches = 0;
};

enum Status { kOk = 0, kInvalid = -1, kUnsupported = -2, kRejected = -5, kEvicted = -6, kNotReady = -7 };

class Scheduler {
 public:
  Scheduler(const Config& cfg, Backend* be) : cfg_(cfg), be_(be), pool_(cfg.pool_bytes) {}

  static size_t out_bytes(const Config& c, int n_point, int n_chan, int64_t n_time);

  // admit a request for the last n_time samples before the ring head
  int submit(int n_point, int chan_lo, int n_chan, int64_t n_time, const double* dircos, double arrival,
             int64_t* id);
  // the writer appends n samples; refuses (kNotReady) to overwrite a leased window unless force
  int advance(int64_t n, bool force);
  int pump();                                   // retire finished launches, issue new ones
  int poll(int64_t id, double* latency) const;  // kOk when done (latency = completed - arrival)
  int cancel(int64_t id);
  int release(int64_t id);                      // give the request's memory back
  const Request* get(int64_t id) const;
  int64_t head() const { return head_; }
  Stats stats() const;
  const PoolAllocator& pool() const { return pool_; }
  std::string last_error;

 private:
  bool next_tile(Request& r, Tile* t);
  void finish_if_done(Request& r);

  Config cfg_;
  Backend* be_;
  PoolAllocator pool_;
  int64_t head_ = 0, next_id_ = 1;
  std::map<int64_t, Request> reqs_;
  std::deque<int64_t> active_;           // round-robin order of requests with tiles to issue
  struct Flight { int64_t handle; std::vector<Tile> tiles; };
  std::deque<Flight> flights_;
  Stats st_;
};

}  // namespace serve
}  // namespace fftbf
