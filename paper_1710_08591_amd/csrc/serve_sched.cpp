// Host-side scheduler of the tied-beam server (see serve_sched.h).
#include "serve_sched.h"

#include <algorithm>
#include <limits>

namespace fftbf {
namespace serve {

// ---------------------------------------------------------------- pool ----

bool PoolAllocator::alloc(size_t bytes, size_t* off) {
  if (bytes == 0) bytes = 1;
  const size_t need = (bytes + align_ - 1) / align_ * align_;
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second >= need) {
      const size_t o = it->first, rest = it->second - need;
      free_.erase(it);
      if (rest) free_[o + need] = rest;
      live_[o] = need;
      used_ += need;
      *off = o;
      return true;
    }
  }
  return false;
}

void PoolAllocator::release(size_t off) {
  auto it = live_.find(off);
  if (it == live_.end()) return;
  size_t o = it->first, sz = it->second;
  used_ -= sz;
  live_.erase(it);
  auto nx = free_.lower_bound(o);
  if (nx != free_.end() && o + sz == nx->first) {   // merge with the following hole
    sz += nx->second;
    nx = free_.erase(nx);
  }
  if (nx != free_.begin()) {                          // merge with the preceding hole
    auto pv = std::prev(nx);
    if (pv->first + pv->second == o) {
      pv->second += sz;
      return;
    }
  }
  free_[o] = sz;
}

size_t PoolAllocator::largest_free() const {
  size_t m = 0;
  for (auto& kv : free_) m = std::max(m, kv.second);
  return m;
}

bool PoolAllocator::check_invariants() const {
  // holes and live blocks tile [0, total) without overlap, holes never adjacent
  std::map<size_t, std::pair<size_t, bool>> all;
  for (auto& kv : free_) all[kv.first] = {kv.second, true};
  for (auto& kv : live_) {
    if (all.count(kv.first)) return false;
    all[kv.first] = {kv.second, false};
  }
  size_t pos = 0, u = 0;
  bool prev_free = false;
  for (auto& kv : all) {
    if (kv.first != pos) return false;
    if (kv.second.second && prev_free) return false;
    prev_free = kv.second.second;
    if (!kv.second.second) u += kv.second.first;
    pos += kv.second.first;
  }
  return pos == total_ && u == used_;
}

// ----------------------------------------------------------- scheduler ----

size_t Scheduler::out_bytes(const Config& c, int n_point, int n_chan, int64_t n_time) {
  return (size_t)(n_time / c.block) * (size_t)n_chan * (size_t)c.n_pol * (size_t)n_point * sizeof(float);
}

int Scheduler::submit(int n_point, int chan_lo, int n_chan, int64_t n_time, const double* dircos,
                      double arrival, int64_t* id) {
  if (id) *id = 0;
  if (!dircos || !id || n_point < 1 || n_point > 4096 || n_chan < 1 || chan_lo < 0 ||
      chan_lo + (int64_t)n_chan > cfg_.n_chan || n_time <= 0 || n_time % cfg_.block) {
    last_error = "submit: invalid request shape";
    return kInvalid;
  }
  if (n_time > cfg_.ring_samples || head_ < n_time) {
    last_error = "submit: window is not in the ring";
    return kEvicted;
  }
  Request r;
  r.id = next_id_;
  r.n_point = n_point;
  r.chan_lo = chan_lo;
  r.n_chan = n_chan;
  r.n_time = n_time;
  r.t_start = head_ - n_time;
  r.arrival = arrival;
  r.admitted = be_->now();
  r.out_bytes = out_bytes(cfg_, n_point, n_chan, n_time);
  if (!pool_.alloc(r.out_bytes, &r.out_offset)) {
    ++st_.rejected;
    last_error = "submit: output does not fit the memory budget";
    return kRejected;
  }
  if (!pool_.alloc((size_t)n_point * 2 * sizeof(double), &r.dir_offset)) {
    pool_.release(r.out_offset);
    ++st_.rejected;
    last_error = "submit: pointing table does not fit the memory budget";
    return kRejected;
  }
  if (!be_->upload_pointings(r.dir_offset, dircos, n_point)) {
    pool_.release(r.out_offset);
    pool_.release(r.dir_offset);
    last_error = "submit: pointing upload failed";
    return kInvalid;
  }
  const int64_t nblk = n_time / cfg_.block;
  const int64_t runs = (nblk + cfg_.blocks_per_tile - 1) / cfg_.blocks_per_tile;
  r.n_tiles = (int64_t)((n_point + 63) / 64) * n_chan * runs;
  ++next_id_;
  ++st_.submitted;
  reqs_[r.id] = r;
  active_.push_back(r.id);
  *id = r.id;
  return kOk;
}

int Scheduler::advance(int64_t n, bool force) {
  if (n < 0) return kInvalid;
  const int64_t new_head = head_ + n;
  const int64_t lost = new_head - cfg_.ring_samples;   // samples before this are overwritten
  bool blocked = false;
  for (auto& kv : reqs_) {
    Request& r = kv.second;
    const bool live = r.state == ReqState::kQueued || r.state == ReqState::kRunning;
    if (live && r.t_start < lost) blocked = true;
  }
  if (blocked && !force) {
    last_error = "advance: a leased window would be overwritten";
    return kNotReady;
  }
  if (blocked) {
    for (auto& kv : reqs_) {
      Request& r = kv.second;
      const bool live = r.state == ReqState::kQueued || r.state == ReqState::kRunning;
      if (live && r.t_start < lost) {
        r.state = ReqState::kEvicted;
        ++st_.evicted;
        finish_if_done(r);
      }
    }
  }
  head_ = new_head;
  return kOk;
}

bool Scheduler::next_tile(Request& r, Tile* t) {
  if (r.state != ReqState::kQueued && r.state != ReqState::kRunning) return false;
  if (r.issued >= r.n_tiles) return false;
  const int64_t nblk = r.n_time / cfg_.block;
  t->req = r.id;
  t->chan = r.chan_lo + r.cur_chan;
  t->ptile = r.cur_ptile;
  t->blk0 = r.cur_blk;
  t->n_blk = (int32_t)std::min<int64_t>(cfg_.blocks_per_tile, nblk - r.cur_blk);
  // advance the cursor: blocks fastest, then channels, then pointing tiles
  r.cur_blk += cfg_.blocks_per_tile;
  if (r.cur_blk >= nblk) {
    r.cur_blk = 0;
    if (++r.cur_chan >= r.n_chan) {
      r.cur_chan = 0;
      ++r.cur_ptile;
    }
  }
  ++r.issued;
  r.state = ReqState::kRunning;
  return true;
}

void Scheduler::finish_if_done(Request& r) {
  if (r.completed >= 0) return;
  if (r.finished != r.issued) return;
  const bool all = r.issued >= r.n_tiles;
  if (r.state == ReqState::kRunning && all) {
    r.state = ReqState::kDone;
    r.completed = be_->now();
    ++st_.completed;
  } else if (r.state == ReqState::kCancelled || r.state == ReqState::kEvicted) {
    r.completed = be_->now();
  }
}

int Scheduler::pump() {
  // retire finished launches (in issue order)
  while (!flights_.empty() && be_->finished(flights_.front().handle)) {
    for (const Tile& t : flights_.front().tiles) {
      auto it = reqs_.find(t.req);
      if (it == reqs_.end()) continue;
      ++it->second.finished;
      ++st_.tiles_done;
      finish_if_done(it->second);
    }
    flights_.pop_front();
  }
  // issue new launches: round-robin quanta over the active requests
  while ((int)flights_.size() < cfg_.max_in_flight && !active_.empty()) {
    std::vector<Tile> batch;
    std::vector<const Request*> rq;
    bool progress = true;
    while (progress && !active_.empty() && (int)batch.size() < cfg_.max_tiles_per_launch) {
      progress = false;
      const size_t n = active_.size();
      for (size_t i = 0; i < n && (int)batch.size() < cfg_.max_tiles_per_launch; ++i) {
        const int64_t id = active_.front();
        active_.pop_front();
        auto it = reqs_.find(id);
        if (it == reqs_.end()) continue;
        Request& r = it->second;
        int took = 0;
        Tile t;
        while (took < cfg_.tiles_per_turn && (int)batch.size() < cfg_.max_tiles_per_launch && next_tile(r, &t)) {
          batch.push_back(t);
          rq.push_back(&r);
          ++took;
        }
        if (took) progress = true;
        if ((r.state == ReqState::kQueued || r.state == ReqState::kRunning) && r.issued < r.n_tiles)
          active_.push_back(id);
      }
    }
    if (batch.empty()) break;
    const int64_t h = be_->launch(batch, rq);
    if (h < 0) {
      last_error = "pump: launch failed";
      return kInvalid;
    }
    ++st_.launches;
    flights_.push_back(Flight{h, std::move(batch)});
  }
  return kOk;
}

int Scheduler::poll(int64_t id, double* latency) const {
  auto it = reqs_.find(id);
  if (it == reqs_.end()) return kInvalid;
  const Request& r = it->second;
  if (r.state == ReqState::kEvicted) return kEvicted;
  if (r.state == ReqState::kCancelled) return kInvalid;
  if (r.state != ReqState::kDone) return kNotReady;
  if (latency) *latency = r.completed - r.arrival;
  return kOk;
}

int Scheduler::cancel(int64_t id) {
  auto it = reqs_.find(id);
  if (it == reqs_.end()) return kInvalid;
  Request& r = it->second;
  if (r.state == ReqState::kQueued || r.state == ReqState::kRunning) {
    r.state = ReqState::kCancelled;
    finish_if_done(r);
  }
  return kOk;
}

int Scheduler::release(int64_t id) {
  auto it = reqs_.find(id);
  if (it == reqs_.end()) return kInvalid;
  Request& r = it->second;
  if (r.finished != r.issued) return kNotReady;   // tiles still on the device
  if (r.state == ReqState::kQueued || r.state == ReqState::kRunning) return kNotReady;
  pool_.release(r.out_offset);
  pool_.release(r.dir_offset);
  reqs_.erase(it);
  return kOk;
}

const Request* Scheduler::get(int64_t id) const {
  auto it = reqs_.find(id);
  return it == reqs_.end() ? nullptr : &it->second;
}

Stats Scheduler::stats() const {
  Stats s = st_;
  s.in_flight = 0;
  for (auto& kv : reqs_)
    if (kv.second.state == ReqState::kQueued || kv.second.state == ReqState::kRunning) ++s.in_flight;
  s.budget_used = (int64_t)pool_.used();
  return s;
}

}  // namespace serve
}  // namespace fftbf
