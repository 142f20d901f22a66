// Host-side tests of the tied-beam server's scheduler against a simulated
// device (no GPU): admission by budget, tiling, batching limits, fairness,
// completion and latency accounting, cancellation, ring leases and eviction,
// and the pool allocator.  Built with g++ (with sanitizers) by
// tests/test_serving_host.py.
#include <cassert>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <set>
#include <tuple>
#include <vector>

#include "serve_sched.h"

using namespace fftbf::serve;

#define CHECK(c)                                                      \
  do {                                                                \
    if (!(c)) {                                                       \
      std::fprintf(stderr, "CHECK failed %s:%d: %s\n", __FILE__, __LINE__, #c); \
      std::exit(1);                                                   \
    }                                                                 \
  } while (0)

// Simulated device: a launch finishes `cost_per_tile * n_tiles` seconds after
// the later of its issue time and the previous launch's end (one stream).
struct FakeBackend : Backend {
  double clock = 0, cost_per_tile = 1e-4, stream_free = 0;
  std::vector<double> ends;
  std::vector<std::vector<Tile>> launched;
  std::map<size_t, int> uploaded;   // pool offset -> n_point
  bool upload_pointings(size_t off, const double* d, int n) override {
    CHECK(d != nullptr);
    uploaded[off] = n;
    return true;
  }
  int64_t launch(const std::vector<Tile>& tiles, const std::vector<const Request*>& reqs) override {
    CHECK(tiles.size() == reqs.size());
    for (size_t i = 0; i < tiles.size(); ++i) CHECK(tiles[i].req == reqs[i]->id);
    const double start = std::max(clock, stream_free);
    stream_free = start + cost_per_tile * tiles.size();
    ends.push_back(stream_free);
    launched.push_back(tiles);
    return (int64_t)ends.size() - 1;
  }
  bool finished(int64_t h) override { return ends[h] <= clock; }
  double now() override { return clock; }
};

static void drain(Scheduler& s, FakeBackend& be, int64_t id, double dt = 1e-4, int max_steps = 10000000) {
  for (int i = 0; i < max_steps; ++i) {
    s.pump();
    double lat;
    if (s.poll(id, &lat) != kNotReady) return;
    be.clock += dt;
  }
  CHECK(false);
}

static void test_pool() {
  PoolAllocator p(1 << 20, 256);
  std::mt19937 rng(1);
  std::vector<size_t> live;
  for (int it = 0; it < 5000; ++it) {
    if (live.empty() || (rng() % 3)) {
      size_t off;
      const size_t sz = 1 + rng() % 20000;
      if (p.alloc(sz, &off)) {
        CHECK(off % 256 == 0);
        live.push_back(off);
      }
    } else {
      const size_t k = rng() % live.size();
      p.release(live[k]);
      live.erase(live.begin() + k);
    }
    CHECK(p.check_invariants());
  }
  for (size_t o : live) p.release(o);
  CHECK(p.used() == 0 && p.largest_free() == (1u << 20) && p.check_invariants());
  size_t a, b;
  CHECK(p.alloc(1 << 20, &a) && !p.alloc(1, &b));
  p.release(a);
  CHECK(p.alloc(1 << 19, &a) && p.alloc(1 << 19, &b) && !p.alloc(256, &a));
}

static Config small_cfg() {
  Config c;
  c.ring_samples = 4096;
  c.pool_bytes = 64 << 20;
  c.n_chan = 32;
  c.n_pol = 1;
  c.blocks_per_tile = 4;
  c.max_tiles_per_launch = 64;
  c.tiles_per_turn = 8;
  c.max_in_flight = 2;
  return c;
}

static void test_validation_and_budget() {
  FakeBackend be;
  Config c = small_cfg();
  c.pool_bytes = 1 << 20;
  Scheduler s(c, &be);
  std::vector<double> d(2 * 300, 0.1);
  int64_t id;
  CHECK(s.submit(4, 0, 4, 1024, d.data(), 0, &id) == kEvicted);     // nothing written yet
  CHECK(s.advance(4096, false) == kOk);
  CHECK(s.submit(0, 0, 4, 1024, d.data(), 0, &id) == kInvalid);
  CHECK(s.submit(4, 30, 4, 1024, d.data(), 0, &id) == kInvalid);    // channels past the end
  CHECK(s.submit(4, 0, 4, 1000, d.data(), 0, &id) == kInvalid);     // not a multiple of 16
  CHECK(s.submit(4, 0, 4, 8192, d.data(), 0, &id) == kEvicted);     // longer than the ring
  CHECK(s.submit(4, 0, 4, 1024, nullptr, 0, &id) == kInvalid);
  // 300 pointings x 32 channels x 256 blocks x 4 B = 9.8 MB > 1 MiB budget
  CHECK(s.submit(300, 0, 32, 4096, d.data(), 0, &id) == kRejected);
  CHECK(s.stats().rejected == 1 && s.stats().budget_used == 0);
  CHECK(s.submit(4, 0, 4, 1024, d.data(), 0, &id) == kOk);
  CHECK(s.stats().budget_used >= (int64_t)Scheduler::out_bytes(c, 4, 4, 1024));
  CHECK(be.uploaded.size() == 1);
}

static void test_tiling_covers_once() {
  FakeBackend be;
  Config c = small_cfg();
  Scheduler s(c, &be);
  s.advance(4096, false);
  std::vector<double> d(2 * 130, 0.0);
  int64_t id;
  CHECK(s.submit(130, 5, 3, 16 * 37, d.data(), 0, &id) == kOk);       // 3 pointing tiles, ragged blocks
  drain(s, be, id);
  std::set<std::tuple<int, int, int64_t>> seen;
  int64_t n = 0;
  for (auto& L : be.launched) {
    CHECK((int)L.size() <= c.max_tiles_per_launch);
    for (auto& t : L) {
      CHECK(t.chan >= 5 && t.chan < 8 && t.ptile >= 0 && t.ptile < 3);
      CHECK(t.n_blk >= 1 && t.n_blk <= c.blocks_per_tile && t.blk0 + t.n_blk <= 37);
      for (int b = 0; b < t.n_blk; ++b) CHECK(seen.insert({t.chan, t.ptile, t.blk0 + b}).second);
      ++n;
    }
  }
  CHECK((int64_t)seen.size() == 3 * 3 * 37);
  CHECK(n == 3 * 3 * ((37 + 3) / 4));
  double lat;
  CHECK(s.poll(id, &lat) == kOk && lat > 0);
}

static void test_fairness_and_inflight_limit() {
  FakeBackend be;
  Config c = small_cfg();
  Scheduler s(c, &be);
  s.advance(4096, false);
  std::vector<double> d(2 * 64, 0.0);
  int64_t big, small;
  CHECK(s.submit(64, 0, 32, 4096, d.data(), 0.0, &big) == kOk);      // 32 x 64 = 2048 tiles
  s.pump();
  CHECK(be.launched.size() == 2);                                      // two launches in flight
  s.pump();
  CHECK(be.launched.size() == 2);                                      // no more until one retires
  be.clock += 1e-6;
  CHECK(s.submit(64, 0, 1, 256, d.data(), be.clock, &small) == kOk);  // 4 tiles, arrives later
  drain(s, be, small);
  double lb, ls;
  CHECK(s.poll(small, &ls) == kOk);
  CHECK(s.poll(big, &lb) == kNotReady);                                // small overtook big
  CHECK(ls < 3 * 64 * be.cost_per_tile + 1e-3);                        // within ~2 launches
  drain(s, be, big);
  CHECK(s.poll(big, &lb) == kOk && lb > ls);
  CHECK(s.stats().completed == 2 && s.stats().tiles_done == 2048 + 4);
  CHECK(s.release(big) == kOk && s.release(small) == kOk && s.stats().budget_used == 0);
}

static void test_cancel_and_release() {
  FakeBackend be;
  Config c = small_cfg();
  Scheduler s(c, &be);
  s.advance(4096, false);
  std::vector<double> d(2 * 64, 0.0);
  int64_t id;
  CHECK(s.submit(64, 0, 32, 4096, d.data(), 0, &id) == kOk);
  s.pump();
  CHECK(s.release(id) == kNotReady);
  CHECK(s.cancel(id) == kOk);
  CHECK(s.release(id) == kNotReady);                  // launched tiles still on the device
  for (int i = 0; i < 100000 && s.release(id) == kNotReady; ++i) {
    be.clock += 1e-4;
    s.pump();
  }
  CHECK(s.get(id) == nullptr && s.stats().budget_used == 0);
  int64_t issued = 0;
  for (auto& L : be.launched) issued += L.size();
  CHECK(issued == 2 * 64);                            // nothing issued after the cancel
  double lat;
  CHECK(s.poll(id, &lat) == kInvalid);
}

static void test_ring_lease_and_eviction() {
  FakeBackend be;
  Config c = small_cfg();
  Scheduler s(c, &be);
  CHECK(s.advance(4096, false) == kOk);
  std::vector<double> d(2, 0.0);
  int64_t a;
  CHECK(s.submit(1, 0, 1, 2048, d.data(), 0, &a) == kOk);    // window [2048, 4096)
  CHECK(s.advance(2048, false) == kOk);                       // overwrites [0, 2048): free
  CHECK(s.advance(16, false) == kNotReady);                   // would overwrite sample 2048
  CHECK(s.head() == 6144);
  CHECK(s.advance(16, true) == kOk);                          // forced: the request is evicted
  double lat;
  CHECK(s.poll(a, &lat) == kEvicted && s.stats().evicted == 1);
  for (int i = 0; i < 1000 && s.release(a) != kOk; ++i) {
    be.clock += 1e-3;
    s.pump();
  }
  CHECK(s.stats().budget_used == 0);
  int64_t b;
  CHECK(s.submit(1, 0, 1, 4096, d.data(), 0, &b) == kOk);
  drain(s, be, b);
  CHECK(s.poll(b, &lat) == kOk);
  CHECK(s.advance(4096, false) == kOk);                       // finished windows hold no lease
}

static void test_random_stream() {
  FakeBackend be;
  Config c = small_cfg();
  c.pool_bytes = 8 << 20;
  Scheduler s(c, &be);
  s.advance(4096, false);
  std::mt19937 rng(7);
  std::vector<double> d(2 * 256, 0.3);
  std::vector<int64_t> ids;
  int rejected = 0;
  for (int i = 0; i < 400; ++i) {
    const int p = 1 + rng() % 256, nc = 1 + rng() % 32, lo = rng() % (33 - nc);
    const int64_t t = 16 * (1 + rng() % 256);
    int64_t id;
    const int r = s.submit(p, lo, nc, t, d.data(), be.clock, &id);
    if (r == kOk) ids.push_back(id);
    else {
      CHECK(r == kRejected);
      ++rejected;
    }
    for (int k = 0; k < 5; ++k) {
      s.pump();
      be.clock += 2e-4;
    }
    for (size_t j = 0; j < ids.size();) {
      double lat;
      if (s.poll(ids[j], &lat) == kOk) {
        CHECK(lat >= 0);
        CHECK(s.release(ids[j]) == kOk);
        ids.erase(ids.begin() + j);
      } else {
        ++j;
      }
    }
    CHECK(s.pool().check_invariants());
    CHECK(s.stats().budget_used <= (int64_t)c.pool_bytes);
  }
  for (int64_t id : ids) {
    drain(s, be, id);
    CHECK(s.release(id) == kOk);
  }
  CHECK(s.stats().budget_used == 0 && s.stats().in_flight == 0);
  CHECK(s.stats().completed + rejected == 400);
}

int main() {
  test_pool();
  test_validation_and_budget();
  test_tiling_covers_once();
  test_fairness_and_inflight_limit();
  test_cancel_and_release();
  test_ring_lease_and_eviction();
  test_random_stream();
  std::printf("ALL OK\n");
  return 0;
}
