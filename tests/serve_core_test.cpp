// Host tests of the serving scheduler core (paper_2301_06763_amd/csrc/
// serve_core.hpp) against a simulated device with a fake clock and fake
// footprints: admission in arrival order under the budget, grouping and
// batch bounds, retirement, requeueing after NMC_ENOMEM and device errors,
// completion of every ticket exactly once, and the ring of serving
// workspace regions (RingArena).  Built and run with
// AddressSanitizer and UndefinedBehaviorSanitizer by test_serve_core_cpu.py.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "../paper_2301_06763_amd/csrc/serve_core.hpp"

#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      std::fprintf(stderr, "FAIL %s:%d: %s\n", __FILE__, __LINE__, #c); \
      std::exit(1);                                                     \
    }                                                                   \
  } while (0)

using nmc::ServeBatch;
using nmc::ServeCore;
using nmc::ServeKey;

// A device whose batches take bytes / rate units of the fake clock; the next
// launches can be made to report NMC_ENOMEM (nothing enqueued) or an error.
struct FakeDevice final : nmc::ServeDevice {
  struct Rec {
    double done_at;
  };
  std::map<uint64_t, size_t> footprint;
  std::map<uint64_t, ServeKey> key;
  double now = 0, rate = 1;
  int enomem_next = 0, fail_next = 0;
  size_t held = 0, peak = 0;
  int live = 0;  // batches launched and not released
  std::vector<std::vector<uint64_t>> launched;
  std::vector<uint64_t> released;

  int poll(const ServeBatch& b) override { return now >= static_cast<const Rec*>(b.dev)->done_at ? 1 : 0; }
  int launch(ServeBatch& b) override {
    CHECK(!b.tickets.empty() && b.dev == nullptr);
    if (fail_next > 0) {
      --fail_next;
      return NMC_EDEVICE;
    }
    if (enomem_next > 0) {
      --enomem_next;
      return NMC_ENOMEM;
    }
    size_t bytes = 0;
    for (uint64_t t : b.tickets) bytes += footprint.at(t);
    b.bytes = bytes;
    b.dev = new Rec{now + (double)bytes / rate};
    held += bytes;
    peak = std::max(peak, held);
    ++live;
    launched.push_back(b.tickets);
    return NMC_OK;
  }
  void release(ServeBatch& b) override {
    held -= b.bytes;
    --live;
    for (uint64_t t : b.tickets) released.push_back(t);
    delete static_cast<Rec*>(b.dev);
    b.dev = nullptr;
  }
};

static uint64_t submit(ServeCore& core, FakeDevice& dev, ServeKey k, size_t bytes) {
  const uint64_t t = core.submit(k, bytes);
  dev.footprint[t] = bytes;
  dev.key[t] = k;
  return t;
}

// Run the fake clock until every batch has retired (a ServeCore leaves the
// device records of batches still in flight to the device side).
static void drain(ServeCore& core, FakeDevice& dev) {
  for (int i = 0; i < 1000 && !core.idle(); ++i) {
    dev.now += 1e6;
    CHECK(core.tick(dev, nullptr) == NMC_OK);
  }
  CHECK(core.idle() && dev.live == 0);
}

// Invariants after every tick.
static void check_state(const ServeCore& core, const FakeDevice& dev) {
  const auto& st = core.stats();
  CHECK(st.inflight_bytes == dev.held);
  if (core.budget()) CHECK(st.inflight_bytes <= core.budget());
  CHECK((int)core.inflight().size() == dev.live);
  CHECK(st.queued == core.queue().size());
  size_t n_inflight = 0;
  for (const auto& b : core.inflight()) n_inflight += b.tickets.size();
  CHECK(st.inflight == n_inflight);
  for (size_t i = 1; i < core.queue().size(); ++i) CHECK(core.queue()[i - 1] < core.queue()[i]);  // arrival order
}

static void test_fifo_admission_under_budget() {
  ServeCore core(100, 32);
  FakeDevice dev;
  const ServeKey k{32, 0, 0};
  const uint64_t a = submit(core, dev, k, 40), b = submit(core, dev, k, 40), c = submit(core, dev, k, 40),
                 d = submit(core, dev, k, 10);
  int n = -1;
  CHECK(core.tick(dev, &n) == NMC_OK);
  // a and b fit (80); c does not, and d, which would fit, waits behind it
  CHECK(n == 2);
  CHECK(core.queue().size() == 2 && core.queue()[0] == c && core.queue()[1] == d);
  // 40 > budget / 4: one request per batch
  CHECK(dev.launched.size() == 2 && dev.launched[0] == std::vector<uint64_t>{a} &&
        dev.launched[1] == std::vector<uint64_t>{b});
  check_state(core, dev);
  // nothing finished yet: no admission
  CHECK(core.tick(dev, &n) == NMC_OK && n == 0);
  dev.now = 40;  // both finish
  CHECK(core.tick(dev, &n) == NMC_OK && n == 2);
  CHECK(core.stats().completed == 2 && core.queue().empty());
  check_state(core, dev);
  dev.now = 1e9;
  CHECK(core.tick(dev, &n) == NMC_OK);
  CHECK(core.idle() && core.stats().completed == 4);
  uint64_t out[8];
  CHECK(core.take_completed(out, 8) == 4);
  CHECK(out[0] == a && out[1] == b && out[2] == c && out[3] == d);
  CHECK(core.find(a) == nullptr);
  std::printf("fifo admission under the budget: ok\n");
}

static void test_grouping_and_batch_bounds() {
  ServeCore core(0, 3);  // no budget, at most 3 requests per batch
  FakeDevice dev;
  const ServeKey k32{32, 1, 0}, k64{64, 1, 0}, k32m{32, 1, 1}, k32d{32, 0, 0};
  std::vector<uint64_t> ts;
  const ServeKey order[] = {k32, k64, k32, k32m, k32, k32, k64, k32d, k32};
  for (const auto& k : order) ts.push_back(submit(core, dev, k, 5));
  int n = 0;
  CHECK(core.tick(dev, &n) == NMC_OK && n == 9);
  size_t total = 0;
  for (const auto& b : dev.launched) {
    CHECK(!b.empty() && b.size() <= 3);
    for (size_t i = 0; i < b.size(); ++i) {
      CHECK(dev.key.at(b[i]) == dev.key.at(b[0]));  // one group per batch
      if (i) CHECK(b[i - 1] < b[i]);                // arrival order inside
    }
    total += b.size();
  }
  CHECK(total == 9);
  // group k32 has 5 requests: batches of 3 and 2
  int k32_batches = 0;
  for (const auto& b : dev.launched)
    if (dev.key.at(b[0]) == k32) ++k32_batches;
  CHECK(k32_batches == 2);
  check_state(core, dev);
  // a byte bound: budget 400 -> batches of at most 100 bytes
  ServeCore core2(400, 32);
  FakeDevice dev2;
  for (int i = 0; i < 8; ++i) submit(core2, dev2, k32, 30);
  CHECK(core2.tick(dev2, &n) == NMC_OK && n == 8);
  for (const auto& b : dev2.launched) CHECK(b.size() * 30 <= 100);
  CHECK(dev2.launched.size() == 3);  // 3 + 3 + 2
  drain(core, dev);
  drain(core2, dev2);
  std::printf("grouping and batch bounds: ok\n");
}

static void test_enomem_and_errors_requeue_in_order() {
  ServeCore core(1000, 32);
  FakeDevice dev;
  const ServeKey ka{32, 0, 0}, kb{64, 0, 0};
  const uint64_t t1 = submit(core, dev, ka, 100), t2 = submit(core, dev, kb, 100), t3 = submit(core, dev, ka, 100);
  // the pool cannot place the first batch and nothing is in flight: ENOMEM,
  // every request back in the queue in arrival order
  dev.enomem_next = 1;
  int n = -1;
  CHECK(core.tick(dev, &n) == NMC_ENOMEM && n == 0);
  CHECK(core.queue().size() == 3 && core.queue()[0] == t1 && core.queue()[1] == t2 && core.queue()[2] == t3);
  check_state(core, dev);
  // the first batch (group ka: t1, t3) launches, the second (t2) reports
  // ENOMEM with work in flight: no error, t2 stays queued
  dev.launched.clear();
  CHECK(core.tick(dev, &n) == NMC_OK && n == 3);  // both launch now
  dev.now = 1e9;
  CHECK(core.tick(dev, &n) == NMC_OK && core.idle());
  const uint64_t u1 = submit(core, dev, ka, 100), u2 = submit(core, dev, kb, 100), u3 = submit(core, dev, kb, 100);
  dev.now = 0;
  dev.enomem_next = 0;
  // first batch launches; make the second report ENOMEM
  struct OneShot final : nmc::ServeDevice {
    FakeDevice& d;
    int calls = 0;
    explicit OneShot(FakeDevice& x) : d(x) {}
    int poll(const ServeBatch& b) override { return d.poll(b); }
    int launch(ServeBatch& b) override { return ++calls == 2 ? NMC_ENOMEM : d.launch(b); }
    void release(ServeBatch& b) override { d.release(b); }
  } once(dev);
  CHECK(core.tick(once, &n) == NMC_OK && n == 1);
  CHECK(core.queue().size() == 2 && core.queue()[0] == u2 && core.queue()[1] == u3);
  (void)u1;
  check_state(core, dev);
  // a device error: reported, the batch and those behind it stay queued
  dev.now = 1e9;
  dev.fail_next = 1;
  CHECK(core.tick(dev, &n) == NMC_EDEVICE && n == 0);
  CHECK(core.queue().size() == 2 && core.queue()[0] == u2);
  check_state(core, dev);
  CHECK(core.tick(dev, &n) == NMC_OK && n == 2);
  dev.now = 2e9;
  CHECK(core.tick(dev, &n) == NMC_OK && core.idle());
  CHECK(core.stats().completed == 6 && core.stats().submitted == 6 && dev.live == 0);
  std::printf("ENOMEM and errors requeue in arrival order: ok\n");
}

// Seeded simulation: Poisson-like arrivals of mixed requests, ticks at
// random times, injected ENOMEM; every ticket completes exactly once and the
// invariants hold after every tick.
static void test_random_simulation() {
  std::mt19937_64 rng(2301);
  for (int round = 0; round < 3; ++round) {
    const size_t budget = round == 2 ? 0 : 4096 + 2048 * round;
    ServeCore core(budget, 32);
    FakeDevice dev;
    dev.rate = 64;
    const int n_req = 3000;
    std::uniform_int_distribution<int> Nd(0, 2), Ld(1, 32), pd(0, 1), md(0, 2), coin(0, 19);
    std::exponential_distribution<double> gap(2.0);
    std::set<uint64_t> submitted, completed;
    double next_arrival = 0;
    int arrived = 0, ticks = 0;
    while (arrived < n_req || !core.idle()) {
      if (arrived < n_req && next_arrival <= dev.now) {
        const int N = 32 << Nd(rng);
        const size_t bytes = (size_t)(N / 32) * (size_t)Ld(rng) * 16;
        submitted.insert(submit(core, dev, ServeKey{N, pd(rng), md(rng)}, bytes));
        ++arrived;
        next_arrival += gap(rng);
        continue;
      }
      if (coin(rng) == 0) dev.enomem_next = 1;
      int n = 0;
      const int rc = core.tick(dev, &n);
      CHECK(rc == NMC_OK || rc == NMC_ENOMEM);
      check_state(core, dev);
      ++ticks;
      uint64_t out[64];
      int k;
      while ((k = core.take_completed(out, 64)) > 0)
        for (int i = 0; i < k; ++i) {
          CHECK(submitted.count(out[i]) == 1);
          CHECK(completed.insert(out[i]).second);  // exactly once
        }
      dev.now += 0.25;
    }
    CHECK(completed.size() == (size_t)n_req);
    CHECK(dev.live == 0 && dev.held == 0);
    const auto& st = core.stats();
    CHECK(st.submitted == (uint64_t)n_req && st.completed == (uint64_t)n_req && st.admitted == (uint64_t)n_req);
    CHECK(st.inflight == 0 && st.queued == 0 && st.inflight_bytes == 0);
    if (budget) CHECK(st.peak_inflight_bytes <= budget);
    std::printf("random simulation (budget %zu): %d requests, %d ticks, %llu batches, peak %zu bytes: ok\n",
                budget, n_req, ticks, (unsigned long long)st.batches, st.peak_inflight_bytes);
  }
}

// The ring of serving workspace regions: regions never overlap, stay in
// bounds, are released oldest first, and a region that fits the free run
// (at the head or, past the end, at the start) is placed.
static void test_ring_arena() {
  nmc::RingArena a(100);
  size_t o = 0;
  CHECK(!a.alloc(0, &o) && !a.alloc(101, &o));
  CHECK(a.alloc(40, &o) && o == 0);
  CHECK(a.alloc(40, &o) && o == 40);
  CHECK(!a.alloc(30, &o));  // 20 left at the end, the start is taken
  CHECK(a.alloc(20, &o) && o == 80);
  a.release_oldest();       // [0, 40) free
  CHECK(!a.alloc(41, &o));
  CHECK(a.alloc(30, &o) && o == 0);  // wrapped
  CHECK(a.alloc(10, &o) && o == 30);
  CHECK(!a.alloc(1, &o));   // full up to the oldest region
  a.release_newest();       // a launch that did not go ahead
  CHECK(a.alloc(10, &o) && o == 30);
  a.release_oldest();
  a.release_oldest();       // [40, 100) free, live: [0, 40)
  CHECK(a.alloc(60, &o) && o == 40);
  CHECK(a.used() == 100);
  a.release_oldest();
  a.release_oldest();
  a.release_oldest();
  CHECK(a.empty() && a.used() == 0);
  CHECK(a.alloc(100, &o) && o == 0);
  a.release_oldest();
  // random FIFO traffic: every placed region is disjoint from the others
  std::mt19937_64 rng(7);
  nmc::RingArena r(1000);
  for (int i = 0; i < 20000; ++i) {
    if (!r.empty() && (rng() % 3 == 0)) {
      r.release_oldest();
      continue;
    }
    const size_t b = 1 + rng() % 300;
    const size_t before = r.used();
    if (r.alloc(b, &o)) {
      CHECK(o + b <= 1000);
      const auto& lv = r.live();
      for (size_t k = 0; k + 1 < lv.size(); ++k)
        CHECK(lv[k].first + lv[k].second <= o || o + b <= lv[k].first);
    } else {
      CHECK(r.used() == before);
      CHECK(before + b > 1000 || !r.empty());  // an empty ring places anything that fits
    }
  }
}

int main() {
  test_ring_arena();
  test_fifo_admission_under_budget();
  test_grouping_and_batch_bounds();
  test_enomem_and_errors_requeue_in_order();
  test_random_simulation();
  std::printf("ALL OK\n");
  return 0;
}
