// Continuous-batching scheduler core of the serving loop (host code only, no
// HIP): admission by footprint in arrival order, grouping of the admitted
// requests by (N, precision, method), batches bounded in requests and bytes,
// retirement of finished batches and requeueing, in arrival order, of what
// could not be launched.  The device side (launching a batch, asking whether
// it finished, releasing what it held) is an interface, implemented over HIP
// streams and events by the library and over a simulated device in the host
// tests.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <tuple>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/nmc.h"

namespace nmc {

// Requests of one group share every launch of a batched solve.
using ServeKey = std::tuple<int, int, int>;  // N, precision, method

struct ServeBatch {
  std::vector<uint64_t> tickets;  // arrival order
  size_t bytes = 0;               // device bytes the batch holds (set by the device)
  void* dev = nullptr;            // the device side's own record of the batch
};

// What the scheduler needs from the device.
class ServeDevice {
 public:
  virtual ~ServeDevice() = default;
  // 1 finished, 0 still running, a negative status on a device error.
  virtual int poll(const ServeBatch& b) = 0;
  // Enqueue the batch; on NMC_OK set b.bytes and b.dev.  NMC_ENOMEM: nothing
  // was enqueued and the batch may be retried once work in flight retires;
  // any other status is an error (nothing of the batch is left running).
  virtual int launch(ServeBatch& b) = 0;
  // The batch finished: release what it held.
  virtual void release(ServeBatch& b) = 0;
};

// Regions of the serving workspace in one allocation of `size` bytes, used
// as a ring: batches retire in launch order, so regions are released oldest
// first and the free space is one run (wrapping at the end).  The device
// side holds the allocation; this tracks offsets only.
class RingArena {
 public:
  RingArena() = default;
  explicit RingArena(size_t size) : size_(size) {}
  // A region of `bytes` after the newest one, or at the start once the end
  // is reached; false when it does not fit beside the regions in use.
  bool alloc(size_t bytes, size_t* off) {
    if (bytes == 0 || bytes > size_) return false;
    size_t at = 0;
    if (!live_.empty()) {
      const size_t tail = live_.front().first;
      const size_t head = live_.back().first + live_.back().second;
      const bool wrapped = live_.back().first < tail;
      if (!wrapped && head + bytes <= size_) at = head;
      else if (!wrapped && bytes <= tail) at = 0;
      else if (wrapped && head + bytes <= tail) at = head;
      else return false;
    }
    live_.emplace_back(at, bytes);
    *off = at;
    return true;
  }
  void release_oldest() {
    if (!live_.empty()) live_.pop_front();
  }
  void release_newest() {  // a launch that did not go ahead
    if (!live_.empty()) live_.pop_back();
  }
  bool empty() const { return live_.empty(); }
  size_t size() const { return size_; }
  size_t used() const {
    size_t u = 0;
    for (const auto& r : live_) u += r.second;
    return u;
  }
  const std::deque<std::pair<size_t, size_t>>& live() const { return live_; }

 private:
  size_t size_ = 0;
  std::deque<std::pair<size_t, size_t>> live_;  // (offset, bytes), oldest first
};

class ServeCore {
 public:
  enum State { kQueued = 0, kInflight = 1, kDone = 2 };
  struct Item {
    ServeKey key;
    size_t bytes;  // admission footprint
    int state;
  };

  ServeCore(size_t budget, int max_batch_requests) : budget_(budget), max_requests_(max_batch_requests) {
    stats_ = nmc_serve_stats{};
    stats_.budget_bytes = budget;
  }

  // Queue a request (the caller has checked that bytes <= budget).
  uint64_t submit(ServeKey key, size_t bytes) {
    const uint64_t t = next_ticket_++;
    items_[t] = Item{key, bytes, kQueued};
    queue_.push_back(t);
    stats_.submitted++;
    stats_.queued = queue_.size();
    return t;
  }

  // One scheduler step: retire finished batches, admit queued requests in
  // arrival order while the footprint of the work in flight fits the budget,
  // launch them as batches (one group each, at most max_batch_requests
  // requests and a quarter of the budget, so that several batches overlap on
  // the device).  Requests whose batch could not be launched go back to the
  // front of the queue in arrival order, and so do all that follow a failed
  // launch.  Returns NMC_OK, the device's error, or NMC_ENOMEM when a batch
  // does not fit with nothing in flight.
  int tick(ServeDevice& dev, int* launched) {
    int n_launched = 0;
    if (launched) *launched = 0;
    int rc = retire(dev);
    if (rc) return rc;
    std::vector<uint64_t> admitted;
    size_t bytes = stats_.inflight_bytes;
    while (!queue_.empty()) {
      const Item& it = items_.at(queue_.front());
      if (budget_ && bytes + it.bytes > budget_) break;
      bytes += it.bytes;
      admitted.push_back(queue_.front());
      queue_.pop_front();
    }
    std::vector<uint64_t> requeue;
    int err = NMC_OK;
    for (auto& ts : make_batches(admitted)) {
      if (!requeue.empty() || err) {  // keep arrival order behind a batch that did not launch
        requeue.insert(requeue.end(), ts.begin(), ts.end());
        continue;
      }
      ServeBatch b;
      b.tickets = ts;
      const int lrc = dev.launch(b);
      if (lrc) {
        requeue.insert(requeue.end(), ts.begin(), ts.end());
        if (lrc != NMC_ENOMEM) err = lrc;
        continue;
      }
      for (uint64_t t : ts) items_.at(t).state = kInflight;
      stats_.admitted += ts.size();
      stats_.inflight += ts.size();
      stats_.batches++;
      stats_.inflight_bytes += b.bytes;
      stats_.peak_inflight_bytes = std::max(stats_.peak_inflight_bytes, stats_.inflight_bytes);
      n_launched += (int)ts.size();
      inflight_.push_back(std::move(b));
    }
    std::sort(requeue.begin(), requeue.end());  // tickets grow with arrival
    for (auto it = requeue.rbegin(); it != requeue.rend(); ++it) queue_.push_front(*it);
    stats_.queued = queue_.size();
    if (launched) *launched = n_launched;
    if (err) return err;
    if (!requeue.empty() && inflight_.empty()) return NMC_ENOMEM;
    return NMC_OK;
  }

  // Retire the finished batches at the head of the in-flight list (batches
  // retire in launch order).
  int retire(ServeDevice& dev) {
    while (!inflight_.empty()) {
      ServeBatch& b = inflight_.front();
      const int q = dev.poll(b);
      if (q < 0) return q;
      if (q == 0) break;
      for (uint64_t t : b.tickets) {
        items_.at(t).state = kDone;
        completed_.push_back(t);
        stats_.completed++;
      }
      stats_.inflight_bytes -= b.bytes;
      stats_.inflight -= b.tickets.size();
      dev.release(b);
      inflight_.pop_front();
    }
    return NMC_OK;
  }

  // Admitted tickets (arrival order) as batches: one group per batch, arrival
  // order inside, at most max_requests_ requests and, under a budget, a
  // quarter of it (a single larger request still forms a batch).
  std::vector<std::vector<uint64_t>> make_batches(const std::vector<uint64_t>& admitted) const {
    const size_t max_bytes = budget_ ? std::max<size_t>(budget_ / 4, 1) : SIZE_MAX;
    std::map<ServeKey, std::vector<uint64_t>> groups;
    for (uint64_t t : admitted) groups[items_.at(t).key].push_back(t);
    std::vector<std::vector<uint64_t>> batches;
    for (auto& kv : groups) {
      std::vector<uint64_t> cur;
      size_t cur_bytes = 0;
      for (uint64_t t : kv.second) {
        const size_t b = items_.at(t).bytes;
        if (!cur.empty() && ((int)cur.size() >= max_requests_ || cur_bytes + b > max_bytes)) {
          batches.push_back(std::move(cur));
          cur.clear();
          cur_bytes = 0;
        }
        cur.push_back(t);
        cur_bytes += b;
      }
      if (!cur.empty()) batches.push_back(std::move(cur));
    }
    return batches;
  }

  // Moves up to cap completed tickets (oldest first) to out and forgets them.
  int take_completed(uint64_t* out, int cap) {
    int k = 0;
    while (k < cap && !completed_.empty()) {
      out[k++] = completed_.front();
      items_.erase(completed_.front());
      completed_.pop_front();
    }
    return k;
  }

  // The item of a ticket, or null.
  const Item* find(uint64_t t) const {
    auto it = items_.find(t);
    return it == items_.end() ? nullptr : &it->second;
  }
  bool idle() const { return queue_.empty() && inflight_.empty(); }
  const ServeBatch* oldest_inflight() const { return inflight_.empty() ? nullptr : &inflight_.front(); }
  const std::deque<ServeBatch>& inflight() const { return inflight_; }
  const std::deque<uint64_t>& queue() const { return queue_; }
  const nmc_serve_stats& stats() const { return stats_; }
  size_t budget() const { return budget_; }

 private:
  size_t budget_;
  int max_requests_;
  uint64_t next_ticket_ = 1;
  std::unordered_map<uint64_t, Item> items_;
  std::deque<uint64_t> queue_;
  std::deque<ServeBatch> inflight_;
  std::deque<uint64_t> completed_;
  nmc_serve_stats stats_;
};

}  // namespace nmc
