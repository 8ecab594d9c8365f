// serving.h -- host-side admission and scheduling for the serving calls.
//
// Plain C++ (no HIP): a first-fit map over one fixed device pool, and a FIFO
// scheduler whose slot threads each run one admitted event at a time.  An
// event is admitted when it is at the head of the queue, a slot is idle and
// the pool holds a free block of the event's size; its block returns to the
// pool when the event completes.  Events that arrive while others run are
// admitted as slots and memory free up, so their device work overlaps.
#pragma once

#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

namespace dotpe {

// First-fit allocator of byte ranges in [0, size); every block starts at a
// multiple of kPoolAlign and free neighbours coalesce.
class PoolMap {
 public:
  static constexpr uint64_t kPoolAlign = 256;
  explicit PoolMap(uint64_t size) : size_(size / kPoolAlign * kPoolAlign) {
    if (size_) free_[0] = size_;
  }
  static uint64_t round(uint64_t n) { return (n + kPoolAlign - 1) / kPoolAlign * kPoolAlign; }
  uint64_t size() const { return size_; }
  // first free block that holds n bytes; false if none does
  bool alloc(uint64_t n, uint64_t* off) {
    n = round(n ? n : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      uint64_t o = it->first, s = it->second;
      free_.erase(it);
      if (s > n) free_[o + n] = s - n;
      used_[o] = n;
      *off = o;
      return true;
    }
    return false;
  }
  // return a block obtained from alloc (unknown offsets are ignored)
  void release(uint64_t off) {
    auto u = used_.find(off);
    if (u == used_.end()) return;
    uint64_t o = off, s = u->second;
    used_.erase(u);
    auto nx = free_.lower_bound(o);
    if (nx != free_.end() && o + s == nx->first) {
      s += nx->second;
      nx = free_.erase(nx);
    }
    if (nx != free_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == o) {
        pv->second += s;
        return;
      }
    }
    free_[o] = s;
  }
  bool fits(uint64_t n) const {
    n = round(n ? n : 1);
    for (const auto& f : free_)
      if (f.second >= n) return true;
    return false;
  }
  uint64_t used_bytes() const {
    uint64_t t = 0;
    for (const auto& u : used_) t += u.second;
    return t;
  }
  size_t n_free_blocks() const { return free_.size(); }

 private:
  uint64_t size_;
  std::map<uint64_t, uint64_t> free_;   // offset -> size
  std::map<uint64_t, uint64_t> used_;   // offset -> size
};

struct JobTimes {
  double t_submit_ms = 0, t_start_ms = 0, t_done_ms = 0;   // since scheduler creation
  uint64_t bytes = 0;
  int slot = -1;
};

// FIFO scheduler over n_slots threads and one pool.  run(slot, offset) does
// the job's work with the pool block at `offset` and returns a status code.
class Scheduler {
 public:
  typedef std::function<int(int slot, uint64_t off)> RunFn;

  Scheduler(int n_slots, uint64_t pool_bytes, std::function<void(int)> slot_init)
      : pool_(pool_bytes), t0_(std::chrono::steady_clock::now()) {
    for (int s = 0; s < n_slots; ++s)
      threads_.emplace_back([this, s, slot_init] {
        if (slot_init) slot_init(s);
        loop(s);
      });
  }
  // finishes every submitted job, then stops the slot threads
  ~Scheduler() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : threads_) t.join();
  }
  uint64_t pool_bytes() const { return pool_.size(); }
  // false if the job can never be admitted (larger than the pool)
  bool admissible(uint64_t bytes) const { return PoolMap::round(bytes) <= pool_.size(); }
  int64_t submit(uint64_t bytes, RunFn run) {
    auto j = std::make_shared<Job>();
    j->bytes = bytes;
    j->run = std::move(run);
    j->times.t_submit_ms = now_ms();
    j->times.bytes = bytes;
    int64_t t;
    {
      std::lock_guard<std::mutex> lk(mu_);
      t = j->ticket = next_ticket_++;
      jobs_[t] = j;
      queue_.push_back(j);
    }
    cv_.notify_all();
    return t;
  }
  // 1 done, 0 pending, -1 unknown ticket
  int poll(int64_t t) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = jobs_.find(t);
    if (it == jobs_.end()) return -1;
    return it->second->done ? 1 : 0;
  }
  // blocks until the job is done, forgets it and returns its status;
  // -1 for an unknown ticket
  int wait(int64_t t, JobTimes* times) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = jobs_.find(t);
    if (it == jobs_.end()) return kUnknown;
    auto j = it->second;
    done_cv_.wait(lk, [&] { return j->done; });
    jobs_.erase(t);
    if (times) *times = j->times;
    return j->rc;
  }
  int in_flight() {
    std::lock_guard<std::mutex> lk(mu_);
    return running_;
  }
  uint64_t pool_used() {
    std::lock_guard<std::mutex> lk(mu_);
    return pool_.used_bytes();
  }
  static constexpr int kUnknown = -1000;

 private:
  struct Job {
    int64_t ticket = 0;
    uint64_t bytes = 0;
    RunFn run;
    int rc = 0;
    bool done = false;
    JobTimes times;
  };
  double now_ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0_).count();
  }
  void loop(int slot) {
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
      cv_.wait(lk, [&] {
        return (!queue_.empty() && pool_.fits(queue_.front()->bytes)) || (stop_ && queue_.empty());
      });
      if (queue_.empty()) return;   // stop_ and drained
      auto j = queue_.front();
      queue_.pop_front();
      uint64_t off = 0;
      pool_.alloc(j->bytes, &off);   // fits() held under the same lock
      ++running_;
      j->times.t_start_ms = now_ms();
      j->times.slot = slot;
      lk.unlock();
      cv_.notify_all();   // the next head may fit in what is left
      int rc = j->run(slot, off);
      lk.lock();
      pool_.release(off);
      --running_;
      j->rc = rc;
      j->times.t_done_ms = now_ms();
      j->done = true;
      j->run = nullptr;
      done_cv_.notify_all();
      cv_.notify_all();
    }
  }

  PoolMap pool_;
  std::chrono::steady_clock::time_point t0_;
  std::mutex mu_;
  std::condition_variable cv_, done_cv_;
  std::deque<std::shared_ptr<Job>> queue_;
  std::map<int64_t, std::shared_ptr<Job>> jobs_;
  std::vector<std::thread> threads_;
  int64_t next_ticket_ = 1;
  int running_ = 0;
  bool stop_ = false;
};

}  // namespace dotpe
