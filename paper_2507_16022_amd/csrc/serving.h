// serving.h -- host-side admission and scheduling for the serving calls.
//
// Plain C++ (no HIP): a first-fit map over one fixed device pool, and a FIFO
// scheduler whose slot threads each run a batch of admitted events at a
// time.  An event is admitted when it is at the head of the queue, a slot is
// idle and the pool holds a free block of the event's size; an idle slot
// takes the head and then, while they fit, the events queued behind it, up
// to the batch limit, and runs them together (their passes packed into
// shared launches).  Each block returns to the pool when its batch
// completes.  Events that arrive while others run are admitted as slots and
// memory free up, so their device work overlaps.
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
  int batch = 0;    // jobs in the batch that ran it
};

// FIFO scheduler over n_slots threads and one pool.  run(slot, offset) does
// the job's work with the pool block at `offset` and returns a status code.
// With a batch function and max_batch > 1, a slot takes up to max_batch
// queued jobs at once and batch(slot, items) runs them all, setting each
// item's status; a job's run function is then not called.  A batch of more
// than one job also holds at most batch_work units of work (as given to
// submit), so that a job large enough to fill the device runs alone and the
// jobs packed together are small ones: a batch completes when its largest
// job does, and a small job packed with a large one would wait for it.
class Scheduler {
 public:
  typedef std::function<int(int slot, uint64_t off)> RunFn;
  struct BatchItem {
    void* payload;    // as given to submit
    uint64_t off;     // pool block
    int rc;           // set by the batch function
  };
  typedef std::function<void(int slot, std::vector<BatchItem>& items)> BatchFn;

  Scheduler(int n_slots, uint64_t pool_bytes, std::function<void(int)> slot_init,
            int max_batch = 1, BatchFn batch = nullptr, double batch_work = 0.0)
      : pool_(pool_bytes),
        t0_(std::chrono::steady_clock::now()),
        max_batch_(batch && max_batch > 1 ? max_batch : 1),
        batch_(std::move(batch)),
        batch_work_(batch_work) {
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
  int64_t submit(uint64_t bytes, RunFn run, std::shared_ptr<void> payload = nullptr,
                 double work = 0.0) {
    auto j = std::make_shared<Job>();
    j->bytes = bytes;
    j->work = work;
    j->run = std::move(run);
    j->payload = std::move(payload);
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
    std::shared_ptr<void> payload;
    double work = 0.0;
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
      // the head (fits() held under the same lock), then while they fit
      // the jobs behind it, in order, up to the batch limit
      std::vector<std::shared_ptr<Job>> batch;
      std::vector<BatchItem> items;
      double work = 0.0;
      while (!queue_.empty() && (int)batch.size() < max_batch_) {
        if (!batch.empty() && work + queue_.front()->work > batch_work_) break;
        uint64_t off = 0;
        if (!pool_.alloc(queue_.front()->bytes, &off)) break;
        work += queue_.front()->work;
        auto j = queue_.front();
        queue_.pop_front();
        j->times.t_start_ms = now_ms();
        j->times.slot = slot;
        batch.push_back(j);
        items.push_back(BatchItem{j->payload.get(), off, 0});
      }
      running_ += (int)batch.size();
      lk.unlock();
      cv_.notify_all();   // the next head may fit in what is left
      if (batch_) {
        batch_(slot, items);
      } else {
        for (size_t q = 0; q < batch.size(); ++q) items[q].rc = batch[q]->run(slot, items[q].off);
      }
      lk.lock();
      const double t_done = now_ms();
      for (size_t q = 0; q < batch.size(); ++q) {
        pool_.release(items[q].off);
        batch[q]->rc = items[q].rc;
        batch[q]->times.t_done_ms = t_done;
        batch[q]->times.batch = (int)batch.size();
        batch[q]->done = true;
        batch[q]->run = nullptr;
        batch[q]->payload.reset();
      }
      running_ -= (int)batch.size();
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
  int max_batch_ = 1;
  BatchFn batch_;
  double batch_work_ = 0.0;
  int64_t next_ticket_ = 1;
  int running_ = 0;
  bool stop_ = false;
};

}  // namespace dotpe
