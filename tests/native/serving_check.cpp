// Host-only checks of the serving scheduler (pool map, FIFO admission by
// memory, slot limit, drain on destruction).  Built with g++ by the tests.
#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "serving.h"

#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::fprintf(stderr, "FAIL %s:%d %s\n", __FILE__, __LINE__, #c); \
      std::exit(1);                                                \
    }                                                              \
  } while (0)

using dotpe::PoolMap;
using dotpe::Scheduler;

static void pool_checks() {
  PoolMap p(4096 + 100);            // rounded down to whole 256-byte units
  CHECK(p.size() == 4096);
  uint64_t a, b, c, d;
  CHECK(p.alloc(1000, &a) && a == 0);        // 1024 bytes
  CHECK(p.alloc(256, &b) && b == 1024);
  CHECK(p.alloc(1, &c) && c == 1280);        // 256 bytes
  CHECK(p.used_bytes() == 1536);
  CHECK(!p.alloc(4096, &d));
  CHECK(p.fits(2560) && !p.fits(2561));
  p.release(b);                               // hole of 256 between a and c
  CHECK(p.alloc(200, &d) && d == 1024);       // first fit takes the hole
  p.release(d);
  p.release(a);                               // coalesces with the hole: [0, 1280)
  CHECK(p.fits(1280));
  CHECK(p.alloc(1280, &d) && d == 0);
  p.release(d);
  p.release(c);                               // everything free again, one block
  CHECK(p.n_free_blocks() == 1 && p.used_bytes() == 0 && p.fits(4096));
  p.release(12345);                           // unknown offsets are ignored
  CHECK(p.used_bytes() == 0);
}

static void sched_checks() {
  const uint64_t pool = 1 << 20;
  std::atomic<int> running{0}, max_running{0};
  std::atomic<uint64_t> bytes_live{0}, max_bytes{0};
  std::mutex m;
  std::vector<int64_t> start_order;
  std::vector<int64_t> tickets;
  {
    Scheduler s(3, pool, nullptr);
    CHECK(s.admissible(pool) && !s.admissible(pool + 1));
    // sizes: the 4th job needs most of the pool, so it waits until the
    // first three are done; the small jobs behind it must not overtake it
    std::vector<uint64_t> sizes = {200000, 200000, 200000, 900000, 10000, 10000, 10000, 500000,
                                   500000, 1000};
    for (size_t q = 0; q < sizes.size(); ++q) {
      const uint64_t n = sizes[q];
      const int64_t id = (int64_t)q;
      tickets.push_back(s.submit(n, [&, n, id](int slot, uint64_t off) {
        CHECK(slot >= 0 && slot < 3);
        CHECK(off % PoolMap::kPoolAlign == 0 && off + n <= pool);
        {
          std::lock_guard<std::mutex> lk(m);
          start_order.push_back(id);
        }
        int r = ++running;
        int mr = max_running.load();
        while (r > mr && !max_running.compare_exchange_weak(mr, r)) {}
        uint64_t b = (bytes_live += PoolMap::round(n));
        uint64_t mb = max_bytes.load();
        while (b > mb && !max_bytes.compare_exchange_weak(mb, b)) {}
        std::this_thread::sleep_for(std::chrono::milliseconds(20));
        bytes_live -= PoolMap::round(n);
        --running;
        return (int)id;
      }));
    }
    // wait returns each job's status; a waited ticket is forgotten
    dotpe::JobTimes t;
    CHECK(s.wait(tickets[0], &t) == 0);
    CHECK(t.t_start_ms >= t.t_submit_ms && t.t_done_ms >= t.t_start_ms + 15.0);
    CHECK(s.poll(tickets[0]) == -1 && s.wait(tickets[0], nullptr) == Scheduler::kUnknown);
    // admission is first in, first out: admission times (taken under the
    // scheduler's lock) follow submission order
    double last = t.t_start_ms;
    for (size_t q = 1; q < 8; ++q) {
      dotpe::JobTimes tq;
      CHECK(s.wait(tickets[q], &tq) == (int)q);
      CHECK(tq.t_start_ms >= last);
      last = tq.t_start_ms;
    }
    // tickets 8 and 9 are left for the destructor to drain
  }
  CHECK(start_order.size() == 10);
  std::vector<int64_t> sorted_order = start_order;
  std::sort(sorted_order.begin(), sorted_order.end());
  for (size_t q = 0; q < sorted_order.size(); ++q) CHECK(sorted_order[q] == (int64_t)q);
  CHECK(max_running.load() <= 3 && max_running.load() >= 2);
  CHECK(max_bytes.load() <= pool);
}

// batches: an idle slot takes the head and the jobs queued behind it while
// they fit, up to the batch limit, in order; a job too large for what is
// left waits for the next batch (and nothing behind it overtakes it)
static void batch_checks() {
  const uint64_t pool = 1 << 20;
  std::mutex m;
  std::vector<std::vector<int64_t>> batches;
  {
    Scheduler::BatchFn fn = [&](int slot, std::vector<Scheduler::BatchItem>& items) {
      CHECK(slot == 0);
      std::vector<int64_t> b;
      for (auto& it : items) {
        const int64_t id = *(const int64_t*)it.payload;
        b.push_back(id);
        it.rc = (int)id;
        CHECK(it.off % PoolMap::kPoolAlign == 0);
      }
      {
        std::lock_guard<std::mutex> lk(m);
        batches.push_back(b);
      }
      std::this_thread::sleep_for(std::chrono::milliseconds(30));
    };
    Scheduler s(1, pool, nullptr, 3, fn);
    // job 0 runs alone (the slot is idle when it arrives); 1..3 then queue
    // and run as one batch of 3; 4 (most of the pool) and 5 come next: 4
    // alone would leave no room for 5, so they run as two batches
    std::vector<uint64_t> sizes = {1000, 1000, 1000, 1000, 1000000, 100000, 1000};
    std::vector<int64_t> tickets;
    auto submit = [&](size_t q) {
      auto id = std::make_shared<int64_t>((int64_t)q);
      tickets.push_back(s.submit(sizes[q], [](int, uint64_t) { return -1; }, id));
    };
    submit(0);
    std::this_thread::sleep_for(std::chrono::milliseconds(10));
    for (size_t q = 1; q < sizes.size(); ++q) submit(q);
    for (size_t q = 0; q < tickets.size(); ++q) {
      dotpe::JobTimes t;
      CHECK(s.wait(tickets[q], &t) == (int)q);
      CHECK(t.batch >= 1 && t.batch <= 3);
    }
  }
  std::vector<int64_t> flat;
  for (auto& b : batches) {
    CHECK(!b.empty() && b.size() <= 3);
    for (int64_t id : b) flat.push_back(id);
  }
  CHECK(flat.size() == 7);
  for (size_t q = 0; q < flat.size(); ++q) CHECK(flat[q] == (int64_t)q);   // first in, first out
  CHECK(batches[0].size() == 1 && batches[0][0] == 0);
  CHECK(batches[1].size() == 3);
  // job 4 fills the pool: its batch holds no other job
  for (auto& b : batches)
    if (std::find(b.begin(), b.end(), 4) != b.end()) CHECK(b.size() == 1);
}

// the work budget: a batch of several jobs holds at most batch_work units;
// a job above the budget runs alone
static void budget_checks() {
  std::mutex m;
  std::vector<std::vector<int64_t>> batches;
  {
    Scheduler::BatchFn fn = [&](int, std::vector<Scheduler::BatchItem>& items) {
      std::vector<int64_t> b;
      for (auto& it : items) {
        b.push_back(*(const int64_t*)it.payload);
        it.rc = 0;
      }
      {
        std::lock_guard<std::mutex> lk(m);
        batches.push_back(b);
      }
      std::this_thread::sleep_for(std::chrono::milliseconds(30));
    };
    Scheduler s(1, 1 << 20, nullptr, 8, fn, 10.0);
    // 0 alone (idle slot); then [1, 2, 3] (4 + 3 + 3 = 10); [4] (50, over
    // the budget, alone); [5, 6] (6 + 4); [7]
    std::vector<double> work = {1, 4, 3, 3, 50, 6, 4, 9};
    std::vector<int64_t> tickets;
    auto submit = [&](size_t q) {
      auto id = std::make_shared<int64_t>((int64_t)q);
      tickets.push_back(s.submit(100, [](int, uint64_t) { return -1; }, id, work[q]));
    };
    submit(0);
    std::this_thread::sleep_for(std::chrono::milliseconds(10));
    for (size_t q = 1; q < work.size(); ++q) submit(q);
    for (int64_t t : tickets) CHECK(s.wait(t, nullptr) == 0);
  }
  const std::vector<std::vector<int64_t>> want = {{0}, {1, 2, 3}, {4}, {5, 6}, {7}};
  CHECK(batches == want);
}

int main() {
  pool_checks();
  sched_checks();
  batch_checks();
  budget_checks();
  std::printf("serving_check OK\n");
  return 0;
}
