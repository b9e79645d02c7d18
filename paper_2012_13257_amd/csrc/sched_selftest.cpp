// CPU harness of the serving scheduler: the real Scheduler driven by a fake
// executor whose batches "complete" after a programmable delay, so admission,
// slot and budget accounting, ticket lifecycle, concurrency of batches and
// shutdown can be tested without a GPU.  Built with the host compiler into
// libgmmsched_test.so; only the test-suite loads it.
#include <chrono>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

#include "scheduler.hpp"

namespace {

using gmm::serve::Job;
using gmm::serve::now_ns;

struct FakeReq {
  int64_t delay_us;
  int fail;  // the batch holding this request reports an error
};

class FakeExecutor {
 public:
  FakeExecutor(int contexts, int max_batch) : ctx_(contexts), max_batch_(max_batch) {}
  int contexts() const { return (int)ctx_.size(); }
  int max_batch() const { return max_batch_; }
  void thread_init() {}

  int launch(int c, std::vector<Job<FakeReq>*>& jobs) {
    std::lock_guard<std::mutex> g(mu_);
    int64_t d = 0;
    bool f = false;
    for (auto* j : jobs) {
      d = std::max(d, j->req.delay_us);
      f = f || j->req.fail;
      // arena ranges of everything on the device must be disjoint
      for (auto& r : live_) {
        const int64_t a0 = j->arena_off, a1 = j->arena_off + (int64_t)j->bytes;
        if (a0 < r.second && r.first < a1) ++overlaps_;
      }
    }
    for (auto* j : jobs) live_.push_back({j->arena_off, j->arena_off + (int64_t)j->bytes});
    ctx_[c].done_at = now_ns() + d * 1000;
    ctx_[c].fail = f;
    ctx_[c].ranges.clear();
    for (auto* j : jobs) ctx_[c].ranges.push_back({j->arena_off, j->arena_off + (int64_t)j->bytes});
    max_jobs_in_batch_ = std::max(max_jobs_in_batch_, (int)jobs.size());
    return INTERP_OK;
  }

  int query(int c) {
    std::lock_guard<std::mutex> g(mu_);
    if (now_ns() < ctx_[c].done_at) return 0;
    for (auto& r : ctx_[c].ranges) {
      for (size_t k = 0; k < live_.size(); ++k) {
        if (live_[k] == r) { live_.erase(live_.begin() + k); break; }
      }
    }
    ctx_[c].ranges.clear();
    return ctx_[c].fail ? INTERP_EHIP : 1;
  }

  void wait(int c) {
    int64_t t;
    {
      std::lock_guard<std::mutex> g(mu_);
      t = ctx_[c].done_at;
    }
    while (now_ns() < t) std::this_thread::sleep_for(std::chrono::microseconds(50));
  }

  int overlaps() {
    std::lock_guard<std::mutex> g(mu_);
    return overlaps_;
  }
  int max_jobs_in_batch() {
    std::lock_guard<std::mutex> g(mu_);
    return max_jobs_in_batch_;
  }

 private:
  struct Ctx {
    int64_t done_at = 0;
    bool fail = false;
    std::vector<std::pair<int64_t, int64_t>> ranges;
  };
  std::mutex mu_;
  std::vector<Ctx> ctx_;
  int max_batch_;
  std::vector<std::pair<int64_t, int64_t>> live_;
  int overlaps_ = 0;
  int max_jobs_in_batch_ = 0;
};

struct Harness {
  FakeExecutor ex;
  gmm::serve::Scheduler<FakeReq, FakeExecutor> sched;
  Harness(uint64_t budget, int slots, int queue, int contexts, int max_batch)
      : ex(contexts, max_batch), sched(&ex, budget, slots, queue) {}
};

}  // namespace

extern "C" {

void* gmm_fake_create(uint64_t budget, int slots, int queue, int contexts, int max_batch) {
  return new Harness(budget, slots, queue, contexts, max_batch);
}

int gmm_fake_submit(void* h, uint64_t bytes, int64_t delay_us, int fail, uint64_t* ticket) {
  return static_cast<Harness*>(h)->sched.submit(FakeReq{delay_us, fail}, bytes, ticket);
}

// n requests of bytes[i] bytes in one call (delay_us and fail as above)
int gmm_fake_submit_many(void* h, const uint64_t* bytes, int n, int64_t delay_us, int fail,
                         uint64_t* tickets, int* accepted) {
  std::vector<FakeReq> rq(n, FakeReq{delay_us, fail});
  return static_cast<Harness*>(h)->sched.submit_many(rq.data(), bytes, n, tickets, accepted);
}

int gmm_fake_poll(void* h, uint64_t ticket, interp_status* st) {
  return static_cast<Harness*>(h)->sched.poll(ticket, st);
}

int gmm_fake_drain(void* h, int64_t timeout_ms) {
  return static_cast<Harness*>(h)->sched.drain(timeout_ms);
}

// stats: [peak arena bytes, peak slots, batches, peak concurrent batches,
//         arena overlaps seen, largest batch]
void gmm_fake_stats(void* h, int64_t* out6) {
  auto* x = static_cast<Harness*>(h);
  out6[0] = (int64_t)x->sched.peak_arena();
  out6[1] = x->sched.peak_slots();
  out6[2] = x->sched.batches();
  out6[3] = x->sched.peak_concurrent_batches();
  out6[4] = x->ex.overlaps();
  out6[5] = x->ex.max_jobs_in_batch();
}

void gmm_fake_shutdown(void* h) { static_cast<Harness*>(h)->sched.shutdown(); }

void gmm_fake_destroy(void* h) {
  auto* x = static_cast<Harness*>(h);
  x->sched.shutdown();
  delete x;
}

// Arena checks: allocate/release a scripted sequence, return the number of
// fragments left (1 when everything coalesced back) or -1 on an invariant
// violation (overlap of live ranges or a failed allocation that should fit).
int gmm_arena_selftest(uint64_t size, int n, const int64_t* sizes, const int* release_order) {
  gmm::serve::Arena a(size);
  std::vector<int64_t> off(n);
  for (int i = 0; i < n; ++i) {
    off[i] = a.alloc((uint64_t)sizes[i]);
    if (off[i] < 0) return -2;
    for (int k = 0; k < i; ++k) {
      const int64_t a0 = off[i], a1 = off[i] + (int64_t)gmm::serve::Arena::round(sizes[i]);
      const int64_t b0 = off[k], b1 = off[k] + (int64_t)gmm::serve::Arena::round(sizes[k]);
      if (a0 < b1 && b0 < a1) return -1;
    }
  }
  for (int i = 0; i < n; ++i) a.release((uint64_t)off[release_order[i]], (uint64_t)sizes[release_order[i]]);
  if (a.used() != 0) return -3;
  const int frag = (int)a.fragments();
  if (a.alloc(size) != 0) return -4;  // everything coalesced back into one range
  return frag;
}

}  // extern "C"
