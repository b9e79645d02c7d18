// Host-side scheduler of the serving loop: request queue, HBM-budget arena,
// job slots, admission, batch formation and completion.  It contains no HIP
// code: the device work is delegated to an Executor, so the same scheduler
// drives the GPU executor (server.hip) and a fake executor in CPU tests.
//
// Continuous batching: a scheduling round first retires finished batches
// (freeing their slots and arena ranges), then admits queued requests in
// arrival order while a job slot is free and the arena can hold the request's
// device state, then launches everything admitted and not yet launched as one
// batch, provided the executor has a free batch context.  Batches run
// concurrently (one context each), so requests that arrive while others are
// on the device start as soon as resources free up instead of waiting for a
// whole batch to drain.
#pragma once

#include <time.h>

#include <algorithm>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "gmminterp.h"

namespace gmm {
namespace serve {

inline int64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (int64_t)ts.tv_sec * 1000000000LL + ts.tv_nsec;
}

// First-fit allocator over [0, size) with coalescing of free neighbours.
class Arena {
 public:
  static constexpr uint64_t kGrain = 256;
  explicit Arena(uint64_t size) : size_(size) {
    if (size) free_[0] = size;
  }
  uint64_t size() const { return size_; }
  uint64_t used() const { return used_; }
  static uint64_t round(uint64_t n) { return (n + kGrain - 1) / kGrain * kGrain; }
  // offset of a free range of n bytes, or -1
  int64_t alloc(uint64_t n) {
    n = round(n ? n : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      const uint64_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > n) free_[off + n] = len - n;
      used_ += n;
      return (int64_t)off;
    }
    return -1;
  }
  void release(uint64_t off, uint64_t n) {
    n = round(n ? n : 1);
    used_ -= n;
    auto it = free_.emplace(off, n).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t fragments() const { return free_.size(); }

 private:
  uint64_t size_;
  uint64_t used_ = 0;
  std::map<uint64_t, uint64_t> free_;
};

template <class Payload>
struct Job {
  uint64_t ticket = 0;
  Payload req{};
  uint64_t bytes = 0;
  int64_t arena_off = -1;
  int32_t state = INTERP_QUEUED;
  int32_t err = INTERP_OK;
  int64_t t_submit = 0, t_admit = 0, t_done = 0;
};

// Executor interface (duck-typed):
//   int  contexts() const;                       number of concurrent batches
//   int  max_batch() const;                      jobs per batch
//   int  launch(int ctx, std::vector<Job<P>*>&); start a batch (async); INTERP_* code
//   int  query(int ctx);                         1 done, 0 running, <0 INTERP_* error
//   void wait(int ctx);                          block until the batch is done
//   void thread_init();                          called once on the scheduler thread
template <class Payload, class Exec>
class Scheduler {
 public:
  using J = Job<Payload>;

  Scheduler(Exec* ex, uint64_t budget, int max_slots, int max_queue)
      : ex_(ex), arena_(budget), max_slots_(max_slots), max_queue_(max_queue) {
    ctx_busy_.assign(ex_->contexts(), false);
    ctx_jobs_.resize(ex_->contexts());
    thread_ = std::thread([this] { loop(); });
  }

  ~Scheduler() { shutdown(); }

  int submit(const Payload& p, uint64_t bytes, uint64_t* ticket) {
    int accepted = 0;
    return submit_many(&p, &bytes, 1, ticket, &accepted);
  }

  // Queues p[0..n) in order under one lock: the first request that cannot be
  // queued (ENOMEM: it can never fit the budget; EAGAIN: the queue is full or
  // the server stops) ends the call with its code, and *accepted (tickets[0..
  // *accepted)) counts the ones queued before it.
  int submit_many(const Payload* p, const uint64_t* bytes, int n, uint64_t* tickets,
                  int* accepted) {
    *accepted = 0;
    // the jobs are built before the lock is taken, so that a large batch
    // holds the scheduler thread up only while it is linked into the queue
    std::vector<std::unique_ptr<J>> js(n);
    for (int i = 0; i < n; ++i) {
      js[i] = std::make_unique<J>();
      js[i]->req = p[i];
      js[i]->bytes = bytes[i];
    }
    std::unique_lock<std::mutex> lk(mu_);
    int rc = INTERP_OK;
    const int64_t t = now_ns();
    for (int i = 0; i < n; ++i) {
      if (stop_) { rc = INTERP_EAGAIN; break; }
      if (Arena::round(bytes[i]) > arena_.size()) { rc = INTERP_ENOMEM; break; }
      if ((int)queue_.size() >= max_queue_) { rc = INTERP_EAGAIN; break; }
      J* j = js[i].get();
      j->ticket = ++next_ticket_;
      j->t_submit = t;
      tickets[i] = j->ticket;
      queue_.push_back(j);
      jobs_[j->ticket] = std::move(js[i]);
      ++outstanding_;
      ++*accepted;
    }
    // When nothing runs or waits, the requests are admitted and launched from
    // the caller's thread at once: waking the scheduler thread first would
    // cost a small request a noticeable part of its latency.  (The thread
    // is still notified: it polls the batch to completion.)
    if (*accepted > 0 && !in_round_ && queue_.size() == (size_t)*accepted && pending_.empty() &&
        !any_busy()) {
      in_round_ = true;
      round(lk);
      in_round_ = false;
      if (outstanding_ == 0) done_cv_.notify_all();
    }
    lk.unlock();
    cv_.notify_all();
    return rc;
  }

  int poll(uint64_t ticket, interp_status* st) {
    std::lock_guard<std::mutex> g(mu_);
    auto it = jobs_.find(ticket);
    if (it == jobs_.end()) return INTERP_ENOTFOUND;
    J* j = it->second.get();
    st->state = j->state;
    st->err = j->err;
    st->t_submit_ns = j->t_submit;
    st->t_admit_ns = j->t_admit;
    st->t_done_ns = j->t_done;
    if (j->state == INTERP_DONE || j->state == INTERP_FAILED) jobs_.erase(it);
    return INTERP_OK;
  }

  // Waits until every submitted request is DONE or FAILED.
  int drain(int64_t timeout_ms) {
    std::unique_lock<std::mutex> lk(mu_);
    auto done = [this] { return outstanding_ == 0; };
    if (timeout_ms < 0) {
      done_cv_.wait(lk, done);
      return INTERP_OK;
    }
    return done_cv_.wait_for(lk, std::chrono::milliseconds(timeout_ms), done) ? INTERP_OK
                                                                            : INTERP_EAGAIN;
  }

  void shutdown() {
    {
      std::lock_guard<std::mutex> g(mu_);
      if (stop_ && !thread_.joinable()) return;
      stop_ = true;
    }
    cv_.notify_all();
    if (thread_.joinable()) thread_.join();
  }

  // statistics (for tests)
  uint64_t peak_arena() const { return peak_arena_; }
  int peak_slots() const { return peak_slots_; }
  int batches() const { return batches_; }
  int peak_concurrent_batches() const { return peak_ctx_; }

 private:
  bool any_busy() const {
    for (bool b : ctx_busy_)
      if (b) return true;
    return false;
  }

  void finish(J* j, int32_t state, int32_t err) {
    j->state = state;
    j->err = err;
    j->t_done = now_ns();
    if (j->arena_off >= 0) {
      arena_.release((uint64_t)j->arena_off, j->bytes);
      j->arena_off = -1;
      --slots_used_;
    }
    --outstanding_;
  }

  // One scheduling round; returns true if a batch is in flight.  Entered and
  // left with the lock held, which is released around every executor call
  // (event queries, table uploads, graph launches can take a while and must
  // not hold up submit / poll).  One round runs at a time (in_round_, taken
  // under the lock by the scheduler thread or by a submit that finds the
  // scheduler idle): only the round touches the contexts, the pending list
  // and the arena; a job's request and arena range do not change while it
  // runs, and poll never frees a running job.
  bool round(std::unique_lock<std::mutex>& lk) {
    // 1. retire finished batches
    std::vector<int> busy, status;
    for (size_t c = 0; c < ctx_busy_.size(); ++c)
      if (ctx_busy_[c]) busy.push_back((int)c);
    if (!busy.empty()) {
      status.resize(busy.size());
      lk.unlock();
      for (size_t k = 0; k < busy.size(); ++k) status[k] = ex_->query(busy[k]);
      lk.lock();
      for (size_t k = 0; k < busy.size(); ++k) {
        const int c = busy[k], q = status[k];
        if (q == 0) continue;
        for (J* j : ctx_jobs_[c]) finish(j, q > 0 ? INTERP_DONE : INTERP_FAILED, q > 0 ? INTERP_OK : q);
        ctx_jobs_[c].clear();
        ctx_busy_[c] = false;
      }
    }
    // 2. admit in arrival order while a slot and arena space are free
    while (!queue_.empty() && slots_used_ < max_slots_) {
      J* j = queue_.front();
      const int64_t off = arena_.alloc(j->bytes);
      if (off < 0) break;
      queue_.pop_front();
      j->arena_off = off;
      j->state = INTERP_RUNNING;
      j->t_admit = now_ns();
      ++slots_used_;
      pending_.push_back(j);
    }
    if (arena_.used() > peak_arena_) peak_arena_ = arena_.used();
    if (slots_used_ > peak_slots_) peak_slots_ = slots_used_;
    // 3. launch the admitted jobs as batches on free contexts, shared evenly
    // among them: a burst then runs as concurrent batches whose phases
    // overlap on the device, rather than as one large batch whose every
    // phase waits for the slowest of its jobs
    std::vector<int> go;
    size_t nfree = 0;
    for (bool b : ctx_busy_) nfree += !b;
    while (!pending_.empty() && nfree > 0) {
      int c = -1;
      for (size_t k = 0; k < ctx_busy_.size(); ++k)
        if (!ctx_busy_[k]) { c = (int)k; break; }
      const size_t n = std::min({pending_.size(), (size_t)ex_->max_batch(),
                                 (pending_.size() + nfree - 1) / nfree});
      --nfree;
      ctx_jobs_[c].assign(pending_.begin(), pending_.begin() + n);
      pending_.erase(pending_.begin(), pending_.begin() + n);
      ctx_busy_[c] = true;
      go.push_back(c);
    }
    if (!go.empty()) {
      std::vector<int> rc(go.size());
      lk.unlock();
      for (size_t k = 0; k < go.size(); ++k) rc[k] = ex_->launch(go[k], ctx_jobs_[go[k]]);
      lk.lock();
      for (size_t k = 0; k < go.size(); ++k) {
        const int c = go[k];
        if (rc[k] == INTERP_OK) {
          ++batches_;
          continue;
        }
        for (J* j : ctx_jobs_[c]) finish(j, INTERP_FAILED, rc[k]);
        ctx_jobs_[c].clear();
        ctx_busy_[c] = false;
      }
    }
    int nbusy = 0;
    for (bool b : ctx_busy_) nbusy += b;
    if (nbusy > peak_ctx_) peak_ctx_ = nbusy;
    return nbusy > 0;
  }

  void loop() {
    ex_->thread_init();
    std::unique_lock<std::mutex> lk(mu_);
    while (true) {
      if (in_round_) {  // a submit runs a round on its own thread: let it finish
        lk.unlock();
        std::this_thread::yield();
        lk.lock();
        continue;
      }
      in_round_ = true;
      const bool busy = round(lk);
      in_round_ = false;
      if (outstanding_ == 0) done_cv_.notify_all();
      if (stop_) break;
      if (busy) {
        // a batch is on the device: poll its completion again at once (a
        // timed wait would sleep for the timer's slack, tens of microseconds,
        // which small requests would see as latency); the lock is dropped
        // so that submit and poll get in between rounds
        lk.unlock();
        std::this_thread::yield();
        lk.lock();
      } else {
        cv_.wait_for(lk, std::chrono::milliseconds(2), [this] {
          return stop_ || !queue_.empty() || !pending_.empty() || any_busy();
        });
      }
    }
    // shutdown: fail what never started, finish what runs
    while (!queue_.empty()) {
      finish(queue_.front(), INTERP_FAILED, INTERP_EAGAIN);
      queue_.pop_front();
    }
    for (J* j : pending_) finish(j, INTERP_FAILED, INTERP_EAGAIN);
    pending_.clear();
    for (size_t c = 0; c < ctx_busy_.size(); ++c) {
      if (!ctx_busy_[c]) continue;
      lk.unlock();
      ex_->wait((int)c);
      const int q = ex_->query((int)c);
      lk.lock();
      for (J* j : ctx_jobs_[c]) finish(j, q > 0 ? INTERP_DONE : INTERP_FAILED, q > 0 ? INTERP_OK : q);
      ctx_jobs_[c].clear();
      ctx_busy_[c] = false;
    }
    done_cv_.notify_all();
  }

  Exec* ex_;
  Arena arena_;
  const int max_slots_, max_queue_;
  std::mutex mu_;
  std::condition_variable cv_, done_cv_;
  std::deque<J*> queue_;
  std::vector<J*> pending_;
  std::unordered_map<uint64_t, std::unique_ptr<J>> jobs_;
  std::vector<bool> ctx_busy_;
  std::vector<std::vector<J*>> ctx_jobs_;
  uint64_t next_ticket_ = 0;
  int slots_used_ = 0;
  int64_t outstanding_ = 0;
  bool stop_ = false;
  bool in_round_ = false;
  uint64_t peak_arena_ = 0;
  int peak_slots_ = 0, batches_ = 0, peak_ctx_ = 0;
  std::thread thread_;
};

}  // namespace serve
}  // namespace gmm
