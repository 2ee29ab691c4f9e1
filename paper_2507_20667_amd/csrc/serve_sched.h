// Serve scheduler: a request queue, admission by device footprint, batching
// of requests on one plan, and the worker loop (continuous batching).  Plain
// C++ (no HIP): the device side comes in through Backend, so the CPU tests run
// this same code with a fake backend that models footprints and durations.
//
// Admission follows the memory model of Section 3.1: a request is admitted
// when the workspace of its batch fits the free arena now.  Each idle worker
// walks the queue in arrival order, plan by plan (first appearance), and takes
// the first plan whose requests fit, as many of them as fit (halving the batch
// until the reservation succeeds); requests of other plans behind a request
// that does not fit yet are not held up, until the oldest request has waited
// `age_ms`: then only its plan is admitted.  When nothing fits, the worker waits
// for memory to come back (a batch ending, or any release in the arena; the
// arena is also used by synchronous calls, which do not signal, so the wait
// is bounded and polls).  A request fails with TN_E_NOMEM only when its
// workspace alone exceeds what transient allocations could ever hold (the
// arena minus persistent plan data), or when it has not fit for `stall_ms`
// while no serve batch was running.
//
// A batch that fails as a whole is run again request by request, so that a
// failure stays with the request that causes it.  stop() cancels every queued
// request (TN_E_CANCELLED), lets running batches finish and joins the
// workers.
#pragma once

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

namespace tn {
namespace sched {

// status values (the same as include/tn.h)
enum : int32_t {
  kOk = 0,
  kPending = 1,
  kNoMem = -3,
  kAgain = -5,
  kCancelled = -6,
  kUnknown = -7
};

typedef std::chrono::steady_clock clk;

struct Req {
  uint64_t ticket = 0;
  const void *plan = nullptr;   // requests with the same plan batch together
  int32_t status = kPending;
  clk::time_point submitted, finished;
  virtual ~Req() {}
};

class Backend {
 public:
  virtual ~Backend() {}
  // workspace bytes of a batch made of the first n requests of `batch`
  virtual size_t footprint(const std::vector<Req *> &batch, size_t n) = 0;
  // arena reservation (offset, or -1 when it does not fit now) and release
  virtual int64_t reserve(size_t bytes) = 0;
  virtual void release(int64_t off, size_t bytes) = 0;
  // bytes transient reservations could ever hold at once
  virtual size_t capacity() = 0;
  // releases seen so far in the arena (any user): a change means memory came back
  virtual uint64_t releases() = 0;
  // per-worker resources (streams, staging), created and destroyed on the worker
  virtual void *worker_begin() = 0;
  virtual void worker_end(void *w) = 0;
  // run a batch in the reserved workspace, without the scheduler's lock:
  // writes each request's result into the request and its status into st,
  // or returns an error for the batch as a whole (st then ignored).  The
  // scheduler publishes the statuses under its lock afterwards.
  virtual int32_t run(void *w, const std::vector<Req *> &batch, int64_t ws, size_t bytes,
                      std::vector<int32_t> &st) = 0;
};

struct Options {
  int workers = 2;
  size_t max_queue = 65536;
  size_t max_batch = 4096;
  int wait_ms = 2;       // bounded wait while nothing fits
  int age_ms = 500;      // a head request older than this is admitted before anything else
  int stall_ms = 2000;   // fits in principle, but not for this long with the serve side idle
};

class Scheduler {
 public:
  Scheduler(Backend *b, const Options &o) : b_(b), opt_(o) {
    for (int i = 0; i < std::max(1, opt_.workers); ++i) th_.emplace_back([this] { worker(); });
  }
  ~Scheduler() { stop(); }

  // takes ownership of r on success; kAgain (queue full, r not taken) otherwise
  int32_t submit(Req *r, uint64_t *ticket) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (stopped_ || queue_.size() >= opt_.max_queue) return kAgain;
      r->ticket = next_++;
      r->status = kPending;
      r->submitted = clk::now();
      reqs_[r->ticket] = r;
      queue_.push_back(r);
      *ticket = r->ticket;
    }
    cv_.notify_one();
    return kOk;
  }

  // kUnknown, kPending, or the final status; with a final status the request
  // is handed to f (under the lock) and then deleted: the ticket is consumed
  template <typename F>
  int32_t take(uint64_t ticket, F &&f) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return kUnknown;
    Req *r = it->second;
    if (r->status == kPending) return kPending;
    const int32_t st = f(r);
    if (st == kPending) return st;  // f refused (bad arguments): keep it
    reqs_.erase(it);
    delete r;
    return st;
  }

  int pending_on(const void *plan) {
    std::lock_guard<std::mutex> lk(mu_);
    int n = 0;
    for (auto &kv : reqs_)
      if (kv.second->plan == plan && kv.second->status == kPending) ++n;
    return n;
  }

  size_t queued() {
    std::lock_guard<std::mutex> lk(mu_);
    return queue_.size();
  }

  // cancel what is queued, let running batches finish, join the workers
  void stop() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (stopped_ && th_.empty()) return;
      stopped_ = true;
      const clk::time_point now = clk::now();
      for (Req *r : queue_) {
        r->status = kCancelled;
        r->finished = now;
      }
      queue_.clear();
    }
    cv_.notify_all();
    for (std::thread &t : th_) t.join();
    th_.clear();
  }

  // requests not yet consumed are deleted with the scheduler
  void drop_all() {
    std::lock_guard<std::mutex> lk(mu_);
    for (auto &kv : reqs_) delete kv.second;
    reqs_.clear();
  }

 private:
  // under mu_: pick a batch that fits now and reserve its workspace
  bool pick(std::vector<Req *> &batch, int64_t &ws, size_t &bytes) {
    std::vector<const void *> seen;
    const size_t cap = b_->capacity();
    // aging: once the oldest request has waited age_ms, only its plan is
    // considered, so that smaller requests cannot keep it out for ever
    const bool aged = !queue_.empty() &&
                      clk::now() - queue_.front()->submitted > std::chrono::milliseconds(opt_.age_ms);
    for (size_t i = 0; i < queue_.size();) {
      const void *plan = queue_[i]->plan;
      if (aged && plan != queue_.front()->plan) {
        ++i;
        continue;
      }
      if (std::find(seen.begin(), seen.end(), plan) != seen.end()) {
        ++i;
        continue;
      }
      seen.push_back(plan);
      std::vector<Req *> cand;
      for (Req *r : queue_)
        if (r->plan == plan && cand.size() < opt_.max_batch) cand.push_back(r);
      // a request that can never fit fails now, alone
      if (b_->footprint(cand, 1) > cap) {
        fail(cand[0], kNoMem);
        seen.pop_back();
        i = 0;
        continue;
      }
      for (size_t n = cand.size(); n > 0; n /= 2) {
        const size_t need = b_->footprint(cand, n);
        if (need > cap) continue;
        const int64_t off = b_->reserve(need);
        if (off >= 0) {
          cand.resize(n);
          batch.swap(cand);
          ws = off;
          bytes = need;
          return true;
        }
      }
      ++i;
    }
    return false;
  }

  void fail(Req *r, int32_t st) {
    queue_.erase(std::find(queue_.begin(), queue_.end(), r));
    r->status = st;
    r->finished = clk::now();
  }

  void worker() {
    void *w = b_->worker_begin();
    std::unique_lock<std::mutex> lk(mu_);
    clk::time_point blocked_since;
    bool blocked = false;
    while (true) {
      if (stopped_) break;
      if (queue_.empty()) {
        blocked = false;
        cv_.wait(lk, [&] { return stopped_ || !queue_.empty(); });
        continue;
      }
      std::vector<Req *> batch;
      int64_t ws = -1;
      size_t bytes = 0;
      if (!pick(batch, ws, bytes)) {
        const clk::time_point now = clk::now();
        if (!blocked || running_ > 0) {
          blocked = true;
          blocked_since = now;
        } else if (now - blocked_since > std::chrono::milliseconds(opt_.stall_ms) && !queue_.empty()) {
          // nothing of ours runs and the head still does not fit: give up on it
          fail(queue_.front(), kNoMem);
          blocked = false;
          continue;
        }
        // a short bounded wait; against the system clock, whose timed wait
        // (pthread_cond_timedwait) thread sanitizers follow, unlike the
        // steady clock's
        const uint64_t seen = b_->releases();
        cv_.wait_until(lk, std::chrono::system_clock::now() + std::chrono::milliseconds(opt_.wait_ms),
                       [&] { return stopped_ || b_->releases() != seen; });
        continue;
      }
      blocked = false;
      for (Req *r : batch) queue_.erase(std::find(queue_.begin(), queue_.end(), r));
      ++running_;
      lk.unlock();
      std::vector<int32_t> st(batch.size(), kOk);
      const int32_t rc = b_->run(w, batch, ws, bytes, st);
      if (rc < 0 && batch.size() > 1) {
        // isolate the failure: each request alone, in the same workspace
        // when its own footprint fits there
        for (size_t i = 0; i < batch.size(); ++i) {
          std::vector<Req *> one{batch[i]};
          std::vector<int32_t> s1(1, kOk);
          const int32_t e = b_->footprint(one, 1) <= bytes ? b_->run(w, one, ws, bytes, s1) : rc;
          st[i] = e < 0 ? e : s1[0];
        }
      } else if (rc < 0) {
        st[0] = rc;
      }
      b_->release(ws, bytes);
      lk.lock();
      const clk::time_point now = clk::now();
      for (size_t i = 0; i < batch.size(); ++i) {
        batch[i]->status = st[i];
        batch[i]->finished = now;
      }
      --running_;
      cv_.notify_all();
    }
    lk.unlock();
    b_->worker_end(w);
  }

  Backend *b_;
  Options opt_;
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<Req *> queue_;
  std::unordered_map<uint64_t, Req *> reqs_;
  std::vector<std::thread> th_;
  uint64_t next_ = 1;
  int running_ = 0;
  bool stopped_ = false;
};

}  // namespace sched
}  // namespace tn
