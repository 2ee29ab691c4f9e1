// CPU tests of the serve scheduler (paper_2507_20667_amd/csrc/serve_sched.h) with a
// fake backend: footprints of (fixed + per-request) bytes in a real Arena over
// a fake range, durations as sleeps, optional gates that hold a batch, and
// requests marked to fail.  Built and run by tests/test_sched.py, also under
// ThreadSanitizer and AddressSanitizer.  Prints one line per case and exits
// non-zero on the first failed check.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "arena.h"
#include "serve_sched.h"

using namespace tn;
using sched::Req;

#define CHECK(c)                                                               \
  do {                                                                         \
    if (!(c)) {                                                                \
      fprintf(stderr, "FAILED %s:%d: %s\n", __FILE__, __LINE__, #c);          \
      exit(1);                                                                 \
    }                                                                          \
  } while (0)

struct FakePlan {
  size_t fixed, perq;
  int us;  // run time of a batch: us * (1 + n / 8)
};

struct FakeReq : Req {
  const FakePlan *fp = nullptr;
  bool poison = false;   // the batch holding it fails, and so does it alone
  int value = 0;         // "result": written by run
  int input = 0;
};

class Gate {
 public:
  void close() {
    std::lock_guard<std::mutex> g(mu_);
    open_ = false;
  }
  void open() {
    {
      std::lock_guard<std::mutex> g(mu_);
      open_ = true;
    }
    cv_.notify_all();
  }
  void pass() {
    std::unique_lock<std::mutex> lk(mu_);
    ++waiting_;
    cv_.notify_all();
    cv_.wait(lk, [&] { return open_; });
    --waiting_;
  }
  void wait_for_waiters(int n) {
    std::unique_lock<std::mutex> lk(mu_);
    cv_.wait(lk, [&] { return waiting_ >= n; });
  }

 private:
  std::mutex mu_;
  std::condition_variable cv_;
  bool open_ = true;
  int waiting_ = 0;
};

class FakeBackend : public sched::Backend {
 public:
  explicit FakeBackend(size_t cap) { arena.init(nullptr, cap); }
  size_t footprint(const std::vector<Req *> &b, size_t n) override {
    const FakePlan *fp = static_cast<FakeReq *>(b[0])->fp;
    return Arena::round(fp->fixed + n * fp->perq);
  }
  int64_t reserve(size_t bytes) override {
    const int64_t off = arena.alloc(bytes);
    if (off >= 0) {
      const size_t now = (in_use += bytes);
      size_t m = peak.load();
      while (now > m && !peak.compare_exchange_weak(m, now)) {
      }
    }
    return off;
  }
  void release(int64_t off, size_t bytes) override {
    in_use -= bytes;
    arena.release(off, bytes);
  }
  size_t capacity() override { return arena.work_capacity(); }
  uint64_t releases() override { return arena.releases(); }
  void *worker_begin() override { return new int(0); }
  void worker_end(void *w) override { delete static_cast<int *>(w); }
  int32_t run(void *, const std::vector<Req *> &b, int64_t ws, size_t bytes,
              std::vector<int32_t> &st) override {
    CHECK(ws >= 0 && (size_t)ws + bytes <= arena.bytes());
    CHECK(footprint(b, b.size()) <= bytes);
    if (gate) gate->pass();
    const FakePlan *fp = static_cast<FakeReq *>(b[0])->fp;
    std::this_thread::sleep_for(std::chrono::microseconds(fp->us * (1 + (int)b.size() / 8)));
    batches++;
    if (b.size() > 1) multi++;
    for (Req *r : b) {
      CHECK(static_cast<FakeReq *>(r)->fp == fp);
      if (static_cast<FakeReq *>(r)->poison) return -4;
    }
    for (size_t i = 0; i < b.size(); ++i) {
      FakeReq *r = static_cast<FakeReq *>(b[i]);
      r->value = 2 * r->input + 1;
      st[i] = sched::kOk;
    }
    return sched::kOk;
  }
  Arena arena;
  Gate *gate = nullptr;
  std::atomic<size_t> in_use{0}, peak{0};
  std::atomic<int> batches{0}, multi{0};
};

static int32_t wait_result(sched::Scheduler &s, uint64_t t, int *value, double timeout_s = 20.0) {
  const auto t0 = std::chrono::steady_clock::now();
  while (true) {
    int v = 0;
    const int32_t st = s.take(t, [&](Req *r) {
      v = static_cast<FakeReq *>(r)->value;
      return r->status;
    });
    if (st != sched::kPending) {
      if (value) *value = v;
      return st;
    }
    CHECK(std::chrono::steady_clock::now() - t0 < std::chrono::duration<double>(timeout_s));
    std::this_thread::sleep_for(std::chrono::microseconds(100));
  }
}

static FakeReq *mk(const FakePlan *fp, int input, bool poison = false) {
  FakeReq *r = new FakeReq;
  r->fp = fp;
  r->plan = fp;
  r->input = input;
  r->poison = poison;
  return r;
}

// Many requests on three plans from two submitting threads: every result is
// right, reservations never exceed the arena, requests batch together.
static void test_mix() {
  FakeBackend b(1 << 20);
  sched::Options o;
  o.workers = 4;
  sched::Scheduler s(&b, o);
  const FakePlan plans[3] = {{4096, 20000, 300}, {1024, 100000, 200}, {65536, 4096, 100}};
  const int N = 600;
  std::vector<uint64_t> tickets(N);
  std::vector<int> which(N);
  auto submitter = [&](int lo, int hi, unsigned seed) {
    std::mt19937 rng(seed);
    for (int i = lo; i < hi; ++i) {
      which[i] = (int)(rng() % 3);
      CHECK(s.submit(mk(&plans[which[i]], i), &tickets[i]) == sched::kOk);
      if (rng() % 4 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 300));
    }
  };
  std::thread t1(submitter, 0, N / 2, 1u), t2(submitter, N / 2, N, 2u);
  t1.join();
  t2.join();
  for (int i = 0; i < N; ++i) {
    int v = -1;
    CHECK(wait_result(s, tickets[i], &v) == sched::kOk);
    CHECK(v == 2 * i + 1);
  }
  s.stop();
  CHECK(b.peak.load() <= b.arena.bytes());
  CHECK(b.in_use.load() == 0 && b.arena.used() == 0);
  CHECK(b.multi.load() > 0);
  printf("mix: %d requests in %d batches (%d of several), peak reservation %zu of %zu bytes\n", N,
         b.batches.load(), b.multi.load(), b.peak.load(), b.arena.bytes());
}

// A full queue answers kAgain; the accepted requests still complete.
static void test_bounded_queue() {
  FakeBackend b(1 << 20);
  Gate gate;
  gate.close();
  b.gate = &gate;
  sched::Options o;
  o.workers = 1;
  o.max_queue = 8;
  o.max_batch = 1;
  sched::Scheduler s(&b, o);
  const FakePlan fp{0, 1024, 10};
  std::vector<uint64_t> ok;
  uint64_t t;
  CHECK(s.submit(mk(&fp, 0), &t) == sched::kOk);  // taken by the worker, held at the gate
  ok.push_back(t);
  gate.wait_for_waiters(1);
  int again = 0;
  for (int i = 1; i < 20; ++i) {
    FakeReq *r = mk(&fp, i);
    if (s.submit(r, &t) == sched::kOk) {
      ok.push_back(t);
    } else {
      delete r;
      ++again;
    }
  }
  CHECK(ok.size() == 9 && again == 11);
  gate.open();
  for (uint64_t tk : ok) CHECK(wait_result(s, tk, nullptr) == sched::kOk);
  CHECK(s.take(ok[0], [](Req *r) { return r->status; }) == sched::kUnknown);  // consumed
  printf("bounded queue: 9 accepted, 11 refused with kAgain, all accepted completed\n");
}

// stop() while a batch runs: the running batch completes, the queued requests
// end cancelled, and nothing is admitted afterwards.
static void test_cancel_on_stop() {
  FakeBackend b(1 << 20);
  Gate gate;
  gate.close();
  b.gate = &gate;
  sched::Options o;
  o.workers = 1;
  o.max_batch = 1;
  sched::Scheduler s(&b, o);
  const FakePlan fp{0, 1024, 10};
  uint64_t t0, t;
  CHECK(s.submit(mk(&fp, 0), &t0) == sched::kOk);
  gate.wait_for_waiters(1);
  std::vector<uint64_t> queued;
  for (int i = 1; i <= 5; ++i) {
    CHECK(s.submit(mk(&fp, i), &t) == sched::kOk);
    queued.push_back(t);
  }
  std::thread opener([&] {
    std::this_thread::sleep_for(std::chrono::milliseconds(50));
    gate.open();
  });
  s.stop();
  opener.join();
  int v = 0;
  CHECK(wait_result(s, t0, &v) == sched::kOk && v == 1);
  for (uint64_t tk : queued) CHECK(wait_result(s, tk, nullptr) == sched::kCancelled);
  FakeReq *late = mk(&fp, 9);
  CHECK(s.submit(late, &t) == sched::kAgain);
  delete late;
  printf("cancel on stop: running batch completed, 5 queued requests cancelled\n");
}

// A batch with one failing request: that request fails, the others succeed.
static void test_failure_isolated() {
  FakeBackend b(1 << 20);
  Gate gate;
  gate.close();
  b.gate = &gate;
  sched::Options o;
  o.workers = 1;
  sched::Scheduler s(&b, o);
  const FakePlan other{0, 512, 10}, fp{0, 1024, 10};
  uint64_t th, t;
  CHECK(s.submit(mk(&other, 0), &th) == sched::kOk);  // holds the worker
  gate.wait_for_waiters(1);
  std::vector<uint64_t> tk;
  for (int i = 0; i < 8; ++i) {
    CHECK(s.submit(mk(&fp, i, i == 5), &t) == sched::kOk);
    tk.push_back(t);
  }
  gate.open();
  CHECK(wait_result(s, th, nullptr) == sched::kOk);
  for (int i = 0; i < 8; ++i) {
    int v = 0;
    const int32_t st = wait_result(s, tk[i], &v);
    if (i == 5) {
      CHECK(st == -4);
    } else {
      CHECK(st == sched::kOk && v == 2 * i + 1);
    }
  }
  printf("failure isolated: 1 of 8 batched requests failed alone\n");
}

// A request larger than the arena fails with kNoMem at once; others run.
static void test_never_fits() {
  FakeBackend b(1 << 20);
  sched::Options o;
  sched::Scheduler s(&b, o);
  const FakePlan big{0, 2 << 20, 10}, small{0, 1024, 10};
  uint64_t tb, ts;
  CHECK(s.submit(mk(&big, 0), &tb) == sched::kOk);
  CHECK(s.submit(mk(&small, 1), &ts) == sched::kOk);
  CHECK(wait_result(s, tb, nullptr) == sched::kNoMem);
  CHECK(wait_result(s, ts, nullptr) == sched::kOk);
  // persistent data counts: what is left for workspaces decides
  const int64_t pers = b.arena.alloc(600 << 10, true);
  CHECK(pers >= 0);
  const FakePlan mid{0, 512 << 10, 10};
  CHECK(s.submit(mk(&mid, 2), &tb) == sched::kOk);
  CHECK(wait_result(s, tb, nullptr) == sched::kNoMem);
  b.arena.release(pers, 600 << 10, true);
  CHECK(s.submit(mk(&mid, 3), &tb) == sched::kOk);
  CHECK(wait_result(s, tb, nullptr) == sched::kOk);
  printf("never fits: kNoMem for a request above the arena and above the arena minus persistent data\n");
}

// No head-of-line blocking: a request that cannot fit while another batch
// holds memory does not keep a later, smaller request of another plan out;
// it runs once the memory comes back.
static void test_no_head_of_line_blocking() {
  FakeBackend b(1 << 20);
  Gate gate;
  gate.close();
  b.gate = &gate;
  sched::Options o;
  o.workers = 2;
  o.age_ms = 60000;
  sched::Scheduler s(&b, o);
  const FakePlan holder{0, 600 << 10, 10}, big{0, 700 << 10, 10}, small{0, 64 << 10, 10};
  uint64_t th, tb, tsm;
  CHECK(s.submit(mk(&holder, 0), &th) == sched::kOk);
  gate.wait_for_waiters(1);
  CHECK(s.submit(mk(&big, 1), &tb) == sched::kOk);
  CHECK(s.submit(mk(&small, 2), &tsm) == sched::kOk);
  // the small request passes the waiting big one and reaches the gate
  gate.wait_for_waiters(2);
  CHECK(s.queued() == 1);
  gate.open();
  CHECK(wait_result(s, tsm, nullptr) == sched::kOk);
  CHECK(wait_result(s, th, nullptr) == sched::kOk);
  CHECK(wait_result(s, tb, nullptr) == sched::kOk);
  printf("no head-of-line blocking: a small request ran while a large one waited for memory\n");
}

// Memory released by someone else (a synchronous call on the same arena)
// admits a waiting request without any batch ending.
static void test_external_release() {
  FakeBackend b(1 << 20);
  sched::Options o;
  o.workers = 1;
  sched::Scheduler s(&b, o);
  const int64_t ext = b.arena.alloc(900 << 10);
  CHECK(ext >= 0);
  const FakePlan fp{0, 512 << 10, 10};
  uint64_t t;
  CHECK(s.submit(mk(&fp, 0), &t) == sched::kOk);
  std::this_thread::sleep_for(std::chrono::milliseconds(30));
  CHECK(s.queued() == 1);
  b.arena.release(ext, 900 << 10);
  CHECK(wait_result(s, t, nullptr) == sched::kOk);
  printf("external release: a waiting request ran once another user freed memory\n");
}

// A request that fits in principle but not for stall_ms with nothing of the
// scheduler's own running ends with kNoMem instead of waiting for ever.
static void test_stall_limit() {
  FakeBackend b(1 << 20);
  sched::Options o;
  o.workers = 1;
  o.stall_ms = 50;
  sched::Scheduler s(&b, o);
  const int64_t ext = b.arena.alloc(900 << 10);
  const FakePlan fp{0, 512 << 10, 10}, small{0, 1024, 10};
  uint64_t t, ts;
  CHECK(s.submit(mk(&fp, 0), &t) == sched::kOk);
  CHECK(s.submit(mk(&small, 1), &ts) == sched::kOk);
  CHECK(wait_result(s, ts, nullptr) == sched::kOk);
  CHECK(wait_result(s, t, nullptr) == sched::kNoMem);
  b.arena.release(ext, 900 << 10);
  printf("stall limit: kNoMem after the limit with the scheduler idle\n");
}

int main() {
  test_mix();
  test_bounded_queue();
  test_cancel_on_stop();
  test_failure_isolated();
  test_never_fits();
  test_no_head_of_line_blocking();
  test_external_release();
  test_stall_limit();
  printf("ALL PASSED\n");
  return 0;
}
