// Host test of the scoring server's scheduler (srv_core.hpp) with a simulated executor:
// no GPU.  tests/test_host_sanitized.py builds it with the address and
// undefined-behaviour sanitizers and again with the thread sanitizer, and runs it.
//
// The simulated executor checks, at every dispatch, what the scheduler promises:
// admitted regions lie inside the arena and never overlap the regions in flight;
// a region covers the footprint of what runs in it; the head of every launch is the
// oldest request not yet admitted (arrival order, so no request is overtaken forever);
// groups hold 2..max_batch small scoring requests.  Failures are injected at dispatch
// (a request that cannot start) and at completion (device flags), and the waiters
// check every outcome against what was injected.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <thread>
#include <vector>

#include "srv_core.hpp"

#ifdef SIM_TSAN_CLOCKWAIT
#include <pthread.h>
#include <time.h>
// This toolchain's thread sanitizer does not intercept pthread_cond_clockwait, which
// libstdc++ uses for timed waits on the steady clock, so it would miss the unlock inside
// those waits and report false races.  The thread-sanitizer build routes them through
// pthread_cond_timedwait (same deadline, measured on the realtime clock), which it sees.
extern "C" int pthread_cond_clockwait(pthread_cond_t* cond, pthread_mutex_t* mutex, clockid_t clock,
                                      const struct timespec* abstime) {
  struct timespec now_c, now_r;
  clock_gettime(clock, &now_c);
  clock_gettime(CLOCK_REALTIME, &now_r);
  long long rem = (long long)(abstime->tv_sec - now_c.tv_sec) * 1000000000LL + (abstime->tv_nsec - now_c.tv_nsec);
  if (rem < 0) rem = 0;
  const long long t = (long long)now_r.tv_sec * 1000000000LL + now_r.tv_nsec + rem;
  struct timespec abs_r;
  abs_r.tv_sec = (time_t)(t / 1000000000LL);
  abs_r.tv_nsec = (long)(t % 1000000000LL);
  return pthread_cond_timedwait(cond, mutex, &abs_r);
}
#endif

#define CHECK(c)                                                               \
  do {                                                                         \
    if (!(c)) {                                                                \
      std::fprintf(stderr, "CHECK failed at %s:%d: %s\n", __FILE__, __LINE__, #c); \
      std::abort();                                                            \
    }                                                                          \
  } while (0)

using cqsrv::aup;
using cqsrv::Clock;
using cqsrv::Req;

// Footprints restated from their definitions (labels, workspace, result; a group adds the
// item list of 16 bytes per label id), independent of the scheduler's helpers.
static size_t foot_alone(const Req& r) {
  const size_t lab = (r.kind == 0 ? 1 : 2) * aup(4 * (size_t)r.n);
  const size_t res = r.kind == 0 ? sizeof(cq_score_result) : sizeof(cq_compare_result);
  return lab + aup(r.ws_bytes) + aup(res);
}
static size_t foot_group(const std::vector<Req*>& g) {
  size_t lab = 0, ws = 0, items = 0;
  for (const Req* r : g) {
    lab += aup(4 * (size_t)r->n);
    ws += aup(r->group_ws);
    items += 16 * (size_t)r->L;
  }
  return lab + aup(ws + aup(items)) + aup(sizeof(cq_score_result) * g.size());
}

// Injected failures, by ticket (tickets are 1, 2, 3, ... in submission order).
static bool fails_at_dispatch(uint64_t id) { return id % 97 == 5; }
static bool fails_on_device(uint64_t id) { return id % 89 == 7; }

class SimExec final : public cqsrv::Executor {
 public:
  SimExec(int slots, size_t cap, int max_batch, unsigned seed) : runs_(slots), cap_(cap), max_batch_(max_batch), rng_(seed) {}

  void dispatch(int slot, const std::vector<Req*>& reqs, bool grouped, size_t off, size_t len) override {
    std::lock_guard<std::mutex> lk(mu_);
    Run& run = runs_[slot];
    CHECK(!run.busy);
    CHECK(off % cqsrv::kAlign == 0);
    CHECK(off + aup(len) <= cap_);
    for (const Run& o : runs_)
      if (o.busy) CHECK(off + aup(len) <= o.off || o.off + aup(o.len) <= off);
    CHECK(!reqs.empty());
    if (grouped) {
      CHECK(reqs.size() >= 2 && (int)reqs.size() <= max_batch_);
      for (const Req* r : reqs) CHECK(r->small && r->kind == 0);
      CHECK(len >= foot_group(reqs));
    } else {
      CHECK(reqs.size() == 1);
      CHECK(len >= foot_alone(*reqs[0]));
    }
    // arrival order: the head is the oldest request not yet admitted
    CHECK(reqs[0]->id == next_expected_);
    for (size_t i = 1; i < reqs.size(); ++i) CHECK(reqs[i]->id > reqs[0]->id);
    double us = 0;
    for (Req* r : reqs) {
      CHECK(admitted_.insert(r->id).second);
      us += 5.0 + (double)r->n / 2000.0;
      if (fails_at_dispatch(r->id)) r->status = CQ_E_DEVICE;
    }
    while (admitted_.count(next_expected_)) ++next_expected_;
    us += std::uniform_real_distribution<double>(0.0, 50.0)(rng_) + extra_us_;
    run.busy = true;
    run.off = off;
    run.len = len;
    run.end = Clock::now() + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double, std::micro>(us));
    ++launches_;
  }

  bool finished(int slot) override {
    std::lock_guard<std::mutex> lk(mu_);
    return Clock::now() >= runs_[slot].end;
  }

  void collect(int slot, const std::vector<Req*>& reqs, bool) override {
    std::lock_guard<std::mutex> lk(mu_);
    CHECK(runs_[slot].busy);
    runs_[slot].busy = false;
    for (Req* r : reqs) {
      if (r->status != CQ_OK) continue;
      if (fails_on_device(r->id)) {
        r->status = CQ_E_LABEL_RANGE;
        continue;
      }
      if (r->kind == 0) {
        r->sres.n = r->n;
        r->sres.K = (int64_t)r->id;  // lets the waiter check it got its own result
      } else {
        r->cres.n = r->n;
        r->cres.nnz = (int64_t)r->id;
      }
    }
  }

  void set_extra_us(double us) {
    std::lock_guard<std::mutex> lk(mu_);
    extra_us_ = us;
  }
  int64_t launches() {
    std::lock_guard<std::mutex> lk(mu_);
    return launches_;
  }

 private:
  struct Run {
    bool busy = false;
    size_t off = 0, len = 0;
    Clock::time_point end{};
  };
  std::mutex mu_;
  std::vector<Run> runs_;
  size_t cap_;
  int max_batch_;
  std::mt19937_64 rng_;
  std::set<uint64_t> admitted_;
  uint64_t next_expected_ = 1;
  double extra_us_ = 0;
  int64_t launches_ = 0;
};

static const int32_t kDummyLabels[1] = {0};

static Req* make_req(std::mt19937_64& rng, size_t arena) {
  Req* r = new Req();
  std::uniform_real_distribution<double> u(0.0, 1.0);
  r->kind = u(rng) < 0.7 ? 0 : 1;
  r->n = (int32_t)(100 + (int64_t)(u(rng) * u(rng) * 400000));
  r->ha = kDummyLabels;
  r->hb = kDummyLabels;
  if (r->kind == 0) {
    r->L = 1 + (int32_t)(u(rng) * 5000);
    r->small = u(rng) < 0.6;
    r->ws_bytes = (size_t)(u(rng) * 3e6);
    // a few requests need most of the arena, so the head waits for memory
    if (u(rng) < 0.03) r->ws_bytes = arena / 2 + (size_t)(u(rng) * (double)arena / 3);
    r->group_ws = r->ws_bytes / 2 + 1000;
  } else {
    r->La = 1 + (int32_t)(u(rng) * 3000);
    r->Lb = 1 + (int32_t)(u(rng) * 3000);
    r->ws_bytes = (size_t)(u(rng) * 2e6);
  }
  return r;
}

// Many requests from several submitting threads, several waiting threads.
static void test_mixed_load() {
  const size_t arena = 48u << 20;
  const int slots = 4, max_batch = 8, total = 3000, submitters = 4, waiters = 4;
  SimExec ex(slots, arena, max_batch, 11);
  cqsrv::Config cfg;
  cfg.num_slots = slots;
  cfg.max_batch = max_batch;
  cfg.arena_bytes = arena;
  cqsrv::Scheduler s(cfg, &ex);
  s.start();
  std::vector<std::vector<std::pair<uint64_t, int>>> tickets(submitters);  // (ticket, kind)
  std::vector<std::thread> th;
  std::atomic<int> rejected{0};
  for (int t = 0; t < submitters; ++t)
    th.emplace_back([&, t] {
      std::mt19937_64 rng(100 + t);
      for (int i = 0; i < total / submitters; ++i) {
        Req* r = make_req(rng, arena);
        const int kind = r->kind;
        uint64_t tk = 0;
        const cq_status st = s.submit(r, &tk, nullptr);
        if (st == CQ_E_BUSY) {
          ++rejected;
          continue;
        }
        CHECK(st == CQ_OK);
        tickets[t].push_back({tk, kind});
        if (i % 64 == 0) std::this_thread::sleep_for(std::chrono::microseconds(200));
      }
    });
  for (auto& x : th) x.join();
  th.clear();
  std::atomic<int64_t> ok{0}, failed{0};
  for (int w = 0; w < waiters; ++w)
    th.emplace_back([&, w] {
      for (int t = 0; t < submitters; ++t)
        for (size_t i = w; i < tickets[t].size(); i += waiters) {
          const auto [tk, kind] = tickets[t][i];
          cqsrv::Outcome o;
          CHECK(s.wait(tk, -1.0, &o, nullptr) == CQ_OK);
          CHECK(o.kind == kind);
          CHECK(o.latency_ms >= 0.0);
          if (fails_at_dispatch(tk)) {
            CHECK(o.status == CQ_E_DEVICE);
            ++failed;
          } else if (fails_on_device(tk)) {
            CHECK(o.status == CQ_E_LABEL_RANGE);
            ++failed;
          } else {
            CHECK(o.status == CQ_OK);
            CHECK((kind == 0 ? o.sres.K : o.cres.nnz) == (int64_t)tk);
            ++ok;
          }
          // a released ticket is unknown
          CHECK(s.wait(tk, 0.0, nullptr, nullptr) == CQ_E_INVALID_ARG);
        }
    });
  for (auto& x : th) x.join();
  cq_server_stats st;
  s.stats(&st);
  CHECK(st.submitted == ok + failed);
  CHECK(st.completed == ok);
  CHECK(st.failed == failed);
  CHECK(st.rejected == rejected);
  CHECK(st.launches == ex.launches());
  CHECK(st.launches <= st.submitted);
  CHECK(st.grouped_requests > 0);
  CHECK(st.p50_ms <= st.p99_ms && st.p99_ms <= st.max_ms);
  CHECK(st.peak_bytes > 0 && (size_t)st.peak_bytes <= arena);
  CHECK(s.arena_in_use() == 0);
  CHECK(s.arena_free_blocks() == 1);
  s.shutdown();
  std::printf("mixed load: %lld ok, %lld failed, %d rejected, %lld launches, %lld grouped\n", (long long)ok.load(),
              (long long)failed.load(), rejected.load(), (long long)st.launches, (long long)st.grouped_requests);
}

// A request larger than the arena is refused at submit and never queued.
static void test_oversize() {
  SimExec ex(1, 1u << 20, 1, 3);
  cqsrv::Config cfg;
  cfg.arena_bytes = 1u << 20;
  cqsrv::Scheduler s(cfg, &ex);
  s.start();
  Req* r = new Req();
  r->n = 1000;
  r->ha = kDummyLabels;
  r->ws_bytes = 1u << 20;
  uint64_t tk = 0;
  const char* why = nullptr;
  CHECK(s.submit(r, &tk, &why) == CQ_E_BUSY);
  CHECK(why != nullptr);
  // exactly the arena fits
  r = new Req();
  r->n = 64;
  r->ha = kDummyLabels;
  r->ws_bytes = (1u << 20) - aup(256) - aup(sizeof(cq_score_result));
  CHECK(s.submit(r, &tk, nullptr) == CQ_OK);
  cqsrv::Outcome o;
  CHECK(s.wait(tk, -1.0, &o, nullptr) == CQ_OK);
  cq_server_stats st;
  s.stats(&st);
  CHECK(st.rejected == 1 && st.submitted == 1);
  CHECK((size_t)st.peak_bytes == (1u << 20));
  std::printf("oversize: ok\n");
}

// Timeouts, a second waiter, unknown tickets.
static void test_wait_rules() {
  SimExec ex(1, 16u << 20, 1, 5);
  ex.set_extra_us(60000.0);  // every launch takes about 60 ms
  cqsrv::Config cfg;
  cfg.arena_bytes = 16u << 20;
  cqsrv::Scheduler s(cfg, &ex);
  s.start();
  Req* r = new Req();
  r->n = 1000;
  r->ha = kDummyLabels;
  uint64_t tk = 0;
  CHECK(s.submit(r, &tk, nullptr) == CQ_OK);
  CHECK(s.wait(tk, 0.0, nullptr, nullptr) == CQ_E_BUSY);  // not finished yet; the ticket stays valid
  CHECK(s.wait(tk + 1000, 0.0, nullptr, nullptr) == CQ_E_INVALID_ARG);
  std::atomic<bool> got{false};
  std::thread w([&] {
    // the main thread's zero-timeout polls may hold the ticket for an instant
    for (int tries = 0;; ++tries) {
      cqsrv::Outcome o;
      const cq_status st = s.wait(tk, -1.0, &o, nullptr);
      if (st == CQ_OK) {
        CHECK(o.status == CQ_OK && o.latency_ms > 0.0);
        break;
      }
      CHECK(st == CQ_E_INVALID_ARG && tries < 1000);
      std::this_thread::sleep_for(std::chrono::microseconds(100));
    }
    got = true;
  });
  // within the launch's 60 ms, a second waiter on the same ticket is refused
  bool seen = false;
  for (int i = 0; i < 30 && !seen; ++i) {
    std::this_thread::sleep_for(std::chrono::milliseconds(1));
    const char* why = nullptr;
    const cq_status st = s.wait(tk, 0.0, nullptr, &why);
    CHECK(st == CQ_E_BUSY || st == CQ_E_INVALID_ARG);
    seen = st == CQ_E_INVALID_ARG;
  }
  CHECK(seen);
  w.join();
  CHECK(got);
  std::printf("wait rules: ok\n");
}

// Shutdown with queued requests and waiting threads: the admitted request finishes, the
// queued ones are cancelled, every waiter returns, later submits are refused.
static void test_shutdown() {
  SimExec ex(1, 16u << 20, 1, 7);
  ex.set_extra_us(50000.0);
  cqsrv::Config cfg;
  cfg.arena_bytes = 16u << 20;
  cqsrv::Scheduler s(cfg, &ex);
  s.start();
  const int nreq = 24;
  std::vector<uint64_t> tk(nreq);
  for (int i = 0; i < nreq; ++i) {
    Req* r = new Req();
    r->n = 1000;
    r->ha = kDummyLabels;
    CHECK(s.submit(r, &tk[i], nullptr) == CQ_OK);
  }
  std::atomic<int> done{0}, cancelled{0};
  std::vector<std::thread> th;
  for (int w = 0; w < 8; ++w)
    th.emplace_back([&, w] {
      for (int i = w; i < nreq; i += 8) {
        cqsrv::Outcome o;
        CHECK(s.wait(tk[i], -1.0, &o, nullptr) == CQ_OK);
        if (o.status == CQ_E_CANCELLED) ++cancelled;
        else CHECK(o.status == CQ_OK);
        ++done;
      }
    });
  std::this_thread::sleep_for(std::chrono::milliseconds(10));
  s.shutdown();
  for (auto& x : th) x.join();
  CHECK(done == nreq);
  CHECK(cancelled >= 1 && cancelled < nreq);
  Req* r = new Req();
  r->n = 10;
  r->ha = kDummyLabels;
  uint64_t t2 = 0;
  CHECK(s.submit(r, &t2, nullptr) == CQ_E_CANCELLED);
  std::printf("shutdown: %d finished, %d cancelled\n", nreq - cancelled.load(), cancelled.load());
}

// The arena against a byte-map model: first fit, no overlap, merging, accounting.
static void test_arena() {
  const size_t cap = 256 * 512;
  cqsrv::Arena a(cap + 100);  // capacity rounds down to whole 256-byte units
  std::vector<int> owner(cap / 256, -1);
  std::vector<std::pair<size_t, size_t>> live;
  std::mt19937_64 rng(9);
  size_t used = 0;
  for (int step = 0; step < 20000; ++step) {
    if (live.empty() || rng() % 3 != 0) {
      const size_t len = 1 + rng() % (256 * 40);
      const size_t units = aup(len) / 256;
      size_t first = SIZE_MAX;  // lowest fitting free run in the model
      for (size_t i = 0, run = 0; i < owner.size(); ++i) {
        run = owner[i] < 0 ? run + 1 : 0;
        if (run == units) {
          first = i + 1 - units;
          break;
        }
      }
      size_t off = 0;
      const bool ok = a.alloc(len, &off);
      // first fit over free blocks equals the lowest fitting run: free neighbours are always merged
      CHECK(ok == (first != SIZE_MAX));
      if (!ok) continue;
      CHECK(off == first * 256);
      for (size_t i = 0; i < units; ++i) {
        CHECK(owner[first + i] < 0);
        owner[first + i] = step;
      }
      live.push_back({off, len});
      used += aup(len);
    } else {
      const size_t k = rng() % live.size();
      const auto [off, len] = live[k];
      live.erase(live.begin() + (long)k);
      a.release(off, len);
      for (size_t i = 0; i < aup(len) / 256; ++i) owner[off / 256 + i] = -1;
      used -= aup(len);
    }
    CHECK(a.in_use() == used);
    CHECK(a.peak() >= used);
  }
  for (const auto& [off, len] : live) a.release(off, len);
  CHECK(a.in_use() == 0);
  CHECK(a.free_blocks().size() == 1 && a.free_blocks().begin()->second == cap);
  std::printf("arena: ok\n");
}

int main() {
  test_arena();
  test_oversize();
  test_wait_rules();
  test_shutdown();
  test_mixed_load();
  std::printf("srv_sim: all passed\n");
  return 0;
}
