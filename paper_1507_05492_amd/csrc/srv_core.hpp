// Request scheduler of the scoring server: the request table, first-fit admission into
// one device arena in arrival order, grouping of small scoring requests, completion and
// latency bookkeeping, waiting and shutdown.  Host code only: the device work goes
// through the Executor interface, so the library runs this scheduler with its HIP
// executor (streams, events, kernels) and the host tests run the same code with a
// simulated executor under the address, undefined-behaviour and thread sanitizers.
#pragma once

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "cq.h"

namespace cqsrv {

using Clock = std::chrono::steady_clock;

constexpr size_t kAlign = 256;
inline size_t aup(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

struct Req {
  uint64_t id = 0;
  int kind = 0;                 // 0 score, 1 compare
  const void* graph = nullptr;  // the library's graph handle (score requests)
  int32_t n = 0, L = 0, La = 0, Lb = 0;
  const int32_t* ha = nullptr;
  const int32_t* hb = nullptr;
  size_t ws_bytes = 0;  // workspace when run alone
  size_t group_ws = 0;  // workspace inside a grouped launch (score requests)
  size_t foot = 0;      // device bytes when run alone (set by submit)
  bool small = false;   // may join a grouped launch
  Clock::time_point t_submit, t_done;
  cq_status status = CQ_OK;
  cq_score_result sres{};
  cq_compare_result cres{};
  bool done = false;
  bool waited = false;  // a thread is waiting for it (one waiter per ticket)
};

// Device bytes of one request run alone: its labels (one or two int32 arrays), its
// workspace and its result.
inline size_t req_footprint(const Req& r) {
  if (r.kind == 0) return aup(4 * (size_t)r.n) + aup(r.ws_bytes) + aup(sizeof(cq_score_result));
  return 2 * aup(4 * (size_t)r.n) + aup(r.ws_bytes) + aup(sizeof(cq_compare_result));
}

// Device bytes of small scoring requests run as one batched launch: every request's
// labels, the workspaces and the group pass's item list (16 bytes per label id), the
// results.
inline size_t group_footprint(const std::vector<Req*>& g) {
  size_t lab = 0, ws = 0, items = 0;
  for (const Req* r : g) {
    lab += aup(4 * (size_t)r->n);
    ws += aup(r->group_ws);
    items += 16 * (size_t)r->L;
  }
  return lab + aup(ws + aup(items)) + aup(sizeof(cq_score_result) * g.size());
}

// First-fit allocator over [0, capacity) of the arena; offsets and lengths are
// multiples of kAlign, and freed blocks merge with their free neighbours.
class Arena {
 public:
  explicit Arena(size_t capacity) {
    const size_t c = capacity & ~(kAlign - 1);
    if (c) free_[0] = c;
  }
  bool alloc(size_t len, size_t* off) {
    len = aup(len);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < len) continue;
      *off = it->first;
      const size_t rest = it->second - len, noff = it->first + len;
      free_.erase(it);
      if (rest) free_[noff] = rest;
      in_use_ += len;
      peak_ = std::max(peak_, in_use_);
      return true;
    }
    return false;
  }
  void release(size_t off, size_t len) {
    len = aup(len);
    in_use_ -= len;
    auto it = free_.emplace(off, len).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t in_use() const { return in_use_; }
  size_t peak() const { return peak_; }
  void reset_peak() { peak_ = in_use_; }
  const std::map<size_t, size_t>& free_blocks() const { return free_; }

 private:
  std::map<size_t, size_t> free_;  // offset -> length
  size_t in_use_ = 0, peak_ = 0;
};

// Runs admitted work on the device.  Only the scheduler's worker thread calls it.
class Executor {
 public:
  virtual ~Executor() = default;
  // Called once on the worker thread before anything else (binds the device).
  virtual void worker_init() {}
  // Start the work of `slot`: one request, or (grouped) small scoring requests run as one
  // batched launch, whose device memory is arena bytes [off, off + len).  Returns at once;
  // a request that cannot be started gets a failing status here.
  virtual void dispatch(int slot, const std::vector<Req*>& reqs, bool grouped, size_t off, size_t len) = 0;
  // True once the slot's work has finished; never blocks.
  virtual bool finished(int slot) = 0;
  // The finished slot's results: fills the result and status of every request whose
  // status is still CQ_OK.
  virtual void collect(int slot, const std::vector<Req*>& reqs, bool grouped) = 0;
};

struct Config {
  int num_slots = 1;
  int max_batch = 1;
  size_t arena_bytes = 0;
};

// What a finished request hands back to its waiter.
struct Outcome {
  int kind = 0;
  cq_status status = CQ_OK;
  cq_score_result sres{};
  cq_compare_result cres{};
  double latency_ms = 0;
};

class Scheduler {
 public:
  Scheduler(const Config& cfg, Executor* ex)
      : cfg_(cfg), cap_(cfg.arena_bytes & ~(kAlign - 1)), ex_(ex), arena_(cfg.arena_bytes), slots_(cfg.num_slots) {}
  Scheduler(const Scheduler&) = delete;
  Scheduler& operator=(const Scheduler&) = delete;
  ~Scheduler() {
    shutdown();
    for (auto& kv : reqs_) delete kv.second;
  }

  void start() { worker_ = std::thread([this] { loop(); }); }

  // Takes ownership of r.  CQ_E_BUSY: the request can never fit the arena (it is not
  // queued); CQ_E_CANCELLED: the server is shutting down.
  cq_status submit(Req* r, uint64_t* ticket, const char** why) {
    r->foot = req_footprint(*r);
    if (r->foot > cap_) {
      delete r;
      std::lock_guard<std::mutex> lk(mu_);
      ++rejected_;
      if (why) *why = "the request needs more device memory than the whole server arena";
      return CQ_E_BUSY;
    }
    r->t_submit = Clock::now();
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (stop_) {
        delete r;
        if (why) *why = "the server is shutting down";
        return CQ_E_CANCELLED;
      }
      r->id = next_id_++;
      reqs_[r->id] = r;
      pending_.push_back(r);
      ++submitted_;
      *ticket = r->id;
    }
    cv_work_.notify_one();
    return CQ_OK;
  }

  // Waits for a ticket (timeout_ms < 0: no limit).  CQ_OK: *out holds the outcome and the
  // ticket is released.  CQ_E_BUSY: not finished in time (the ticket stays valid).
  // CQ_E_INVALID_ARG: unknown ticket, or another thread is waiting for it.
  cq_status wait(uint64_t ticket, double timeout_ms, Outcome* out, const char** why) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) {
      if (why) *why = "unknown ticket";
      return CQ_E_INVALID_ARG;
    }
    Req* r = it->second;
    if (r->waited) {
      if (why) *why = "another thread is waiting for this ticket";
      return CQ_E_INVALID_ARG;
    }
    r->waited = true;
    ++waiters_;
    auto ready = [&] { return r->done; };
    bool ok = true;
    if (timeout_ms < 0) cv_done_.wait(lk, ready);
    else ok = cv_done_.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), ready);
    r->waited = false;
    if (--waiters_ == 0 && stop_) cv_done_.notify_all();  // shutdown waits for the last waiter
    if (!ok) return CQ_E_BUSY;
    if (out) {
      out->kind = r->kind;
      out->status = r->status;
      out->sres = r->sres;
      out->cres = r->cres;
      out->latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
    }
    reqs_.erase(it);
    delete r;
    return CQ_OK;
  }

  void stats(cq_server_stats* out) {
    std::lock_guard<std::mutex> lk(mu_);
    std::memset(out, 0, sizeof(*out));
    out->submitted = submitted_;
    out->completed = completed_;
    out->failed = failed_;
    out->rejected = rejected_;
    out->launches = launches_;
    out->grouped_requests = grouped_;
    out->busy_s = busy_s_;
    out->peak_bytes = (int64_t)arena_.peak();
    std::vector<double> v = lat_ms_;
    if (!v.empty()) {
      std::sort(v.begin(), v.end());
      auto q = [&](double f) { return v[std::min(v.size() - 1, (size_t)(f * (double)(v.size() - 1) + 0.5))]; };
      out->p50_ms = q(0.50);
      out->p99_ms = q(0.99);
      out->max_ms = v.back();
      double sum = 0;
      for (double x : v) sum += x;
      out->mean_ms = sum / (double)v.size();
    }
  }

  void reset_stats() {
    std::lock_guard<std::mutex> lk(mu_);
    lat_ms_.clear();
    submitted_ = completed_ = failed_ = launches_ = grouped_ = rejected_ = 0;
    busy_s_ = 0;
    arena_.reset_peak();
    if (inflight_ > 0) busy_since_ = Clock::now();
  }

  // Cancels the requests not yet admitted (CQ_E_CANCELLED), lets the admitted ones
  // finish, stops the worker and returns once no thread is inside wait().  Idempotent.
  void shutdown() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
      for (Req* r : pending_) {
        r->status = CQ_E_CANCELLED;
        r->t_done = Clock::now();
        r->done = true;
      }
      pending_.clear();
    }
    cv_work_.notify_all();
    if (worker_.joinable()) worker_.join();
    std::unique_lock<std::mutex> lk(mu_);
    cv_done_.notify_all();
    cv_done_.wait(lk, [&] { return waiters_ == 0; });
  }

  // Arena state, for the host tests (call with no request admitted).
  size_t arena_in_use() {
    std::lock_guard<std::mutex> lk(mu_);
    return arena_.in_use();
  }
  size_t arena_free_blocks() {
    std::lock_guard<std::mutex> lk(mu_);
    return arena_.free_blocks().size();
  }

 private:
  struct Slot {
    bool busy = false;
    bool grouped = false;
    std::vector<Req*> reqs;
    size_t off = 0, len = 0;
  };

  // Completions, then admissions into free slots in arrival order.  A small scoring
  // request at the head takes the small scoring requests queued behind it (up to
  // max_batch, as many as fit the arena) into one grouped launch; any other head waits
  // until its own footprint fits, so later requests never overtake it.
  void loop() {
    ex_->worker_init();
    for (;;) {
      bool progress = false;
      for (int i = 0; i < (int)slots_.size(); ++i) {
        Slot& sl = slots_[i];
        if (!sl.busy || !ex_->finished(i)) continue;
        const auto now = Clock::now();
        std::lock_guard<std::mutex> lk(mu_);
        ex_->collect(i, sl.reqs, sl.grouped);
        for (Req* r : sl.reqs) {
          r->t_done = now;
          r->done = true;
          lat_ms_.push_back(std::chrono::duration<double, std::milli>(now - r->t_submit).count());
          if (r->status == CQ_OK) ++completed_;
          else ++failed_;
        }
        arena_.release(sl.off, sl.len);
        sl.busy = false;
        sl.reqs.clear();
        if (--inflight_ == 0) busy_s_ += std::chrono::duration<double>(now - busy_since_).count();
        progress = true;
        cv_done_.notify_all();
      }
      std::unique_lock<std::mutex> lk(mu_);
      for (;;) {
        if (pending_.empty()) break;
        int si = -1;
        for (int i = 0; i < (int)slots_.size(); ++i)
          if (!slots_[i].busy) {
            si = i;
            break;
          }
        if (si < 0) break;
        Req* head = pending_.front();
        std::vector<Req*> take = {head};
        size_t off = 0, len = 0;
        bool grouped = false;
        if (head->small && cfg_.max_batch > 1) {
          for (size_t i = 1; i < pending_.size() && (int)take.size() < cfg_.max_batch; ++i)
            if (pending_[i]->small) take.push_back(pending_[i]);
          while (take.size() > 1) {
            len = group_footprint(take);
            if (arena_.alloc(len, &off)) break;
            take.pop_back();
          }
          grouped = take.size() > 1;
        }
        if (!grouped) {
          len = head->foot;
          if (!arena_.alloc(len, &off)) break;  // wait for memory (arrival order is kept)
        }
        for (Req* r : take) pending_.erase(std::find(pending_.begin(), pending_.end(), r));
        Slot& sl = slots_[si];
        sl.reqs = take;
        sl.grouped = grouped;
        sl.off = off;
        sl.len = len;
        sl.busy = true;
        if (inflight_++ == 0) busy_since_ = Clock::now();
        ++launches_;
        if (grouped) grouped_ += (int64_t)take.size();
        lk.unlock();
        ex_->dispatch(si, sl.reqs, grouped, off, len);
        lk.lock();
        progress = true;
      }
      if (stop_ && pending_.empty() && inflight_ == 0) break;
      if (!progress) {
        if (inflight_ > 0) {
          lk.unlock();
          std::this_thread::yield();
        } else {
          cv_work_.wait_for(lk, std::chrono::microseconds(200));
        }
      }
    }
  }

  Config cfg_;
  size_t cap_;  // usable arena bytes
  Executor* ex_;
  Arena arena_;
  std::vector<Slot> slots_;  // touched by the worker thread only
  std::mutex mu_;
  std::condition_variable cv_work_, cv_done_;
  std::deque<Req*> pending_;
  std::map<uint64_t, Req*> reqs_;
  uint64_t next_id_ = 1;
  bool stop_ = false;
  std::thread worker_;
  std::vector<double> lat_ms_;
  int64_t submitted_ = 0, completed_ = 0, failed_ = 0, launches_ = 0, grouped_ = 0, rejected_ = 0;
  int inflight_ = 0;  // busy slots
  int waiters_ = 0;   // threads inside wait()
  double busy_s_ = 0;
  Clock::time_point busy_since_;
};

}  // namespace cqsrv
