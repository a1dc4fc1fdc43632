// Host core of the serving engine: lanes of step-level continuous batching, workspace
// slots, admission, in-flight ticks and completion.  Plain C++ (threads, no device
// code): the library instantiates it with an executor that plans requests and runs
// their steps on the GPU (server.hpp); the host tests drive the same core with a fake
// executor under the thread and address sanitizers.
//
// Model.  A request is a sequence of steps (for a phi-action: the mu-mode products and
// node sums of phiks_apply, in order).  Requests are routed at submission to a lane
// (the server's size classes).  Each lane has a worker thread that repeatedly
//   1. admits queued requests of its lane in arrival order while the arena has a slot
//      for the head request and the lane has fewer than max_active requests running
//      (a slot is allocated on admission and released when the request completes);
//   2. prepares the newly admitted requests (Exec::prepare: plan and step list);
//   3. issues one tick: the next step of every running request of the lane
//      (Exec::issue), so a request admitted now joins the lane's running schedule at
//      the next step boundary instead of waiting for the others to finish;
// keeping at most ticks_in_flight ticks queued on the device.  A completer thread per
// lane waits for the lane's ticks in order (Exec::wait), completes the requests whose
// last step was in the tick, releases their slots and wakes their waiters.  Lanes are
// independent (their own streams in the library), so the steps of small requests do not
// wait behind the steps of large ones.
//
// Deadlines.  A request may carry a timeout (Request::timeout, seconds from submission;
// 0 = none).  Still queued when it passes, the request completes with kTimedOut
// without being prepared or run (the worker wakes for the earliest queued deadline).
// Running when it passes, it is issued no further step: it leaves the running set at the
// next tick boundary and completes with kTimedOut once every tick holding one of its
// steps has completed (its slot is in use until then).  Its output is then partial.
//
// Executor interface (called without the engine's lock held):
//   int  prepare(Request& r);            plan + steps; sets r.nsteps >= 1; status
//   int  issue(int lane, const std::vector<Request*>& reqs, const std::vector<int>& step,
//              void** token);            step[i] of reqs[i]; on failure no work may remain
//                                        queued for the tick (the executor waits for it)
//   int  wait(int lane, void* token);    blocks until the tick's work is done; status
//   void finish(Request& r);             the request is complete (before its waiter wakes)
#pragma once

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <iterator>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

namespace phiks_serve {

// Status of a request whose deadline passed (the library's PHIKS_ETIMEDOUT).
constexpr int kTimedOut = -7;

inline double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Lane of a request of n_values doubles among `lanes` size classes: lane 0 up to 2^18
// values (2D up to 512^2, 3D up to 64^3), then one lane per factor 8 (3D: each doubling
// of the side).  Pure host function.
inline int lane_of(int64_t n_values, int lanes) {
  int lg = 0;
  while (lg < 62 && ((int64_t)1 << lg) < n_values) ++lg;
  const int l = lg <= 18 ? 0 : (lg - 16) / 3;
  return std::max(0, std::min(lanes - 1, l));
}

// First-fit allocator of workspace slots: offsets and sizes in doubles, rounded up to
// even counts so every slot is 16-byte aligned.
class Arena {
 public:
  explicit Arena(size_t cap) : cap_(cap & ~(size_t)1) {
    if (cap_) free_[0] = cap_;
  }
  static size_t round(size_t n) { return (n + 1) & ~(size_t)1; }
  size_t capacity() const { return cap_; }
  size_t used() const { return used_; }

  bool alloc(size_t n, size_t* off) {
    n = round(n);
    if (n == 0) n = 2;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      *off = it->first;
      const size_t start = it->first + n, rest = it->second - n;
      free_.erase(it);
      if (rest) free_[start] = rest;
      used_ += n;
      return true;
    }
    return false;
  }

  void release(size_t off, size_t n) {
    n = round(n);
    if (n == 0) n = 2;
    used_ -= n;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + n == next->first) {
      n += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += n;
        return;
      }
    }
    free_[off] = n;
  }

  // Free blocks inside the arena, disjoint and not adjacent; used + free = capacity.
  bool consistent() const {
    size_t free_total = 0, end = 0;
    bool first = true;
    for (const auto& kv : free_) {
      if (kv.second == 0 || kv.first + kv.second > cap_) return false;
      if (!first && kv.first <= end) return false;   // overlapping or adjacent (unmerged)
      end = kv.first + kv.second;
      free_total += kv.second;
      first = false;
    }
    return free_total + used_ == cap_;
  }

 private:
  size_t cap_, used_ = 0;
  std::map<size_t, size_t> free_;   // offset -> size
};

struct Request {
  int64_t ticket = 0;
  int lane = 0;
  size_t ws_doubles = 0;   // slot size (doubles)
  size_t ws_off = 0;       // slot offset in the arena (doubles), valid once admitted
  int nsteps = 0, next = 0;
  int status = 0;
  bool done = false;
  double timeout = 0.0;    // seconds from submission to the deadline; 0: none
  double deadline = 0.0;   // set by submit: t_submit + timeout (0: none)
  double t_submit = 0.0, t_admit = 0.0, t_done = 0.0;
  void* ctx = nullptr;     // the executor's state of this request
};

struct EngineStats {
  int64_t submitted = 0, admitted = 0, completed = 0, ticks = 0;
  int64_t timed_out = 0;   // completed with kTimedOut (queued or running)
};

template <class Exec>
class Engine {
 public:
  Engine(Exec* ex, size_t arena_doubles, int lanes, int max_active, int ticks_in_flight)
      : ex_(ex), arena_(arena_doubles), L_(std::max(1, lanes)),
        max_active_(std::max(1, max_active)), kif_(std::max(1, ticks_in_flight)),
        lanes_(L_) {
    for (int l = 0; l < L_; ++l) {
      lanes_[l].worker = std::thread(&Engine::worker, this, l);
      lanes_[l].completer = std::thread(&Engine::completer, this, l);
    }
  }
  ~Engine() { shutdown(); }
  Engine(const Engine&) = delete;
  Engine& operator=(const Engine&) = delete;

  size_t arena_capacity() const { return arena_.capacity(); }

  // Queues r (r->lane, r->ws_doubles set; the slot must fit an empty arena).  False
  // once shutdown has begun.
  bool submit(Request* r) {
    std::lock_guard<std::mutex> lk(mu_);
    if (stopping_ || r->lane < 0 || r->lane >= L_) return false;
    r->t_submit = now_s();
    r->deadline = r->timeout > 0.0 ? r->t_submit + r->timeout : 0.0;
    reqs_[r->ticket] = r;
    lanes_[r->lane].pending.push_back(r);
    ++stats_.submitted;
    lanes_[r->lane].cv.notify_all();
    return true;
  }

  // Blocks until the request is done and hands it back to the caller (who owns it
  // from then on); nullptr for an unknown ticket or one another caller already waits for.
  Request* wait(int64_t ticket) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return nullptr;
    Request* r = it->second;
    reqs_.erase(it);   // claimed by this caller
    cv_done_.wait(lk, [&] { return r->done; });
    return r;
  }

  EngineStats stats() {
    std::lock_guard<std::mutex> lk(mu_);
    return stats_;
  }

  // After shutdown: every request never waited for, handed back to the caller.
  std::vector<Request*> take_all() {
    std::lock_guard<std::mutex> lk(mu_);
    std::vector<Request*> v;
    for (auto& kv : reqs_) v.push_back(kv.second);
    reqs_.clear();
    return v;
  }

  // Arena invariants (tests).
  bool arena_consistent() {
    std::lock_guard<std::mutex> lk(mu_);
    return arena_.consistent();
  }

  // Runs everything queued, then stops the threads.  Idempotent.
  void shutdown() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (joined_) return;
      stopping_ = true;
      for (Lane& ln : lanes_) ln.cv.notify_all();
    }
    for (Lane& ln : lanes_) {
      if (ln.worker.joinable()) ln.worker.join();
      if (ln.completer.joinable()) ln.completer.join();
    }
    std::lock_guard<std::mutex> lk(mu_);
    joined_ = true;
  }

 private:
  struct Tick {
    void* token = nullptr;
    int status = 0;                    // nonzero: the tick failed when issued
    std::vector<Request*> finishing;   // requests whose last step is in this tick
    std::vector<Request*> expired;     // running requests stopped by their deadline
  };
  struct Lane {
    std::deque<Request*> pending;
    std::deque<Tick> inflight;
    int queued_ticks = 0;   // issued and not yet completed
    bool worker_done = false;
    std::condition_variable cv;        // worker: work, slots, tick completions, stop
    std::condition_variable cv_comp;   // completer: ticks, worker done
    std::thread worker, completer;
  };

  // Completes r under the lock: releases its slot (if admitted), records the time and
  // status.
  void complete_locked(Request* r, int status, double t, bool admitted = true) {
    if (admitted) arena_.release(r->ws_off, r->ws_doubles);
    r->status = status;
    r->t_done = t;
    r->done = true;
    ++stats_.completed;
    if (status == kTimedOut) ++stats_.timed_out;
  }

  static bool expired_at(const Request* r, double now) { return r->deadline > 0.0 && now >= r->deadline; }

  void worker(int l) {
    Lane& ln = lanes_[l];
    std::vector<Request*> active;   // this worker's running requests, in admission order
    for (;;) {
      std::vector<Request*> fresh, stale;   // admitted now; queued past their deadline
      {
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
          const double now = now_s();
          double wake = 0.0;   // earliest deadline still queued
          for (auto it = ln.pending.begin(); it != ln.pending.end();) {
            if (expired_at(*it, now)) {
              stale.push_back(*it);
              it = ln.pending.erase(it);
            } else {
              if ((*it)->deadline > 0.0 && (wake == 0.0 || (*it)->deadline < wake)) wake = (*it)->deadline;
              ++it;
            }
          }
          while (!ln.pending.empty() && (int)(active.size() + fresh.size()) < max_active_) {
            Request* r = ln.pending.front();
            size_t off = 0;
            if (!arena_.alloc(r->ws_doubles, &off)) break;   // no overtaking: wait for a slot
            r->ws_off = off;
            r->t_admit = now_s();
            ln.pending.pop_front();
            fresh.push_back(r);
            ++stats_.admitted;
          }
          if (!stale.empty()) break;
          if ((!active.empty() || !fresh.empty()) && ln.queued_ticks < kif_) break;
          if (stopping_ && ln.pending.empty() && active.empty() && fresh.empty()) {
            ln.worker_done = true;
            ln.cv_comp.notify_all();
            return;
          }
          if (wake > 0.0) {
            // Sleep until the earliest queued deadline, at most 10 ms at a time.  The wait
            // is on the system clock (pthread_cond_timedwait, which the thread sanitizer
            // follows; a steady-clock wait_for maps to pthread_cond_clockwait, which it does
            // not); the deadlines themselves are compared on the steady clock above, so a
            // step of the system clock delays an expiry by at most the 10 ms cap.
            const double dt = std::min(0.01, std::max(0.0, wake - now_s())) + 1e-6;
            ln.cv.wait_until(lk, std::chrono::system_clock::now() +
                                     std::chrono::duration_cast<std::chrono::system_clock::duration>(
                                         std::chrono::duration<double>(dt)));
          } else {
            ln.cv.wait(lk);
          }
        }
      }
      for (Request* r : stale) {   // never admitted: no slot, nothing issued
        ex_->finish(*r);
        std::lock_guard<std::mutex> lk(mu_);
        complete_locked(r, kTimedOut, now_s(), false);
        cv_done_.notify_all();
      }
      for (Request* r : fresh) {
        const int rc = ex_->prepare(*r);
        if (rc != 0 || r->nsteps < 1) {
          ex_->finish(*r);
          std::lock_guard<std::mutex> lk(mu_);
          complete_locked(r, rc != 0 ? rc : -1, now_s());
          cv_done_.notify_all();
          for (Lane& o : lanes_) o.cv.notify_all();   // a slot was released
        } else {
          active.push_back(r);
        }
      }
      if (active.empty()) continue;
      Tick t;
      {
        // running requests past their deadline get no further step
        const double now = now_s();
        std::vector<Request*> live;
        for (Request* r : active) (expired_at(r, now) ? t.expired : live).push_back(r);
        active.swap(live);
      }
      if (!active.empty()) {
        std::vector<int> step(active.size());
        for (size_t i = 0; i < active.size(); ++i) step[i] = active[i]->next++;
        t.status = ex_->issue(l, active, step, &t.token);
      }
      std::vector<Request*> still;
      for (Request* r : active) {
        if (t.status != 0 || r->next >= r->nsteps) t.finishing.push_back(r);
        else still.push_back(r);
      }
      active.swap(still);
      std::lock_guard<std::mutex> lk(mu_);
      if (t.token || t.status != 0) ++stats_.ticks;   // a tick of expiries only issues nothing
      ++ln.queued_ticks;
      ln.inflight.push_back(std::move(t));
      ln.cv_comp.notify_all();
    }
  }

  void completer(int l) {
    Lane& ln = lanes_[l];
    for (;;) {
      Tick t;
      {
        std::unique_lock<std::mutex> lk(mu_);
        ln.cv_comp.wait(lk, [&] { return !ln.inflight.empty() || ln.worker_done; });
        if (ln.inflight.empty()) return;   // the worker is done and every tick completed
        t = std::move(ln.inflight.front());
        ln.inflight.pop_front();
      }
      int status = t.status;
      if (t.token) {
        const int ws = ex_->wait(l, t.token);
        if (status == 0) status = ws;
      }
      // ticks complete in order, so every earlier step of an expired request is done
      const double now = now_s();
      for (Request* r : t.finishing) ex_->finish(*r);
      for (Request* r : t.expired) ex_->finish(*r);
      std::lock_guard<std::mutex> lk(mu_);
      for (Request* r : t.finishing) complete_locked(r, status, now);
      for (Request* r : t.expired) complete_locked(r, kTimedOut, now);
      --ln.queued_ticks;
      cv_done_.notify_all();
      for (Lane& o : lanes_) o.cv.notify_all();   // slots released, a tick fewer queued
    }
  }

  Exec* ex_;
  Arena arena_;
  const int L_, max_active_, kif_;
  std::mutex mu_;
  std::condition_variable cv_done_;
  std::vector<Lane> lanes_;
  std::unordered_map<int64_t, Request*> reqs_;
  EngineStats stats_;
  bool stopping_ = false, joined_ = false;
};

}  // namespace phiks_serve
