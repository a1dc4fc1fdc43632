// Host check of the serving engine core (paper_2210_07667_amd/csrc/server_core.hpp)
// driven by a fake executor: a simulated device per lane runs each tick after an
// injected latency.  Run under the thread sanitizer (the engine's worker, completer,
// submitter and waiter threads) and under the address and undefined-behaviour
// sanitizers.  Checked:
//   * every request's steps are issued in order 0..nsteps-1, each once, and only while
//     the request holds its workspace slot;
//   * the slots of the requests running at any time (all lanes) are disjoint;
//   * a request is completed only after every tick holding one of its steps completed;
//   * admission within a lane follows submission order;
//   * every request completes once, with the executor's status (injected failures of
//     prepare and of issue included); the arena is whole again at the end;
//   * deadlines: a request queued past its deadline completes with kTimedOut without
//     being prepared; one running past it is issued no further step and completes with
//     kTimedOut only after its issued steps completed; requests without a deadline are
//     unaffected.
// Exit status 0 when every check holds.
#include <atomic>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <map>
#include <mutex>
#include <random>
#include <set>
#include <thread>
#include <vector>

#include "server_core.hpp"

using phiks_serve::Engine;
using phiks_serve::kTimedOut;
using phiks_serve::Request;

static std::atomic<int> g_fail{0};
#define CHECK(c)                                                              \
  do {                                                                        \
    if (!(c)) {                                                               \
      std::fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #c);    \
      g_fail.store(1);                                                        \
    }                                                                         \
  } while (0)

struct Spec {           // what the fake executor knows of a request
  int nsteps = 1;
  bool fail_prepare = false;
  std::vector<int> issued;   // step indices in issue order
  int pending_ticks = 0;     // issued ticks holding a step of it, not yet completed
  bool finished = false;
};

struct Token {
  std::vector<Request*> reqs;
  bool done = false;
  int status = 0;
};

struct FakeExec {
  int lanes;
  std::mutex mu;
  std::condition_variable cv;
  std::vector<std::deque<Token*>> queue;    // simulated device queue per lane
  std::vector<std::vector<int64_t>> admitted;
  std::map<int64_t, std::pair<size_t, size_t>> running;   // ticket -> slot
  bool stop = false;
  std::vector<std::thread> devices;
  std::atomic<int> tick_no{0};
  int fail_every;   // issue fails on every fail_every-th tick (0: never)

  FakeExec(int L, int fe) : lanes(L), queue(L), admitted(L), fail_every(fe) {
    for (int l = 0; l < L; ++l) devices.emplace_back([this, l] { device(l); });
  }
  ~FakeExec() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    cv.notify_all();
    for (auto& t : devices) t.join();
  }

  void device(int l) {
    std::mt19937 rng(1234 + l);
    for (;;) {
      Token* t = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return stop || !queue[l].empty(); });
        if (queue[l].empty()) return;
        t = queue[l].front();
      }
      std::this_thread::sleep_for(std::chrono::microseconds(20 + rng() % 300));
      std::lock_guard<std::mutex> lk(mu);
      for (Request* r : t->reqs) --((Spec*)r->ctx)->pending_ticks;
      t->done = true;
      queue[l].pop_front();
      cv.notify_all();
    }
  }

  int prepare(Request& r) {
    Spec& s = *(Spec*)r.ctx;
    std::lock_guard<std::mutex> lk(mu);
    admitted[r.lane].push_back(r.ticket);
    for (auto& kv : running) {   // disjoint slots
      const size_t a0 = kv.second.first, a1 = a0 + kv.second.second;
      CHECK(r.ws_off + r.ws_doubles <= a0 || a1 <= r.ws_off);
    }
    running[r.ticket] = {r.ws_off, r.ws_doubles};
    if (s.fail_prepare) return -8;
    r.nsteps = s.nsteps;
    return 0;
  }

  int issue(int lane, const std::vector<Request*>& reqs, const std::vector<int>& step, void** token) {
    std::lock_guard<std::mutex> lk(mu);
    std::set<int64_t> seen;
    for (size_t i = 0; i < reqs.size(); ++i) {
      Spec& s = *(Spec*)reqs[i]->ctx;
      CHECK(seen.insert(reqs[i]->ticket).second);
      CHECK(running.count(reqs[i]->ticket) == 1);
      CHECK(step[i] == (int)s.issued.size());
      CHECK(step[i] < s.nsteps);
      CHECK(reqs[i]->lane == lane);
      s.issued.push_back(step[i]);
    }
    const int k = ++tick_no;
    if (fail_every > 0 && k % fail_every == 0) {
      *token = nullptr;
      return -9;   // nothing queued for a failed tick
    }
    Token* t = new Token;
    t->reqs = reqs;
    for (Request* r : reqs) ++((Spec*)r->ctx)->pending_ticks;
    queue[lane].push_back(t);
    *token = t;
    cv.notify_all();
    return 0;
  }

  int wait(int, void* token) {
    Token* t = (Token*)token;
    std::unique_lock<std::mutex> lk(mu);
    cv.wait(lk, [&] { return t->done; });
    const int st = t->status;
    delete t;
    return st;
  }

  void finish(Request& r) {
    Spec& s = *(Spec*)r.ctx;
    std::lock_guard<std::mutex> lk(mu);
    CHECK(!s.finished);
    CHECK(s.pending_ticks == 0);
    s.finished = true;
    running.erase(r.ticket);
  }
};

static int run(int lanes, int max_active, size_t arena, int fail_every, int nreq, int threads,
               unsigned seed, bool deadlines = false) {
  FakeExec ex(lanes, fail_every);
  std::vector<Request*> all(nreq);
  std::vector<Spec*> spec(nreq);
  std::mt19937 rng(seed);
  for (int i = 0; i < nreq; ++i) {
    all[i] = new Request;
    spec[i] = new Spec;
    all[i]->ticket = i + 1;
    all[i]->lane = (int)(rng() % lanes);
    all[i]->ws_doubles = phiks_serve::Arena::round(1 + rng() % (arena / 3));
    spec[i]->nsteps = 1 + (int)(rng() % 12);
    spec[i]->fail_prepare = (rng() % 29) == 0;
    if (deadlines && rng() % 4 == 0) all[i]->timeout = 1e-6 * (50 + rng() % 3000);
    all[i]->ctx = spec[i];
  }
  {
    Engine<FakeExec> eng(&ex, arena, lanes, max_active, 2);
    std::vector<std::thread> subs;
    std::atomic<int> next{0};
    std::mutex order_mu;
    std::vector<std::vector<int64_t>> submit_order(lanes);
    for (int t = 0; t < threads; ++t) {
      subs.emplace_back([&, t] {
        std::mt19937 r2(seed * 31 + t);
        std::vector<int> mine;
        for (;;) {
          const int i = next.fetch_add(1);
          if (i >= nreq) break;
          {
            // submission order per lane as the engine sees it
            std::lock_guard<std::mutex> lk(order_mu);
            CHECK(eng.submit(all[i]));
            submit_order[all[i]->lane].push_back(all[i]->ticket);
          }
          mine.push_back(i);
          if (r2() % 3 == 0) std::this_thread::sleep_for(std::chrono::microseconds(r2() % 400));
        }
        for (int i : mine) {
          Request* r = eng.wait(all[i]->ticket);
          CHECK(r == all[i]);
          CHECK(r && r->done);
          if (r) {
            const Spec& s = *spec[i];
            if (r->status == kTimedOut) {
              CHECK(r->timeout > 0.0 && r->t_done >= r->deadline);
              CHECK((int)s.issued.size() < s.nsteps);
            } else if (s.fail_prepare) {
              CHECK(r->status == -8 && s.issued.empty());
            } else if (r->status == 0) {
              CHECK((int)s.issued.size() == s.nsteps);
            } else {
              CHECK(r->status == -9);
            }
            CHECK(r->t_done >= r->t_submit);
          }
        }
      });
    }
    for (auto& t : subs) t.join();
    CHECK(eng.wait(1) == nullptr);   // every ticket already claimed
    const auto st = eng.stats();
    int64_t n_admitted = 0, n_timed_out = 0;
    for (int l = 0; l < lanes; ++l) n_admitted += (int64_t)ex.admitted[l].size();
    for (int i = 0; i < nreq; ++i) n_timed_out += all[i]->status == kTimedOut;
    CHECK(st.submitted == nreq && st.completed == nreq && st.admitted == n_admitted);
    CHECK(st.timed_out == n_timed_out);
    if (!deadlines) CHECK(n_admitted == nreq && n_timed_out == 0);
    eng.shutdown();
    CHECK(eng.arena_consistent());
    CHECK(eng.take_all().empty());
    // admission follows submission order (requests expired in the queue are skipped)
    for (int l = 0; l < lanes; ++l) {
      std::vector<int64_t> expect;
      std::set<int64_t> adm(ex.admitted[l].begin(), ex.admitted[l].end());
      for (int64_t t : submit_order[l])
        if (adm.count(t)) expect.push_back(t);
      CHECK(ex.admitted[l] == expect);
      for (int64_t t : submit_order[l])
        if (!adm.count(t)) CHECK(all[t - 1]->status == kTimedOut && spec[t - 1]->issued.empty());
    }
    std::printf("lanes %d max_active %d arena %zu fail_every %d%s: %d requests, %lld ticks, "
                "%lld timed out\n", lanes, max_active, arena, fail_every,
                deadlines ? " deadlines" : "", nreq, (long long)st.ticks, (long long)n_timed_out);
  }
  for (int i = 0; i < nreq; ++i) {
    CHECK(spec[i]->finished);
    delete spec[i];
    delete all[i];
  }
  return g_fail.load();
}

// Deterministic deadlines: one slot, so B waits behind A and expires in the queue; C
// runs far longer than its timeout and is stopped at a step boundary; D (no deadline)
// and A complete normally.
static void deadline_scenarios() {
  FakeExec ex(1, 0);
  Request r[4];
  Spec sp[4];
  const int steps[4] = {40, 3, 1000, 5};
  for (int i = 0; i < 4; ++i) {
    r[i].ticket = 100 + i;
    r[i].lane = 0;
    r[i].ws_doubles = 64;
    sp[i].nsteps = steps[i];
    r[i].ctx = &sp[i];
  }
  r[1].timeout = 1e-3;
  r[2].timeout = 2e-3;
  {
    Engine<FakeExec> eng(&ex, 64, 1, 4, 2);
    CHECK(eng.submit(&r[0]));
    CHECK(eng.submit(&r[1]));
    Request* b = eng.wait(101);
    CHECK(b == &r[1] && b->status == kTimedOut && sp[1].issued.empty());
    CHECK(b->t_done >= b->deadline);
    Request* a = eng.wait(100);
    CHECK(a == &r[0] && a->status == 0 && (int)sp[0].issued.size() == 40);
    CHECK(eng.submit(&r[2]));
    CHECK(eng.submit(&r[3]));
    Request* c = eng.wait(102);
    CHECK(c == &r[2] && c->status == kTimedOut);
    CHECK(!sp[2].issued.empty() && (int)sp[2].issued.size() < 1000 && sp[2].finished);
    Request* d = eng.wait(103);
    CHECK(d == &r[3] && d->status == 0 && (int)sp[3].issued.size() == 5);
    const auto st = eng.stats();
    CHECK(st.timed_out == 2 && st.completed == 4 && st.admitted == 3);
    eng.shutdown();
    CHECK(eng.arena_consistent());
    std::printf("deadlines: B expired in the queue, C stopped after %zu of 1000 steps\n",
                sp[2].issued.size());
  }
}

int main() {
  // arena allocator alone: random alloc/release against a reference bitmap
  {
    phiks_serve::Arena a(1000);
    std::mt19937 rng(7);
    std::vector<std::pair<size_t, size_t>> live;
    std::vector<char> used(1000, 0);
    for (int it = 0; it < 20000; ++it) {
      if (!live.empty() && (rng() % 2)) {
        const size_t k = rng() % live.size();
        a.release(live[k].first, live[k].second);
        for (size_t x = 0; x < live[k].second; ++x) used[live[k].first + x] = 0;
        live.erase(live.begin() + k);
      } else {
        const size_t n = phiks_serve::Arena::round(1 + rng() % 200);
        size_t off = 0;
        if (a.alloc(n, &off)) {
          CHECK(off % 2 == 0 && off + n <= 1000);
          for (size_t x = 0; x < n; ++x) {
            CHECK(!used[off + x]);
            used[off + x] = 1;
          }
          live.push_back({off, n});
        }
      }
      CHECK(a.consistent());
    }
  }
  CHECK(phiks_serve::lane_of(1, 3) == 0 && phiks_serve::lane_of(1 << 18, 3) == 0);
  CHECK(phiks_serve::lane_of((1 << 18) + 1, 3) == 1 && phiks_serve::lane_of(1 << 21, 3) == 1);
  CHECK(phiks_serve::lane_of(192 * 192 * 192, 3) == 2 && phiks_serve::lane_of(1LL << 40, 3) == 2);
  CHECK(phiks_serve::lane_of(1 << 30, 1) == 0);
  run(1, 1, 64, 0, 60, 1, 1);
  run(3, 3, 400, 0, 300, 4, 2);
  run(2, 8, 1000, 37, 300, 3, 3);
  run(4, 2, 150, 11, 200, 4, 4);
  run(2, 3, 300, 0, 300, 4, 5, true);
  run(3, 8, 1000, 23, 300, 3, 6, true);
  deadline_scenarios();
  if (g_fail.load()) {
    std::fprintf(stderr, "server core check FAILED\n");
    return 1;
  }
  std::printf("server core check passed\n");
  return 0;
}
