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
//     prepare and of issue included); the arena is whole again at the end.
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
    if (s.fail_prepare) return -7;
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
               unsigned seed) {
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
            if (s.fail_prepare) CHECK(r->status == -7 && s.issued.empty());
            else if (r->status == 0) CHECK((int)s.issued.size() == s.nsteps);
            else CHECK(r->status == -9);
            CHECK(r->t_done >= r->t_submit);
          }
        }
      });
    }
    for (auto& t : subs) t.join();
    CHECK(eng.wait(1) == nullptr);   // every ticket already claimed
    const auto st = eng.stats();
    CHECK(st.submitted == nreq && st.completed == nreq && st.admitted == nreq);
    eng.shutdown();
    CHECK(eng.arena_consistent());
    CHECK(eng.take_all().empty());
    for (int l = 0; l < lanes; ++l) CHECK(ex.admitted[l] == submit_order[l]);
    std::printf("lanes %d max_active %d arena %zu fail_every %d: %d requests, %lld ticks\n", lanes,
                max_active, arena, fail_every, nreq, (long long)st.ticks);
  }
  for (int i = 0; i < nreq; ++i) {
    CHECK(spec[i]->finished);
    delete spec[i];
    delete all[i];
  }
  return g_fail.load();
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
  if (g_fail.load()) {
    std::fprintf(stderr, "server core check FAILED\n");
    return 1;
  }
  std::printf("server core check passed\n");
  return 0;
}
