// Serving: same-vector requests submitted one at a time, run in groups.
//
// A request is one phiks_apply (outputs as eq. scaldiffphi) on caller-owned device
// vectors.  Inside the server:
//   * operators are registered once (host copies of A_1..A_d) and named by an id;
//   * plan cache: the plans (host plan + the small exponentials of Section 3.1 on the
//     device) keyed on (operator id, tau, p, n_scales, tol); requests of one operator
//     and step share one plan.  LRU eviction of unused plans keeps the
//     cache within the HBM budget less the workspace arena.
//   * admission: the worker takes pending requests in arrival order that share the
//     first one's (p, n_scales), as long as their workspaces fit the arena and the
//     group has at most max_group requests (continuous batching: whatever arrived
//     while the previous group ran forms the next one).  Both this choice and the
//     eviction choice are pure host functions (select_group, select_evictions), also
//     exported for tests of the policy without a device.
//   * execution: a group runs as the grouped launches of phiks_batch_apply (so every
//     result is bitwise what phiks_apply returns for that request alone); host
//     planning of the next group overlaps the device work of the previous ones.
//   * completion: a second thread waits on each group's event in order, stamps the
//     completion time and wakes the callers blocked in phiks_server_wait.
// Requests are planned with the relative reading of the tolerance (vnorms = NULL), so
// the plan does not depend on the vector.
//
// Included once, at the end of phiks.hip, after batch.hpp.
#pragma once

#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct PlanKey {
  std::vector<char> bytes;  // operator id, tau, p, n_scales, tol
  uint64_t hash = 0;
  bool operator==(const PlanKey& o) const { return hash == o.hash && bytes == o.bytes; }
};
struct PlanKeyHash {
  size_t operator()(const PlanKey& k) const { return (size_t)k.hash; }
};

struct CachedPlan {
  phiks_plan_s* plan = nullptr;
  size_t bytes = 0;        // device bytes of its matrices
  int refs = 0;            // requests admitted and not yet completed
  uint64_t last_use = 0;   // LRU tick
};

struct ServerOperator {
  int d = 0;
  int64_t n[PHIKS_MAX_D] = {0};
  int64_t N = 1;
  std::vector<std::vector<double>> A;  // host copies, row-major
};

struct ServerRequest {
  int64_t ticket = 0;
  PlanKey key;
  const ServerOperator* op = nullptr;
  double tau = 0.0, tol = 0.0;
  int p = 0, ns = 1;
  const double* v = nullptr;
  double* out = nullptr;
  size_t ws_bound = 0;     // workspace doubles for the largest q (admission)
  double t_submit = 0.0, t_done = 0.0;
  int status = PHIKS_OK;
  bool done = false;
  CachedPlan* cp = nullptr;
};

struct InFlightGroup {
  hipEvent_t ev = nullptr;
  std::vector<ServerRequest*> reqs;
};

// ------------------------------------------------ scheduling policy (host only)
// The worker and the plan cache decide through these two functions alone, so the policy
// can be exercised without a device (phiks_server_select_group / _select_evictions).

struct GroupCandidate {
  int p, ns;
  size_t ws;   // workspace doubles the request may need
};

// The next group from the pending requests c (arrival order): the requests with the
// first one's (p, n_scales), in order, while their workspaces (each rounded up to an
// even count of doubles) fit the arena together, at most max_group of them.  The first
// request of that class that does not fit ends the group, so none overtakes another of
// its class; requests of other classes wait for a later group.  Indices into c.
std::vector<int> select_group(const std::vector<GroupCandidate>& c, size_t arena_doubles,
                              int max_group) {
  std::vector<int> g;
  if (c.empty()) return g;
  const int p0 = c[0].p, ns0 = c[0].ns;
  size_t ws = 0;
  for (int i = 0; i < (int)c.size() && (int)g.size() < max_group; ++i) {
    if (c[i].p != p0 || c[i].ns != ns0) continue;
    const size_t need = (c[i].ws + 1) & ~(size_t)1;
    if (ws + need > arena_doubles) break;
    ws += need;
    g.push_back(i);
  }
  return g;
}

struct CacheEntryDesc {
  size_t bytes;
  int refs;            // requests admitted and not yet completed
  uint64_t last_use;   // LRU tick
};

// Plans to evict before a new plan of new_bytes joins a cache of cache_bytes with
// capacity cap: unreferenced entries, least recently used first, until the new plan
// fits; when every remaining entry is referenced the cache runs over its budget.
// Indices into e, in eviction order.
std::vector<int> select_evictions(const std::vector<CacheEntryDesc>& e, size_t cache_bytes,
                                  size_t new_bytes, size_t cap) {
  std::vector<int> v;
  std::vector<char> gone(e.size(), 0);
  while (cache_bytes + new_bytes > cap) {
    int victim = -1;
    for (int i = 0; i < (int)e.size(); ++i)
      if (!gone[i] && e[i].refs == 0 && (victim < 0 || e[i].last_use < e[victim].last_use))
        victim = i;
    if (victim < 0) break;
    gone[victim] = 1;
    cache_bytes -= e[victim].bytes;
    v.push_back(victim);
  }
  return v;
}

uint64_t fnv1a(const char* p, size_t n, uint64_t h = 1469598103934665603ull) {
  for (size_t i = 0; i < n; ++i) {
    h ^= (unsigned char)p[i];
    h *= 1099511628211ull;
  }
  return h;
}

}  // namespace

struct phiks_server_s {
  size_t budget = 0, arena_doubles = 0;
  int max_group = 1;
  hipStream_t stream = nullptr;
  int device = 0;
  double* arena = nullptr;
  GroupTables tab;
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_inflight;
  std::deque<ServerRequest*> pending;
  std::unordered_map<int64_t, ServerRequest*> tickets;
  std::unordered_map<int64_t, ServerOperator> ops;
  int64_t next_op = 1;
  std::unordered_map<PlanKey, CachedPlan, PlanKeyHash> cache;
  size_t cache_bytes = 0;
  std::deque<InFlightGroup> inflight;
  bool stop = false, worker_done = false;
  int64_t next_ticket = 1;
  uint64_t tick = 0;
  phiks_server_stats_t st{};
  std::thread worker, completer;
};

namespace {

void server_finish(phiks_server_s& S, ServerRequest* r, int status, double t) {
  r->status = status;
  r->t_done = t;
  r->done = true;
  ++S.st.completed;
}

// Cached plan for r (built on a miss); called by the worker without the lock held.
int server_plan(phiks_server_s& S, ServerRequest* r) {
  {
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.cache.find(r->key);
    if (it != S.cache.end()) {
      r->cp = &it->second;
      ++r->cp->refs;
      r->cp->last_use = ++S.tick;
      ++S.st.cache_hits;
      return PHIKS_OK;
    }
  }
  const ServerOperator& op = *r->op;
  std::vector<const double*> A(op.d);
  for (int mu = 0; mu < op.d; ++mu) A[mu] = op.A[mu].data();
  phiks_plan_t plan = nullptr;
  int rc = phiks_plan(op.d, op.n, A.data(), r->tau, r->p, r->ns, r->tol, PHIKS_SAME_VECTOR,
                      nullptr, PHIKS_FP64, S.stream, &plan);
  if (rc != PHIKS_OK) return rc;
  const size_t bytes = plan_device_doubles(*plan) * sizeof(double);
  std::vector<phiks_plan_s*> evict;
  {
    std::lock_guard<std::mutex> lk(S.mu);
    ++S.st.cache_misses;
    // least recently used plans that no admitted request holds, until the new one fits
    const size_t cap = S.budget > S.arena_doubles * sizeof(double)
                           ? S.budget - S.arena_doubles * sizeof(double) : 0;
    std::vector<decltype(S.cache)::iterator> its;
    std::vector<CacheEntryDesc> desc;
    for (auto it = S.cache.begin(); it != S.cache.end(); ++it) {
      its.push_back(it);
      desc.push_back({it->second.bytes, it->second.refs, it->second.last_use});
    }
    for (int i : select_evictions(desc, S.cache_bytes, bytes, cap)) {
      S.cache_bytes -= its[i]->second.bytes;
      evict.push_back(its[i]->second.plan);
      S.cache.erase(its[i]);
      ++S.st.evictions;
    }
    auto ins = S.cache.emplace(r->key, CachedPlan{plan, bytes, 1, ++S.tick});
    r->cp = &ins.first->second;
    S.cache_bytes += bytes;
    S.st.cache_bytes = (int64_t)S.cache_bytes;
  }
  for (phiks_plan_s* P : evict) phiks_plan_destroy(P);  // stream-ordered release
  return PHIKS_OK;
}

void server_worker(phiks_server_s* Sp) {
  phiks_server_s& S = *Sp;
  (void)hipSetDevice(S.device);
  for (;;) {
    std::vector<ServerRequest*> group;
    {
      std::unique_lock<std::mutex> lk(S.mu);
      S.cv_work.wait(lk, [&] { return S.stop || !S.pending.empty(); });
      if (S.pending.empty()) break;  // stop requested and drained
      std::vector<GroupCandidate> cand;
      for (const ServerRequest* r : S.pending) cand.push_back({r->p, r->ns, r->ws_bound});
      const std::vector<int> pick = select_group(cand, S.arena_doubles, S.max_group);
      std::vector<char> taken(S.pending.size(), 0);
      for (int i : pick) {
        group.push_back(S.pending[i]);
        taken[i] = 1;
      }
      std::deque<ServerRequest*> rest;
      for (size_t i = 0; i < S.pending.size(); ++i)
        if (!taken[i]) rest.push_back(S.pending[i]);
      S.pending.swap(rest);
    }
    // plans (cache lookups; misses are planned here, overlapping earlier groups)
    std::vector<ServerRequest*> run;
    for (ServerRequest* r : group) {
      const int rc = server_plan(S, r);
      if (rc != PHIKS_OK) {
        std::lock_guard<std::mutex> lk(S.mu);
        server_finish(S, r, rc, now_s());
      } else {
        run.push_back(r);
      }
    }
    if (run.empty()) {
      S.cv_done.notify_all();
      continue;
    }
    GroupWork W;
    W.p = run[0]->p;
    W.ns = run[0]->ns;
    size_t off = 0;
    for (ServerRequest* r : run) {
      W.plans.push_back(r->cp->plan);
      W.v.push_back(r->v);
      W.out.push_back(r->out);
      W.ws.push_back(S.arena + off);
      off += (workspace_doubles(*r->cp->plan) + 1) & ~(size_t)1;
    }
    BatchSchedule sched;
    build_group_schedule(W, sched);
    int rc = run_group(S.tab, sched, S.stream);
    hipEvent_t ev = nullptr;
    if (rc == PHIKS_OK && (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
                           hipEventRecord(ev, S.stream) != hipSuccess)) {
      rc = PHIKS_EDEVICE;
      if (ev) (void)hipEventDestroy(ev);
      ev = nullptr;
    }
    std::lock_guard<std::mutex> lk(S.mu);
    ++S.st.groups;
    if (rc != PHIKS_OK) {
      (void)hipStreamSynchronize(S.stream);
      const double t = now_s();
      for (ServerRequest* r : run) {
        --r->cp->refs;
        server_finish(S, r, rc, t);
      }
      S.cv_done.notify_all();
      continue;
    }
    S.inflight.push_back({ev, run});
    S.cv_inflight.notify_all();
  }
  std::lock_guard<std::mutex> lk(S.mu);
  S.worker_done = true;
  S.cv_inflight.notify_all();
}

void server_completer(phiks_server_s* Sp) {
  phiks_server_s& S = *Sp;
  (void)hipSetDevice(S.device);
  for (;;) {
    InFlightGroup g;
    {
      std::unique_lock<std::mutex> lk(S.mu);
      S.cv_inflight.wait(lk, [&] { return !S.inflight.empty() || S.worker_done; });
      if (S.inflight.empty()) break;
      g = S.inflight.front();
      S.inflight.pop_front();
    }
    const int status = (hipEventSynchronize(g.ev) == hipSuccess) ? PHIKS_OK : PHIKS_EDEVICE;
    const double t = now_s();
    (void)hipEventDestroy(g.ev);
    {
      std::lock_guard<std::mutex> lk(S.mu);
      for (ServerRequest* r : g.reqs) {
        --r->cp->refs;
        server_finish(S, r, status, t);
      }
    }
    S.cv_done.notify_all();
  }
}

}  // namespace

extern "C" {

int phiks_server_select_group(int count, const int* p, const int* n_scales,
                              const size_t* ws_doubles, size_t arena_doubles, int max_group,
                              int* picked, int* npicked) {
  if (count < 0 || max_group < 1 || !npicked || (count > 0 && (!p || !n_scales || !ws_doubles || !picked)))
    return PHIKS_EINVAL;
  std::vector<GroupCandidate> c(count);
  for (int i = 0; i < count; ++i) c[i] = {p[i], n_scales[i], ws_doubles[i]};
  const std::vector<int> g = select_group(c, arena_doubles, max_group);
  for (size_t i = 0; i < g.size(); ++i) picked[i] = g[i];
  *npicked = (int)g.size();
  return PHIKS_OK;
}

int phiks_server_select_evictions(int count, const size_t* bytes, const int* refs,
                                  const uint64_t* last_use, size_t cache_bytes, size_t new_bytes,
                                  size_t capacity, int* victims, int* nvictims) {
  if (count < 0 || !nvictims || (count > 0 && (!bytes || !refs || !last_use || !victims)))
    return PHIKS_EINVAL;
  std::vector<CacheEntryDesc> e(count);
  for (int i = 0; i < count; ++i) e[i] = {bytes[i], refs[i], last_use[i]};
  const std::vector<int> v = select_evictions(e, cache_bytes, new_bytes, capacity);
  for (size_t i = 0; i < v.size(); ++i) victims[i] = v[i];
  *nvictims = (int)v.size();
  return PHIKS_OK;
}

int phiks_server_create(size_t hbm_budget, size_t workspace_bytes, int max_group,
                        void* hip_stream, phiks_server_t* out) {
  if (!out) return PHIKS_EINVAL;
  *out = nullptr;
  if (max_group < 1 || workspace_bytes < 16 || hbm_budget < workspace_bytes) return PHIKS_EINVAL;
  phiks_server_s* S = new (std::nothrow) phiks_server_s;
  if (!S) return PHIKS_ENOMEM;
  S->budget = hbm_budget;
  S->arena_doubles = workspace_bytes / sizeof(double);
  S->max_group = max_group;
  S->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&S->device) != hipSuccess) {
    delete S;
    set_error("hipGetDevice failed");
    return PHIKS_EDEVICE;
  }
  if (hipMalloc((void**)&S->arena, S->arena_doubles * sizeof(double)) != hipSuccess) {
    delete S;
    set_error("hipMalloc of the server workspace failed");
    return PHIKS_ENOMEM;
  }
  S->worker = std::thread(server_worker, S);
  S->completer = std::thread(server_completer, S);
  *out = S;
  return PHIKS_OK;
}

int phiks_server_register(phiks_server_t server, int d, const int64_t* n,
                          const double* const* A, int64_t* op_id) {
  if (!server || !op_id) return PHIKS_EINVAL;
  // any valid same-vector problem on these matrices (tau, p and tol are checked at submit)
  int rc = validate_problem(d, n, A, 1.0, 0, 1, 1.0, PHIKS_SAME_VECTOR, nullptr);
  if (rc != PHIKS_OK) return rc;
  ServerOperator op;
  op.d = d;
  op.A.resize(d);
  for (int mu = 0; mu < d; ++mu) {
    op.n[mu] = n[mu];
    op.N *= n[mu];
    op.A[mu].assign(A[mu], A[mu] + n[mu] * n[mu]);
  }
  std::lock_guard<std::mutex> lk(server->mu);
  *op_id = server->next_op++;
  server->ops.emplace(*op_id, std::move(op));
  return PHIKS_OK;
}

int phiks_server_submit(phiks_server_t server, int64_t op_id, double tau, int p, int n_scales,
                        double tol, const double* v, double* out, int64_t* ticket) {
  if (!server || !v || !out || !ticket) return PHIKS_EINVAL;
  if (p < 0 || p > PHIKS_MAX_P || n_scales < 1 || n_scales > 16) return PHIKS_EINVAL;
  if (!std::isfinite(tau) || !std::isfinite(tol)) return PHIKS_ENONFINITE;
  if (!(tau > 0.0) || !(tol > 0.0)) return PHIKS_EINVAL;
  ServerRequest* r = new (std::nothrow) ServerRequest;
  if (!r) return PHIKS_ENOMEM;
  r->tau = tau;
  r->tol = tol;
  r->p = p;
  r->ns = n_scales;
  r->v = v;
  r->out = out;
  auto put = [&](const void* src, size_t bytes) {
    const char* c = (const char*)src;
    r->key.bytes.insert(r->key.bytes.end(), c, c + bytes);
  };
  put(&op_id, sizeof(op_id));
  put(&tau, sizeof(tau));
  put(&p, sizeof(p));
  put(&n_scales, sizeof(n_scales));
  put(&tol, sizeof(tol));
  r->key.hash = fnv1a(r->key.bytes.data(), r->key.bytes.size());
  std::lock_guard<std::mutex> lk(server->mu);
  auto it = server->ops.find(op_id);
  if (it == server->ops.end() || server->stop) {
    delete r;
    return PHIKS_EINVAL;
  }
  r->op = &it->second;
  const int64_t t = std::max<int64_t>({(int64_t)kQMax - 1, (int64_t)p, 1});
  r->ws_bound = (size_t)(2 * t + 2 * p) * r->op->N;
  // refused unless select_group could admit it alone (same rounding to even doubles)
  if (((r->ws_bound + 1) & ~(size_t)1) > server->arena_doubles) {
    delete r;
    set_error("request workspace exceeds the server's workspace arena");
    return PHIKS_EWORKSPACE;
  }
  r->ticket = server->next_ticket++;
  r->t_submit = now_s();
  server->tickets[r->ticket] = r;
  server->pending.push_back(r);
  *ticket = r->ticket;
  server->cv_work.notify_one();
  return PHIKS_OK;
}

int phiks_server_wait(phiks_server_t server, int64_t ticket, double* latency_s) {
  if (!server) return PHIKS_EINVAL;
  std::unique_lock<std::mutex> lk(server->mu);
  auto it = server->tickets.find(ticket);
  if (it == server->tickets.end()) return PHIKS_EINVAL;
  ServerRequest* r = it->second;
  server->cv_done.wait(lk, [&] { return r->done; });
  const int status = r->status;
  if (latency_s) *latency_s = r->t_done - r->t_submit;
  server->tickets.erase(it);
  delete r;
  return status;
}

int phiks_server_stats(phiks_server_t server, phiks_server_stats_t* out) {
  if (!server || !out) return PHIKS_EINVAL;
  std::lock_guard<std::mutex> lk(server->mu);
  *out = server->st;
  out->cache_bytes = (int64_t)server->cache_bytes;
  out->cached_plans = (int64_t)server->cache.size();
  return PHIKS_OK;
}

void phiks_server_destroy(phiks_server_t server) {
  if (!server) return;
  {
    std::lock_guard<std::mutex> lk(server->mu);
    server->stop = true;
  }
  server->cv_work.notify_all();
  server->worker.join();      // runs what is pending, then stops
  server->completer.join();   // every group has completed
  (void)hipStreamSynchronize(server->stream);
  for (auto& kv : server->cache) phiks_plan_destroy(kv.second.plan);
  (void)hipStreamSynchronize(server->stream);
  free_group_tables(server->tab);
  if (server->arena) (void)hipFree(server->arena);
  for (auto& kv : server->tickets) delete kv.second;
  delete server;
}

}  // extern "C"
