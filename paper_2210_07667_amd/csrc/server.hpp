// Serving: phi-action requests submitted one at a time, run by step-level continuous
// batching on the GPU.
//
// A request is one phiks_apply (outputs as eq. scaldiffphi) on caller-owned device
// vectors, in FP64, FP32 or BF16x3 mu-mode arithmetic.  Inside the server:
//   * operators are registered once (host copies of A_1..A_d) and named by an id;
//   * plan cache: the plans (host plan + the small exponentials of Section 3.1 on the
//     device) keyed on (operator, tau, p, n_scales, tol, precision); least recently
//     used plans that no running request holds are evicted when the cache would exceed
//     the HBM budget less the workspace arena (select_evictions);
//   * lanes: requests are routed by size (phiks_serve::lane_of) to lanes, each with its
//     own stream, so small requests never wait behind the steps of large ones; the
//     lanes' kernels overlap on the device;
//   * within a lane, the engine of server_core.hpp admits requests in arrival order as
//     workspace slots free up (one slot per request, allocated on admission, released
//     on completion) and runs ticks: one step of every running request of the lane.
//     A request's steps are the launches of phiks_apply -- for FP64 one mu-mode product
//     or node-sum pass each, grouped across the lane's requests into the launches of
//     the batched path (BatchSchedule); for FP32 / BF16x3 one Tucker operator each,
//     issued as phiks_apply issues it -- so every result is bitwise what phiks_apply
//     returns for that request alone, whatever else is running.  A request submitted
//     while others run joins its lane's schedule at the next tick.
// Requests are planned with the relative reading of the tolerance (vnorms = NULL), so
// the plan does not depend on the vector.
//
// Included once, at the end of phiks.hip, after batch.hpp.
#pragma once

#include <atomic>
#include <memory>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "server_core.hpp"

namespace {

struct PlanKey {
  std::vector<char> bytes;  // operator id, tau, p, n_scales, tol, precision, options generation
  uint64_t hash = 0;
  bool operator==(const PlanKey& o) const { return hash == o.hash && bytes == o.bytes; }
};
struct PlanKeyHash {
  size_t operator()(const PlanKey& k) const { return (size_t)k.hash; }
};

struct CachedPlan {
  phiks_plan_s* plan = nullptr;
  size_t bytes = 0;        // device bytes of its matrices
  int refs = 0;            // admitted requests not yet completed
  uint64_t last_use = 0;   // LRU tick
};

struct ServerOperator {
  int d = 0;
  int64_t n[PHIKS_MAX_D] = {0};
  int64_t N = 1;
  std::vector<std::vector<double>> A;  // host copies, row-major
};

// ------------------------------------------------ scheduling policy (host only)
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

// Workspace doubles a request may need: phiks_apply's workspace for the largest q.
size_t request_ws_bound(int p, int64_t N) {
  const int64_t t = std::max<int64_t>({(int64_t)kQMax - 1, (int64_t)p, 1});
  return (size_t)(2 * t + 2 * std::max(p, 1)) * N;
}

// One step of a served request.
struct ReqStep {
  enum Kind { Gemm = 0, Combine = 1, Tucker = 2 } kind = Gemm;
  StepGemm sg{};            // Gemm: one FP64 mu-mode product (grouped across requests)
  CombineArgs ca{};         // Combine: the node sums (grouped)
  // Tucker: one mixed-precision Tucker operator, issued as phiks_apply issues it
  MatSel sel = MatSel::Level;
  int idx = 0, nbatch = 1;
  const double* in = nullptr;
  int64_t in_stride = 0;
  double* out = nullptr;
  bool lincomb = false;
  EpiLinComb lin{};
};

// Executor state of one request (phiks_serve::Request::ctx).
struct ServedRequest {
  PlanKey key;
  const ServerOperator* op = nullptr;
  double tau = 0.0, tol = 0.0;
  int p = 0, ns = 1, precision = PHIKS_FP64;
  const double* v = nullptr;
  double* out = nullptr;
  CachedPlan* cp = nullptr;
  double *ta = nullptr, *tb = nullptr;
  std::vector<ReqStep> steps;
};

// The steps of phiks_apply for plan P on v into out with workspace ws, in its order
// (eqs. integrandsimul and simul, then the exponential outputs): FP64 plans one step
// per mu-mode product (the views of tucker_args) or node-sum pass, mixed-precision plans
// one step per Tucker operator.
void request_steps(const phiks_plan_s& P, const double* v, double* out, double* ws,
                   ServedRequest& R) {
  std::vector<ReqStep>& steps = R.steps;
  steps.clear();
  const int64_t N = P.N;
  const int p = P.p, ns = P.ns, s = P.s, q = P.q, d = P.d;
  const int64_t tcount = std::max<int64_t>({(int64_t)q - 1, (int64_t)p, 1});
  double* ta = ws;
  double* tb = ta + tcount * N;
  double* pa = tb + tcount * N;
  double* pb = pa + (int64_t)p * N;
  R.ta = ta;
  R.tb = tb;
  auto slot = [&](int level, int ell) { return out + ((int64_t)level * (p + 1) + ell) * N; };
  const bool f64 = (P.precision == PHIKS_FP64);
  EpiLinComb lin;
  std::memset(&lin, 0, sizeof(lin));
  lin.N = N;
  lin.p = p;
  for (int ell = 1; ell <= p; ++ell) {
    const double sc = std::ldexp(1.0, -ell);
    lin.a[ell - 1] = sc;
    for (int k = 1; k <= ell; ++k) lin.c[ell - 1][k - 1] = sc / factorial(ell - k);
  }
  auto tucker_steps = [&](MatSel sel, int idx, const double* in, int64_t in_stride, int nbatch,
                          double* dst, const double* Y) {
    if (f64) {
      double* L[PHIKS_MAX_D];
      int64_t stride[PHIKS_MAX_D];
      for (int mu = 0; mu < d; ++mu) {
        const int64_t nn = P.n[mu] * P.n[mu];
        stride[mu] = (sel == MatSel::AllNodes) ? nn : 0;
        L[mu] = (sel == MatSel::Level) ? P.E[mu] + (size_t)idx * nn
                                       : P.Lnode[mu] + (size_t)(sel == MatSel::Node ? idx : 0) * nn;
      }
      GemmArgs gs[PHIKS_MAX_D];
      tucker_args(d, P.n, N, in, in_stride, L, stride, nbatch, dst, ta, tb, gs);
      for (int mu = 1; mu <= d; ++mu) {
        ReqStep st;
        st.kind = ReqStep::Gemm;
        const bool lc = (mu == d) && Y != nullptr;
        st.sg = StepGemm{gs[mu - 1], mu == 1, lc, lc ? Y : nullptr, N, p};
        steps.push_back(st);
      }
      return;
    }
    ReqStep st;
    st.kind = ReqStep::Tucker;
    st.sel = sel;
    st.idx = idx;
    st.in = in;
    st.in_stride = in_stride;
    st.nbatch = nbatch;
    st.out = dst;
    st.lincomb = Y != nullptr;
    st.lin = lin;
    st.lin.Y = Y;
    steps.push_back(st);
  };
  if (p > 0) {
    const int nodes = q - 1;
    double* wbuf = tucker_free_buffer(d, ta, tb);
    tucker_steps(MatSel::AllNodes, 0, v, 0, nodes, wbuf, nullptr);
    double* cur = (s < ns) ? slot(s, 1) : pa;
    ReqStep cs;
    cs.kind = ReqStep::Combine;
    CombineArgs& ca = cs.ca;
    std::memset(&ca, 0, sizeof(ca));
    ca.nin = nodes + 1;
    for (int i = 0; i < nodes; ++i) ca.in[i] = wbuf + (int64_t)i * N;
    ca.in[nodes] = v;
    ca.out = cur;
    ca.out_stride = N;
    ca.nout = p;
    ca.beta = 0.0;
    ca.N = N;
    for (int ell = 1; ell <= p; ++ell)
      for (int i = 0; i < q; ++i)
        ca.coef[ell - 1][i] = P.w[i] * std::pow(P.theta[i], ell - 1) / factorial(ell - 1);
    ca.vec = combine_vec_ok(ca) ? 1 : 0;
    steps.push_back(cs);
    for (int j = s; j >= 1; --j) {
      double* dst = (j - 1 < ns) ? slot(j - 1, 1) : ((cur == pa) ? pb : pa);
      tucker_steps(MatSel::Level, j, cur, N, p, dst, cur);
      cur = dst;
    }
  }
  for (int lev = 0; lev < ns; ++lev) tucker_steps(MatSel::Level, lev, v, 0, 1, slot(lev, 0), nullptr);
}

struct ServerExec;

}  // namespace

struct phiks_server_s {
  size_t budget = 0, arena_doubles = 0;
  int lanes = 1, max_active = 1;
  int device = 0;
  double* arena = nullptr;
  std::vector<hipStream_t> streams;                 // one per lane
  std::vector<std::vector<GroupTables>> rings;      // launch tables per lane, one per tick in flight + 1
  std::vector<int> ring_next;
  std::mutex ev_mu;
  std::vector<hipEvent_t> event_pool;
  std::mutex mu;                                    // operators, cache, stats
  std::unordered_map<int64_t, ServerOperator> ops;
  int64_t next_op = 1;
  std::unordered_map<PlanKey, CachedPlan, PlanKeyHash> cache;
  size_t cache_bytes = 0;
  uint64_t tick = 0;
  phiks_server_stats_t st{};
  std::atomic<int64_t> next_ticket{1};
  std::unique_ptr<ServerExec> exec;
  std::unique_ptr<phiks_serve::Engine<ServerExec>> engine;
};

namespace {

constexpr int kTicksInFlight = 2;

// Cached plan for R on the lane's stream (built on a miss).  Plans of one operator
// all have its size and so serve one lane only.
int server_plan(phiks_server_s& S, ServedRequest& R, hipStream_t st) {
  {
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.cache.find(R.key);
    if (it != S.cache.end()) {
      R.cp = &it->second;
      ++R.cp->refs;
      R.cp->last_use = ++S.tick;
      ++S.st.cache_hits;
      return PHIKS_OK;
    }
  }
  const ServerOperator& op = *R.op;
  std::vector<const double*> A(op.d);
  for (int mu = 0; mu < op.d; ++mu) A[mu] = op.A[mu].data();
  phiks_plan_t plan = nullptr;
  int rc = phiks_plan(op.d, op.n, A.data(), R.tau, R.p, R.ns, R.tol, PHIKS_SAME_VECTOR, nullptr,
                      R.precision, st, &plan);
  if (rc != PHIKS_OK) return rc;
  const size_t bytes = plan_device_doubles(*plan) * sizeof(double);
  std::vector<phiks_plan_s*> evict;
  {
    std::lock_guard<std::mutex> lk(S.mu);
    ++S.st.cache_misses;
    auto it = S.cache.find(R.key);
    if (it != S.cache.end()) {
      // (not reached: a key's requests all run on one lane, whose worker plans them one
      // at a time) the cached plan wins and the new one is released
      R.cp = &it->second;
      ++R.cp->refs;
      R.cp->last_use = ++S.tick;
      evict.push_back(plan);
    } else {
      const size_t cap = S.budget > S.arena_doubles * sizeof(double)
                             ? S.budget - S.arena_doubles * sizeof(double) : 0;
      std::vector<decltype(S.cache)::iterator> its;
      std::vector<CacheEntryDesc> desc;
      for (auto e = S.cache.begin(); e != S.cache.end(); ++e) {
        its.push_back(e);
        desc.push_back({e->second.bytes, e->second.refs, e->second.last_use});
      }
      for (int i : select_evictions(desc, S.cache_bytes, bytes, cap)) {
        S.cache_bytes -= its[i]->second.bytes;
        evict.push_back(its[i]->second.plan);
        S.cache.erase(its[i]);
        ++S.st.evictions;
      }
      auto ins = S.cache.emplace(R.key, CachedPlan{plan, bytes, 1, ++S.tick});
      R.cp = &ins.first->second;
      S.cache_bytes += bytes;
    }
  }
  for (phiks_plan_s* P : evict) phiks_plan_destroy(P);  // stream-ordered on its lane
  return PHIKS_OK;
}

struct ServerExec {
  phiks_server_s* S;

  int prepare(phiks_serve::Request& r) {
    (void)hipSetDevice(S->device);
    ServedRequest& R = *(ServedRequest*)r.ctx;
    RET_IF(server_plan(*S, R, S->streams[r.lane]));
    request_steps(*R.cp->plan, R.v, R.out, S->arena + r.ws_off, R);
    r.nsteps = (int)R.steps.size();
    return PHIKS_OK;
  }

  hipEvent_t get_event() {
    {
      std::lock_guard<std::mutex> lk(S->ev_mu);
      if (!S->event_pool.empty()) {
        hipEvent_t e = S->event_pool.back();
        S->event_pool.pop_back();
        return e;
      }
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
  }

  int issue_steps(int lane, const std::vector<phiks_serve::Request*>& reqs,
                  const std::vector<int>& step) {
    hipStream_t st = S->streams[lane];
    BatchSchedule sch;
    // A tick groups the next steps of a lane's few running requests: 128 x 64 tiles for the
    // squaring epilogue (the batched workload's tuned rule) halve its work-groups there,
    // which costs more than their operand reuse gains (600 requests/s: p50 17 ms and p99
    // 156-163 ms with them, 10-12 ms and 117-127 ms without).  The tile class does not
    // change any result bit.
    sch.tune.wide_lc = 0;
    std::vector<StepGemm> gemms;
    std::vector<CombineArgs> combs;
    std::vector<std::pair<ServedRequest*, const ReqStep*>> tuckers;
    for (size_t i = 0; i < reqs.size(); ++i) {
      ServedRequest& R = *(ServedRequest*)reqs[i]->ctx;
      const ReqStep& x = R.steps[step[i]];
      if (x.kind == ReqStep::Gemm) {
        gemms.push_back(x.sg);
        if (x.sg.lincomb) sch.set_lin(x.sg.p);
      } else if (x.kind == ReqStep::Combine) {
        combs.push_back(x.ca);
      } else {
        tuckers.push_back({&R, &x});
      }
    }
    if (!gemms.empty()) sch.add_gemm_step(gemms);
    if (!combs.empty()) sch.add_combine_step(combs);
    if (!sch.launches.empty()) {
      GroupTables& T = S->rings[lane][S->ring_next[lane]];
      S->ring_next[lane] = (S->ring_next[lane] + 1) % (int)S->rings[lane].size();
      RET_IF(upload_group(T, sch, st));
      RET_IF(issue_group(T, sch, st));
    }
    for (auto& t : tuckers) {
      const phiks_plan_s& P = *t.first->cp->plan;
      const ReqStep& x = *t.second;
      if (x.lincomb)
        RET_IF(plan_tucker(P, x.sel, x.idx, x.in, x.in_stride, x.nbatch, x.out, t.first->ta,
                           t.first->tb, x.lin, st));
      else
        RET_IF(plan_tucker(P, x.sel, x.idx, x.in, x.in_stride, x.nbatch, x.out, t.first->ta,
                           t.first->tb, EpiStore{1.0, 0.0}, st));
    }
    return PHIKS_OK;
  }

  int issue(int lane, const std::vector<phiks_serve::Request*>& reqs, const std::vector<int>& step,
            void** token) {
    (void)hipSetDevice(S->device);
    *token = nullptr;
    int rc = issue_steps(lane, reqs, step);
    hipEvent_t ev = nullptr;
    if (rc == PHIKS_OK) {
      ev = get_event();
      if (!ev || hipEventRecord(ev, S->streams[lane]) != hipSuccess) rc = PHIKS_EDEVICE;
    }
    if (rc != PHIKS_OK) {
      // nothing of the failed tick may remain queued once its requests are completed
      (void)hipStreamSynchronize(S->streams[lane]);
      (void)hipGetLastError();
      if (ev) {
        std::lock_guard<std::mutex> lk(S->ev_mu);
        S->event_pool.push_back(ev);
      }
      return rc;
    }
    *token = ev;
    return PHIKS_OK;
  }

  int wait(int, void* token) {
    (void)hipSetDevice(S->device);
    hipEvent_t ev = (hipEvent_t)token;
    const int rc = hipEventSynchronize(ev) == hipSuccess ? PHIKS_OK : PHIKS_EDEVICE;
    std::lock_guard<std::mutex> lk(S->ev_mu);
    S->event_pool.push_back(ev);
    return rc;
  }

  void finish(phiks_serve::Request& r) {
    ServedRequest& R = *(ServedRequest*)r.ctx;
    std::lock_guard<std::mutex> lk(S->mu);
    if (R.cp) --R.cp->refs;
    R.cp = nullptr;
    ++S->st.completed;
  }
};

void server_release(phiks_server_s* S) {
  if (S->engine) S->engine->shutdown();
  for (hipStream_t s : S->streams) (void)hipStreamSynchronize(s);
  for (auto& kv : S->cache) phiks_plan_destroy(kv.second.plan);
  for (hipStream_t s : S->streams) (void)hipStreamSynchronize(s);
  for (auto& ring : S->rings)
    for (GroupTables& T : ring) free_group_tables(T);
  for (hipEvent_t e : S->event_pool) (void)hipEventDestroy(e);
  for (hipStream_t s : S->streams) (void)hipStreamDestroy(s);
  if (S->arena) (void)hipFree(S->arena);
}

}  // namespace

extern "C" {

int phiks_server_lane(int64_t n_values, int lanes) {
  if (n_values < 1 || lanes < 1) return PHIKS_EINVAL;
  return phiks_serve::lane_of(n_values, lanes);
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

int phiks_server_create(size_t hbm_budget, size_t workspace_bytes, int max_active, int lanes,
                        phiks_server_t* out) {
  if (!out) return PHIKS_EINVAL;
  *out = nullptr;
  if (max_active < 1 || lanes < 1 || lanes > PHIKS_SERVER_MAX_LANES || workspace_bytes < 16 ||
      hbm_budget < workspace_bytes)
    return PHIKS_EINVAL;
  phiks_server_s* S = new (std::nothrow) phiks_server_s;
  if (!S) return PHIKS_ENOMEM;
  S->budget = hbm_budget;
  S->arena_doubles = (workspace_bytes / sizeof(double)) & ~(size_t)1;
  S->max_active = max_active;
  S->lanes = lanes;
  auto fail = [&](int code, const char* msg) {
    set_error(msg);
    server_release(S);
    delete S;
    return code;
  };
  if (hipGetDevice(&S->device) != hipSuccess) return fail(PHIKS_EDEVICE, "hipGetDevice failed");
  if (hipMalloc((void**)&S->arena, S->arena_doubles * sizeof(double)) != hipSuccess) {
    S->arena = nullptr;
    return fail(PHIKS_ENOMEM, "hipMalloc of the server workspace failed");
  }
  for (int l = 0; l < lanes; ++l) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
      return fail(PHIKS_EDEVICE, "hipStreamCreate failed");
    S->streams.push_back(s);
  }
  S->rings.assign(lanes, std::vector<GroupTables>(kTicksInFlight + 1));
  S->ring_next.assign(lanes, 0);
  S->exec.reset(new (std::nothrow) ServerExec{S});
  if (!S->exec) return fail(PHIKS_ENOMEM, "out of host memory");
  S->engine.reset(new (std::nothrow) phiks_serve::Engine<ServerExec>(
      S->exec.get(), S->arena_doubles, lanes, max_active, kTicksInFlight));
  if (!S->engine) return fail(PHIKS_ENOMEM, "out of host memory");
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

static_assert(phiks_serve::kTimedOut == PHIKS_ETIMEDOUT, "one status for expired requests");

int phiks_server_submit(phiks_server_t server, int64_t op_id, double tau, int p, int n_scales,
                        double tol, int precision, double timeout_s, const double* v,
                        double* out, int64_t* ticket) {
  if (!server || !v || !out || !ticket) return PHIKS_EINVAL;
  if (p < 0 || p > PHIKS_MAX_P || n_scales < 1 || n_scales > 16) return PHIKS_EINVAL;
  if (precision != PHIKS_FP64 && precision != PHIKS_FP32 && precision != PHIKS_BF16X3)
    return PHIKS_EINVAL;
  if (!std::isfinite(tau) || !std::isfinite(tol)) return PHIKS_ENONFINITE;
  if (!(tau > 0.0) || !(tol > 0.0)) return PHIKS_EINVAL;
  if (!std::isfinite(timeout_s) || timeout_s < 0.0) return PHIKS_EINVAL;
  std::unique_ptr<ServedRequest> R(new (std::nothrow) ServedRequest);
  std::unique_ptr<phiks_serve::Request> r(new (std::nothrow) phiks_serve::Request);
  if (!R || !r) return PHIKS_ENOMEM;
  R->tau = tau;
  R->tol = tol;
  R->p = p;
  R->ns = n_scales;
  R->precision = precision;
  R->v = v;
  R->out = out;
  auto put = [&](const void* src, size_t bytes) {
    const char* c = (const char*)src;
    R->key.bytes.insert(R->key.bytes.end(), c, c + bytes);
  };
  put(&op_id, sizeof(op_id));
  put(&tau, sizeof(tau));
  put(&p, sizeof(p));
  put(&n_scales, sizeof(n_scales));
  put(&tol, sizeof(tol));
  put(&precision, sizeof(precision));
  // plans made under other planner options are not reused
  PlannerOptions popt;
  uint64_t pgen = 0;
  planner_options(popt, &pgen);
  put(&pgen, sizeof(pgen));
  R->key.hash = fnv1a(R->key.bytes.data(), R->key.bytes.size());
  {
    std::lock_guard<std::mutex> lk(server->mu);
    auto it = server->ops.find(op_id);
    if (it == server->ops.end()) return PHIKS_EINVAL;
    R->op = &it->second;   // operators stay registered until destroy
  }
  r->lane = phiks_serve::lane_of(R->op->N, server->lanes);
  r->ws_doubles = phiks_serve::Arena::round(request_ws_bound(p, R->op->N));
  if (r->ws_doubles > server->arena_doubles) {
    set_error("request workspace exceeds the server's workspace arena");
    return PHIKS_EWORKSPACE;
  }
  r->ticket = server->next_ticket.fetch_add(1);
  r->timeout = timeout_s;
  r->ctx = R.get();
  if (!server->engine->submit(r.get())) return PHIKS_EINVAL;
  *ticket = r->ticket;
  R.release();
  r.release();
  return PHIKS_OK;
}

int phiks_server_wait(phiks_server_t server, int64_t ticket, double* latency_s, double* done_s) {
  if (!server) return PHIKS_EINVAL;
  phiks_serve::Request* r = server->engine->wait(ticket);
  if (!r) return PHIKS_EINVAL;
  const int status = r->status;
  if (latency_s) *latency_s = r->t_done - r->t_submit;
  if (done_s) *done_s = r->t_done;
  delete (ServedRequest*)r->ctx;
  delete r;
  return status;
}

int phiks_server_stats(phiks_server_t server, phiks_server_stats_t* out) {
  if (!server || !out) return PHIKS_EINVAL;
  const phiks_serve::EngineStats es = server->engine->stats();
  std::lock_guard<std::mutex> lk(server->mu);
  *out = server->st;
  out->ticks = es.ticks;
  out->timed_out = es.timed_out;
  out->cache_bytes = (int64_t)server->cache_bytes;
  out->cached_plans = (int64_t)server->cache.size();
  return PHIKS_OK;
}

double phiks_server_clock(void) { return phiks_serve::now_s(); }

void phiks_server_destroy(phiks_server_t server) {
  if (!server) return;
  server_release(server);
  // requests never waited for
  for (phiks_serve::Request* r : server->engine->take_all()) {
    delete (ServedRequest*)r->ctx;
    delete r;
  }
  server->engine.reset();
  delete server;
}

}  // extern "C"
