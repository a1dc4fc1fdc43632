// Host code of the library under the address and undefined-behaviour sanitizers: the
// planner (through phiks_plan_params and phiks_plan_params_complex), the batched launch
// schedule with its tables and capture fork plan (phiks_batch_dryrun, which checks
// every table entry against the problem's buffers), and the server policy functions.
// Linked against a host-only build of the library (no device code runs).
//
//   batch_plan_check <problems file>
// The file (written by tests/test_host_sanitize.py from the batched workload) holds
// little-endian records: int32 count; per distinct matrix size: int32 n, then n*n
// float64 (row-major), terminated by n = 0; per problem: int32 d, d int32 sizes,
// float64 tau.  Exit status 0 when every call succeeds and every check holds.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <vector>

#include "phiks.h"

static int failures = 0;
#define CHECK(c)                                                           \
  do {                                                                     \
    if (!(c)) {                                                            \
      std::fprintf(stderr, "CHECK failed at line %d: %s (%s)\n", __LINE__, #c, \
                   phiks_last_error());                                    \
      ++failures;                                                          \
    }                                                                      \
  } while (0)

template <class T>
static bool rd(FILE* f, T* x, size_t n = 1) {
  return std::fread(x, sizeof(T), n, f) == n;
}

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int count = 0;
  if (!rd(f, &count) || count < 1) return 2;
  std::map<int, std::vector<double>> mats;
  for (;;) {
    int n = 0;
    if (!rd(f, &n)) return 2;
    if (n == 0) break;
    std::vector<double> A((size_t)n * n);
    if (!rd(f, A.data(), A.size())) return 2;
    mats[n] = std::move(A);
  }
  std::vector<int> d(count);
  std::vector<std::vector<int64_t>> n(count);
  std::vector<double> tau(count);
  for (int i = 0; i < count; ++i) {
    if (!rd(f, &d[i])) return 2;
    std::vector<int> sz(d[i]);
    if (!rd(f, sz.data(), sz.size()) || !rd(f, &tau[i])) return 2;
    n[i].assign(sz.begin(), sz.end());
  }
  std::fclose(f);

  // planner on every problem (same vector, p = 3, one scale, tolerance 2^-53 relative)
  std::vector<int> s(count), q(count);
  for (int i = 0; i < count; ++i) {
    std::vector<const double*> A(d[i]);
    for (int mu = 0; mu < d[i]; ++mu) A[mu] = mats[(int)n[i][mu]].data();
    int t = 0;
    CHECK(phiks_plan_params(d[i], n[i].data(), A.data(), tau[i], 3, 1, std::ldexp(1.0, -53),
                            PHIKS_SAME_VECTOR, nullptr, &s[i], &q[i], &t) == PHIKS_OK);
    int s2 = 0, q2 = 0, t2 = 0;   // the combination task too
    CHECK(phiks_plan_params(d[i], n[i].data(), A.data(), tau[i], 3, 2, std::ldexp(1.0, -53),
                            PHIKS_LINCOMB, nullptr, &s2, &q2, &t2) == PHIKS_OK);
  }
  // complex operators: tau (1 + i) times the first few matrices
  for (auto& kv : mats) {
    const int m = kv.first;
    std::vector<double> C(2 * (size_t)m * m);
    for (size_t e = 0; e < (size_t)m * m; ++e) C[2 * e] = C[2 * e + 1] = kv.second[e];
    const double* A[2] = {C.data(), C.data()};
    const int64_t nn[2] = {m, m};
    int a = 0, b = 0, c = 0;
    CHECK(phiks_plan_params_complex(2, nn, A, 1e-3, 1e-3, 4, 2, 1e-12, PHIKS_SAME_VECTOR, nullptr,
                                    &a, &b, &c) == PHIKS_OK);
  }
  // planner options: norm-centred rectangles and a narrower q range on the first problems,
  // then the defaults back (the rest of the run plans with them)
  {
    phiks_planner_options_t prev{}, opt{5, 9, 40, PHIKS_RECT_NORM_CENTERED}, bad{2, 12, 64, 0};
    CHECK(phiks_planner_options(&opt, &prev) == PHIKS_OK);
    CHECK(prev.q_min == 3 && prev.q_max == 12 && prev.s_max == 64 && prev.rect == PHIKS_RECT_BENDIXSON);
    CHECK(phiks_planner_options(&bad, nullptr) == PHIKS_EINVAL);
    for (int i = 0; i < (count < 64 ? count : 64); ++i) {
      std::vector<const double*> A(d[i]);
      for (int mu = 0; mu < d[i]; ++mu) A[mu] = mats[(int)n[i][mu]].data();
      int a = 0, b = 0, c = 0;
      const int rc = phiks_plan_params(d[i], n[i].data(), A.data(), tau[i], 3, 1,
                                       std::ldexp(1.0, -53), PHIKS_SAME_VECTOR, nullptr, &a, &b, &c);
      CHECK(rc == PHIKS_OK || rc == PHIKS_ENOPLAN);
      if (rc == PHIKS_OK) CHECK(b >= 5 && b <= 9 && a <= 40);
      double xi[4];
      CHECK(phiks_range_rectangle(n[i][0], A[0], PHIKS_RECT_NORM_CENTERED, xi) == PHIKS_OK);
      CHECK(xi[0] <= xi[1] && xi[2] <= xi[3]);
    }
    CHECK(phiks_planner_options(&prev, nullptr) == PHIKS_OK);
  }
  // the batched schedule of every problem, and of a few subsets and settings
  std::vector<const int64_t*> np(count);
  for (int i = 0; i < count; ++i) np[i] = n[i].data();
  int64_t L = 0, T = 0, V = 0;
  CHECK(phiks_batch_dryrun(count, d.data(), np.data(), s.data(), q.data(), 3, 1, 4, &L, &T, &V) ==
        PHIKS_OK);
  CHECK(V == 0);
  std::printf("batch of %d: %lld launches, %lld table bytes\n", count, (long long)L, (long long)T);
  const int sub = count < 17 ? count : 17;
  for (int p = 0; p <= 4; ++p)
    for (int ns = 1; ns <= 2; ++ns)
      for (int fk = 0; fk <= 5; fk += 5) {
        std::vector<int> ss(s.begin(), s.begin() + sub);
        for (int& x : ss) x = std::max(x, ns - 1);
        CHECK(phiks_batch_dryrun(sub, d.data(), np.data(), ss.data(), q.data(), p, ns, fk, &L, &T,
                                 &V) == PHIKS_OK);
        CHECK(V == 0);
      }
  // server policy functions on random inputs
  std::mt19937 rng(11);
  for (int it = 0; it < 2000; ++it) {
    const int cnt = (int)(rng() % 20);
    std::vector<size_t> bytes(cnt);
    std::vector<int> refs(cnt), victims(cnt + 1);
    std::vector<uint64_t> last(cnt);
    size_t total = 0;
    for (int k = 0; k < cnt; ++k) {
      bytes[k] = 1 + rng() % 1000;
      refs[k] = (int)(rng() % 3 == 0);
      last[k] = rng() % 100;
      total += bytes[k];
    }
    int nv = -1;
    CHECK(phiks_server_select_evictions(cnt, bytes.data(), refs.data(), last.data(), total,
                                        1 + rng() % 500, rng() % 4000, victims.data(), &nv) ==
          PHIKS_OK);
    CHECK(nv >= 0 && nv <= cnt);
    for (int k = 0; k < nv; ++k) CHECK(victims[k] >= 0 && victims[k] < cnt && refs[victims[k]] == 0);
    const int lanes = 1 + (int)(rng() % 4);
    const int lane = phiks_server_lane(1 + (int64_t)(rng() % (1u << 30)), lanes);
    CHECK(lane >= 0 && lane < lanes);
  }
  if (failures) {
    std::fprintf(stderr, "batch / planner check FAILED (%d)\n", failures);
    return 1;
  }
  std::printf("batch / planner check passed\n");
  return 0;
}
