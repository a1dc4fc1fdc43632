// Runtime and C ABI of the phiks library for MI355X (gfx950).
//
// phiks_plan:    host planning (planner.cpp), then the small exponentials on the
//                device: degree-24 Taylor with scaling and squaring for every node matrix
//                exp((1-theta_i) tau A_mu / 2^s), and exp(tau A_mu / 2^j) for j = s..0
//                by squaring (Section 3.1).
// phiks_apply:   same vector, eqs. integrandsimul / simul.
// phiks_combine: linear combination, eqs. integrandcomb / comb.
// Every exponential of K is a Tucker operator (eq. Tuckerprod): d mu-mode products,
// each one FP64 MFMA GEMM launch (gemm_f64.hpp) with no tensor permutation; the
// weighted sums and the squaring recurrences are fused into the epilogue of the
// last mu-mode product or done by one memory-bound pass (kernels.hpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "gemm_f32.hpp"
#include "gemm_f64.hpp"
#include "kernels.hpp"
#include "phiks.h"
#include "plan.hpp"
#include "planner.hpp"
#include "runtime.hpp"
#include "stage.hpp"
#include "tucker_mixed.hpp"
#include "tucker_f64.hpp"

using namespace phiks;

namespace {

int64_t sq(int64_t x) { return x * x; }

// Which small matrices a Tucker operator of the phi recurrence uses.
enum class MatSel { AllNodes, Node, Level };

// Tucker operator of the plan in its precision: matrices of every node theta_i < 1
// batched (AllNodes), of one node (Node, idx), or exp(B/2^idx) (Level, idx).
template <class Epi>
int plan_tucker(const phiks_plan_s& P, MatSel sel, int idx, const double* in,
                int64_t in_stride, int nbatch, double* out, double* ta, double* tb,
                const Epi& epi, hipStream_t st) {
  int64_t stride[PHIKS_MAX_D];
  for (int mu = 0; mu < P.d; ++mu) stride[mu] = (sel == MatSel::AllNodes) ? P.n[mu] * P.n[mu] : 0;
  if (P.cplx) {
    double* Lr[PHIKS_MAX_D];
    double* Ls[PHIKS_MAX_D];
    int64_t sr[PHIKS_MAX_D], ss[PHIKS_MAX_D];
    for (int mu = 0; mu < P.d; ++mu) {
      const int64_t nn = P.n[mu] * P.n[mu];
      const size_t k = (sel == MatSel::AllNodes) ? 0 : (size_t)idx;
      Lr[mu] = (sel == MatSel::Level) ? P.E[mu] + k * 4 * nn : P.Lnode[mu] + k * 4 * nn;
      Ls[mu] = (sel == MatSel::Level) ? P.Esplit[mu] + k * 2 * nn : P.Lsplit[mu] + k * 2 * nn;
      sr[mu] = 4 * stride[mu];
      ss[mu] = 2 * stride[mu];
    }
    return tucker_complex(P, in, in_stride, Lr, sr, Ls, ss, nbatch, out, ta, tb, epi, st);
  }
  if (P.precision != PHIKS_FP64) {
    float* L[PHIKS_MAX_D];
    for (int mu = 0; mu < P.d; ++mu) {
      const int64_t nn = P.n[mu] * P.n[mu];
      L[mu] = (sel == MatSel::Level) ? P.E32[mu] + (size_t)idx * nn
                                     : P.Lnode32[mu] + (size_t)(sel == MatSel::Node ? idx : 0) * nn;
    }
    if (P.precision == PHIKS_BF16X3)
      return tucker_mixed<PHIKS_BF16X3>(P, in, in_stride, L, stride, nbatch, out, ta, tb, epi, st);
    return tucker_mixed<PHIKS_FP32>(P, in, in_stride, L, stride, nbatch, out, ta, tb, epi, st);
  }
  double* L[PHIKS_MAX_D];
  for (int mu = 0; mu < P.d; ++mu) {
    const int64_t nn = P.n[mu] * P.n[mu];
    L[mu] = (sel == MatSel::Level) ? P.E[mu] + (size_t)idx * nn
                                   : P.Lnode[mu] + (size_t)(sel == MatSel::Node ? idx : 0) * nn;
  }
  return tucker(P, in, in_stride, L, stride, nbatch, out, ta, tb, epi, st);
}

// the buffer (ta or tb) that the last mode does not read
double* tucker_free_buffer(int d, double* ta, double* tb) {
  if (d == 1) return ta;
  return ((d - 1) % 2 == 1) ? tb : ta;
}

// 16-byte accesses: even N and output stride, 16-byte aligned bases
bool combine_vec_ok(const CombineArgs& a) {
  bool v = (a.N % 2 == 0) && (a.out_stride % 2 == 0) && ((uintptr_t)a.out % 16 == 0);
  for (int t = 0; t < a.nin; ++t) v = v && ((uintptr_t)a.in[t] % 16 == 0);
  return v;
}

int launch_combine(const CombineArgs& a_in, hipStream_t st) {
  if (a_in.N <= 0 || a_in.nout <= 0) return PHIKS_OK;
  CombineArgs a = a_in;
  a.vec = combine_vec_ok(a) ? 1 : 0;
  int64_t blocks = (a.N + 255) / 256;
  blocks = std::min<int64_t>(blocks, 8192);
  (void)hipGetLastError();
  hipLaunchKernelGGL(combine_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a);
  CHECK_LAUNCH();
  return PHIKS_OK;
}

double factorial(int k) {
  double f = 1.0;
  for (int i = 2; i <= k; ++i) f *= i;
  return f;
}

// ------------------------------------------------- small matrix exponentials
// exp(c B) for the node matrices and exp(B / 2^s), B = tau A_mu shifted by
// sigma_mu I (Section 3.1 notes the shift leaves the method unchanged): scaling and
// squaring around a degree-24 Taylor polynomial.  For ||X||_1 <= 2 its truncation
// error is below 2^25 / 25! = 2.2e-18, under 2^-53 of ||exp(X)|| >= e^-2.
const double kTaylorTheta = 2.0;
const int kTaylorDegree = 24;
// bound on c (re_hi - sigma) for the shifted exponentials: e^512 < 2^739 leaves room below
// the largest double for the Taylor factor e^2, the squarings' sums and the dimension
const double kShiftHeadroom = 512.0;

// One small operator: the shifted B - sigma I (host, row-major), sigma, its 1-norm.
struct ExpmOp {
  int64_t n;
  std::vector<double> Bshift;
  double sigma;
  double norm1;
};

struct ExpmRequest {
  int op;                  // index into the operator list
  double c;                // exp(c B_op) is requested
  double* dst;             // n^2 destination
  double* dst2 = nullptr;  // optional second destination of the same values
};

// C_i = A_i B_i (+ beta C_i) for pointer arrays of equal-size n x n products; the
// pointer table is staged through S and the launch goes through S.later.
int ptr_gemm(const std::vector<const double*>& a, const std::vector<const double*>& b,
             const std::vector<double*>& c, int n, double beta, Stager& S, hipStream_t st) {
  if (a.empty()) return PHIKS_OK;
  const size_t nb = a.size();
  std::vector<void*> hp(3 * nb);
  for (size_t i = 0; i < nb; ++i) {
    hp[i] = (void*)a[i];
    hp[nb + i] = (void*)b[i];
    hp[2 * nb + i] = (void*)c[i];
  }
  void** dp = nullptr;
  RET_IF(S.table(hp.data(), hp.size(), &dp));
  GemmArgs g = empty_args();
  g.M = g.N = g.K = n;
  g.lda = g.ldb = g.ldc = n;
  g.nb1 = (int)nb;
  g.pA = (const double* const*)dp;
  g.pB = (const double* const*)(dp + nb);
  g.pC = (double* const*)(dp + 2 * nb);
  std::vector<const void*> ptrs;
  for (size_t i = 0; i < nb; ++i) {
    ptrs.push_back(a[i]);
    ptrs.push_back(b[i]);
    ptrs.push_back(c[i]);
  }
  return S.later([g, beta, st, ptrs]() { return launch_gemm<false>(g, EpiStore{1.0, beta}, st, ptrs); });
}

// Computes exp(c_r B_{op_r}) for every request on the device, into dst (and dst2).
// Tables and the work buffer come from S, launches go through S.later (held until
// S.submit when S is deferred).
int batched_expm(const std::vector<ExpmOp>& ops, const std::vector<ExpmRequest>& reqs,
                 Stager& S, hipStream_t st) {
  const size_t nops = ops.size();
  if (reqs.empty()) return PHIKS_OK;
  // Bh = Bshift / beta with beta a power of two >= ||Bshift||_1 (an exact scaling)
  std::vector<double> beta(nops);
  for (size_t o = 0; o < nops; ++o)
    beta[o] = ops[o].norm1 > 0.0 ? std::ldexp(1.0, (int)std::ceil(std::log2(ops[o].norm1))) : 1.0;
  // squarings t_r and polynomial argument X_r = g_r Bh with ||X_r||_1 <= theta
  std::vector<int> tsq(reqs.size());
  std::vector<double> gam(reqs.size());
  for (size_t r = 0; r < reqs.size(); ++r) {
    const int o = reqs[r].op;
    const double x = std::fabs(reqs[r].c) * ops[o].norm1;
    int t = (x > kTaylorTheta) ? (int)std::ceil(std::log2(x / kTaylorTheta)) : 0;
    tsq[r] = std::max(t, 0);
    gam[r] = reqs[r].c * beta[o] / std::ldexp(1.0, tsq[r]);
  }
  // work buffer (freed with S): Bh of every operator, one after the other; per operator
  // Bh^2..Bh^5; per request D_0..D_4 and one squaring buffer
  size_t total = 0;
  std::vector<size_t> b1_off(nops), op_off(nops), req_off(reqs.size());
  for (size_t o = 0; o < nops; ++o) { b1_off[o] = total; total += sq(ops[o].n); }
  for (size_t o = 0; o < nops; ++o) { op_off[o] = total; total += (kTaylorBlocks - 1) * sq(ops[o].n); }
  for (size_t r = 0; r < reqs.size(); ++r) {
    req_off[r] = total;
    total += (kTaylorBlocks + 1) * sq(ops[reqs[r].op].n);
  }
  double* work = nullptr;
  RET_IF(S.scratch(total * sizeof(double), (void**)&work));
  auto pw_ptr = [&](size_t o, int k) {  // Bh^k, k = 1..5
    return k == 1 ? work + b1_off[o] : work + op_off[o] + (size_t)(k - 2) * sq(ops[o].n);
  };
  auto d_ptr = [&](size_t r, int i) { return work + req_off[r] + (size_t)i * sq(ops[reqs[r].op].n); };
  {
    // one upload per operator into the side-by-side region: a deferred S joins those that
    // follow each other in its staging block as on the device into one copy, and no
    // staging block has to hold every operator of a large batch at once
    std::vector<double> h;
    for (size_t o = 0; o < nops; ++o) {
      h.resize(ops[o].Bshift.size());
      for (size_t e = 0; e < h.size(); ++e) h[e] = ops[o].Bshift[e] / beta[o];
      RET_IF(S.upload(pw_ptr(o, 1), h.data(), sizeof(double) * h.size()));
    }
  }
  // operators grouped by size for the pointer-array GEMMs
  std::vector<int64_t> sizes;
  for (size_t o = 0; o < nops; ++o)
    if (std::find(sizes.begin(), sizes.end(), ops[o].n) == sizes.end()) sizes.push_back(ops[o].n);
  // shared powers in three dependent levels: Bh^2 = Bh Bh; Bh^3 = Bh^2 Bh and
  // Bh^4 = Bh^2 Bh^2; Bh^5 = Bh^4 Bh
  static_assert(kTaylorBlocks == 5, "the power levels below form Bh^2 .. Bh^5");
  const int levels[3][2][3] = {{{2, 1, 1}, {0, 0, 0}}, {{3, 2, 1}, {4, 2, 2}}, {{5, 4, 1}, {0, 0, 0}}};
  for (const auto& lev : levels) {
    for (int64_t nsz : sizes) {
      std::vector<const double*> a, b;
      std::vector<double*> c;
      for (const auto& prod : lev) {
        if (prod[0] == 0) continue;
        for (size_t o = 0; o < nops; ++o) {
          if (ops[o].n != nsz) continue;
          a.push_back(pw_ptr(o, prod[1]));
          b.push_back(pw_ptr(o, prod[2]));
          c.push_back(pw_ptr(o, prod[0]));
        }
      }
      RET_IF(ptr_gemm(a, b, c, (int)nsz, 0.0, S, st));
    }
  }
  // D_i of every request
  std::vector<TaylorJob> jobs(reqs.size());
  int64_t nmax = 0;
  for (size_t r = 0; r < reqs.size(); ++r) {
    const int o = reqs[r].op;
    TaylorJob& J = jobs[r];
    std::memset(&J, 0, sizeof(J));
    J.n = (int)ops[o].n;
    nmax = std::max(nmax, ops[o].n);
    for (int k = 1; k < kTaylorBlocks; ++k) J.pw[k] = pw_ptr(o, k);
    double gk = 1.0;  // g^j / j!
    for (int j = 0; j <= kTaylorDegree; ++j) {
      J.coef[j / kTaylorBlocks][j % kTaylorBlocks] = gk;
      gk *= gam[r] / (j + 1);
    }
    for (int i = 0; i < kTaylorBlocks; ++i) J.D[i] = d_ptr(r, i);
  }
  TaylorJob* djobs = nullptr;
  RET_IF(S.table(jobs.data(), jobs.size(), &djobs));
  const unsigned eblocks = (unsigned)std::min<int64_t>((sq(nmax) + 255) / 256, 1024);
  const unsigned njobs = (unsigned)jobs.size();
  RET_IF(S.later([=]() {
    (void)hipGetLastError();
    hipLaunchKernelGGL(taylor_form_kernel, dim3(eblocks, njobs), dim3(256), 0, st, djobs);
    CHECK_LAUNCH();
    return PHIKS_OK;
  }));
  // Horner in S = Bh^5: D_i <- D_(i+1) S + D_i, i = 3..0; D_0 then holds T(X)
  for (int i = kTaylorBlocks - 2; i >= 0; --i) {
    for (int64_t nsz : sizes) {
      std::vector<const double*> a, b;
      std::vector<double*> c;
      for (size_t r = 0; r < reqs.size(); ++r) {
        if (ops[reqs[r].op].n != nsz) continue;
        a.push_back(d_ptr(r, i + 1));
        b.push_back(pw_ptr(reqs[r].op, kTaylorBlocks));
        c.push_back(d_ptr(r, i));
      }
      RET_IF(ptr_gemm(a, b, c, (int)nsz, 1.0, S, st));
    }
  }
  // squarings: X <- X^2 (ping-pong through the request's last buffer)
  std::vector<double*> curp(reqs.size()), othp(reqs.size());
  int tmax = 0;
  for (size_t r = 0; r < reqs.size(); ++r) {
    curp[r] = d_ptr(r, 0);
    othp[r] = d_ptr(r, kTaylorBlocks);
    tmax = std::max(tmax, tsq[r]);
  }
  for (int t = 0; t < tmax; ++t) {
    for (int64_t nsz : sizes) {
      std::vector<const double*> a, b;
      std::vector<double*> c;
      std::vector<size_t> idx;
      for (size_t r = 0; r < reqs.size(); ++r) {
        if (ops[reqs[r].op].n != nsz || tsq[r] <= t) continue;
        a.push_back(curp[r]);
        b.push_back(curp[r]);
        c.push_back(othp[r]);
        idx.push_back(r);
      }
      RET_IF(ptr_gemm(a, b, c, (int)nsz, 0.0, S, st));
      for (size_t r : idx) std::swap(curp[r], othp[r]);
    }
  }
  // dst (and dst2) = e^{c sigma} X
  std::vector<ScaleJob> sj;
  for (size_t r = 0; r < reqs.size(); ++r) {
    const double scale = std::exp(reqs[r].c * ops[reqs[r].op].sigma);
    const int n = (int)ops[reqs[r].op].n;
    sj.push_back({curp[r], reqs[r].dst, scale, n});
    if (reqs[r].dst2) sj.push_back({curp[r], reqs[r].dst2, scale, n});
  }
  ScaleJob* dsj = nullptr;
  RET_IF(S.table(sj.data(), sj.size(), &dsj));
  const unsigned nsj = (unsigned)sj.size();
  return S.later([=]() {
    (void)hipGetLastError();
    hipLaunchKernelGGL(scale_copy_kernel, dim3(eblocks, nsj), dim3(256), 0, st, dsj);
    CHECK_LAUNCH();
    return PHIKS_OK;
  });
}

// The GEMM views of a mu-mode product hold prod(n_<mu) and prod(n_>mu) (times `mult`
// doubles per value: 2 for complex data) in 32-bit fields; shapes beyond that are refused.
bool views_fit_int32(int d, const int64_t* n, int64_t mult) {
  for (int mu = 0; mu < d; ++mu) {
    int64_t lo = mult, hi = 1;
    for (int k = 0; k < mu; ++k) lo *= n[k];
    for (int k = mu + 1; k < d; ++k) hi *= n[k];
    if (lo > 0x7fffffffLL || hi > 0x7fffffffLL) return false;
  }
  return true;
}

int validate_problem(int d, const int64_t* n, const double* const* A, double tau, int p,
                     int n_scales, double tol, int task, const double* vnorms) {
  if (d < 1 || d > PHIKS_MAX_D || !n || !A) return PHIKS_EINVAL;
  if (p < 0 || p > PHIKS_MAX_P || n_scales < 1 || n_scales > 16) return PHIKS_EINVAL;
  if (task != PHIKS_SAME_VECTOR && task != PHIKS_LINCOMB) return PHIKS_EINVAL;
  if (!std::isfinite(tau) || !std::isfinite(tol)) return PHIKS_ENONFINITE;
  if (!(tau > 0.0) || !(tol > 0.0)) return PHIKS_EINVAL;
  int64_t N = 1;
  for (int mu = 0; mu < d; ++mu) {
    if (n[mu] < 1 || n[mu] > PHIKS_MAX_N || !A[mu]) return PHIKS_EINVAL;
    N *= n[mu];
    if (N > (int64_t)1 << 40) return PHIKS_EINVAL;
    for (int64_t e = 0; e < n[mu] * n[mu]; ++e)
      if (!std::isfinite(A[mu][e])) return PHIKS_ENONFINITE;
  }
  if (!views_fit_int32(d, n, 1)) {
    set_error("a mode's leading or trailing extent exceeds 2^31 - 1");
    return PHIKS_EINVAL;
  }
  if (vnorms) {
    const int nv = (task == PHIKS_SAME_VECTOR) ? 1 : p + 1;
    for (int k = 0; k < nv; ++k)
      if (!std::isfinite(vnorms[k]) || vnorms[k] < 0.0) return PHIKS_EINVAL;
  }
  return PHIKS_OK;
}

// host planning shared by phiks_plan and phiks_plan_params
// The process-wide planner options, or EINVAL (with the reason) while the environment
// holds an invalid setting.
int current_planner_options(PlannerOptions& opt) {
  if (planner_options(opt)) return PHIKS_OK;
  set_error("invalid planner setting in PHIKS_QMIN, PHIKS_QMAX, PHIKS_SMAX or PHIKS_PLAN_RECT");
  return PHIKS_EINVAL;
}

void set_noplan_error(const PlannerOptions& opt) {
  char msg[128];
  std::snprintf(msg, sizeof msg, "no (s, q) with s <= %d and %d <= q <= %d meets the tolerance",
                opt.s_max, opt.q_min, opt.q_max);
  set_error(msg);
}

// host planning shared by phiks_plan and phiks_plan_params (tau > 0, so tau scales the
// rectangle, of the kind the planner options select, without reordering its sides);
// re_hi (if not null) receives each mode's tau * right edge
int host_plan(int d, const int64_t* n, const double* const* A, double tau, int p,
              int n_scales, double tol, int task, const double* vnorms, PlanChoice& pc,
              double* re_hi = nullptr) {
  PlannerOptions opt;
  int rc = current_planner_options(opt);
  if (rc != PHIKS_OK) return rc;
  Rect xi{0.0, 0.0, 0.0, 0.0};
  for (int mu = 0; mu < d; ++mu) {
    Rect r = range_rectangle(n[mu], A[mu], opt.rect);
    if (re_hi) re_hi[mu] = tau * r.re_hi;
    xi.re_lo += tau * r.re_lo;
    xi.re_hi += tau * r.re_hi;
    xi.im_lo += tau * r.im_lo;
    xi.im_hi += tau * r.im_hi;
  }
  pc = choose_sq(xi, p, n_scales, tol, task, vnorms, opt);
  if (!pc.ok) {
    set_noplan_error(opt);
    return PHIKS_ENOPLAN;
  }
  return PHIKS_OK;
}

// quadrature nodes theta_i < 1, each of which needs a Tucker operator
int plan_nodes(const phiks_plan_s& P) { return (P.p > 0) ? P.q - 1 : 0; }

// A combination whose node Tuckers of all p input vectors fit (q - 1) p tensors of at
// most 2^24 doubles in all (the small problems, whose launches do not fill the GPU) runs
// them as one batched launch per mode and sums the nodes in one pass; larger ones take
// one input vector at a time.  FP64 real plans only.
constexpr int64_t kCombineBatchDoubles = int64_t(1) << 24;
bool combine_batches_vectors(const phiks_plan_s& P) {
  return P.task == PHIKS_LINCOMB && !P.cplx && P.precision == PHIKS_FP64 && P.p > 0 &&
         (int64_t)(P.q - 1) * P.p * plan_vec_doubles(P) <= kCombineBatchDoubles;
}

// Tensors per Tucker buffer: max(q - 1, p) (the node Tuckers of one input, batched over
// the nodes, or the p tensors of a squaring step), or (q - 1) p for a combination whose
// node Tuckers of all inputs run together.
int64_t tucker_buffer_tensors(const phiks_plan_s& P) {
  const int64_t t = std::max<int64_t>({(int64_t)P.q - 1, (int64_t)P.p, 1});
  return combine_batches_vectors(P) ? std::max<int64_t>(t, (int64_t)(P.q - 1) * P.p) : t;
}

size_t workspace_doubles(const phiks_plan_s& P) {
  const int64_t N = plan_vec_doubles(P);
  // same vector and combination alike: two Tucker buffers and the double-buffered p
  // running sums
  return (size_t)(2 * tucker_buffer_tensors(P) + 2 * std::max(P.p, 1)) * N;
}


// Fills P with the problem and its host plan (no device work).
int plan_init_host(phiks_plan_s& P, int d, const int64_t* n, const double* const* A, double tau,
                   int p, int n_scales, double tol, int task, const double* vnorms,
                   int precision) {
  int rc = validate_problem(d, n, A, tau, p, n_scales, tol, task, vnorms);
  if (rc != PHIKS_OK) return rc;
  if (precision != PHIKS_FP64 && precision != PHIKS_FP32 && precision != PHIKS_BF16X3)
    return PHIKS_EINVAL;
  PlanChoice pc;
  rc = host_plan(d, n, A, tau, p, n_scales, tol, task, vnorms, pc, P.re_hi);
  if (rc != PHIKS_OK) return rc;
  P.d = d;
  P.N = 1;
  for (int mu = 0; mu < d; ++mu) { P.n[mu] = n[mu]; P.N *= n[mu]; }
  P.tau = tau;
  P.p = p;
  P.ns = n_scales;
  P.task = task;
  P.precision = precision;
  P.s = pc.s;
  P.q = pc.q;
  P.t_paper = pc.tucker_paper;
  if (p > 0) gll_rule(pc.q, P.theta, P.w);
  const int nodes = plan_nodes(P);
  if (task == PHIKS_SAME_VECTOR) P.t_exec = nodes + pc.s * p + n_scales;
  else P.t_exec = nodes * p + pc.s * p + n_scales;
  return PHIKS_OK;
}

// Complex problems: A_mu complex (re/im interleaved, row-major), tau complex and
// nonzero.  The rectangle (of the kind the planner options select) is that of each
// B_mu = tau A_mu, summed.
int plan_init_host_complex(phiks_plan_s& P, int d, const int64_t* n, const double* const* A,
                           double tau_re, double tau_im, int p, int n_scales, double tol,
                           int task, const double* vnorms) {
  if (d < 1 || d > PHIKS_MAX_D || !n || !A) return PHIKS_EINVAL;
  if (p < 0 || p > PHIKS_MAX_P || n_scales < 1 || n_scales > 16) return PHIKS_EINVAL;
  if (task != PHIKS_SAME_VECTOR && task != PHIKS_LINCOMB) return PHIKS_EINVAL;
  if (!std::isfinite(tau_re) || !std::isfinite(tau_im) || !std::isfinite(tol)) return PHIKS_ENONFINITE;
  if ((tau_re == 0.0 && tau_im == 0.0) || !(tol > 0.0)) return PHIKS_EINVAL;
  PlannerOptions opt;
  int orc = current_planner_options(opt);
  if (orc != PHIKS_OK) return orc;
  int64_t N = 1;
  Rect xi{0.0, 0.0, 0.0, 0.0};
  for (int mu = 0; mu < d; ++mu) {
    if (n[mu] < 1 || n[mu] > PHIKS_MAX_N || !A[mu]) return PHIKS_EINVAL;
    N *= n[mu];
    if (N > (int64_t)1 << 39) return PHIKS_EINVAL;
    const int64_t m = n[mu];
    std::vector<double> B(2 * m * m);
    for (int64_t e = 0; e < m * m; ++e) {
      const double ar = A[mu][2 * e], ai = A[mu][2 * e + 1];
      if (!std::isfinite(ar) || !std::isfinite(ai)) return PHIKS_ENONFINITE;
      B[2 * e] = tau_re * ar - tau_im * ai;
      B[2 * e + 1] = tau_re * ai + tau_im * ar;
    }
    const Rect r = range_rectangle_complex(m, B.data(), opt.rect);
    P.re_hi[mu] = r.re_hi;   // also that of the real form's symmetric part
    xi.re_lo += r.re_lo;
    xi.re_hi += r.re_hi;
    xi.im_lo += r.im_lo;
    xi.im_hi += r.im_hi;
  }
  if (!views_fit_int32(d, n, 2)) {
    set_error("a mode's leading or trailing extent exceeds 2^31 - 1");
    return PHIKS_EINVAL;
  }
  if (vnorms) {
    const int nv = (task == PHIKS_SAME_VECTOR) ? 1 : p + 1;
    for (int k = 0; k < nv; ++k)
      if (!std::isfinite(vnorms[k]) || vnorms[k] < 0.0) return PHIKS_EINVAL;
  }
  const PlanChoice pc = choose_sq(xi, p, n_scales, tol, task, vnorms, opt);
  if (!pc.ok) {
    set_noplan_error(opt);
    return PHIKS_ENOPLAN;
  }
  P.d = d;
  P.N = N;
  for (int mu = 0; mu < d; ++mu) P.n[mu] = n[mu];
  P.tau = tau_re;
  P.tau_im = tau_im;
  P.cplx = 1;
  P.p = p;
  P.ns = n_scales;
  P.task = task;
  P.precision = PHIKS_FP64;
  P.s = pc.s;
  P.q = pc.q;
  P.t_paper = pc.tucker_paper;
  if (p > 0) gll_rule(pc.q, P.theta, P.w);
  const int nodes = plan_nodes(P);
  if (task == PHIKS_SAME_VECTOR) P.t_exec = nodes + pc.s * p + n_scales;
  else P.t_exec = nodes * p + pc.s * p + n_scales;
  return PHIKS_OK;
}

// Doubles per mode of the mixed-precision copies: the FP32 node matrices and exp(B/2^j)
// (each block rounded up to whole doubles), then for PHIKS_BF16X3 the same blocks again
// as pair words, the whole rounded up to an even count so the pair copy keeps the FP32
// copy's 16-byte alignment.
size_t mixed_doubles(const phiks_plan_s& P, int mu) {
  if (P.precision == PHIKS_FP64) return 0;
  const size_t nn = sq(P.n[mu]);
  const size_t f32 = ((size_t)plan_nodes(P) * nn + 3) / 2 + 1 + ((size_t)(P.s + 1) * nn + 3) / 2 + 1;
  return P.precision == PHIKS_BF16X3 ? 2 * ((f32 + 1) / 2 * 2) : f32;
}

// Plan-lifetime device memory in doubles: per mode the node matrices and exp(B/2^j),
// j = 0..s, then (mixed precision) their copies of mixed_doubles.
size_t plan_device_doubles(const phiks_plan_s& P) {
  const int nodes = plan_nodes(P);
  size_t total = 0;
  if (P.cplx) {  // real forms (4 n^2) and [Re | Im] forms (2 n^2) of every matrix
    for (int mu = 0; mu < P.d; ++mu) total += (size_t)(nodes + P.s + 1) * 6 * sq(P.n[mu]);
    return total;
  }
  for (int mu = 0; mu < P.d; ++mu) total += (size_t)(nodes + P.s + 1) * sq(P.n[mu]);
  for (int mu = 0; mu < P.d; ++mu) total += mixed_doubles(P, mu);
  return total;
}

// Points P's matrices into base (plan_device_doubles(P) doubles, 16-byte aligned).
void plan_assign(phiks_plan_s& P, double* base) {
  const int nodes = plan_nodes(P);
  size_t total = 0;
  if (P.cplx) {
    for (int mu = 0; mu < P.d; ++mu) {
      const size_t nn = sq(P.n[mu]);
      P.Lnode[mu] = base + total;
      total += (size_t)nodes * 4 * nn;
      P.E[mu] = base + total;
      total += (size_t)(P.s + 1) * 4 * nn;
      P.Lsplit[mu] = base + total;
      total += (size_t)nodes * 2 * nn;
      P.Esplit[mu] = base + total;
      total += (size_t)(P.s + 1) * 2 * nn;
    }
    return;
  }
  for (int mu = 0; mu < P.d; ++mu) {
    P.Lnode[mu] = base + total;
    total += (size_t)nodes * sq(P.n[mu]);
    P.E[mu] = base + total;
    total += (size_t)(P.s + 1) * sq(P.n[mu]);
  }
  if (P.precision != PHIKS_FP64) {
    for (int mu = 0; mu < P.d; ++mu) {
      const size_t start = total;
      P.Lnode32[mu] = (float*)(base + total);
      total += ((size_t)nodes * sq(P.n[mu]) + 3) / 2 + 1;
      P.E32[mu] = (float*)(base + total);
      total += ((size_t)(P.s + 1) * sq(P.n[mu]) + 3) / 2 + 1;
      // the pair copy starts half-way into the mode's block: mixed_doubles / 2 doubles,
      // i.e. mixed_doubles floats, after Lnode32
      if (P.precision == PHIKS_BF16X3) P.pair_off[mu] = (int64_t)mixed_doubles(P, mu);
      total = start + mixed_doubles(P, mu);
    }
  }
}

// Builds the small exponentials of every plan in one device pass (Section 3.1): one
// batched_expm over all their operators for the node matrices exp((1-theta_i) B/2^s)
// (theta_1 = 0 gives exp(B/2^s) itself) or exp(B/2^s) alone when p = 0, then
// exp(B/2^(j-1)) = exp(B/2^j)^2 for j = s..1 grouped over plans and modes of equal
// size, then the FP32 copies of the mixed-precision plans.  A[i] are plan i's host
// matrices; every plan's device pointers must already be assigned.
int build_plan_matrices(const std::vector<phiks_plan_s*>& plans,
                        const std::vector<const double* const*>& A, hipStream_t st) {
  Stager S(st);
  S.defer();   // every table of the exponentials in one upload, then their launches
  std::vector<ExpmOp> ops;
  std::vector<ExpmRequest> reqs;
  for (size_t i = 0; i < plans.size(); ++i) {
    const phiks_plan_s& P = *plans[i];
    const int nodes = plan_nodes(P);
    const double inv2s = std::ldexp(1.0, -P.s);
    for (int mu = 0; mu < P.d; ++mu) {
      // shifted operator B - sigma I, sigma = tr(B)/n (the shift remark of Section 3.1);
      // a complex B = tau A is taken in its real form (2n x 2n, blocks [[Re, -Im],
      // [Im, Re]]), whose exponential is the real form of exp(B)
      const int64_t nc = P.n[mu];
      const int64_t m = P.cplx ? 2 * nc : nc;
      ExpmOp op;
      op.n = m;
      op.Bshift.resize(m * m);
      if (P.cplx) {
        const double* Ac = A[i][mu];
        for (int64_t r = 0; r < nc; ++r)
          for (int64_t c = 0; c < nc; ++c) {
            const double ar = Ac[2 * (r * nc + c)], ai = Ac[2 * (r * nc + c) + 1];
            const double br = P.tau * ar - P.tau_im * ai, bi = P.tau * ai + P.tau_im * ar;
            op.Bshift[(2 * r) * m + 2 * c] = br;
            op.Bshift[(2 * r) * m + 2 * c + 1] = -bi;
            op.Bshift[(2 * r + 1) * m + 2 * c] = bi;
            op.Bshift[(2 * r + 1) * m + 2 * c + 1] = br;
          }
      } else {
        for (int64_t e = 0; e < m * m; ++e) op.Bshift[e] = P.tau * A[i][mu][e];
      }
      // shift sigma = tr(B)/m, raised where exp(c (B - sigma I)) could overflow: the
      // largest c taken is 2^-s, and ||exp(c (B - sigma I))|| <= exp(c (re_hi - sigma)),
      // so sigma >= re_hi - kShiftHeadroom 2^s keeps it below e^kShiftHeadroom (the
      // factor e^{c sigma} applied afterwards restores exp(c B) exactly in exact arithmetic)
      double tr = 0.0;
      for (int64_t k = 0; k < m; ++k) tr += op.Bshift[k * m + k];
      op.sigma = std::max(tr / m, P.re_hi[mu] - std::ldexp(kShiftHeadroom, P.s));
      for (int64_t k = 0; k < m; ++k) op.Bshift[k * m + k] -= op.sigma;
      double nrm = 0.0;
      for (int64_t c = 0; c < m; ++c) {
        double col = 0.0;
        for (int64_t r = 0; r < m; ++r) col += std::fabs(op.Bshift[r * m + c]);
        nrm = std::max(nrm, col);
      }
      op.norm1 = nrm;
      const int o = (int)ops.size();
      ops.push_back(std::move(op));
      if (nodes > 0) {
        // theta_1 = 0: that node matrix is exp(B/2^s) itself, written to both places
        for (int k = 0; k < nodes; ++k)
          reqs.push_back({o, (1.0 - P.theta[k]) * inv2s, P.Lnode[mu] + (size_t)k * sq(m),
                          k == 0 ? P.E[mu] + (size_t)P.s * sq(m) : nullptr});
      } else {
        reqs.push_back({o, inv2s, P.E[mu] + (size_t)P.s * sq(m)});
      }
      (void)nc;
    }
  }
  RET_IF(batched_expm(ops, reqs, S, st));
  int smax = 0;
  for (phiks_plan_s* P : plans) smax = std::max(smax, P->s);
  // exp(B/2^(j-1)) = exp(B/2^j)^2, j = s..1, grouped by size
  for (int j = smax; j >= 1; --j) {
    auto opn = [](const phiks_plan_s* P, int mu) { return P->cplx ? 2 * P->n[mu] : P->n[mu]; };
    std::vector<int64_t> sizes;
    for (phiks_plan_s* P : plans)
      if (P->s >= j)
        for (int mu = 0; mu < P->d; ++mu)
          if (std::find(sizes.begin(), sizes.end(), opn(P, mu)) == sizes.end()) sizes.push_back(opn(P, mu));
    for (int64_t nsz : sizes) {
      std::vector<const double*> a;
      std::vector<double*> c;
      for (phiks_plan_s* P : plans) {
        if (P->s < j) continue;
        for (int mu = 0; mu < P->d; ++mu) {
          if (opn(P, mu) != nsz) continue;
          a.push_back(P->E[mu] + (size_t)j * sq(nsz));
          c.push_back(P->E[mu] + (size_t)(j - 1) * sq(nsz));
        }
      }
      RET_IF(ptr_gemm(a, a, c, (int)nsz, 0.0, S, st));
    }
  }
  RET_IF(S.submit());
  // complex plans: the [Re | Im] forms used by the modes > 1
  std::vector<ScaleJob> splits;
  for (phiks_plan_s* P : plans) {
    if (!P->cplx) continue;
    const int nodes = plan_nodes(*P);
    for (int mu = 0; mu < P->d; ++mu) {
      const int64_t nn = sq(P->n[mu]);
      for (int k = 0; k < nodes; ++k)
        splits.push_back({P->Lnode[mu] + (size_t)k * 4 * nn, P->Lsplit[mu] + (size_t)k * 2 * nn, 1.0,
                          (int)P->n[mu]});
      for (int k = 0; k <= P->s; ++k)
        splits.push_back({P->E[mu] + (size_t)k * 4 * nn, P->Esplit[mu] + (size_t)k * 2 * nn, 1.0,
                          (int)P->n[mu]});
    }
  }
  if (!splits.empty()) {
    ScaleJob* dsj = nullptr;
    RET_IF(S.table(splits.data(), splits.size(), &dsj));
    int64_t nmax = 0;
    for (const ScaleJob& j : splits) nmax = std::max<int64_t>(nmax, j.n);
    (void)hipGetLastError();
    hipLaunchKernelGGL(complex_split_kernel,
                       dim3((unsigned)std::min<int64_t>((2 * sq(nmax) + 255) / 256, 1024),
                            (unsigned)splits.size()),
                       dim3(256), 0, st, dsj);
    CHECK_LAUNCH();
  }
  // FP32 copies of every node matrix and of exp(B/2^j): the mixed-precision paths
  // multiply by these; everything else stays FP64
  for (phiks_plan_s* P : plans) {
    if (P->precision == PHIKS_FP64) continue;
    const int nodes = plan_nodes(*P);
    for (int mu = 0; mu < P->d; ++mu) {
      const int64_t ln = (int64_t)nodes * sq(P->n[mu]);
      const int64_t le = (int64_t)(P->s + 1) * sq(P->n[mu]);
      (void)hipGetLastError();
      if (ln > 0)
        hipLaunchKernelGGL(to_f32_kernel, dim3((unsigned)std::min<int64_t>((ln + 255) / 256, 4096)),
                           dim3(256), 0, st, (const double*)P->Lnode[mu], P->Lnode32[mu], ln);
      hipLaunchKernelGGL(to_f32_kernel, dim3((unsigned)std::min<int64_t>((le + 255) / 256, 4096)),
                         dim3(256), 0, st, (const double*)P->E[mu], P->E32[mu], le);
      if (P->precision == PHIKS_BF16X3) {
        if (ln > 0)
          hipLaunchKernelGGL(to_pair_kernel, dim3((unsigned)std::min<int64_t>((ln + 255) / 256, 4096)),
                             dim3(256), 0, st, (const double*)P->Lnode[mu],
                             reinterpret_cast<unsigned*>(P->Lnode32[mu] + P->pair_off[mu]), ln);
        hipLaunchKernelGGL(to_pair_kernel, dim3((unsigned)std::min<int64_t>((le + 255) / 256, 4096)),
                           dim3(256), 0, st, (const double*)P->E[mu],
                           reinterpret_cast<unsigned*>(P->E32[mu] + P->pair_off[mu]), le);
      }
      CHECK_LAUNCH();
    }
  }
  return PHIKS_OK;
}

}  // namespace

namespace {

// ------------------------------------------------ fixed scratch (no allocation)
// Workspace of phiks_apply_noalloc: a file-scope device array, one copy per device
// (the code object places it on every device the library runs on, where it stays
// until the process ends).  Host code never uses the name `scratch` as an address:
// the array's device address on a device comes from hipGetSymbolAddress, taken once
// per device with that device current, and only that address reaches kernels.
__device__ __align__(256) double scratch[PHIKS_NOALLOC_SCRATCH_BYTES / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {nullptr};

// Device address of `scratch` on `device` (looked up on the first call for it).
int noalloc_scratch(int device, void** ptr) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("phiks_apply_noalloc: device index out of range");
    return PHIKS_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = 0;
    HIP_OK(hipGetDevice(&cur));
    if (cur != device) HIP_OK(hipSetDevice(device));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) HIP_OK(hipSetDevice(cur));
    if (e != hipSuccess || p == nullptr) {
      set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return PHIKS_EDEVICE;
    }
    g_scratch_ptr[device] = p;
  }
  *ptr = g_scratch_ptr[device];
  return PHIKS_OK;
}

}  // namespace

// =================================================================== C ABI
extern "C" {

const char* phiks_status_string(int status) {
  switch (status) {
    case PHIKS_OK: return "ok";
    case PHIKS_EINVAL: return "invalid argument";
    case PHIKS_ENOPLAN: return "no (s, q) meets the tolerance";
    case PHIKS_ENOMEM: return "out of memory";
    case PHIKS_EDEVICE: return "device error";
    case PHIKS_EWORKSPACE: return "workspace missing or too small";
    case PHIKS_ENONFINITE: return "non-finite input";
    case PHIKS_ETIMEDOUT: return "deadline passed before the request finished";
    default: return "unknown status";
  }
}

const char* phiks_last_error(void) { return g_last_error.c_str(); }

int phiks_gll(int q, double* theta, double* w) {
  if (q < 2 || q > kQMax || !theta || !w) return PHIKS_EINVAL;
  gll_rule(q, theta, w);
  return PHIKS_OK;
}

int phiks_rectangle(int64_t n, const double* B, double* xi) {
  if (n < 1 || n > PHIKS_MAX_N || !B || !xi) return PHIKS_EINVAL;
  for (int64_t e = 0; e < n * n; ++e)
    if (!std::isfinite(B[e])) return PHIKS_ENONFINITE;
  Rect r = bendixson_rectangle(n, B);
  xi[0] = r.re_lo;
  xi[1] = r.re_hi;
  xi[2] = r.im_lo;
  xi[3] = r.im_hi;
  return PHIKS_OK;
}

int phiks_range_rectangle(int64_t n, const double* B, int rect, double* xi) {
  if (n < 1 || n > PHIKS_MAX_N || !B || !xi) return PHIKS_EINVAL;
  if (rect != PHIKS_RECT_BENDIXSON && rect != PHIKS_RECT_NORM_CENTERED) return PHIKS_EINVAL;
  for (int64_t e = 0; e < n * n; ++e)
    if (!std::isfinite(B[e])) return PHIKS_ENONFINITE;
  const Rect r = range_rectangle(n, B, (RectKind)rect);
  xi[0] = r.re_lo;
  xi[1] = r.re_hi;
  xi[2] = r.im_lo;
  xi[3] = r.im_hi;
  return PHIKS_OK;
}

int phiks_planner_options(const phiks_planner_options_t* set, phiks_planner_options_t* get) {
  PlannerOptions cur;
  const bool env_ok = planner_options(cur);
  if (get) {
    get->q_min = cur.q_min;
    get->q_max = cur.q_max;
    get->s_max = cur.s_max;
    get->rect = (int)cur.rect;
  }
  if (set) {
    PlannerOptions o;
    o.q_min = set->q_min;
    o.q_max = set->q_max;
    o.s_max = set->s_max;
    if (set->rect != PHIKS_RECT_BENDIXSON && set->rect != PHIKS_RECT_NORM_CENTERED) {
      set_error("planner options: unknown rectangle kind");
      return PHIKS_EINVAL;
    }
    o.rect = (RectKind)set->rect;
    if (!set_planner_options(o)) {
      set_error("planner options: need 3 <= q_min <= q_max <= 12 and 0 <= s_max <= 64");
      return PHIKS_EINVAL;
    }
    return PHIKS_OK;
  }
  if (!env_ok) {
    set_error("invalid planner setting in PHIKS_QMIN, PHIKS_QMAX, PHIKS_SMAX or PHIKS_PLAN_RECT");
    return PHIKS_EINVAL;
  }
  return PHIKS_OK;
}

int phiks_remainder(int q, int p, double w_re, double w_im, double* err) {
  if (q < 2 || q > kQMax || p < 1 || p > PHIKS_MAX_P || !err) return PHIKS_EINVAL;
  if (!std::isfinite(w_re) || !std::isfinite(w_im)) return PHIKS_ENONFINITE;
  remainder(q, p, w_re, w_im, err);
  return PHIKS_OK;
}

int phiks_plan_params(int d, const int64_t* n, const double* const* A, double tau, int p,
                      int n_scales, double tol, int task, const double* vnorms, int* s,
                      int* q, int* tucker_paper) {
  int rc = validate_problem(d, n, A, tau, p, n_scales, tol, task, vnorms);
  if (rc != PHIKS_OK) return rc;
  PlanChoice pc;
  rc = host_plan(d, n, A, tau, p, n_scales, tol, task, vnorms, pc);
  if (rc != PHIKS_OK) return rc;
  if (s) *s = pc.s;
  if (q) *q = pc.q;
  if (tucker_paper) *tucker_paper = pc.tucker_paper;
  return PHIKS_OK;
}

int finish_plan(phiks_plan_s* P, const double* const* A, void* hip_stream, phiks_plan_t* out);

int phiks_plan(int d, const int64_t* n, const double* const* A, double tau, int p,
               int n_scales, double tol, int task, const double* vnorms, int precision,
               void* hip_stream, phiks_plan_t* out) {
  if (!out) return PHIKS_EINVAL;
  *out = nullptr;
  phiks_plan_s* P = new (std::nothrow) phiks_plan_s;
  if (!P) return PHIKS_ENOMEM;
  int rc = plan_init_host(*P, d, n, A, tau, p, n_scales, tol, task, vnorms, precision);
  if (rc != PHIKS_OK) {
    delete P;
    return rc;
  }
  return finish_plan(P, A, hip_stream, out);
}

int phiks_plan_complex(int d, const int64_t* n, const double* const* A, double tau_re,
                       double tau_im, int p, int n_scales, double tol, int task,
                       const double* vnorms, void* hip_stream, phiks_plan_t* out) {
  if (!out) return PHIKS_EINVAL;
  *out = nullptr;
  phiks_plan_s* P = new (std::nothrow) phiks_plan_s;
  if (!P) return PHIKS_ENOMEM;
  int rc = plan_init_host_complex(*P, d, n, A, tau_re, tau_im, p, n_scales, tol, task, vnorms);
  if (rc != PHIKS_OK) {
    delete P;
    return rc;
  }
  return finish_plan(P, A, hip_stream, out);
}

int phiks_plan_params_complex(int d, const int64_t* n, const double* const* A, double tau_re,
                              double tau_im, int p, int n_scales, double tol, int task,
                              const double* vnorms, int* s, int* q, int* tucker_paper) {
  phiks_plan_s P;
  int rc = plan_init_host_complex(P, d, n, A, tau_re, tau_im, p, n_scales, tol, task, vnorms);
  if (rc != PHIKS_OK) return rc;
  if (s) *s = P.s;
  if (q) *q = P.q;
  if (tucker_paper) *tucker_paper = P.t_paper;
  return PHIKS_OK;
}

// Device part of phiks_plan / phiks_plan_complex: allocation and the small exponentials.
int finish_plan(phiks_plan_s* P, const double* const* A, void* hip_stream, phiks_plan_t* out) {
  int rc = PHIKS_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  auto fail = [&](int code) {
    phiks_plan_destroy(P);
    return code;
  };
  if (hipGetDevice(&P->device) != hipSuccess) { set_error("hipGetDevice failed"); return fail(PHIKS_EDEVICE); }
  P->stream = st;
  if (hipMallocAsync(&P->dmem, std::max<size_t>(plan_device_doubles(*P), 1) * sizeof(double), st) !=
      hipSuccess) {
    P->dmem = nullptr;
    set_error("hipMallocAsync of plan matrices failed");
    return fail(PHIKS_ENOMEM);
  }
  plan_assign(*P, (double*)P->dmem);
  rc = build_plan_matrices({P}, {A}, st);
  if (rc != PHIKS_OK) return fail(rc);
  *out = P;
  return PHIKS_OK;
}

void phiks_plan_destroy(phiks_plan_t plan) {
  if (!plan) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(plan->device);
  if (plan->dmem) (void)hipFreeAsync(plan->dmem, plan->stream);
  (void)hipSetDevice(cur);
  delete plan;
}

int phiks_plan_info(phiks_plan_t plan, int* s, int* q, int* tucker_paper, int* tucker_exec) {
  if (!plan) return PHIKS_EINVAL;
  if (s) *s = plan->s;
  if (q) *q = plan->q;
  if (tucker_paper) *tucker_paper = plan->t_paper;
  if (tucker_exec) *tucker_exec = plan->t_exec;
  return PHIKS_OK;
}

int phiks_plan_matrix(phiks_plan_t plan, int mu, int kind, int index, double* dst,
                      void* hip_stream) {
  if (!plan || !dst || mu < 0 || mu >= plan->d) return PHIKS_EINVAL;
  const int64_t m = plan->cplx ? 2 * plan->n[mu] : plan->n[mu];
  const double* src = nullptr;
  if (kind == PHIKS_MATRIX_NODE) {
    if (index < 0 || index >= plan_nodes(*plan)) return PHIKS_EINVAL;
    src = plan->Lnode[mu] + (size_t)index * sq(m);
  } else if (kind == PHIKS_MATRIX_LEVEL) {
    if (index < 0 || index > plan->s) return PHIKS_EINVAL;
    src = plan->E[mu] + (size_t)index * sq(m);
  } else {
    return PHIKS_EINVAL;
  }
  HIP_OK(hipMemcpyAsync(dst, src, sq(m) * sizeof(double), hipMemcpyDeviceToDevice,
                        (hipStream_t)hip_stream));
  return PHIKS_OK;
}

int phiks_device_count(int* count) {
  if (!count) return PHIKS_EINVAL;
  *count = 0;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) return PHIKS_OK;  // no device: count 0
  *count = n;
  return PHIKS_OK;
}

int phiks_device_alloc(size_t bytes, void** ptr) {
  if (!ptr) return PHIKS_EINVAL;
  *ptr = nullptr;
  if (bytes == 0) bytes = 8;
  if (hipMalloc(ptr, bytes) != hipSuccess) {
    set_error("hipMalloc failed");
    *ptr = nullptr;
    return PHIKS_ENOMEM;
  }
  return PHIKS_OK;
}

int phiks_device_free(void* ptr) {
  if (!ptr) return PHIKS_OK;
  HIP_OK(hipFree(ptr));
  return PHIKS_OK;
}

int phiks_memcpy_htod(void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return PHIKS_OK;
  if (!dst || !src) return PHIKS_EINVAL;
  HIP_OK(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
  return PHIKS_OK;
}

int phiks_memcpy_dtoh(void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return PHIKS_OK;
  if (!dst || !src) return PHIKS_EINVAL;
  HIP_OK(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost));
  return PHIKS_OK;
}

int phiks_memcpy_dtod(void* dst, const void* src, size_t bytes, void* hip_stream) {
  if (bytes == 0) return PHIKS_OK;
  if (!dst || !src) return PHIKS_EINVAL;
  HIP_OK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, (hipStream_t)hip_stream));
  return PHIKS_OK;
}

int phiks_device_synchronize(void) {
  HIP_OK(hipDeviceSynchronize());
  return PHIKS_OK;
}

int phiks_stream_create(void** stream) {
  if (!stream) return PHIKS_EINVAL;
  *stream = nullptr;
  hipStream_t s = nullptr;
  HIP_OK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  *stream = s;
  return PHIKS_OK;
}

int phiks_stream_destroy(void* stream) {
  if (!stream) return PHIKS_OK;
  HIP_OK(hipStreamDestroy((hipStream_t)stream));
  return PHIKS_OK;
}

int phiks_stream_order(void* first, void* then) {
  if (first == then) return PHIKS_OK;
  hipEvent_t e = nullptr;
  HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  int rc = PHIKS_OK;
  if (hipEventRecord(e, (hipStream_t)first) != hipSuccess ||
      hipStreamWaitEvent((hipStream_t)then, e, 0) != hipSuccess) {
    set_error("event record or stream wait failed");
    rc = PHIKS_EDEVICE;
  }
  // released by the runtime once the recorded work has completed
  (void)hipEventDestroy(e);
  return rc;
}

int phiks_stream_synchronize(void* stream) {
  HIP_OK(hipStreamSynchronize((hipStream_t)stream));
  return PHIKS_OK;
}

int phiks_kernel_timing(int enable) {
  std::lock_guard<std::mutex> lk(g_timing_mu);
  g_timing = (enable != 0);
  return PHIKS_OK;
}

int phiks_kernel_timing_read(double* total_ms, int64_t* launches, double* flops) {
  if (!total_ms || !launches || !flops) return PHIKS_EINVAL;
  std::lock_guard<std::mutex> lk(g_timing_mu);
  double ms = 0.0, fl = 0.0;
  for (size_t i = 0; i < g_timed.size(); ++i) {
    const TimedLaunch& t = g_timed[i];
    HIP_OK(hipEventSynchronize(t.b));
    float x = 0.0f;
    HIP_OK(hipEventElapsedTime(&x, t.a, t.b));
    // kernels of one stream run one after another: a start stamp taken before the previous
    // timed launch on the stream ended is clipped to that end
    if (i > 0 && g_timed[i - 1].st == t.st) {
      float gap = 0.0f;
      HIP_OK(hipEventElapsedTime(&gap, g_timed[i - 1].b, t.a));
      if (gap < 0.0f) HIP_OK(hipEventElapsedTime(&x, g_timed[i - 1].b, t.b));
    }
    ms += x;
    fl += t.flops;
  }
  for (auto& t : g_timed) {
    g_event_pool.push_back(t.a);
    g_event_pool.push_back(t.b);
  }
  *total_ms = ms;
  *launches = (int64_t)g_timed.size();
  *flops = fl;
  g_timed.clear();
  return PHIKS_OK;
}

int phiks_tucker(int d, const int64_t* n, const double* const* L, const double* v,
                 double* out, void* ws, size_t ws_bytes, void* hip_stream) {
  if (d < 1 || d > PHIKS_MAX_D || !n || !L || !v || !out) return PHIKS_EINVAL;
  phiks_plan_s P;
  P.d = d;
  P.N = 1;
  for (int mu = 0; mu < d; ++mu) {
    if (n[mu] < 1 || n[mu] > PHIKS_MAX_N || !L[mu]) return PHIKS_EINVAL;
    P.n[mu] = n[mu];
    P.N *= n[mu];
    if (P.N > (int64_t)1 << 40) return PHIKS_EINVAL;
  }
  if (!views_fit_int32(d, n, 1)) return PHIKS_EINVAL;
  const size_t need = (d >= 2) ? 2 * (size_t)P.N * sizeof(double) : 0;
  if (need > 0 && (!ws || ws_bytes < need)) return PHIKS_EWORKSPACE;
  double* ta = (double*)ws;
  double* tb = ta ? ta + P.N : nullptr;
  double* Ls[PHIKS_MAX_D];
  int64_t zero_stride[PHIKS_MAX_D] = {0};
  for (int mu = 0; mu < d; ++mu) Ls[mu] = const_cast<double*>(L[mu]);
  return tucker(P, v, 0, Ls, zero_stride, 1, out, ta, tb, EpiStore{1.0, 0.0},
                (hipStream_t)hip_stream);
}

int phiks_vector_op(int op, int64_t n, double a, const double* x, double b, const double* y,
                    double* out, void* hip_stream) {
  if (op < PHIKS_VOP_AXPBY || op > PHIKS_VOP_BRUSS_V || n < 0 || (n > 0 && (!x || !out)))
    return PHIKS_EINVAL;
  if (!std::isfinite(a) || !std::isfinite(b)) return PHIKS_ENONFINITE;
  if (n == 0) return PHIKS_OK;
  VecOpArgs v{op, n, a, b, x, y, out};
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  (void)hipGetLastError();
  hipLaunchKernelGGL(vector_op_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)hip_stream, v);
  CHECK_LAUNCH();
  return PHIKS_OK;
}

int phiks_workspace_size(phiks_plan_t plan, size_t* bytes) {
  if (!plan || !bytes) return PHIKS_EINVAL;
  *bytes = workspace_doubles(*plan) * sizeof(double);
  return PHIKS_OK;
}

static int apply_body(const phiks_plan_s& P, const double* v, double* out, void* ws,
                      hipStream_t st);

int phiks_apply(phiks_plan_t plan, const double* v, double* out, void* ws, size_t ws_bytes,
                void* hip_stream) {
  if (!plan || !v || !out) return PHIKS_EINVAL;
  if (plan->task != PHIKS_SAME_VECTOR) return PHIKS_EINVAL;
  const size_t need = workspace_doubles(*plan) * sizeof(double);
  if (!ws || ws_bytes < need) return PHIKS_EWORKSPACE;
  return apply_body(*plan, v, out, ws, (hipStream_t)hip_stream);
}

int phiks_apply_noalloc(phiks_plan_t plan, const double* v, double* out, void* hip_stream) {
  if (!plan || !v || !out) return PHIKS_EINVAL;
  if (plan->task != PHIKS_SAME_VECTOR) return PHIKS_EINVAL;
  const size_t need = workspace_doubles(*plan) * sizeof(double);
  if (need > (size_t)PHIKS_NOALLOC_SCRATCH_BYTES) {
    set_error("phiks_apply_noalloc: the plan needs " + std::to_string(need) +
              " workspace bytes, more than the fixed scratch of " +
              std::to_string((size_t)PHIKS_NOALLOC_SCRATCH_BYTES));
    return PHIKS_EWORKSPACE;
  }
  void* ws = nullptr;
  RET_IF(noalloc_scratch(plan->device, &ws));
  return apply_body(*plan, v, out, ws, (hipStream_t)hip_stream);
}

// Body of phiks_apply once the arguments are checked; ws holds workspace_doubles(P).
static int apply_body(const phiks_plan_s& P, const double* v, double* out, void* ws,
                      hipStream_t st) {
  const int64_t N = plan_vec_doubles(P);  // doubles per vector
  const int p = P.p, ns = P.ns, s = P.s, q = P.q, d = P.d;
  const int64_t tcount = tucker_buffer_tensors(P);
  double* ta = (double*)ws;
  double* tb = ta + tcount * N;
  double* pa = tb + tcount * N;
  double* pb = pa + (int64_t)p * N;
  auto slot = [&](int level, int ell) { return out + ((int64_t)level * (p + 1) + ell) * N; };

  if (p > 0) {
    // eq. integrandsimul: one Tucker per node theta_i < 1, all nodes in one batch
    const int nodes = q - 1;
    double* wbuf = tucker_free_buffer(d, ta, tb);
    RET_IF(plan_tucker(P, MatSel::AllNodes, 0, v, 0, nodes, wbuf, ta, tb, EpiStore{1.0, 0.0}, st));
    double* cur = (s < ns) ? slot(s, 1) : pa;
    CombineArgs ca;
    std::memset(&ca, 0, sizeof(ca));
    ca.nin = nodes + 1;
    for (int i = 0; i < nodes; ++i) ca.in[i] = wbuf + (int64_t)i * N;
    ca.in[nodes] = v;  // theta_q = 1: exp(0) v = v
    ca.out = cur;
    ca.out_stride = N;
    ca.nout = p;
    ca.beta = 0.0;
    ca.N = N;
    for (int ell = 1; ell <= p; ++ell)
      for (int i = 0; i < q; ++i)
        ca.coef[ell - 1][i] = P.w[i] * std::pow(P.theta[i], ell - 1) / factorial(ell - 1);
    RET_IF(launch_combine(ca, st));
    // eq. simul: j = s..1, fused into the last mu-mode product of Tucker(P_l; E_j)
    for (int j = s; j >= 1; --j) {
      double* dst = (j - 1 < ns) ? slot(j - 1, 1) : ((cur == pa) ? pb : pa);
      EpiLinComb epi;
      std::memset(&epi, 0, sizeof(epi));
      epi.Y = cur;
      epi.N = N;
      epi.p = p;
      for (int ell = 1; ell <= p; ++ell) {
        const double sc = std::ldexp(1.0, -ell);
        epi.a[ell - 1] = sc;
        for (int k = 1; k <= ell; ++k) epi.c[ell - 1][k - 1] = sc / factorial(ell - k);
      }
      RET_IF(plan_tucker(P, MatSel::Level, j, cur, N, p, dst, ta, tb, epi, st));
      cur = dst;
    }
  }
  // exponential outputs exp(2^-j tau K) v (eq. tucker with exp(B/2^j))
  for (int lev = 0; lev < ns; ++lev) {
    RET_IF(plan_tucker(P, MatSel::Level, lev, v, 0, 1, slot(lev, 0), ta, tb, EpiStore{1.0, 0.0}, st));
  }
  return PHIKS_OK;
}

}  // extern "C"

namespace {

// Node Tuckers (every node theta_i < 1) of the inputs v[act[0]], ..., v[act[na-1]] of a
// combination with an FP64 real plan, entry (node i, input j) written at out + (i na + j) N.
// The views are tucker_args' for one input, widened to all of them: mode 1 by its free
// batch index z0 (one launch when the inputs lie equally far apart in memory, else one
// launch per input), modes > 1 by folding the input index into their trailing batch z0
// (input j's tensor of a node lies j N after input 0's, since N = n_<mu n_mu n_>mu).
int node_tuckers_of_inputs(const phiks_plan_s& P, const double* const* v, const std::vector<int>& act,
                           double* out, double* ta, double* tb, hipStream_t st) {
  const int na = (int)act.size();
  const int64_t N = P.N;
  double* L[PHIKS_MAX_D];
  int64_t ls[PHIKS_MAX_D];
  for (int mu = 0; mu < P.d; ++mu) {
    L[mu] = P.Lnode[mu];
    ls[mu] = P.n[mu] * P.n[mu];
  }
  GemmArgs gs[PHIKS_MAX_D];
  tucker_args(P.d, P.n, N, v[act[0]], 0, L, ls, plan_nodes(P), out, ta, tb, gs);
  // mode 1: A = the input (rows of N / n_1), B = the node matrices
  GemmArgs g1 = gs[0];
  g1.sC1 = (int64_t)na * N;
  const auto addr = [&](int j) { return (int64_t)(uintptr_t)v[act[j]]; };
  bool even = na > 1 && (addr(1) - addr(0)) % (int64_t)sizeof(double) == 0;
  const int64_t gap = na > 1 ? addr(1) - addr(0) : 0;
  for (int j = 2; j < na && even; ++j) even = addr(j) - addr(j - 1) == gap;
  if (even || na == 1) {
    g1.nb0 = na;
    g1.sA0 = gap / (int64_t)sizeof(double);
    g1.sB0 = 0;
    g1.sC0 = N;
    RET_IF((launch_gemm<true>(g1, EpiStore{1.0, 0.0}, st)));
  } else {
    for (int j = 0; j < na; ++j) {
      GemmArgs g = g1;
      g.A = v[act[j]];
      g.C = g1.C + (int64_t)j * N;
      RET_IF((launch_gemm<true>(g, EpiStore{1.0, 0.0}, st)));
    }
  }
  // modes > 1: B = the previous mode's entries, z0 = j n_>mu + (trailing index)
  for (int mu = 2; mu <= P.d; ++mu) {
    GemmArgs g = gs[mu - 1];
    g.nb0 *= na;
    g.sB1 = (int64_t)na * N;
    g.sC1 = (int64_t)na * N;
    RET_IF((launch_gemm<false>(g, EpiStore{1.0, 0.0}, st)));
  }
  return PHIKS_OK;
}

}  // namespace

extern "C" {

int phiks_combine(phiks_plan_t plan, const double* const* v, double* out, void* ws,
                  size_t ws_bytes, void* hip_stream) {
  if (!plan || !v || !out) return PHIKS_EINVAL;
  if (plan->task != PHIKS_LINCOMB) return PHIKS_EINVAL;
  const phiks_plan_s& P = *plan;
  const size_t need = workspace_doubles(P) * sizeof(double);
  if (!ws || ws_bytes < need) return PHIKS_EWORKSPACE;
  hipStream_t st = (hipStream_t)hip_stream;
  const int64_t N = plan_vec_doubles(P);  // doubles per vector
  const int p = P.p, ns = P.ns, s = P.s, q = P.q, d = P.d;
  const int64_t tcount = tucker_buffer_tensors(P);
  double* ta = (double*)ws;
  double* tb = ta + tcount * N;
  double* qa = tb + tcount * N;
  double* qb = qa + (int64_t)std::max(p, 1) * N;
  bool any = false;
  for (int k = 1; k <= p; ++k) any = any || (v[k] != nullptr);

  // Node sums of eq. integrandcomb, Q_l = sum_i w_i Tucker_i(U_il) with node inputs
  // U_il = sum_{k<=l} theta_i^(l-k)/(l-k)! v_{p+1-k} / 2^((l-k+1)s).  The Tucker operator
  // is linear, so Q_l = sum_{k<=l} sum_i c_ilk Tucker_i(v_{p+1-k}) with
  // c_ilk = w_i theta_i^(l-k)/(l-k)! / 2^((l-k+1)s): one Tucker of each input vector per
  // node, all nodes of one vector in one batched launch per mode (as the same-vector
  // path), their weighted sums accumulated into Q_k..Q_p; for small problems the nodes of
  // all input vectors in one batched launch per mode and one node sum into Q_1..Q_p.  The
  // U_il are never formed.
  auto coef = [&](int i, int ell, int k) {
    return P.w[i] * std::pow(P.theta[i], ell - k) / factorial(ell - k) *
           std::ldexp(1.0, -(ell - k + 1) * s);
  };
  auto emit = [&](int lev, const double* Q) -> int {
    double* o = out + (int64_t)lev * N;
    if (v[0]) {
      if (Q) {
        EpiLinComb epi;
        std::memset(&epi, 0, sizeof(epi));
        epi.Y = Q + (int64_t)(p - 1) * N;
        epi.N = N;
        epi.p = 1;
        epi.a[0] = 1.0;
        epi.c[0][0] = 1.0;
        return plan_tucker(P, MatSel::Level, lev, v[0], 0, 1, o, ta, tb, epi, st);
      }
      return plan_tucker(P, MatSel::Level, lev, v[0], 0, 1, o, ta, tb, EpiStore{1.0, 0.0}, st);
    }
    if (Q) {
      HIP_OK(hipMemcpyAsync(o, Q + (int64_t)(p - 1) * N, N * sizeof(double),
                            hipMemcpyDeviceToDevice, st));
      return PHIKS_OK;
    }
    HIP_OK(hipMemsetAsync(o, 0, N * sizeof(double), st));
    return PHIKS_OK;
  };

  const double* Qcur = nullptr;
  if (p > 0 && any) {
    if (combine_batches_vectors(P)) {
      // the node Tuckers of every input at once, then one node sum (possibly in several
      // passes of at most kMaxIn inputs) over them and the theta_q = 1 terms
      std::vector<int> act;   // input vectors present, v_act[j]
      for (int vi = 1; vi <= p; ++vi)
        if (v[vi]) act.push_back(vi);
      const int na = (int)act.size();
      const int nodes = q - 1;
      double* wbuf = tucker_free_buffer(d, ta, tb);
      RET_IF(node_tuckers_of_inputs(P, v, act, wbuf, ta, tb, st));
      std::vector<const double*> in;
      std::vector<std::array<double, 8>> cf;   // coefficient of input t for Q_1..Q_p
      for (int j = 0; j < na; ++j) {
        const int k = p + 1 - act[j];
        for (int i = 0; i <= nodes; ++i) {
          // i < nodes: entry (i, j) of the node results; i = nodes: theta_q = 1, v itself
          in.push_back(i < nodes ? wbuf + ((int64_t)i * na + j) * N : v[act[j]]);
          std::array<double, 8> c{};
          for (int ell = k; ell <= p; ++ell) c[ell - 1] = coef(i, ell, k);
          cf.push_back(c);
        }
      }
      for (size_t t0 = 0; t0 < in.size(); t0 += kMaxIn) {
        CombineArgs ca;
        std::memset(&ca, 0, sizeof(ca));
        ca.out = qa;
        ca.out_stride = N;
        ca.nout = p;
        ca.beta = (t0 == 0) ? 0.0 : 1.0;
        ca.N = N;
        ca.nin = (int)std::min<size_t>(kMaxIn, in.size() - t0);
        for (int t = 0; t < ca.nin; ++t) {
          ca.in[t] = in[t0 + t];
          for (int ell = 1; ell <= p; ++ell) ca.coef[ell - 1][t] = cf[t0 + t][ell - 1];
        }
        RET_IF(launch_combine(ca, st));
      }
    } else {
      double* Q = qa;
      // node theta_q = 1 (exp(0) = I, no Tucker): Q_l = sum_{k<=l} c_qlk v_{p+1-k}
      {
        CombineArgs ca;
        std::memset(&ca, 0, sizeof(ca));
        ca.out = Q;
        ca.out_stride = N;
        ca.nout = p;
        ca.beta = 0.0;
        ca.N = N;
        int t = 0;
        for (int vi = 1; vi <= p; ++vi) {
          if (!v[vi]) continue;
          const int k = p + 1 - vi;
          ca.in[t] = v[vi];
          for (int ell = k; ell <= p; ++ell) ca.coef[ell - 1][t] = coef(q - 1, ell, k);
          ++t;
        }
        ca.nin = t;
        RET_IF(launch_combine(ca, st));
      }
      // nodes theta_i < 1, one input vector at a time
      const int nodes = q - 1;
      double* wbuf = tucker_free_buffer(d, ta, tb);
      for (int vi = 1; vi <= p; ++vi) {
        if (!v[vi]) continue;
        const int k = p + 1 - vi;
        RET_IF(plan_tucker(P, MatSel::AllNodes, 0, v[vi], 0, nodes, wbuf, ta, tb,
                           EpiStore{1.0, 0.0}, st));
        CombineArgs ca;
        std::memset(&ca, 0, sizeof(ca));
        ca.nin = nodes;
        for (int i = 0; i < nodes; ++i) ca.in[i] = wbuf + (int64_t)i * N;
        ca.out = Q + (int64_t)(k - 1) * N;
        ca.out_stride = N;
        ca.nout = p - k + 1;
        ca.beta = 1.0;
        ca.N = N;
        for (int ell = k; ell <= p; ++ell)
          for (int i = 0; i < nodes; ++i) ca.coef[ell - k][i] = coef(i, ell, k);
        RET_IF(launch_combine(ca, st));
      }
    }
    double* cur = qa;
    if (s < ns) RET_IF(emit(s, cur));
    // eq. comb: Q_l <- Tucker(Q_l; E_j) + sum_{k<=l} Q_k / ((l-k)! 2^((l-k) j))
    for (int j = s; j >= 1; --j) {
      double* dst = (cur == qa) ? qb : qa;
      EpiLinComb epi;
      std::memset(&epi, 0, sizeof(epi));
      epi.Y = cur;
      epi.N = N;
      epi.p = p;
      for (int ell = 1; ell <= p; ++ell) {
        epi.a[ell - 1] = 1.0;
        for (int k = 1; k <= ell; ++k)
          epi.c[ell - 1][k - 1] = std::ldexp(1.0, -(ell - k) * j) / factorial(ell - k);
      }
      RET_IF(plan_tucker(P, MatSel::Level, j, cur, N, p, dst, ta, tb, epi, st));
      cur = dst;
      if (j - 1 < ns) RET_IF(emit(j - 1, cur));
    }
    Qcur = cur;
  } else {
    for (int lev = 0; lev < ns; ++lev) RET_IF(emit(lev, nullptr));
  }
  (void)Qcur;
  return PHIKS_OK;
}

}  // extern "C"

#include "batch.hpp"
#include "server.hpp"
