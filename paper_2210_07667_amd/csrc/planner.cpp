// Host-side planning for phiks (Section 3.3 of the paper).
//
// * Gauss-Lobatto-Legendre nodes on [0,1]: zeros of P'_{q-1}(2t-1) plus the two
//   endpoints, found by Newton's method in long double; weights
//   1/(q(q-1) P_{q-1}(x_i)^2) on [0,1].
// * Numerical-range rectangle: W(K) is the Minkowski sum of the W(A_mu); each is
//   covered by the Bendixson rectangle [lambda(H)] x i[lambda(S)], H and S the
//   Hermitian and skew-Hermitian parts.  Extreme eigenvalues come from a
//   Householder reduction to tridiagonal form (skipped when the part is already
//   tridiagonal, as for finite-difference operators) and Sturm bisection.
// * Remainder: R_q(f_l(., w)) = (1/2 pi) int_0^{2pi} k_q(z) f_l(z, w)
//   (r e^{i zeta} - e^{-i zeta}/(16 r)) d zeta on the ellipse z = r e^{i zeta} + 1/2
//   + e^{-i zeta}/(16 r) with foci 0 and 1, trapezoidal rule in zeta.  The kernel
//   k_q(z) = int_0^1 pi_q(t) / (pi_q(z) (z - t)) dt is evaluated through the
//   three-term recurrence of the orthogonal polynomials underlying the rule:
//   pi_q(t) = t (t - 1) p_{q-2}(t), p_k monic orthogonal for the weight t(1-t) on
//   [0,1], so that int pi_q(t)/(z-t) dt = -rho_{q-2}(z) with rho_k the associated
//   second-kind functions, which are the minimal solution of the same recurrence and
//   are obtained stably by its backward continued fraction.
// * The contour integral does not depend on r; r is picked per point w near the
//   saddle point of the integrand so that the trapezoidal sum does not cancel.
// * (s, q) search as in Section 3.3 (see choose_sq).
#include "planner.hpp"

#include <algorithm>
#include <climits>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <mutex>

namespace phiks {

using cd = std::complex<double>;

// ------------------------------------------------------------ planner options
namespace {
std::mutex g_opt_mu;
bool g_opt_init = false;
bool g_opt_env_bad = false;
uint64_t g_opt_gen = 0;
PlannerOptions g_opt;

// First use: PHIKS_QMIN, PHIKS_QMAX, PHIKS_SMAX (integers) and PHIKS_PLAN_RECT
// (bendixson | normcentered) override the defaults.  A malformed or out-of-range
// setting leaves the defaults in place and marks the options invalid until replaced.
void init_options_locked() {
  if (g_opt_init) return;
  g_opt_init = true;
  PlannerOptions o;
  bool bad = false;
  auto read_int = [&](const char* name, int& dst) {
    const char* v = std::getenv(name);
    if (!v || !*v) return;
    char* end = nullptr;
    const long x = std::strtol(v, &end, 10);
    if (*end != '\0' || x < INT_MIN || x > INT_MAX) {
      bad = true;
      return;
    }
    dst = (int)x;
  };
  read_int("PHIKS_QMIN", o.q_min);
  read_int("PHIKS_QMAX", o.q_max);
  read_int("PHIKS_SMAX", o.s_max);
  const char* r = std::getenv("PHIKS_PLAN_RECT");
  if (r && *r) {
    if (!std::strcmp(r, "bendixson")) o.rect = RectKind::Bendixson;
    else if (!std::strcmp(r, "normcentered")) o.rect = RectKind::NormCentered;
    else bad = true;
  }
  if (bad || !planner_options_valid(o)) g_opt_env_bad = true;
  else g_opt = o;
}
}  // namespace

bool planner_options(PlannerOptions& out, uint64_t* generation) {
  std::lock_guard<std::mutex> lk(g_opt_mu);
  init_options_locked();
  out = g_opt;
  if (generation) *generation = g_opt_gen;
  return !g_opt_env_bad;
}

bool set_planner_options(const PlannerOptions& o) {
  if (!planner_options_valid(o)) return false;
  std::lock_guard<std::mutex> lk(g_opt_mu);
  init_options_locked();
  g_opt = o;
  g_opt_env_bad = false;
  ++g_opt_gen;
  return true;
}

// ------------------------------------------------------------------ GLL rule
void gll_rule(int q, double* theta, double* w) {
  const int n = q - 1;  // Legendre degree
  auto legendre = [n](long double x, long double& p, long double& pm1) {
    long double a = 1.0L, b = x;
    if (n == 0) { p = 1.0L; pm1 = 0.0L; return; }
    for (int k = 2; k <= n; ++k) {
      long double c = ((2 * k - 1) * x * b - (k - 1) * a) / k;
      a = b;
      b = c;
    }
    p = b;
    pm1 = a;
  };
  std::vector<long double> x(q);
  x[0] = -1.0L;
  x[q - 1] = 1.0L;
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int k = 1; k < n; ++k) {
    long double xi = -std::cos(pi * k / n);
    for (int it = 0; it < 100; ++it) {
      long double P, Pm1;
      legendre(xi, P, Pm1);
      long double dP = n * (xi * P - Pm1) / (xi * xi - 1.0L);
      long double d2P = (2.0L * xi * dP - n * (n + 1) * P) / (1.0L - xi * xi);
      long double step = dP / d2P;
      xi -= step;
      if (std::fabs(step) < 1e-19L) break;
    }
    x[k] = xi;
  }
  for (int k = 0; k < q; ++k) {
    long double P, Pm1;
    legendre(x[k], P, Pm1);
    long double wk = 1.0L / ((long double)n * (n + 1) * P * P);  // half of the [-1,1] weight
    theta[k] = (double)((x[k] + 1.0L) / 2.0L);
    w[k] = (double)wk;
  }
  theta[0] = 0.0;
  theta[q - 1] = 1.0;
}

// -------------------------------------------------- extreme eigenvalues (host)
namespace {

// Number of eigenvalues < x of the symmetric tridiagonal (a, b) (Sturm sequence).
int sturm_count(const std::vector<double>& a, const std::vector<double>& b, double x) {
  const size_t n = a.size();
  int cnt = 0;
  double d = 1.0;
  for (size_t k = 0; k < n; ++k) {
    double bb = (k == 0) ? 0.0 : b[k - 1] * b[k - 1];
    d = a[k] - x - (k == 0 ? 0.0 : bb / d);
    if (d == 0.0) d = -std::numeric_limits<double>::min() * 4.0;
    if (d < 0.0) ++cnt;
  }
  return cnt;
}

void tridiag_extremes(const std::vector<double>& a, const std::vector<double>& b,
                      double& lo, double& hi) {
  const size_t n = a.size();
  double glo = std::numeric_limits<double>::infinity();
  double ghi = -glo;
  for (size_t k = 0; k < n; ++k) {
    double r = (k > 0 ? std::fabs(b[k - 1]) : 0.0) + (k + 1 < n ? std::fabs(b[k]) : 0.0);
    glo = std::min(glo, a[k] - r);
    ghi = std::max(ghi, a[k] + r);
  }
  double pad = 1e-14 * std::max(std::fabs(glo), std::fabs(ghi)) + 1e-300;
  glo -= pad;
  ghi += pad;
  const int nn = (int)n;
  // smallest eigenvalue: the smallest x with count(x) >= 1 ... bisect count(x) == 0
  double l = glo, h = ghi;
  for (int it = 0; it < 200 && h - l > 0; ++it) {
    double m = 0.5 * (l + h);
    if (m <= l || m >= h) break;
    if (sturm_count(a, b, m) >= 1) h = m; else l = m;
  }
  lo = 0.5 * (l + h);
  l = glo;
  h = ghi;
  for (int it = 0; it < 200 && h - l > 0; ++it) {
    double m = 0.5 * (l + h);
    if (m <= l || m >= h) break;
    if (sturm_count(a, b, m) >= nn) h = m; else l = m;
  }
  hi = 0.5 * (l + h);
}

// Householder reduction of a dense symmetric (skew = false) or skew-symmetric
// (skew = true) matrix M (n x n row-major, overwritten) to tridiagonal form;
// returns the diagonal a and the sub-diagonal b.
void householder_tridiag(std::vector<double>& M, int64_t n, bool skew,
                         std::vector<double>& a, std::vector<double>& b) {
  std::vector<double> v(n), p(n), wv(n);
  for (int64_t k = 0; k + 2 < n; ++k) {
    const int64_t m = n - k - 1;  // length of the column below the diagonal
    double nrm = 0.0;
    for (int64_t i = 0; i < m; ++i) {
      double x = M[(k + 1 + i) * n + k];
      nrm += x * x;
    }
    nrm = std::sqrt(nrm);
    double x0 = M[(k + 1) * n + k];
    if (nrm == 0.0) continue;
    double alpha = (x0 > 0) ? -nrm : nrm;
    for (int64_t i = 0; i < m; ++i) v[i] = M[(k + 1 + i) * n + k];
    v[0] -= alpha;
    double vtv = 0.0;
    for (int64_t i = 0; i < m; ++i) vtv += v[i] * v[i];
    if (vtv == 0.0) continue;
    double beta = 2.0 / vtv;
    // p = beta * M' v on the trailing block
    for (int64_t i = 0; i < m; ++i) {
      const double* row = &M[(k + 1 + i) * n + (k + 1)];
      double acc = 0.0;
      for (int64_t j = 0; j < m; ++j) acc += row[j] * v[j];
      p[i] = beta * acc;
    }
    if (!skew) {
      double vp = 0.0;
      for (int64_t i = 0; i < m; ++i) vp += v[i] * p[i];
      double K = 0.5 * beta * vp;
      for (int64_t i = 0; i < m; ++i) wv[i] = p[i] - K * v[i];
      for (int64_t i = 0; i < m; ++i) {
        double* row = &M[(k + 1 + i) * n + (k + 1)];
        for (int64_t j = 0; j < m; ++j) row[j] -= v[i] * wv[j] + wv[i] * v[j];
      }
    } else {
      // H S H = S + v p^T - p v^T for skew S (v^T S v = 0)
      for (int64_t i = 0; i < m; ++i) {
        double* row = &M[(k + 1 + i) * n + (k + 1)];
        for (int64_t j = 0; j < m; ++j) row[j] += v[i] * p[j] - p[i] * v[j];
      }
    }
    M[(k + 1) * n + k] = alpha;
    M[k * n + (k + 1)] = skew ? -alpha : alpha;
    for (int64_t i = 1; i < m; ++i) {
      M[(k + 1 + i) * n + k] = 0.0;
      M[k * n + (k + 1 + i)] = 0.0;
    }
  }
  a.assign(n, 0.0);
  b.assign(n > 0 ? n - 1 : 0, 0.0);
  for (int64_t k = 0; k < n; ++k) a[k] = skew ? 0.0 : M[k * n + k];
  for (int64_t k = 0; k + 1 < n; ++k) b[k] = M[(k + 1) * n + k];
}

}  // namespace

Rect bendixson_rectangle(int64_t n, const double* B) {
  Rect r{};
  std::vector<double> a, b;
  // banded fast path: a tridiagonal B has tridiagonal H = (B+B^T)/2 and S = (B-B^T)/2
  bool tri = true;
  for (int64_t i = 0; i < n && tri; ++i)
    for (int64_t j = 0; j < n; ++j)
      if ((j > i + 1 || i > j + 1) && B[i * n + j] != 0.0) { tri = false; break; }
  if (tri) {
    a.resize(n);
    b.resize(n > 0 ? n - 1 : 0);
    for (int64_t k = 0; k < n; ++k) a[k] = B[k * n + k];
    for (int64_t k = 0; k + 1 < n; ++k) b[k] = 0.5 * (B[(k + 1) * n + k] + B[k * n + k + 1]);
    tridiag_extremes(a, b, r.re_lo, r.re_hi);
    for (int64_t k = 0; k + 1 < n; ++k) b[k] = std::fabs(0.5 * (B[(k + 1) * n + k] - B[k * n + k + 1]));
    for (auto& x : a) x = 0.0;
  } else {
    std::vector<double> H(n * n), S(n * n);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t j = 0; j < n; ++j) {
        H[i * n + j] = 0.5 * (B[i * n + j] + B[j * n + i]);
        S[i * n + j] = 0.5 * (B[i * n + j] - B[j * n + i]);
      }
    householder_tridiag(H, n, false, a, b);
    tridiag_extremes(a, b, r.re_lo, r.re_hi);
    // S real skew: the Hermitian matrix S/i has eigenvalues +-omega; its tridiagonal
    // form has zero diagonal and off-diagonal moduli |b_k|
    householder_tridiag(S, n, true, a, b);
    for (auto& x : b) x = std::fabs(x);
    for (auto& x : a) x = 0.0;
  }
  double lo, hi;
  tridiag_extremes(a, b, lo, hi);
  // the spectrum of S/i is symmetric: use the larger modulus on both sides
  const double om = std::max(std::fabs(lo), std::fabs(hi));
  r.im_lo = -om;
  r.im_hi = om;
  if (n == 1) r.im_lo = r.im_hi = 0.0;
  return r;
}

// Bendixson rectangle of a complex matrix (interleaved re/im, row-major): the real
// parts of the numerical range lie between the extreme eigenvalues of H = (B + B^*)/2,
// the imaginary parts between those of G = (B - B^*)/(2i); both are Hermitian.  A
// Hermitian tridiagonal matrix is unitarily similar (diagonal phase scaling) to the
// real symmetric tridiagonal with the moduli of its off-diagonals; a dense Hermitian
// matrix X has the real symmetric form [[Re X, -Im X], [Im X, Re X]], whose
// eigenvalues are those of X, each twice.
Rect bendixson_rectangle_complex(int64_t n, const double* B) {
  auto re = [&](int64_t i, int64_t j) { return B[2 * (i * n + j)]; };
  auto im = [&](int64_t i, int64_t j) { return B[2 * (i * n + j) + 1]; };
  Rect r{};
  bool tri = true;
  for (int64_t i = 0; i < n && tri; ++i)
    for (int64_t j = 0; j < n; ++j)
      if ((j > i + 1 || i > j + 1) && (re(i, j) != 0.0 || im(i, j) != 0.0)) { tri = false; break; }
  std::vector<double> a, b;
  if (tri) {
    a.resize(n);
    b.resize(n > 0 ? n - 1 : 0);
    // H: diagonal Re B_kk, off-diagonal (B_{k+1,k} + conj B_{k,k+1}) / 2
    for (int64_t k = 0; k < n; ++k) a[k] = re(k, k);
    for (int64_t k = 0; k + 1 < n; ++k)
      b[k] = std::hypot(0.5 * (re(k + 1, k) + re(k, k + 1)), 0.5 * (im(k + 1, k) - im(k, k + 1)));
    tridiag_extremes(a, b, r.re_lo, r.re_hi);
    // G: diagonal Im B_kk, off-diagonal (B_{k+1,k} - conj B_{k,k+1}) / (2i)
    for (int64_t k = 0; k < n; ++k) a[k] = im(k, k);
    for (int64_t k = 0; k + 1 < n; ++k)
      b[k] = std::hypot(0.5 * (re(k + 1, k) - re(k, k + 1)), 0.5 * (im(k + 1, k) + im(k, k + 1)));
    tridiag_extremes(a, b, r.im_lo, r.im_hi);
  } else {
    const int64_t m = 2 * n;
    for (int part = 0; part < 2; ++part) {
      // X = H (part 0) or G (part 1) as a complex Hermitian matrix, then its real form
      std::vector<double> R(m * m);
      for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
          double xr, xi;
          if (part == 0) {  // (B_ij + conj B_ji) / 2
            xr = 0.5 * (re(i, j) + re(j, i));
            xi = 0.5 * (im(i, j) - im(j, i));
          } else {          // (B_ij - conj B_ji) / (2i)
            xr = 0.5 * (im(i, j) + im(j, i));
            xi = -0.5 * (re(i, j) - re(j, i));
          }
          R[i * m + j] = xr;
          R[(i + n) * m + (j + n)] = xr;
          R[i * m + (j + n)] = -xi;
          R[(i + n) * m + j] = xi;
        }
      householder_tridiag(R, m, false, a, b);
      if (part == 0) tridiag_extremes(a, b, r.re_lo, r.re_hi);
      else tridiag_extremes(a, b, r.im_lo, r.im_hi);
    }
  }
  return r;
}

// ------------------------------------------------------ kernel k_q and contour
namespace {

constexpr int kM = 128;        // trapezoidal nodes on the ellipse
constexpr int kNR = 48;        // capacities r on a geometric grid
constexpr double kRLo = 0.3;
constexpr double kRHi = 3.0e5;

struct KTable {
  double r[kNR];
  cd z[kNR][kM];               // contour points
  cd g[kNR][kM];               // r e^{i zeta} - e^{-i zeta}/(16 r)
  cd k[kNR][kQMax + 1][kM];    // k_q(z), q = 2..kQMax
};

// Ratios r_j = rho_j / rho_{j-1} of the second-kind functions of the monic
// polynomials orthogonal for t(1-t) on [0,1]: alpha_j = 1/2, beta_0 = 1/6,
// beta_j = j (j+2) / (4 (2j+1)(2j+3)).  Backward continued fraction.
void second_kind(cd z, cd* rho /* rho_0..rho_{kQMax-2} */) {
  const int need = kQMax - 1;
  std::vector<cd> prev(need), cur(need);
  int nu = 64;
  bool first = true;
  for (int rep = 0; rep < 12; ++rep) {
    cd rr = 0.0;
    for (int j = nu; j >= 0; --j) {
      double beta = (j == 0) ? 1.0 / 6.0 : (double)j * (j + 2) / (4.0 * (2 * j + 1) * (2 * j + 3));
      rr = beta / (z - 0.5 - rr);
      if (j < need) cur[j] = rr;
    }
    if (!first) {
      double diff = 0.0;
      for (int j = 0; j < need; ++j) diff = std::max(diff, std::abs(cur[j] - prev[j]) / std::abs(cur[j]));
      if (diff < 1e-17) break;
    }
    prev = cur;
    first = false;
    nu *= 2;
  }
  cd acc = 1.0;
  for (int j = 0; j < need; ++j) {
    acc *= cur[j];
    rho[j] = acc;
  }
}

// monic p_k(z), k = 0..kQMax-2, by the forward recurrence
void monic_poly(cd z, cd* pk) {
  cd a = 0.0, b = 1.0;
  pk[0] = 1.0;
  for (int j = 0; j + 1 <= kQMax - 2; ++j) {
    double beta = (j == 0) ? 0.0 : (double)j * (j + 2) / (4.0 * (2 * j + 1) * (2 * j + 3));
    cd c = (z - 0.5) * b - beta * a;
    a = b;
    b = c;
    pk[j + 1] = b;
  }
}

const KTable& ktable() {
  static KTable* T = nullptr;
  static std::once_flag once;
  std::call_once(once, [] {
    T = new KTable;
    const double two_pi = 6.283185307179586476925286766559;
    for (int ir = 0; ir < kNR; ++ir) {
      double r = kRLo * std::pow(kRHi / kRLo, (double)ir / (kNR - 1));
      T->r[ir] = r;
      for (int m = 0; m < kM; ++m) {
        double zeta = two_pi * m / kM;
        cd e(std::cos(zeta), std::sin(zeta));
        cd z = r * e + 0.5 + std::conj(e) / (16.0 * r);
        T->z[ir][m] = z;
        T->g[ir][m] = r * e - std::conj(e) / (16.0 * r);
        cd rho[kQMax - 1], pk[kQMax - 1];
        second_kind(z, rho);
        monic_poly(z, pk);
        for (int q = 2; q <= kQMax; ++q) {
          // k_q(z) = -rho_{q-2}(z) / (z (z-1) p_{q-2}(z))
          T->k[ir][q][m] = -rho[q - 2] / (z * (z - 1.0) * pk[q - 2]);
        }
      }
    }
  });
  return *T;
}

}  // namespace

bool remainder(int q, int p, double w_re, double w_im, double* err) {
  const KTable& T = ktable();
  const cd w(w_re, w_im);
  const double aw = std::abs(w);
  if (aw == 0.0) {
    for (int l = 0; l < p; ++l) err[l] = 0.0;
    return true;
  }
  // saddle point of |k_q(z) z^(l-1) e^{-z w}| ~ r^(-(2q-l)) e^{r |w|}, l mid-range
  double lmid = 0.5 * (1 + p);
  double rstar = (2.0 * q - lmid) / aw;
  int ir = 0;
  if (rstar <= T.r[0]) ir = 0;
  else if (rstar >= T.r[kNR - 1]) ir = kNR - 1;
  else ir = (int)std::lround(std::log(rstar / kRLo) / std::log(kRHi / kRLo) * (kNR - 1));
  double fact[kMaxP + 1];
  fact[0] = 1.0;
  for (int l = 1; l <= p; ++l) fact[l] = fact[l - 1] * l;
  cd sum[kMaxP];
  for (int l = 0; l < p; ++l) sum[l] = 0.0;
  for (int m = 0; m < kM; ++m) {
    const cd z = T.z[ir][m];
    const cd ex = (1.0 - z) * w;
    if (ex.real() > 700.0) {
      for (int l = 0; l < p; ++l) err[l] = std::numeric_limits<double>::infinity();
      return false;
    }
    const cd base = T.k[ir][q][m] * std::exp(ex) * T.g[ir][m];
    cd zp = 1.0;
    for (int l = 0; l < p; ++l) {
      sum[l] += base * zp / fact[l];
      zp *= z;
    }
  }
  for (int l = 0; l < p; ++l) {
    double v = std::abs(sum[l]) / kM;
    err[l] = std::isfinite(v) ? v : std::numeric_limits<double>::infinity();
  }
  return true;
}

// ------------------------------------------------------------- (s, q) search
namespace {

void boundary_points(const Rect& xi, std::vector<cd>& pts) {
  cd c[4] = {cd(xi.re_lo, xi.im_lo), cd(xi.re_hi, xi.im_lo), cd(xi.re_hi, xi.im_hi),
             cd(xi.re_lo, xi.im_hi)};
  pts.clear();
  for (int k = 0; k < 4; ++k) {
    cd z0 = c[k], z1 = c[(k + 1) % 4];
    for (int m = 0; m < kSidePoints; ++m) pts.push_back(z0 + (z1 - z0) * ((double)m / kSidePoints));
  }
}

int tucker_count(int task, int s, int q, int p, int ns) {
  return task == 0 ? q + s * p + ns : q * p + s * p + ns;
}

bool check(int task, const double* b, int s, int p, double tol, const double* vn) {
  if (task == 0) {
    double nv = vn ? vn[0] : 1.0;
    for (int l = 1; l <= p; ++l)
      if (!(b[l - 1] * nv <= tol * std::ldexp(1.0, l * s))) return false;
    return true;
  }
  for (int l = 1; l <= p; ++l) {
    double tot = 0.0;
    for (int k = 1; k <= l; ++k) {
      double nv = vn ? vn[p + 1 - k] : 1.0;
      tot += b[l - k] * nv * std::ldexp(1.0, -(l - k + 1) * s);
    }
    if (!(tot <= tol)) return false;
  }
  return true;
}

}  // namespace

bool planner_options_valid(const PlannerOptions& o) {
  return o.q_min >= kQMin && o.q_min <= o.q_max && o.q_max <= kQMax && o.s_max >= 0 &&
         o.s_max <= kSMax && (o.rect == RectKind::Bendixson || o.rect == RectKind::NormCentered);
}

Rect norm_centered_rectangle(const Rect& b, double mean_re, double mean_im) {
  const double hr = std::max(mean_re - b.re_lo, b.re_hi - mean_re);
  const double hi = std::max(mean_im - b.im_lo, b.im_hi - mean_im);
  return Rect{mean_re - hr, mean_re + hr, mean_im - hi, mean_im + hi};
}

Rect range_rectangle(int64_t n, const double* B, RectKind kind) {
  Rect r = bendixson_rectangle(n, B);
  if (kind == RectKind::NormCentered) {
    double tr = 0.0;
    for (int64_t k = 0; k < n; ++k) tr += B[k * n + k];
    r = norm_centered_rectangle(r, tr / (double)n, 0.0);
  }
  return r;
}

Rect range_rectangle_complex(int64_t n, const double* B, RectKind kind) {
  Rect r = bendixson_rectangle_complex(n, B);
  if (kind == RectKind::NormCentered) {
    double tr_re = 0.0, tr_im = 0.0;
    for (int64_t k = 0; k < n; ++k) {
      tr_re += B[2 * (k * n + k)];
      tr_im += B[2 * (k * n + k) + 1];
    }
    r = norm_centered_rectangle(r, tr_re / (double)n, tr_im / (double)n);
  }
  return r;
}

PlanChoice choose_sq(const Rect& xi, int p, int n_scales, double tol, int task,
                     const double* vnorms, const PlannerOptions& opt) {
  PlanChoice out;
  const int s0 = std::max(0, n_scales - 1);
  if (s0 > opt.s_max) return out;  // the requested scales need s >= n_scales - 1
  if (p == 0) {
    out.s = s0;
    out.q = 0;
    out.tucker_paper = n_scales;
    out.ok = true;
    return out;
  }
  std::vector<cd> pts;
  boundary_points(xi, pts);
  // a check passes iff the maximum over the points does, so points that repeat exactly
  // (a side of zero length: the real rectangle of a symmetric operator) are evaluated once
  {
    std::vector<cd> uniq;
    for (const cd& z : pts)
      if (std::find(uniq.begin(), uniq.end(), z) == uniq.end()) uniq.push_back(z);
    pts.swap(uniq);
  }
  const double cp = 1.0 + std::sqrt(2.0);
  size_t hot = 0;  // index of the last violating point: tried first
  auto feasible = [&](int s, int q) {
    double b[kMaxP];
    double e[kMaxP];
    for (int l = 0; l < p; ++l) b[l] = 0.0;
    const double sc = std::ldexp(1.0, -s);
    for (size_t t = 0; t < pts.size(); ++t) {
      size_t idx = (t + hot) % pts.size();
      cd w = pts[idx] * sc;
      remainder(q, p, w.real(), w.imag(), e);
      for (int l = 0; l < p; ++l) b[l] = std::max(b[l], cp * e[l]);
      if (!check(task, b, s, p, tol, vnorms)) {
        hot = idx;
        return false;
      }
    }
    return true;
  };
  bool have_prev = false;
  PlanChoice prev;
  double prevT = 0.0;
  for (int s = s0; s <= opt.s_max; ++s) {
    int qf = -1;
    if (feasible(s, opt.q_max)) {
      for (int q = opt.q_min; q <= opt.q_max; ++q) {
        if (q == opt.q_max || feasible(s, q)) { qf = q; break; }
      }
    }
    double T = (qf < 0) ? std::numeric_limits<double>::infinity()
                        : (double)tucker_count(task, s, qf, p, n_scales);
    if (have_prev && T > prevT) return prev;
    prev.s = s;
    prev.q = qf;
    prev.tucker_paper = (qf < 0) ? 0 : (int)T;
    prev.ok = qf >= 0;
    prevT = T;
    have_prev = true;
  }
  return prev;  // ok == false when no s <= opt.s_max was feasible
}

}  // namespace phiks
