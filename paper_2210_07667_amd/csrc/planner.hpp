// Host-side planning for phiks: quadrature rule, numerical-range rectangle,
// quadrature remainder bound and the choice of (s, q) (Section 3.3 of the paper).
#pragma once

#include <cstdint>
#include <vector>

namespace phiks {

constexpr int kQMin = 3;
constexpr int kQMax = 12;
constexpr int kSMax = 64;
constexpr int kSidePoints = 16;  // boundary points per side of the rectangle
constexpr int kMaxP = 8;         // largest phi index

struct Rect {
  double re_lo, re_hi, im_lo, im_hi;
};

// Which rectangle covers the numerical range W(B_mu) (Section 3.3 estimates it from the
// Hermitian and skew-Hermitian parts without fixing the construction):
// * Bendixson: [lambda_min(H), lambda_max(H)] x i[lambda_min(G), lambda_max(G)] with
//   H = (B + B^*)/2, G = (B - B^*)/(2i), the tightest axis-aligned box around W(B);
// * norm-centred: the box centred at sigma = tr(B)/n (the shift of the remark in
//   Section 3.1) with half-widths ||H - Re(sigma) I||_2 and ||G - Im(sigma) I||_2.
enum class RectKind { Bendixson = 0, NormCentered = 1 };

// The planner's search range and rectangle: q in [q_min, q_max] (Section 3.3 uses 3..12),
// s up to s_max.
struct PlannerOptions {
  int q_min = kQMin;
  int q_max = kQMax;
  int s_max = kSMax;
  RectKind rect = RectKind::Bendixson;
};

// True when 3 <= q_min <= q_max <= kQMax and 0 <= s_max <= kSMax.
bool planner_options_valid(const PlannerOptions& o);

// The process-wide options every plan uses (copied under a lock).  Returns false while
// the environment holds an invalid setting that set_planner_options has not replaced;
// `generation` counts the replacements (plan caches key on it).
bool planner_options(PlannerOptions& out, uint64_t* generation = nullptr);
// Replaces the options; false (nothing changed) when they are not valid.
bool set_planner_options(const PlannerOptions& o);

// The norm-centred box from the Bendixson box of the same matrix and the mean of its
// diagonal: ||H - c I||_2 = max(c - lambda_min(H), lambda_max(H) - c) for Hermitian H,
// and likewise for G.
Rect norm_centered_rectangle(const Rect& bendixson, double mean_re, double mean_im);

// The rectangle of the given kind for a real (row-major) or complex (re/im interleaved,
// row-major) n x n matrix.
Rect range_rectangle(int64_t n, const double* B, RectKind kind);
Rect range_rectangle_complex(int64_t n, const double* B, RectKind kind);

// Gauss-Lobatto-Legendre rule on [0,1]: theta[0] = 0 < ... < theta[q-1] = 1.
void gll_rule(int q, double* theta, double* w);

// Bendixson rectangle of a real n x n row-major matrix.
Rect bendixson_rectangle(int64_t n, const double* B);
// Bendixson rectangle of a complex n x n row-major matrix (re/im interleaved).
Rect bendixson_rectangle_complex(int64_t n, const double* B);

// |R_q(f_l(., w))|, l = 1..p, by the contour integral of Section 3.3.
// Returns false (and +inf entries) when the integrand overflows.
bool remainder(int q, int p, double w_re, double w_im, double* err);

struct PlanChoice {
  int s = 0;
  int q = 0;
  int tucker_paper = 0;
  bool ok = false;
};

// task 0 = same vector, 1 = linear combination; vnorms may be null (all ones).
// s runs from n_scales - 1 to opt.s_max, q from opt.q_min to opt.q_max.
PlanChoice choose_sq(const Rect& xi, int p, int n_scales, double tol, int task,
                     const double* vnorms, const PlannerOptions& opt = PlannerOptions());

}  // namespace phiks
