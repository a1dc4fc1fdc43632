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
PlanChoice choose_sq(const Rect& xi, int p, int n_scales, double tol, int task,
                     const double* vnorms);

}  // namespace phiks
