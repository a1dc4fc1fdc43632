// The plan object behind phiks_plan_t: problem shape, the chosen (s, q), the GLL rule
// and the device copies of the small exponentials.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "phiks.h"
#include "planner.hpp"

// ------------------------------------------------------------------- the plan
struct phiks_plan_s {
  int d = 0;
  int64_t n[PHIKS_MAX_D] = {0};
  int64_t N = 0;
  double tau = 0.0, tau_im = 0.0;    // the step (imaginary part: complex plans)
  int p = 0, ns = 1, task = 0, precision = 0;
  int s = 0, q = 0, t_paper = 0, t_exec = 0;
  double theta[phiks::kQMax] = {0}, w[phiks::kQMax] = {0};
  // right edge of the numerical-range rectangle of each B_mu = tau A_mu: at least the
  // largest eigenvalue of its Hermitian part, so ||exp(c B_mu)|| <= exp(c re_hi[mu])
  double re_hi[PHIKS_MAX_D] = {0};
  int device = 0;
  hipStream_t stream = nullptr;         // stream the plan was built on (and is released on)
  void* dmem = nullptr;                 // all plan-lifetime device matrices
  double* Lnode[PHIKS_MAX_D] = {nullptr};  // (q-1) node matrices per mode, stride n^2
  double* E[PHIKS_MAX_D] = {nullptr};      // (s+1) matrices per mode: exp(B/2^j), stride n^2
  float* Lnode32[PHIKS_MAX_D] = {nullptr};  // FP32 copies (mixed precisions)
  float* E32[PHIKS_MAX_D] = {nullptr};
  // PHIKS_BF16X3: the same matrices as pair words (hi | lo << 16 of each FP32 value),
  // at Lnode32[mu] + pair_off[mu] and E32[mu] + pair_off[mu] (a multiple of 4 floats).
  int64_t pair_off[PHIKS_MAX_D] = {0};
  // Complex plans (A_mu or tau complex; vectors of N complex values, re/im interleaved):
  // Lnode / E hold the real forms of the complex matrices (2n x 2n, the 2 x 2 block
  // [[Re, -Im], [Im, Re]] at block (i, j)), stride 4n^2, and Lsplit / Esplit the
  // n x 2n matrices [Re | Im] of the same exponentials, stride 2n^2.
  int cplx = 0;
  double* Lsplit[PHIKS_MAX_D] = {nullptr};
  double* Esplit[PHIKS_MAX_D] = {nullptr};
};

// Doubles per vector of the plan's problem (N, or 2N for complex vectors).
inline int64_t plan_vec_doubles(const phiks_plan_s& P) { return P.cplx ? 2 * P.N : P.N; }
