// Elementwise and small-matrix kernels of the phiks path (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "devptr.hpp"

namespace phiks {

constexpr int kMaxIn = 16;

// out_l[e] = sum_t coef[l][t] * in_t[e]  (+ beta * out_l[e]),  l < nout, t < nin.
// Used for the node sums of eq. integrandsimul (inputs: the node Tucker results and
// v), the node inputs of eq. integrandcomb (inputs: v_1..v_p) and the node
// theta_q = 1 of a combination.  Memory-bound; one pass over the inputs.
struct CombineArgs {
  const double* in[kMaxIn];
  int nin;
  double* out;
  int64_t out_stride;
  int nout;
  double beta;
  int64_t N;
  int vec;              // 1: 16-byte accesses (even N and out_stride, aligned bases)
  double coef[8][kMaxIn];
};

// Elements first, first + stride, ... of one combination.
__device__ __forceinline__ void combine_body(const CombineArgs& a, int64_t first, int64_t stride) {
  PHIKS_GLOBAL double* out = gptr(a.out);
  if (a.vec) {
    // 16-byte accesses (conditions checked by the launcher)
    typedef double d2 __attribute__((ext_vector_type(2)));
    const int64_t N2 = a.N >> 1;
    for (int64_t e = first; e < N2; e += stride) {
      d2 x[kMaxIn];
#pragma unroll
      for (int t = 0; t < kMaxIn; ++t)
        if (t < a.nin) x[t] = reinterpret_cast<const PHIKS_GLOBAL d2*>(gptr(a.in[t]))[e];
      for (int l = 0; l < a.nout; ++l) {
        d2 r = {0.0, 0.0};
#pragma unroll
        for (int t = 0; t < kMaxIn; ++t)
          if (t < a.nin) r += a.coef[l][t] * x[t];
        PHIKS_GLOBAL d2* o = reinterpret_cast<PHIKS_GLOBAL d2*>(out + l * a.out_stride) + e;
        *o = (a.beta == 0.0) ? r : a.beta * (*o) + r;
      }
    }
    return;
  }
  for (int64_t e = first; e < a.N; e += stride) {
    double x[kMaxIn];
#pragma unroll
    for (int t = 0; t < kMaxIn; ++t)
      if (t < a.nin) x[t] = gptr(a.in[t])[e];
    for (int l = 0; l < a.nout; ++l) {
      double r = 0.0;
#pragma unroll
      for (int t = 0; t < kMaxIn; ++t)
        if (t < a.nin) r += a.coef[l][t] * x[t];
      PHIKS_GLOBAL double* o = out + l * a.out_stride + e;
      *o = (a.beta == 0.0) ? r : a.beta * (*o) + r;
    }
  }
}

__global__ void __launch_bounds__(256) combine_kernel(CombineArgs a) {
  combine_body(a, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x);
}

// One combination per blockIdx.y (many independent problems in one launch).
__global__ void __launch_bounds__(256) combine_grouped_kernel(const CombineArgs* __restrict__ items) {
  combine_body(items[blockIdx.y], (int64_t)blockIdx.x * blockDim.x + threadIdx.x,
               (int64_t)gridDim.x * blockDim.x);
}

// Elementwise vector operations for integrators built on the phi-actions (y may be
// null: zero).  Axpby: a x + b y.  Rational: a / (1 + (b x)^2) + y.  Cubic: a (x - x^3) + b y.
// Brusselator reaction terms with x = u, y = v: BrussU a + x^2 y, BrussV a x - x^2 y.
enum { kVopAxpby = 0, kVopRational = 1, kVopCubic = 2, kVopBrussU = 3, kVopBrussV = 4 };
struct VecOpArgs {
  int op;
  int64_t N;
  double a, b;
  const double* x;
  const double* y;
  double* out;
};

__global__ void __launch_bounds__(256) vector_op_kernel(VecOpArgs v) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < v.N;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double x = v.x[e];
    const double y = v.y ? v.y[e] : 0.0;
    double r;
    if (v.op == kVopAxpby) {
      r = v.a * x + v.b * y;
    } else if (v.op == kVopRational) {
      const double bx = v.b * x;
      r = v.a / (1.0 + bx * bx) + y;
    } else if (v.op == kVopCubic) {
      r = v.a * (x - x * x * x) + v.b * y;
    } else if (v.op == kVopBrussU) {
      r = v.a + x * x * y;
    } else {
      r = v.a * x - x * x * y;
    }
    v.out[e] = r;
  }
}

// dst = (float)src, n entries.
__global__ void __launch_bounds__(256) to_f32_kernel(const double* src, float* dst, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = (float)src[e];
}

// ---------------------------------------------------------- Taylor exponential
// Job j evaluates the degree-24 Taylor polynomial of X = g Bh, where Bh is a mode's
// shifted operator divided by a power of two (so that its 1-norm is at most 1) and
// Bh^1 .. Bh^5 are shared by all jobs of that mode (every exponential the plan needs
// is exp of a multiple of the same operator).  Paterson-Stockmeyer form:
//   T(X) = sum_{i=0}^{4} D_i S^i,   S = Bh^5,   D_i = sum_{k=0}^{4} g^(5i+k)/(5i+k)! Bh^k.
// This kernel forms D_0 .. D_4; the Horner steps R <- R S + D_i are GEMMs.
constexpr int kTaylorBlocks = 5;  // degree 24 = 5 * 5 - 1
struct TaylorJob {
  const double* pw[kTaylorBlocks];            // pw[k] = Bh^k, k = 1..4 (pw[0] unused, Bh^0 = I)
  double coef[kTaylorBlocks][kTaylorBlocks];  // coef[i][k] = g^(5i+k) / (5i+k)!
  double* D[kTaylorBlocks];
  int n;
};

__global__ void __launch_bounds__(256) taylor_form_kernel(const TaylorJob* jobs) {
  const TaylorJob& J = jobs[blockIdx.y];
  const int64_t nn = (int64_t)J.n * J.n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double id = (e % (J.n + 1)) == 0 ? 1.0 : 0.0;
    const double p1 = J.pw[1][e], p2 = J.pw[2][e], p3 = J.pw[3][e], p4 = J.pw[4][e];
#pragma unroll
    for (int i = 0; i < kTaylorBlocks; ++i)
      J.D[i][e] = J.coef[i][0] * id + J.coef[i][1] * p1 + J.coef[i][2] * p2 +
                  J.coef[i][3] * p3 + J.coef[i][4] * p4;
  }
}

// dst = scale * src over n*n entries, batched.
struct ScaleJob {
  const double* src;
  double* dst;
  double scale;
  int n;
};

__global__ void __launch_bounds__(256) scale_copy_kernel(const ScaleJob* jobs) {
  const ScaleJob& J = jobs[blockIdx.y];
  const int64_t nn = (int64_t)J.n * J.n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
       e += (int64_t)gridDim.x * blockDim.x)
    J.dst[e] = J.scale * J.src[e];
}

// Complex plans: [Re | Im] form (n x 2n) of a matrix held in its real form R (2n x 2n,
// 2 x 2 blocks [[Re, -Im], [Im, Re]]): dst[i][j] = R[2i][2j], dst[i][n+j] = R[2i+1][2j].
// Batched like the scale jobs (src, dst, n = the complex size).
__global__ void __launch_bounds__(256) complex_split_kernel(const ScaleJob* jobs) {
  const ScaleJob& J = jobs[blockIdx.y];
  const int64_t n = J.n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < 2 * n * n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / (2 * n), c = e % (2 * n);
    const int64_t j = c % n, im = c / n;
    J.dst[e] = J.src[(2 * i + im) * (2 * n) + 2 * j];
  }
}

}  // namespace phiks
