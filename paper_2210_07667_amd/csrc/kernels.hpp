// Elementwise and small-matrix kernels of the phiks path (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

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
  double coef[8][kMaxIn];
};

__global__ void __launch_bounds__(256) combine_kernel(CombineArgs a) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < a.N; e += stride) {
    double x[kMaxIn];
#pragma unroll
    for (int t = 0; t < kMaxIn; ++t)
      if (t < a.nin) x[t] = a.in[t][e];
    for (int l = 0; l < a.nout; ++l) {
      double r = 0.0;
#pragma unroll
      for (int t = 0; t < kMaxIn; ++t)
        if (t < a.nin) r += a.coef[l][t] * x[t];
      double* o = a.out + l * a.out_stride + e;
      *o = (a.beta == 0.0) ? r : a.beta * (*o) + r;
    }
  }
}

// ------------------------------------------------------------ Pade exponential
// Job j computes the [m/m] Pade approximant of X = gamma * Bs (Bs = B - sigma I):
//   S_U = sum_k cu[k] Bs^(2k),  V = sum_k cv[k] Bs^(2k)   (Bs^0 = I)
// so that U = Bs S_U and r_m(X) = (V - U)^-1 (V + U).  The even powers of Bs are
// shared by all jobs of one mode (every node matrix is a multiple of the same Bs).
struct ExpmJob {
  const double* pw[7];  // pw[k] = Bs^(2k), k >= 1 (pw[0] unused)
  double cu[7];
  double cv[7];
  int nk;               // number of even powers used (m = 2 nk + 1)
  int n;
  double* SU;
  double* V;
  double* U;
  double* Q;            // V - U, overwritten by its LU factors
  double* X;            // V + U, overwritten by the solution
};

__global__ void __launch_bounds__(256) expm_form_kernel(const ExpmJob* jobs) {
  const ExpmJob& J = jobs[blockIdx.y];
  const int64_t nn = (int64_t)J.n * J.n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
       e += (int64_t)gridDim.x * blockDim.x) {
    const bool diag = (e % (J.n + 1)) == 0;
    double su = diag ? J.cu[0] : 0.0;
    double v = diag ? J.cv[0] : 0.0;
    for (int k = 1; k <= J.nk; ++k) {
      const double x = J.pw[k][e];
      su += J.cu[k] * x;
      v += J.cv[k] * x;
    }
    J.SU[e] = su;
    J.V[e] = v;
  }
}

__global__ void __launch_bounds__(256) expm_qx_kernel(const ExpmJob* jobs) {
  const ExpmJob& J = jobs[blockIdx.y];
  const int64_t nn = (int64_t)J.n * J.n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double v = J.V[e], u = J.U[e];
    J.Q[e] = v - u;
    J.X[e] = v + u;
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

// Solve Q X = R in place (X overwrites R) by Gaussian elimination with partial
// pivoting; one work-group per system, rows of Q and R row-major, n <= 1024.
constexpr int kSolveThreads = 1024;

__global__ void __launch_bounds__(kSolveThreads) lu_solve_kernel(const ExpmJob* jobs) {
  const ExpmJob& J = jobs[blockIdx.x];
  const int n = J.n;
  double* __restrict__ Q = J.Q;
  double* __restrict__ R = J.X;
  __shared__ double lmul[1024];
  __shared__ double rowq[1024];
  __shared__ double rowr[1024];
  __shared__ double redv[kSolveThreads];
  __shared__ int redi[kSolveThreads];
  const int tid = threadIdx.x;
  for (int k = 0; k < n; ++k) {
    // pivot: argmax_i>=k |Q[i][k]|
    double best = -1.0;
    int bi = k;
    for (int i = k + tid; i < n; i += kSolveThreads) {
      const double a = fabs(Q[(int64_t)i * n + k]);
      if (a > best) { best = a; bi = i; }
    }
    redv[tid] = best;
    redi[tid] = bi;
    __syncthreads();
    for (int off = kSolveThreads / 2; off > 0; off >>= 1) {
      if (tid < off) {
        const double o = redv[tid + off];
        const int oi = redi[tid + off];
        if (o > redv[tid] || (o == redv[tid] && oi < redi[tid])) { redv[tid] = o; redi[tid] = oi; }
      }
      __syncthreads();
    }
    const int piv = redi[0];
    __syncthreads();
    // swap rows k and piv (Q columns k.., R all columns); cache the pivot row
    for (int j = tid; j < n; j += kSolveThreads) {
      if (piv != k) {
        if (j >= k) {
          const double a = Q[(int64_t)k * n + j], b = Q[(int64_t)piv * n + j];
          Q[(int64_t)k * n + j] = b;
          Q[(int64_t)piv * n + j] = a;
        }
        const double c = R[(int64_t)k * n + j], d = R[(int64_t)piv * n + j];
        R[(int64_t)k * n + j] = d;
        R[(int64_t)piv * n + j] = c;
      }
    }
    __syncthreads();
    for (int j = tid; j < n; j += kSolveThreads) {
      rowq[j] = Q[(int64_t)k * n + j];
      rowr[j] = R[(int64_t)k * n + j];
    }
    __syncthreads();
    const double pinv = 1.0 / rowq[k];
    for (int i = k + 1 + tid; i < n; i += kSolveThreads) lmul[i] = Q[(int64_t)i * n + k] * pinv;
    __syncthreads();
    // trailing update: Q[i][j] -= l_i Q[k][j] (j > k), R[i][j] -= l_i R[k][j]
    const int wq = n - k - 1;
    const int width = wq + n;
    const int64_t total = (int64_t)(n - k - 1) * width;
    for (int64_t t = tid; t < total; t += kSolveThreads) {
      const int i = k + 1 + (int)(t / width);
      const int c = (int)(t % width);
      const double l = lmul[i];
      if (c < wq) {
        const int j = k + 1 + c;
        Q[(int64_t)i * n + j] -= l * rowq[j];
      } else {
        const int j = c - wq;
        R[(int64_t)i * n + j] -= l * rowr[j];
      }
    }
    __syncthreads();
  }
  // back substitution, row by row from the bottom
  for (int k = n - 1; k >= 0; --k) {
    const double dinv = 1.0 / Q[(int64_t)k * n + k];
    for (int j = tid; j < n; j += kSolveThreads) {
      const double x = R[(int64_t)k * n + j] * dinv;
      R[(int64_t)k * n + j] = x;
      rowr[j] = x;
    }
    __syncthreads();
    for (int i = tid; i < k; i += kSolveThreads) lmul[i] = Q[(int64_t)i * n + k];
    __syncthreads();
    const int64_t total = (int64_t)k * n;
    for (int64_t t = tid; t < total; t += kSolveThreads) {
      const int i = (int)(t / n);
      const int j = (int)(t % n);
      R[(int64_t)i * n + j] -= lmul[i] * rowr[j];
    }
    __syncthreads();
  }
}

}  // namespace phiks
