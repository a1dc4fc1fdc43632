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
  int vec;              // 1: 16-byte accesses (even N and out_stride, aligned bases)
  double coef[8][kMaxIn];
};

__global__ void __launch_bounds__(256) combine_kernel(CombineArgs a) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (a.vec) {
    // 16-byte accesses (conditions checked by the launcher)
    typedef double d2 __attribute__((ext_vector_type(2)));
    const int64_t N2 = a.N >> 1;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N2; e += stride) {
      d2 x[kMaxIn];
#pragma unroll
      for (int t = 0; t < kMaxIn; ++t)
        if (t < a.nin) x[t] = reinterpret_cast<const d2*>(a.in[t])[e];
      for (int l = 0; l < a.nout; ++l) {
        d2 r = {0.0, 0.0};
#pragma unroll
        for (int t = 0; t < kMaxIn; ++t)
          if (t < a.nin) r += a.coef[l][t] * x[t];
        d2* o = reinterpret_cast<d2*>(a.out + l * a.out_stride) + e;
        *o = (a.beta == 0.0) ? r : a.beta * (*o) + r;
      }
    }
    return;
  }
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

// dst = (float)src, n entries.
__global__ void __launch_bounds__(256) to_f32_kernel(const double* src, float* dst, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = (float)src[e];
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

// Solve Q X = R in place (X overwrites R) by blocked LU with partial pivoting; one
// work-group of 1024 threads per system, rows of Q and R row-major, n <= 1024.
//
// For each block of b columns (b = 16 for n <= 512, else 8): the panel
// Q[kb:n, kb:kb+b] is factored in LDS (pivot search, swap, multipliers, rank-1
// updates within the panel); its row interchanges are then applied to the columns
// right of the panel and to R; U12 = L11^-1 A12 is formed column by column in
// registers; and the trailing rows are updated once per block,
// A22 -= L21 U12 (b fused multiply-adds per element per block, L21 from LDS).  The
// same elimination is applied to R as extra columns.  Back substitution with the
// upper factor is blocked the same way (U11 solves in registers, U01 from LDS).
constexpr int kSolveThreads = 1024;
constexpr int kSolveCols = 256;
constexpr int kSolveRows = kSolveThreads / kSolveCols;
constexpr int kPanelCap = 8192;  // doubles of LDS for the panel (64 KB; gfx950 has 160 KB)

__global__ void __launch_bounds__(kSolveThreads) lu_solve_kernel(const ExpmJob* jobs) {
  const ExpmJob& J = jobs[blockIdx.x];
  const int n = J.n;
  double* __restrict__ Q = J.Q;
  double* __restrict__ R = J.X;
  const int bsz = (n <= 512) ? 16 : 8;  // rows * bsz <= kPanelCap
  __shared__ double panel[kPanelCap];
  __shared__ int piv[16];
  __shared__ double wbest[kSolveThreads / 64];
  __shared__ int wrow[kSolveThreads / 64];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int tx = tid % kSolveCols;
  const int ty = tid / kSolveCols;

  for (int kb = 0; kb < n; kb += bsz) {
    const int bw = min(bsz, n - kb);
    const int rows = n - kb;
    for (int e = tid; e < rows * bw; e += kSolveThreads) {
      const int r = e / bw, c = e - (e / bw) * bw;
      panel[r * bw + c] = Q[(int64_t)(kb + r) * n + kb + c];
    }
    __syncthreads();
    // ---- panel factorization in LDS
    for (int c = 0; c < bw; ++c) {
      double best = -1.0;
      int br = c;
      for (int r = c + tid; r < rows; r += kSolveThreads) {
        const double a = fabs(panel[r * bw + c]);
        if (a > best) { best = a; br = r; }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_down(best, off);
        const int orr = __shfl_down(br, off);
        if (ob > best || (ob == best && orr < br)) { best = ob; br = orr; }
      }
      if (lane == 0) { wbest[wave] = best; wrow[wave] = br; }
      __syncthreads();
      if (tid == 0) {
        double b0 = wbest[0];
        int r0 = wrow[0];
        for (int w = 1; w < kSolveThreads / 64; ++w)
          if (wbest[w] > b0 || (wbest[w] == b0 && wrow[w] < r0)) { b0 = wbest[w]; r0 = wrow[w]; }
        piv[c] = r0;
      }
      __syncthreads();
      const int pr = piv[c];
      if (pr != c && tid < bw) {
        const double a = panel[c * bw + tid];
        panel[c * bw + tid] = panel[pr * bw + tid];
        panel[pr * bw + tid] = a;
      }
      __syncthreads();
      const double pinv = 1.0 / panel[c * bw + c];
      for (int r = c + 1 + tid; r < rows; r += kSolveThreads) {
        const double l = panel[r * bw + c] * pinv;
        panel[r * bw + c] = l;
        for (int cc = c + 1; cc < bw; ++cc) panel[r * bw + cc] -= l * panel[c * bw + cc];
      }
      __syncthreads();
    }
    for (int e = tid; e < rows * bw; e += kSolveThreads) {
      const int r = e / bw, c = e - (e / bw) * bw;
      Q[(int64_t)(kb + r) * n + kb + c] = panel[r * bw + c];
    }
    // ---- interchanges on the columns right of the panel and on R, then U12
    const int wq = n - kb - bw;  // Q columns right of the panel
    for (int col = tid; col < wq + n; col += kSolveThreads) {
      double* base = (col < wq) ? Q + kb + bw + col : R + (col - wq);
      for (int c = 0; c < bw; ++c) {
        const int pr = piv[c];
        if (pr != c) {
          const double a = base[(int64_t)(kb + c) * n];
          base[(int64_t)(kb + c) * n] = base[(int64_t)(kb + pr) * n];
          base[(int64_t)(kb + pr) * n] = a;
        }
      }
      double u[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        if (t < bw) {
          double x = base[(int64_t)(kb + t) * n];
#pragma unroll
          for (int s2 = 0; s2 < t; ++s2) x -= panel[t * bw + s2] * u[s2];
          u[t] = x;
          base[(int64_t)(kb + t) * n] = x;
        }
      }
    }
    __syncthreads();
    // ---- trailing update A22 -= L21 U12 (Q right part and all of R)
    for (int col0 = 0; col0 < wq + n; col0 += kSolveCols) {
      const int col = col0 + tx;
      if (col < wq + n) {
        double* base = (col < wq) ? Q + kb + bw + col : R + (col - wq);
        double u[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) u[t] = (t < bw) ? base[(int64_t)(kb + t) * n] : 0.0;
        for (int r = bw + ty; r < rows; r += kSolveRows) {
          double x = base[(int64_t)(kb + r) * n];
#pragma unroll
          for (int t = 0; t < 16; ++t)
            if (t < bw) x -= panel[r * bw + t] * u[t];
          base[(int64_t)(kb + r) * n] = x;
        }
      }
    }
    __syncthreads();
  }
  // ---- back substitution U X = R, blocks from the bottom
  const int nblk = (n + bsz - 1) / bsz;
  for (int blk = nblk - 1; blk >= 0; --blk) {
    const int kb = blk * bsz;
    const int bw = min(bsz, n - kb);
    // U11 (bw x bw) and U01 (kb x bw) into LDS
    for (int e = tid; e < (kb + bw) * bw; e += kSolveThreads) {
      const int r = e / bw, c = e - (e / bw) * bw;
      panel[r * bw + c] = Q[(int64_t)r * n + kb + c];
    }
    __syncthreads();
    for (int col = tid; col < n; col += kSolveThreads) {
      double x[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) x[t] = (t < bw) ? R[(int64_t)(kb + t) * n + col] : 0.0;
#pragma unroll
      for (int t = 15; t >= 0; --t) {
        if (t < bw) {
          double v = x[t];
#pragma unroll
          for (int s2 = t + 1; s2 < 16; ++s2)
            if (s2 < bw) v -= panel[(kb + t) * bw + s2] * x[s2];
          x[t] = v / panel[(kb + t) * bw + t];
        }
      }
#pragma unroll
      for (int t = 0; t < 16; ++t)
        if (t < bw) R[(int64_t)(kb + t) * n + col] = x[t];
    }
    __syncthreads();
    for (int col0 = 0; col0 < n; col0 += kSolveCols) {
      const int col = col0 + tx;
      if (col < n) {
        double x[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) x[t] = (t < bw) ? R[(int64_t)(kb + t) * n + col] : 0.0;
        for (int r = ty; r < kb; r += kSolveRows) {
          double v = R[(int64_t)r * n + col];
#pragma unroll
          for (int t = 0; t < 16; ++t)
            if (t < bw) v -= panel[r * bw + t] * x[t];
          R[(int64_t)r * n + col] = v;
        }
      }
    }
    __syncthreads();
  }
}

}  // namespace phiks
