// BF16x3 variant of the mu-mode product (see gemm_f64.hpp for the three views and the
// tile order).  Every operand value x (FP64 or FP32 in memory) is split on its way into
// LDS into two bfloat16 numbers, hi = bf16(x) and lo = bf16(x - hi), both rounded to
// nearest even (unit roundoff 2^-8), so that |x - hi - lo| <= 2^-16 |x|.  The product
// of two split operands is taken as hi*hi + hi*lo + lo*hi (the lo*lo term, at most
// 2^-16 |a b|, is dropped), each term a v_mfma_f32_16x16x32_bf16 accumulating in FP32:
// every term a b of a contraction is formed to within 3 * 2^-16 |a b|.
// Intermediate tensors are stored in FP32 (or, in a pair chain, as the hi/lo halves of
// each FP32 value packed in one 32-bit word, so that the next product reads its
// operands already split) and the last mode writes FP64 through the epilogues of the
// FP32 kernel, so the squaring recurrence stays in FP64.
//
// MFMA v_mfma_f32_16x16x32_bf16, per lane l (eight consecutive k per lane):
//   A operand  A[m0 + (l & 15)][k0 + 8 (l >> 4) + t],   t = 0..7
//   B operand  B[k0 + 8 (l >> 4) + t][n0 + (l & 15)],   t = 0..7
//   C result   c[r] = C[m0 + 4 (l >> 4) + r][n0 + (l & 15)]      (checked on the GPU)
//
// LDS: both operands are held k-contiguous, one row of BK bfloat16 per output row
// (A) or column (B), as BK/8 groups of 16 bytes; group g of row r is stored at
// position g ^ swz(r).  A wave's fragment read (16 rows, one group each) and the
// stores (16 rows x 1 group, or 16/G rows x G groups) then cover all 64 banks once.
// The n-contiguous tensor operand of the middle and last modes is transposed on the
// way in: each thread gathers eight k of one column.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "gemm_f32.hpp"
#include "gemm_f64.hpp"

namespace phiks {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float flt2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

#ifndef PHIKS_BF_BK
#define PHIKS_BF_BK 32
#endif
#ifndef PHIKS_BF_MIN_WAVES
#define PHIKS_BF_MIN_WAVES 2
#endif

// Split eight values into their bfloat16 hi and lo parts, packed two per 32-bit word
// (element 2t in the low half of word t, as the MFMA operand expects).
__device__ __forceinline__ void split8(const float (&x)[8], u32x4& hi, u32x4& lo) {
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const flt2 v = {x[2 * t], x[2 * t + 1]};
    const unsigned h = __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2));
    const flt2 r = {v.x - __builtin_bit_cast(float, h << 16),
                    v.y - __builtin_bit_cast(float, h & 0xffff0000u)};
    hi[t] = h;
    lo[t] = __builtin_bit_cast(unsigned, __builtin_convertvector(r, bf16x2));
  }
}

// The split of one value as a pair word: hi in the low 16 bits, lo in the high 16 bits.
// The same two roundings as split8, so a pair word holds exactly the halves split8
// would form from x.
__device__ __forceinline__ unsigned split_pair(float x) {
  const flt2 v = {x, 0.f};
  const unsigned h = __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2)) & 0xffffu;
  const flt2 r = {x - __builtin_bit_cast(float, h << 16), 0.f};
  const unsigned l = __builtin_bit_cast(unsigned, __builtin_convertvector(r, bf16x2)) & 0xffffu;
  return h | (l << 16);
}

// Eight pair words (consecutive k) regrouped into the MFMA operands: the hi halves of
// words 2t and 2t + 1 into word t of hi, the lo halves into word t of lo.
__device__ __forceinline__ void unpair8(const unsigned (&w)[8], u32x4& hi, u32x4& lo) {
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    hi[t] = __builtin_amdgcn_perm(w[2 * t + 1], w[2 * t], 0x05040100u);
    lo[t] = __builtin_amdgcn_perm(w[2 * t + 1], w[2 * t], 0x07060302u);
  }
}

// Intermediate tensors of a pair chain: C holds split_pair of the FP32 product.
struct EpiStorePair {
  __device__ __forceinline__ void operator()(unsigned* C, int64_t e, int64_t, double acc) const {
    C[e] = split_pair((float)acc);
  }
};

// Pair words of FP64 matrices rounded to FP32 (the plan's copies for pair chains).
__global__ void __launch_bounds__(256) to_pair_kernel(const double* src, unsigned* dst, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = split_pair((float)src[e]);
}

// Group position of row r for G groups of 16 bytes per row.
template <int G> __device__ __forceinline__ int swz_bf(int r) {
  return (r / (16 / G)) & (G - 1);
}

// Eight consecutive k (from gk) of row `row` of a k-contiguous operand with leading
// dimension ld.  load() only issues the loads (out-of-range parts read element 0 of
// the operand); get() applies the zero fill and the conversion to FP32.  Keeping the
// two apart lets the loads of the next K chunk stay in flight while the MFMAs of the
// current one run.  VEC: 16-byte loads (K a multiple of 4, so that each four-k half
// is wholly inside or outside).
template <bool VEC, class T>
struct Row8 {
  static constexpr bool kF64 = std::is_same<T, double>::value;
  typedef typename std::conditional<VEC, typename std::conditional<kF64, dbl2, flt4>::type, T>::type V;
  static constexpr int kNV = VEC ? (kF64 ? 4 : 2) : 8;
  V v[kNV];

  __device__ __forceinline__ void load(const T* __restrict__ P, int64_t ld, int row, int rows,
                                       int gk, int K) {
    // (bitwise predicates and selected offsets: short-circuit conditions make the
    // compiler branch around each load)
    const bool rok = row < rows;
    const int64_t base = rok ? (int64_t)row * ld : 0;
    if constexpr (VEC) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const bool ok = rok & (gk + 4 * h < K);
        const T* q = P + (ok ? base + gk + 4 * h : 0);
        if constexpr (kF64) {
          v[2 * h] = *reinterpret_cast<const dbl2*>(q);
          v[2 * h + 1] = *reinterpret_cast<const dbl2*>(q + 2);
        } else {
          v[h] = *reinterpret_cast<const flt4*>(q);
        }
      }
    } else {
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const bool ok = rok & (gk + t < K);
        v[t] = P[ok ? base + gk + t : 0];
      }
    }
  }

  __device__ __forceinline__ void get(int row, int rows, int gk, int K, float (&x)[8]) const {
    const bool rok = row < rows;
    if constexpr (VEC) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const bool ok = rok & (gk + 4 * h < K);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          float e;
          if constexpr (kF64) e = (float)v[2 * h + t / 2][t % 2];
          else e = v[h][t];
          x[4 * h + t] = ok ? e : 0.f;
        }
      }
    } else {
#pragma unroll
      for (int t = 0; t < 8; ++t) x[t] = (rok & (gk + t < K)) ? (float)v[t] : 0.f;
    }
  }
};

// TA: element type of A in memory (FP64 for the first mode of a chain, else FP32); B is
// FP32.  TC: element type of C.  VEC: 16-byte loads of the k-contiguous operands (K,
// lda, strides multiples of 4, 16-byte aligned bases; ldb too when B_KCONTIG).
template <int BM, int BN, int WM, int WN, bool B_KCONTIG, bool VEC, class TA, class TC, class Epi>
__global__ void __launch_bounds__(256, PHIKS_BF_MIN_WAVES) gemm_bf16x3_kernel(GemmArgs g, Epi epi) {
  constexpr int BK = PHIKS_BF_BK;
  constexpr int G = BK / 8;  // 16-byte groups per LDS row
  static_assert(G == 4 || G == 8, "BK is 32 or 64");
  constexpr int WGM = BM / WM;
  constexpr int WGN = BN / WN;
  static_assert(WGM * WGN == 4, "4 waves per work-group");
  constexpr int FM = WM / 16;
  constexpr int FN = WN / 16;
  constexpr int LA = BM * G / 256;  // eight-k groups per thread
  constexpr int LB = BN * G / 256;
  static_assert(LA >= 1 && LB >= 1, "tile too small for 256 threads");

  __shared__ __align__(16) u32x4 Ah[2][BM][G];
  __shared__ __align__(16) u32x4 Al[2][BM][G];
  __shared__ __align__(16) u32x4 Bh[2][BN][G];
  __shared__ __align__(16) u32x4 Bl[2][BN][G];

  int64_t rest = xcd_remap(blockIdx.x, g.total_tiles);
  int tm, tn;
  int64_t z1, z0;
  if constexpr (B_KCONTIG) {
    tn = (int)(rest % g.tiles_n);
    rest /= g.tiles_n;
    z1 = rest % g.nb1;
    rest /= g.nb1;
    tm = (int)(rest % g.tiles_m);
    z0 = rest / g.tiles_m;
  } else {
    z1 = rest % g.nb1;
    rest /= g.nb1;
    tm = (int)(rest % g.tiles_m);
    rest /= g.tiles_m;
    tn = (int)(rest % g.tiles_n);
    z0 = rest / g.tiles_n;
  }
  const TA* __restrict__ A = reinterpret_cast<const TA*>(g.A) + z0 * g.sA0 + z1 * g.sA1;
  const float* __restrict__ B = reinterpret_cast<const float*>(g.B) + z0 * g.sB0 + z1 * g.sB1;
  TC* Cb = reinterpret_cast<TC*>(g.C);
  const int64_t cbase = z0 * g.sC0 + z1 * g.sC1;

  const int m0 = tm * BM;
  const int n0 = tn * BN;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave / WGN) * WM;
  const int wn = (wave % WGN) * WN;

  // raw operand registers of the next K chunk (see Row8)
  Row8<VEC, TA> ra[LA];
  typename std::conditional<B_KCONTIG, Row8<VEC, float>, Row8<false, float>>::type rb[LB];
  auto load_chunk = [&](int k0) {
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      const int e = tid + i * 256;
      ra[i].load(A, g.lda, m0 + e / G, g.M, k0 + 8 * (e % G), g.K);
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int e = tid + i * 256;
      if constexpr (B_KCONTIG) {
        rb[i].load(B, g.ldb, n0 + e / G, g.N, k0 + 8 * (e % G), g.K);
      } else {
        // column n of eight consecutive k rows; lanes take consecutive n (coalesced)
        const int gn = n0 + e % BN, gk = k0 + 8 * (e / BN);
        const bool nok = gn < g.N;
        const int64_t off0 = (int64_t)gk * g.ldb + gn;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const bool ok = nok & (gk + t < g.K);
          const int64_t off = off0 + (int64_t)t * g.ldb;
          rb[i].v[t] = B[ok ? off : 0];
        }
      }
    }
  };
  auto store_chunk = [&](int buf, int k0) {
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      const int e = tid + i * 256;
      const int r = e / G, c = (e % G) ^ swz_bf<G>(e / G);
      float x[8];
      ra[i].get(m0 + r, g.M, k0 + 8 * (e % G), g.K, x);
      u32x4 h, l;
      split8(x, h, l);
      Ah[buf][r][c] = h;
      Al[buf][r][c] = l;
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int e = tid + i * 256;
      int r, c;
      float x[8];
      if constexpr (B_KCONTIG) {
        r = e / G;
        c = (e % G) ^ swz_bf<G>(r);
        rb[i].get(n0 + r, g.N, k0 + 8 * (e % G), g.K, x);
      } else {
        r = e % BN;
        c = (e / BN) ^ swz_bf<G>(r);
        const int gn = n0 + r, gk = k0 + 8 * (e / BN);
#pragma unroll
        for (int t = 0; t < 8; ++t) x[t] = ((gn < g.N) & (gk + t < g.K)) ? rb[i].v[t] : 0.f;
      }
      u32x4 h, l;
      split8(x, h, l);
      Bh[buf][r][c] = h;
      Bl[buf][r][c] = l;
    }
  };

  flt4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = flt4{0.f, 0.f, 0.f, 0.f};

  const int nchunks = (g.K + BK - 1) / BK;
  load_chunk(0);
  store_chunk(0, 0);
  __syncthreads();
  const int lr = lane & 15;
  const int lk = lane >> 4;
  for (int c = 0; c < nchunks; ++c) {
    const int buf = c & 1;
    if (c + 1 < nchunks) load_chunk((c + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < G; kk += 4) {
      const int grp = kk + lk;
      bf16x8 ah[FM], al[FM], bh[FN], bl[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        const int r = wm + i * 16 + lr;
        ah[i] = __builtin_bit_cast(bf16x8, Ah[buf][r][grp ^ swz_bf<G>(r)]);
        al[i] = __builtin_bit_cast(bf16x8, Al[buf][r][grp ^ swz_bf<G>(r)]);
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int r = wn + j * 16 + lr;
        bh[j] = __builtin_bit_cast(bf16x8, Bh[buf][r][grp ^ swz_bf<G>(r)]);
        bl[j] = __builtin_bit_cast(bf16x8, Bl[buf][r][grp ^ swz_bf<G>(r)]);
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
        }
    }
    if (c + 1 < nchunks) store_chunk(buf ^ 1, (c + 1) * BK);
    __syncthreads();
  }

  store_acc_tile<FM, FN, TC>(acc, g, epi, Cb, cbase, z1, m0 + wm, n0 + wn, lr, lk);
}

}  // namespace phiks
