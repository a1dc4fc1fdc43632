// FP32 MFMA variant of the mu-mode product (see gemm_f64.hpp for the three views and
// the tile order).  Operands are converted to FP32 on their way into LDS (the tensor
// may arrive in FP64 -- the first mode of a Tucker operator reads the FP64 vectors of
// the phi recurrence -- or in FP32, the intermediate modes), the products accumulate
// in FP32 on v_mfma_f32_16x16x4_f32, and the last mode writes FP64 through the same
// epilogues as the FP64 kernel (the squaring recurrence stays in FP64).
//
// MFMA v_mfma_f32_16x16x4_f32, per lane l:
//   A operand  A[m0 + (l & 15)][k0 + (l >> 4)]
//   B operand  B[k0 + (l >> 4)][n0 + (l & 15)]
//   C result   c[r] = C[m0 + 4 (l >> 4) + r][n0 + (l & 15)]      (checked on the GPU)
//
// LDS: k-major tiles of floats, 32 k per chunk.  Column c of row k is stored at
// c ^ swz(k) so that a wave's fragment read (16 columns x 4 rows) and its
// transposing stores (8 rows x 8 groups of 4 k) both touch 64 distinct banks.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "gemm_f64.hpp"

namespace phiks {

typedef float flt4 __attribute__((ext_vector_type(4)));

// C = alpha * acc (+ beta * C) for an output of element type T.
template <class T>
struct EpiStoreT {
  double alpha, beta;
  __device__ __forceinline__ void operator()(T* C, int64_t e, int64_t, double acc) const {
    C[e] = (T)((beta == 0.0) ? alpha * acc : alpha * acc + beta * (double)C[e]);
  }
};

template <int BM> __device__ __forceinline__ int swz32_t(int k) {
  return ((16 * (k & 3)) ^ (8 * ((k >> 2) & 7))) & (BM - 1);
}
template <int BN> __device__ __forceinline__ int swz32_n(int k) { return (16 * (k & 3)) & (BN - 1); }

template <class T> struct Vec4;
template <> struct Vec4<float> {
  __device__ __forceinline__ static flt4 load(const float* p) { return *reinterpret_cast<const flt4*>(p); }
};
template <> struct Vec4<double> {
  __device__ __forceinline__ static flt4 load(const double* p) {
    const dbl2 a = *reinterpret_cast<const dbl2*>(p);
    const dbl2 b = *reinterpret_cast<const dbl2*>(p + 2);
    return flt4{(float)a[0], (float)a[1], (float)b[0], (float)b[1]};
  }
};

// Epilogue of the FP32-accumulating kernels: wave fragments acc[i][j] (16 x 16 each,
// c[r] at row 4 (l >> 4) + r, column l & 15) of the output block whose top-left
// corner is (mb, nb), written through Epi.  The squaring epilogue (EpiLinComb)
// forms its FP64 combination one 16-row block at a time.
template <int FM, int FN, class TC, class Epi>
__device__ __forceinline__ void store_acc_tile(const flt4 (&acc)[FM][FN], const GemmArgs& g,
                                               const Epi& epi, TC* Cb, int64_t cbase, int64_t z1,
                                               int mb, int nb, int lr, int lk,
                                               const double* Yb = nullptr, int64_t YN = 0) {
  if constexpr (std::is_same<Epi, EpiLinComb>::value) {
    static_assert(std::is_same<TC, double>::value, "the squaring epilogue writes FP64");
    // one 16-row block at a time (FP64 partial results stay in few registers)
    const int l = (int)z1;
    const double al = epi.a[l];
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      double o[FN][4];
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) o[j][r] = al * (double)acc[i][j][r];
      for (int k = 0; k <= l; ++k) {
        const double ck = epi.c[l][k];
        const double* __restrict__ Yk = (Yb ? Yb : epi.Y) + (int64_t)(k - l) * (Yb ? YN : epi.N);
        double y[FN][4];
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          const int n = nb + j * 16 + lr;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int m = mb + i * 16 + 4 * lk + r;
            const bool ok = m < g.M && n < g.N;
            y[j][r] = ok ? Yk[cbase + (int64_t)m * g.ldc + n] : 0.0;
          }
        }
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) o[j][r] += ck * y[j][r];
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int n = nb + j * 16 + lr;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = mb + i * 16 + 4 * lk + r;
          if (m < g.M && n < g.N) Cb[cbase + (int64_t)m * g.ldc + n] = o[j][r];
        }
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int n = nb + j * 16 + lr;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = mb + i * 16 + 4 * lk + r;
          if (m < g.M && n < g.N) epi(Cb, cbase + (int64_t)m * g.ldc + n, z1, (double)acc[i][j][r]);
        }
      }
  }
}

// TA: element type of A in memory; B is FP32 (a small matrix or an FP32 intermediate)
// unless B_KCONTIG is false and it is the tensor (then it is an FP32 intermediate).
// TC: element type of C.  VEC: 4 elements per load (K, lda, ldb, strides multiples of 4,
// 16-byte aligned bases, and N a multiple of 4 for an n-contiguous B).
#ifndef PHIKS_F32_BK
#define PHIKS_F32_BK 32
#endif
#ifndef PHIKS_F32_MIN_WAVES
#define PHIKS_F32_MIN_WAVES 3
#endif

template <int BM, int BN, int WM, int WN, bool B_KCONTIG, bool VEC, class TA, class TC, class Epi>
__device__ __forceinline__ void gemm_f32_tile(const GemmArgs& g, const Epi& epi, int64_t rest,
                                              const double* Yb = nullptr, int64_t YN = 0) {
  constexpr int BK = PHIKS_F32_BK;
  constexpr int WGM = BM / WM;
  constexpr int WGN = BN / WN;
  static_assert(WGM * WGN == 4, "4 waves per work-group");
  constexpr int FM = WM / 16;
  constexpr int FN = WN / 16;
  constexpr int VW = VEC ? 4 : 1;
  constexpr int LA = BM * BK / (256 * VW);
  constexpr int LB = BN * BK / (256 * VW);
  typedef typename std::conditional<VEC, flt4, float>::type vec_t;

  __shared__ __align__(16) float As[2][BK][BM];
  __shared__ __align__(16) float Bs[2][BK][BN];

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

  // Raw operand registers of the next K chunk: the loads only are issued here; the
  // zero fill of out-of-range elements and the conversion of FP64 input happen when
  // the registers are written to LDS, so the loads stay in flight while the MFMAs of
  // the current chunk run.  Out-of-range elements read a clamped in-range address.
  constexpr bool kA64 = std::is_same<TA, double>::value;
  typedef typename std::conditional<VEC, typename std::conditional<kA64, dbl2, flt4>::type, TA>::type
      rawa_t;
  constexpr int kAV = (VEC && kA64) ? 2 : 1;  // raw registers per A load
  rawa_t ra[LA][kAV];
  vec_t rb[LB];
  auto a_ok = [&](int e, int k0) {
    const int m = e / (BK / VW), k = VW * (e % (BK / VW));
    return (m0 + m < g.M) & (k0 + k < g.K);
  };
  auto b_ok = [&](int e, int k0) {
    int n, k;
    if constexpr (B_KCONTIG) { n = e / (BK / VW); k = VW * (e % (BK / VW)); }
    else { k = e / (BN / VW); n = VW * (e % (BN / VW)); }
    return (n0 + n < g.N) & (k0 + k < g.K);
  };
  static_assert(LA <= 32 && LB <= 32, "one mask bit per load");
  // in-range bits of the loads in flight (the scalar-load variants keep them; the
  // 16-byte ones recompute them, which costs fewer registers)
  uint32_t amask = 0, bmask = 0;
  auto a_in = [&](int i, int e, int k0) -> bool {
    if constexpr (VEC) return a_ok(e, k0);
    else return (amask >> i) & 1;
  };
  auto b_in = [&](int i, int e, int k0) -> bool {
    if constexpr (VEC) return b_ok(e, k0);
    else return (bmask >> i) & 1;
  };
  auto load_chunk = [&](int k0) {
    amask = bmask = 0;
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      const int e = tid + i * 256;
      const int m = e / (BK / VW), k = VW * (e % (BK / VW));
      const bool ok = a_ok(e, k0);
      if constexpr (!VEC) amask |= (uint32_t)ok << i;
      const int64_t off = ok ? (int64_t)(m0 + m) * g.lda + k0 + k : 0;
#pragma unroll
      for (int h = 0; h < kAV; ++h) ra[i][h] = *reinterpret_cast<const rawa_t*>(A + off + 2 * h);
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int e = tid + i * 256;
      int n, k;
      if constexpr (B_KCONTIG) { n = e / (BK / VW); k = VW * (e % (BK / VW)); }
      else { k = e / (BN / VW); n = VW * (e % (BN / VW)); }
      const int gn = n0 + n, gk = k0 + k;
      const bool ok = b_ok(e, k0);
      if constexpr (!VEC) bmask |= (uint32_t)ok << i;
      const int64_t off =
          ok ? (B_KCONTIG ? (int64_t)gn * g.ldb + gk : (int64_t)gk * g.ldb + gn) : 0;
      rb[i] = *reinterpret_cast<const vec_t*>(B + off);
    }
  };
  auto a_value = [&](int i, int e, int k0) -> vec_t {
    const bool ok = a_in(i, e, k0);
    if constexpr (VEC) {
      flt4 x;
      if constexpr (kA64) x = flt4{(float)ra[i][0][0], (float)ra[i][0][1], (float)ra[i][1][0], (float)ra[i][1][1]};
      else x = ra[i][0];
      return ok ? x : flt4{0.f, 0.f, 0.f, 0.f};
    } else {
      return ok ? (float)ra[i][0] : 0.f;
    }
  };
  auto store_chunk = [&](int buf, int k0) {
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      const int e = tid + i * 256;
      const int m = e / (BK / VW), k = VW * (e % (BK / VW));
      const vec_t x = a_value(i, e, k0);
      if constexpr (VEC) {
#pragma unroll
        for (int t = 0; t < 4; ++t) As[buf][k + t][m ^ swz32_t<BM>(k + t)] = x[t];
      } else {
        As[buf][k][m ^ swz32_t<BM>(k)] = x;
      }
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int e = tid + i * 256;
      vec_t x = rb[i];
      if (!b_in(i, e, k0)) x = vec_t(0.f);
      if constexpr (B_KCONTIG) {
        const int n = e / (BK / VW), k = VW * (e % (BK / VW));
        if constexpr (VEC) {
#pragma unroll
          for (int t = 0; t < 4; ++t) Bs[buf][k + t][n ^ swz32_t<BN>(k + t)] = x[t];
        } else {
          Bs[buf][k][n ^ swz32_t<BN>(k)] = x;
        }
      } else {
        const int k = e / (BN / VW), n = VW * (e % (BN / VW));
        if constexpr (VEC) *reinterpret_cast<flt4*>(&Bs[buf][k][n ^ swz32_n<BN>(k)]) = x;
        else Bs[buf][k][n ^ swz32_n<BN>(k)] = x;
      }
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
    for (int kk = 0; kk < BK; kk += 4) {
      const int k = kk + lk;
      float fa[FM], fb[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) fa[i] = As[buf][k][(wm + i * 16 + lr) ^ swz32_t<BM>(k)];
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        if constexpr (B_KCONTIG) fb[j] = Bs[buf][k][(wn + j * 16 + lr) ^ swz32_t<BN>(k)];
        else fb[j] = Bs[buf][k][(wn + j * 16 + lr) ^ swz32_n<BN>(k)];
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i], fb[j], acc[i][j], 0, 0, 0);
    }
    if (c + 1 < nchunks) store_chunk(buf ^ 1, (c + 1) * BK);
    __syncthreads();
  }

  store_acc_tile<FM, FN, TC>(acc, g, epi, Cb, cbase, z1, m0 + wm, n0 + wn, lr, lk, Yb, YN);
}

template <int BM, int BN, int WM, int WN, bool B_KCONTIG, bool VEC, class TA, class TC, class Epi>
__global__ void __launch_bounds__(256, VEC ? PHIKS_F32_MIN_WAVES : 2) gemm_f32_kernel(GemmArgs g, Epi epi) {
  gemm_f32_tile<BM, BN, WM, WN, B_KCONTIG, VEC, TA, TC, Epi>(g, epi, xcd_remap(blockIdx.x, g.total_tiles));
}

// Grouped launch (many independent FP32 products of one configuration in one grid, as
// gemm_f64_grouped): each item runs exactly the tiles gemm_f32_kernel would run for it.
template <int BM, int BN, int WM, int WN, bool B_KCONTIG, bool VEC, class TA, class TC, class Epi>
__global__ void __launch_bounds__(256, VEC ? PHIKS_F32_MIN_WAVES : 2)
    gemm_f32_grouped(const GroupItem* __restrict__ items, const int64_t* __restrict__ first,
                     int nitems, int64_t total, Epi epi) {
  const int64_t t = xcd_remap(blockIdx.x, total);
  const int i = find_group_item(first, nitems, t);
  const GroupItem& it = items[i];
  // the item's pre-step tensors go beside epi, not into a modified copy of it (a local
  // copy indexed by the tensor index lives in scratch memory)
  if constexpr (std::is_same<Epi, EpiLinComb>::value) {
    gemm_f32_tile<BM, BN, WM, WN, B_KCONTIG, VEC, TA, TC, Epi>(it.g, epi, t - first[i], it.Y, it.YN);
  } else {
    gemm_f32_tile<BM, BN, WM, WN, B_KCONTIG, VEC, TA, TC, Epi>(it.g, epi, t - first[i]);
  }
}

}  // namespace phiks
