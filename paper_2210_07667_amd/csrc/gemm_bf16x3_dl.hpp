// BF16x3 mu-mode product with direct-to-LDS operand loads, for modes > 1 of a mixed
// chain (both operands FP32 in memory, the tensor operand n-contiguous).  Same product,
// split and epilogues as gemm_bf16x3_kernel; what differs is the operand path.  The
// register-staged kernel gathers the n-contiguous tensor with eight strided 4-byte loads
// per lane and splits on its way into LDS; here both FP32 tiles reach LDS unchanged by
// 16-byte DMA (gemm_f64_dl.hpp) and every lane splits the values of its own fragments
// when it reads them:
//  * matrix operand A (k-contiguous), rows r < BM, 32 k per chunk as eight 16-byte quads:
//    slot r*8 + (kq ^ ((r / 2) mod 8)); lane group lk reads quads 2lk and 2lk + 1
//    (ds_read_b128 each), i.e. k = 8 lk .. 8 lk + 7 as the BF16 MFMA takes them.
//  * tensor operand B (n-contiguous), rows k < 32, BN/4 column quads per row:
//    slot k*BN/4 + (cq ^ 4 ((k / 8) mod 4)); a lane reads its column at rows 8 lk + t,
//    t = 0..7 (ds_read_b32 each; the four lane groups land on four 64-byte bank groups).
// PAIR: both operands hold pair words (split_pair: hi | lo << 16) instead of FP32 values,
// same layout; a fragment read then only regroups the halves (unpair8), the split having
// been done once by whichever kernel wrote the operand.  The MFMA operands, and so the
// results, are bitwise those of the FP32 form on the values the pairs were split from.
// Requirements (checked by the launcher): K a multiple of 32, N of 4, the leading
// dimensions and strides multiples of 4 floats, 16-byte aligned bases; ragged M/N fetch
// clamped in-range rows or columns.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "gemm_bf16x3.hpp"
#include "gemm_f32_dl.hpp"
#include "gemm_f64_dl.hpp"

namespace phiks {

template <int BM, int BN, int WM, int WN, class TC, class Epi, bool PAIR>
__device__ __forceinline__ void gemm_bf16x3_dl_tile(const GemmArgs& g, const Epi& epi, int64_t rest) {
  constexpr int BK = 32;                  // floats of k per chunk (one BF16 MFMA step)
  constexpr int KQ = BK / 4;              // 16-byte quads per row of A
  constexpr int WGM = BM / WM, WGN = BN / WN;
  static_assert(WGM * WGN == 4, "4 waves per work-group");
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int A_SLOTS = BM * KQ, B_SLOTS = BK * BN / 4;
  static_assert(A_SLOTS % 256 == 0 && B_SLOTS % 256 == 0, "every thread fetches the same count");
  static_assert(BN / 4 >= 16, "column-quad swizzle needs BN >= 64");
  constexpr int LA = A_SLOTS / 256, LB = B_SLOTS / 256;
  constexpr int STAGE = 4 * (A_SLOTS + B_SLOTS);   // floats per stage
  constexpr bool LC = std::is_same<Epi, EpiLinComb>::value;
  constexpr int LDS_FLOATS = (LC && 2 * lc_f32_epilogue_doubles<BM, BN, WM, WN>() > 2 * STAGE)
                                 ? 2 * lc_f32_epilogue_doubles<BM, BN, WM, WN>()
                                 : 2 * STAGE;

  __shared__ __align__(16) float lds[LDS_FLOATS];

  const TileCoords tc = tile_coords<false>(g, rest);
  const PHIKS_GLOBAL float* A =
      (const PHIKS_GLOBAL float*)gptr(g.A) + tc.z0 * g.sA0 + tc.z1 * g.sA1;
  const PHIKS_GLOBAL float* B =
      (const PHIKS_GLOBAL float*)gptr(g.B) + tc.z0 * g.sB0 + tc.z1 * g.sB1;
  TC* Cb = reinterpret_cast<TC*>(g.C);
  const int64_t cbase = tc.z0 * g.sC0 + tc.z1 * g.sC1;
  const int m0 = tc.tm * BM, n0 = tc.tn * BN;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = (wave / WGN) * WM, wn = (wave % WGN) * WN;
  const int lr = lane & 15, lk = lane >> 4;

  const PHIKS_GLOBAL float* asrc[LA];
  const PHIKS_GLOBAL float* bsrc[LB];
#pragma unroll
  for (int i = 0; i < LA; ++i) {
    const int s = i * 256 + tid;
    const int r = s / KQ, kq = (s % KQ) ^ ((r >> 1) & 7);
    asrc[i] = A + (int64_t)min(m0 + r, g.M - 1) * g.lda + 4 * kq;
  }
#pragma unroll
  for (int i = 0; i < LB; ++i) {
    const int s = i * 256 + tid;
    const int k = s / (BN / 4), cq = (s % (BN / 4)) ^ (((k >> 3) & 3) << 2);
    bsrc[i] = B + (int64_t)k * g.ldb + min(n0 + 4 * cq, g.N - 4);
  }
  const int64_t bstep = (int64_t)BK * g.ldb;

  auto issue = [&](int c) {
    float* st = lds + (c & 1) * STAGE;
#pragma unroll
    for (int i = 0; i < LA; ++i)
      dma16(reinterpret_cast<const PHIKS_GLOBAL double*>(asrc[i] + (int64_t)c * BK),
            reinterpret_cast<double*>(st + 4 * (i * 256 + wave * 64)));
#pragma unroll
    for (int i = 0; i < LB; ++i)
      dma16(reinterpret_cast<const PHIKS_GLOBAL double*>(bsrc[i] + (int64_t)c * bstep),
            reinterpret_cast<double*>(st + 4 * A_SLOTS + 4 * (i * 256 + wave * 64)));
  };

  flt4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = flt4{0.f, 0.f, 0.f, 0.f};

  const int nchunks = g.K / BK;
  issue(0);
  for (int c = 0; c < nchunks; ++c) {
    wait_vmcnt<0>();
    wait_lgkmcnt0();
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();   // chunk c visible; every wave is done with chunk c - 1
    asm volatile("" ::: "memory");
    if (c + 1 < nchunks) issue(c + 1);
    const float* as = lds + (c & 1) * STAGE;
    const float* bs = as + 4 * A_SLOTS;
    bf16x8 bh[FN], bl[FN];
#pragma unroll
    for (int jj = 0; jj < FN; ++jj) {
      const int n = wn + jj * 16 + lr;
      float x[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int k = 8 * lk + t;
        x[t] = bs[4 * (k * (BN / 4) + ((n >> 2) ^ (((k >> 3) & 3) << 2))) + (n & 3)];
      }
      u32x4 h, l;
      if constexpr (PAIR) {
        unsigned w[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) w[t] = __builtin_bit_cast(unsigned, x[t]);
        unpair8(w, h, l);
      } else {
        split8(x, h, l);
      }
      bh[jj] = __builtin_bit_cast(bf16x8, h);
      bl[jj] = __builtin_bit_cast(bf16x8, l);
    }
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      const int r = wm + i * 16 + lr;
      const flt4 q0 = *reinterpret_cast<const flt4*>(as + 4 * (r * KQ + ((2 * lk) ^ ((r >> 1) & 7))));
      const flt4 q1 = *reinterpret_cast<const flt4*>(as + 4 * (r * KQ + ((2 * lk + 1) ^ ((r >> 1) & 7))));
      const float x[8] = {q0[0], q0[1], q0[2], q0[3], q1[0], q1[1], q1[2], q1[3]};
      u32x4 h, l;
      if constexpr (PAIR) {
        unsigned w[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) w[t] = __builtin_bit_cast(unsigned, x[t]);
        unpair8(w, h, l);
      } else {
        split8(x, h, l);
      }
      const bf16x8 ah = __builtin_bit_cast(bf16x8, h), al = __builtin_bit_cast(bf16x8, l);
#pragma unroll
      for (int jj = 0; jj < FN; ++jj) {
        acc[i][jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[jj], acc[i][jj], 0, 0, 0);
        acc[i][jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[jj], acc[i][jj], 0, 0, 0);
        acc[i][jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[jj], acc[i][jj], 0, 0, 0);
      }
    }
  }

  if constexpr (LC)
    lincomb_epilogue_f32<BM, BN, WM, WN>(acc, g, epi, epi.Y, epi.N, Cb, cbase, tc.z1,
                                         reinterpret_cast<double*>(lds), m0, n0, wave, tid);
  else
    store_acc_tile<FM, FN, TC>(acc, g, epi, Cb, cbase, tc.z1, m0 + wm, n0 + wn, lr, lk);
}

#ifndef PHIKS_BFDL_MIN_WAVES
#define PHIKS_BFDL_MIN_WAVES 2
#endif

template <int BM, int BN, int WM, int WN, class TC, class Epi, bool PAIR>
__global__ void __launch_bounds__(256, PHIKS_BFDL_MIN_WAVES) gemm_bf16x3_dl_kernel(GemmArgs g, Epi epi) {
  gemm_bf16x3_dl_tile<BM, BN, WM, WN, TC, Epi, PAIR>(g, epi, xcd_remap(blockIdx.x, g.total_tiles));
}

}  // namespace phiks
