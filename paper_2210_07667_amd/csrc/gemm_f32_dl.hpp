// FP32 MFMA mu-mode product with direct-to-LDS operand loads.  Same products, tile
// order and per-element arithmetic as gemm_f32_kernel; the squaring epilogue streams its
// FP64 pre-step tensors through LDS (lincomb_lds_epilogue_f32, also used by the BF16x3
// direct-to-LDS kernel).  The operand path is the one of gemm_f64_dl.hpp with 16-byte
// slots holding four floats:
//  * k-contiguous operand, rows r < R, k < 16 per chunk: slot of (r, k quad kq) is
//    r*4 + (kq ^ ((r / 4) mod 4)).  Lane group lk = l >> 4 reads quad lk of its row
//    (ds_read_b128) and feeds four MFMA steps: step h takes k = 4 lk + h, for both
//    operands.
//  * A in FP64 (TA = double: the first mode of a chain, which reads the FP64 vectors):
//    its rows reach LDS unconverted, eight 16-byte slots of two doubles per row and
//    chunk, slot r*8 + (kp ^ ((r / 2) mod 8)); lane group lk reads slots 2 lk and 2 lk + 1
//    (k = 4 lk .. 4 lk + 3) and rounds them to FP32 there, as gemm_f32_kernel does on
//    its way into LDS.
//  * n-contiguous operand, k < 16, columns c < BN: slot of (k, column quad cq) is
//    k*BN/4 + (cq ^ 4 ((k / 4) mod 4)); fragment reads are 4 bytes, the four rows of one
//    read land on four different 64-byte bank groups.
// MFMA v_mfma_f32_16x16x4_f32: A[m0 + (l & 15)][k(l >> 4)], B[k(l >> 4)][n0 + (l & 15)],
// c[r] = C[m0 + 4 (l >> 4) + r][n0 + (l & 15)].  K must be a multiple of 4, the leading
// dimensions and strides multiples of 4 floats, N too for an n-contiguous B (the
// launcher checks); ragged M/N fetch clamped in-range rows or columns.  A K that is not a
// multiple of 16 ends in a partial chunk: its slots past K fetch an in-range address of the
// same operand, and the lane groups whose four k lie past K zero both fragments, so those
// k add exact zeros (the chunks before it run as for any K).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "gemm_f32.hpp"
#include "gemm_f64_dl.hpp"

namespace phiks {

#ifndef PHIKS_F32DL_MIN_WAVES
#define PHIKS_F32DL_MIN_WAVES 4
#endif

__device__ __forceinline__ int swz_kq(int r) { return (r >> 2) & 3; }
__device__ __forceinline__ int swz_nq(int k) { return ((k >> 2) & 3) << 2; }

// Y slice buffers of the squaring epilogue below: three while a slice is at most 16 KB,
// else two (the buffers overlay the operand ring once the K loop is done).
template <int BM, int BN, int WM>
constexpr int lc_f32_bufs() { return (BM / WM) * 16 * BN * 8 <= 16384 ? 3 : 2; }
template <int BM, int BN, int WM>
constexpr int lc_f32_lds_doubles() { return lc_f32_bufs<BM, BN, WM>() * (BM / WM) * 16 * BN; }

// Squaring epilogue of the FP32-accumulating direct-to-LDS kernels: out = a_l acc +
// sum_{k <= l} c_lk Y_k in FP64, with the pre-step tensors Y_k streamed through LDS by
// 16-byte DMA (the scheme of lincomb_lds_epilogue in gemm_f64_dl.hpp, for the FP32
// accumulator layout c[r] at row 4 (l >> 4) + r).  Rounds run fragment row by fragment
// row (round i (l + 1) + k: slice of fragment row i of every wave, of Y_k), so only one
// row block of FP64 partial sums is live; per element the arithmetic is the register
// epilogue's (a_l acc, then one fma per k in k order).  Slice layout: WGM * 16 rows of
// BN columns as column pairs, slot rho * BN/2 + (cp ^ 8 ((rho / 4) mod 2)): the two row
// groups 4 apart that one 32-lane read touches land on different bank halves.  YB
// buffers, DMA YB - 1 rounds ahead.  Needs lincomb_dl_ok (checked by the launchers).
template <int BM, int BN, int WM, int WN, int FM, int FN>
__device__ __forceinline__ void lincomb_lds_epilogue_f32(const flt4 (&acc)[FM][FN], const GemmArgs& g,
                                                         const EpiLinComb& epi, const double* Yb,
                                                         int64_t YN, double* Cb,
                                                         int64_t cbase, int64_t z1, double* lds,
                                                         int m0, int n0, int wave, int tid) {
  constexpr int WGM = BM / WM, WGN = BN / WN;
  constexpr int ROWS = WGM * 16, CP = BN / 2;
  constexpr int YSLICE = ROWS * BN;                     // doubles
  constexpr int YB = lc_f32_bufs<BM, BN, WM>();
  constexpr int SLOTS = ROWS * CP, LY = SLOTS / 256;
  static_assert(SLOTS % 256 == 0, "every thread fetches the same count");
  static_assert(CP >= 16, "column-pair swizzle needs BN >= 32");
  const int lane = tid & 63, lr = lane & 15, lk = lane >> 4;
  const int wgm = wave / WGN, wn = (wave % WGN) * WN;
  const int l = (int)z1, nk = l + 1;
  const int rounds = FM * nk;

  // this thread's slots: source offset of slice row rho (fragment row 0), clamped column
  int64_t off[LY];
#pragma unroll
  for (int q = 0; q < LY; ++q) {
    const int s = q * 256 + tid;
    const int rho = s / CP, cp = (s % CP) ^ (((rho >> 2) & 1) << 3);
    const int row = (rho / 16) * WM + rho % 16;
    off[q] = (int64_t)row * g.ldc + min(n0 + 2 * cp, g.N - 2);
  }
  const PHIKS_GLOBAL double* Y0 = gptr(Yb) + cbase - (int64_t)l * YN;   // Y_0 at this tile
  auto issue = [&](int r) {
    const int i = r / nk, k = r - i * nk;
    const PHIKS_GLOBAL double* Yk = Y0 + (int64_t)k * YN;
    double* buf = lds + (r % YB) * YSLICE;
#pragma unroll
    for (int q = 0; q < LY; ++q) {
      const int s = q * 256 + tid;
      const int rho = s / CP;
      const int row = (rho / 16) * WM + rho % 16;
      const int grow = min(m0 + row + i * 16, g.M - 1);
      dma16(Yk + off[q] + (int64_t)(grow - row) * g.ldc, buf + 2 * (q * 256 + wave * 64));
    }
  };

  // every wave is done with the operand ring before its memory is overwritten
  wait_lgkmcnt0();
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
#pragma unroll
  for (int r = 0; r < YB - 1; ++r)
    if (r < rounds) issue(r);
  const double al = epi.a[l];
  const int ml = m0 + wgm * WM + 4 * lk, nl = n0 + wn + lr;
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    double o[FN][4];
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) o[j][rr] = al * (double)acc[i][j][rr];
    for (int k = 0; k < nk; ++k) {
      const int r = i * nk + k;
      // round r has landed once at most the later rounds' loads are outstanding (stores
      // of earlier row blocks issued after them only make this wait longer)
      if (r + YB - 2 < rounds) wait_vmcnt<(YB - 2) * LY>();
      else wait_vmcnt<0>();
      wait_lgkmcnt0();
      asm volatile("" ::: "memory");
      __builtin_amdgcn_s_barrier();
      asm volatile("" ::: "memory");
      if (r + YB - 1 < rounds) issue(r + YB - 1);     // into the buffer round r - 1 used
      const double* buf = lds + (r % YB) * YSLICE;
      const double ck = epi.c[l][k];
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int c = wn + j * 16 + lr;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const int rho = wgm * 16 + 4 * lk + rr;
          const double y = buf[2 * (rho * CP + ((c >> 1) ^ (((rho >> 2) & 1) << 3))) + (c & 1)];
          o[j][rr] = __builtin_fma(ck, y, o[j][rr]);
        }
      }
    }
    const int64_t base = cbase + (int64_t)(ml + i * 16) * g.ldc + nl;
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr)
        if ((ml + i * 16 + rr < g.M) & (nl + j * 16 < g.N))
          Cb[base + (int64_t)rr * g.ldc + j * 16] = o[j][rr];
  }
}

#ifndef PHIKS_F32_LC_WAVE
#define PHIKS_F32_LC_WAVE 1  // 1: wave-private pre-step slices (lincomb_wave_epilogue_f32)
#endif
#ifndef PHIKS_F32_LC_FNP
#define PHIKS_F32_LC_FNP 2   // 16-column fragments per round of the wave-private epilogue
#endif

// Wave-private form of the squaring epilogue above (the scheme of lincomb_wave_epilogue in
// gemm_f64_dl.hpp): round r = ((i * JP) + jp) * (l + 1) + k brings, for this wave only, 16
// rows (fragment row i) by FNP * 16 columns (column part jp) of Y_k into one of its YB
// buffers, YB - 1 rounds ahead, and waits only on the wave's own loads.  A wave's slice is
// FNP * 2 KB, so the epilogue needs 4 * YB * FNP * 2 KB of LDS (32 KB with FNP = 2, where
// the shared slices of a 64 x 64 or 128 x 64 tile needed 48 KB and of a 64 x 128 tile
// 64 KB: 5 work-groups per CU instead of 3 or 2; FP32 batch of 512 problems 27.0 -> 26.4
// ms).  Slice layout: slice row
// t = 4 (r mod 4) + r / 4 for tile row r (the four rows 4 lk + rr one read touches are
// consecutive), column pairs swizzled by ((r / 4) mod 2) (CPS / 2).  Per element the
// arithmetic and its order are the shared form's: a_l acc, then one fma per k in k order.
template <int FN>
constexpr int lc_f32w_fnp() { return FN < PHIKS_F32_LC_FNP ? FN : PHIKS_F32_LC_FNP; }
template <int WN, int YB>
constexpr int lc_f32w_lds_doubles() { return 4 * YB * 16 * lc_f32w_fnp<WN / 16>() * 16; }

template <int WM, int WN, int YB, int FM, int FN>
__device__ __forceinline__ void lincomb_wave_epilogue_f32(const flt4 (&acc)[FM][FN], const GemmArgs& g,
                                                          const EpiLinComb& epi, const double* Yb,
                                                          int64_t YN, double* Cb,
                                                          int64_t cbase, int64_t z1, double* lds,
                                                          int mw, int nw, int wave, int lane) {
  constexpr int FNP = lc_f32w_fnp<FN>(), JP = FN / FNP;
  static_assert(FN % FNP == 0, "whole column parts");
  constexpr int CPS = FNP * 8;                 // column pairs per slice row
  constexpr int SLICE = 16 * FNP * 16;         // doubles per wave slice
  constexpr int LW = 16 * CPS / 64;            // 16-byte loads per lane per round
  const int lr = lane & 15, lk = lane >> 4;
  const int l = (int)z1, nk = l + 1;
  const int rounds = FM * JP * nk;
  double* wbuf = lds + wave * YB * SLICE;
  const PHIKS_GLOBAL double* Y0 = gptr(Yb) + cbase - (int64_t)l * YN;   // Y_0 at this tile
  auto issue = [&](int r) {
    const int ij = r / nk, k = r - ij * nk;
    const int i = ij / JP, jp = ij - i * JP;
    const PHIKS_GLOBAL double* Yk = Y0 + (int64_t)k * YN;
    double* buf = wbuf + (r % YB) * SLICE;
    // computed per round (not hoisted out of the loops: held across them they would not fit)
    int64_t ldc = g.ldc;
    int M = g.M, N = g.N;
    int mr = __builtin_amdgcn_readfirstlane(mw), nc = __builtin_amdgcn_readfirstlane(nw);   // wave-uniform
    asm volatile("" : "+s"(ldc), "+s"(M), "+s"(N), "+s"(mr), "+s"(nc));
#pragma unroll
    for (int q = 0; q < LW; ++q) {
      const int s = q * 64 + lane;
      const int t = s / CPS, row = (t & 3) * 4 + (t >> 2);
      const int cp = (s % CPS) ^ (((row >> 2) & 1) * (CPS / 2));
      const int grow = min(mr + i * 16 + row, M - 1), gcol = min(nc + jp * FNP * 16 + 2 * cp, N - 2);
      dma16(Yk + (int64_t)grow * ldc + gcol, buf + 2 * (q * 64));
    }
  };

  // every wave is done with the operand ring before its memory is overwritten
  wait_lgkmcnt0();
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
#pragma unroll
  for (int r = 0; r < YB - 1; ++r)
    if (r < rounds) issue(r);
  const double al = epi.a[l];
  const int ml = mw + 4 * lk, nl = nw + lr;
#pragma unroll
  for (int i = 0; i < FM; ++i) {
#pragma unroll
    for (int jp = 0; jp < JP; ++jp) {
      double o[FNP][4];
#pragma unroll
      for (int j = 0; j < FNP; ++j)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) o[j][rr] = al * (double)acc[i][jp * FNP + j][rr];
      for (int k = 0; k < nk; ++k) {
        const int r = (i * JP + jp) * nk + k;
        // round r has landed once at most the later rounds' loads are outstanding (stores
        // of earlier parts issued after them only make this wait longer)
        if (r + YB - 2 < rounds) wait_vmcnt<(YB - 2) * LW>();
        else wait_vmcnt<0>();
        asm volatile("" ::: "memory");
        // the buffer round r - 1 used is free: its reads fed the fmas above
        if (r + YB - 1 < rounds) issue(r + YB - 1);
        const double* buf = wbuf + (r % YB) * SLICE;
        const double ck = epi.c[l][k];
#pragma unroll
        for (int j = 0; j < FNP; ++j) {
          const int c = j * 16 + lr;
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int row = 4 * lk + rr, t = rr * 4 + lk;   // t = slice row of tile row `row`
            const double y = buf[2 * (t * CPS + ((c >> 1) ^ (((row >> 2) & 1) * (CPS / 2)))) + (c & 1)];
            o[j][rr] = __builtin_fma(ck, y, o[j][rr]);
          }
        }
      }
      const int64_t base = cbase + (int64_t)(ml + i * 16) * g.ldc + nl + jp * FNP * 16;
#pragma unroll
      for (int j = 0; j < FNP; ++j)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
          if ((ml + i * 16 + rr < g.M) & (nl + (jp * FNP + j) * 16 < g.N))
            Cb[base + (int64_t)rr * g.ldc + j * 16] = o[j][rr];
    }
  }
}

// Which form a tile takes: the wave-private one below 128 x 128 (the tiles of small and
// mid-sized products, whose shared slices needed 48 or 64 KB of LDS), the shared one for
// 128 x 128 tiles (large products: register-bound anyway, they keep more bytes in flight
// per work-group with shared slices: 256^3 FP32 call 9.50 against 9.66 ms, BF16x3 6.11
// against 6.41 ms with the wave form).
template <int BM, int BN>
constexpr bool lc_f32_wave_form() { return PHIKS_F32_LC_WAVE == 1 && BM * BN < 128 * 128; }

// LDS doubles the squaring epilogue of a tile needs
template <int BM, int BN, int WM, int WN>
constexpr int lc_f32_epilogue_doubles() {
  return lc_f32_wave_form<BM, BN>() ? lc_f32w_lds_doubles<WN, 2>() : lc_f32_lds_doubles<BM, BN, WM>();
}

// The squaring epilogue of the FP32-accumulating direct-to-LDS kernels (either form; the
// same operations in the same order per element).
template <int BM, int BN, int WM, int WN, int FM, int FN>
__device__ __forceinline__ void lincomb_epilogue_f32(const flt4 (&acc)[FM][FN], const GemmArgs& g,
                                                     const EpiLinComb& epi, const double* Yb,
                                                     int64_t YN, double* Cb, int64_t cbase,
                                                     int64_t z1, double* lds, int m0, int n0,
                                                     int wave, int tid) {
  if constexpr (lc_f32_wave_form<BM, BN>()) {
    constexpr int WGN = BN / WN;
    lincomb_wave_epilogue_f32<WM, WN, 2>(acc, g, epi, Yb, YN, Cb, cbase, z1, lds, m0 + (wave / WGN) * WM,
                                         n0 + (wave % WGN) * WN, wave, tid & 63);
  } else {
    lincomb_lds_epilogue_f32<BM, BN, WM, WN>(acc, g, epi, Yb, YN, Cb, cbase, z1, lds, m0, n0, wave, tid);
  }
}

template <int BM, int BN, int WM, int WN, bool B_KCONTIG, class TA, class TC, class Epi>
__device__ __forceinline__ void gemm_f32_dl_tile(const GemmArgs& g, const Epi& epi, int64_t rest,
                                                 const double* Yb, int64_t YN) {
  constexpr int BK = 16;                 // floats of k per chunk
  constexpr int KQ = BK / 4;             // 16-byte slots per k-contiguous FP32 row
  constexpr bool AD = std::is_same<TA, double>::value;
  constexpr int AQ = AD ? 2 * KQ : KQ;   // 16-byte slots per row of A
  constexpr int WGM = BM / WM, WGN = BN / WN;
  static_assert(WGM * WGN == 4, "4 waves per work-group");
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int A_SLOTS = BM * AQ, B_SLOTS = BN * KQ;
  static_assert(A_SLOTS % 256 == 0 && B_SLOTS % 256 == 0, "every thread fetches the same count");
  static_assert(B_KCONTIG || BN / 4 >= 16, "column-quad swizzle needs BN >= 64");
  constexpr int LA = A_SLOTS / 256, LB = B_SLOTS / 256;
  constexpr int STAGE = 4 * (A_SLOTS + B_SLOTS);   // floats per stage
  constexpr bool LC = std::is_same<Epi, EpiLinComb>::value;
  constexpr int LDS_FLOATS = (LC && 2 * lc_f32_epilogue_doubles<BM, BN, WM, WN>() > 2 * STAGE)
                                 ? 2 * lc_f32_epilogue_doubles<BM, BN, WM, WN>()
                                 : 2 * STAGE;

  __shared__ __align__(16) float lds[LDS_FLOATS];

  const TileCoords tc = tile_coords<B_KCONTIG>(g, rest);
  const PHIKS_GLOBAL TA* A = (const PHIKS_GLOBAL TA*)gptr(g.A) + tc.z0 * g.sA0 + tc.z1 * g.sA1;
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

  const PHIKS_GLOBAL TA* asrc[LA];
  const PHIKS_GLOBAL float* bsrc[LB];
#pragma unroll
  for (int i = 0; i < LA; ++i) {
    const int s = i * 256 + tid;
    const int r = s / AQ, q = (s % AQ) ^ (AD ? (r >> 1) & 7 : swz_kq(r));
    asrc[i] = A + (int64_t)min(m0 + r, g.M - 1) * g.lda + (16 / (int)sizeof(TA)) * q;
  }
#pragma unroll
  for (int i = 0; i < LB; ++i) {
    const int s = i * 256 + tid;
    if constexpr (B_KCONTIG) {
      const int r = s / KQ, kq = (s % KQ) ^ swz_kq(s / KQ);
      bsrc[i] = B + (int64_t)min(n0 + r, g.N - 1) * g.ldb + 4 * kq;
    } else {
      const int k = s / (BN / 4), cq = (s % (BN / 4)) ^ swz_nq(s / (BN / 4));
      bsrc[i] = B + (int64_t)k * g.ldb + min(n0 + 4 * cq, g.N - 4);
    }
  }
  const int64_t bstep = B_KCONTIG ? BK : (int64_t)BK * g.ldb;

  const int nchunks = (g.K + BK - 1) / BK;
  const int ktail = g.K % BK;   // k in the last chunk when K is not a multiple of 16 (4-aligned)
  auto issue = [&](int c) {
    float* st = lds + (c & 1) * STAGE;
    const bool tail = ktail != 0 && c == nchunks - 1;   // wave-uniform
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      const PHIKS_GLOBAL TA* src = asrc[i] + (int64_t)c * BK;
      if (tail) {
        // k of the slot within the chunk; past K: the row's first slot (k = 0, in range)
        const int s = i * 256 + tid;
        const int r = s / AQ, q = (s % AQ) ^ (AD ? (r >> 1) & 7 : swz_kq(r));
        if ((16 / (int)sizeof(TA)) * q >= ktail) src = asrc[i] - (16 / (int)sizeof(TA)) * q;
      }
      dma16(reinterpret_cast<const PHIKS_GLOBAL double*>(src),
            reinterpret_cast<double*>(st + 4 * (i * 256 + wave * 64)));
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const PHIKS_GLOBAL float* src = bsrc[i] + (int64_t)c * bstep;
      if (tail) {
        const int s = i * 256 + tid;
        if constexpr (B_KCONTIG) {
          const int kq = (s % KQ) ^ swz_kq(s / KQ);
          if (4 * kq >= ktail) src = bsrc[i] - 4 * kq;
        } else {
          const int k = s / (BN / 4);   // row of the chunk; past K: the last row of K
          if (k >= ktail) src += (int64_t)(ktail - 1 - k) * g.ldb;
        }
      }
      dma16(reinterpret_cast<const PHIKS_GLOBAL double*>(src),
            reinterpret_cast<double*>(st + 4 * A_SLOTS + 4 * (i * 256 + wave * 64)));
    }
  };

  flt4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = flt4{0.f, 0.f, 0.f, 0.f};

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
    flt4 fa[FM], fb[FN];
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      const int r = wm + i * 16 + lr;
      if constexpr (AD) {
        const dbl2 p0 = *reinterpret_cast<const dbl2*>(as + 4 * (r * AQ + ((2 * lk) ^ ((r >> 1) & 7))));
        const dbl2 p1 = *reinterpret_cast<const dbl2*>(as + 4 * (r * AQ + ((2 * lk + 1) ^ ((r >> 1) & 7))));
        fa[i] = flt4{(float)p0[0], (float)p0[1], (float)p1[0], (float)p1[1]};
      } else {
        fa[i] = *reinterpret_cast<const flt4*>(as + 4 * (r * KQ + (lk ^ swz_kq(r))));
      }
    }
#pragma unroll
    for (int jj = 0; jj < FN; ++jj) {
      const int n = wn + jj * 16 + lr;
      if constexpr (B_KCONTIG) {
        fb[jj] = *reinterpret_cast<const flt4*>(bs + 4 * (n * KQ + (lk ^ swz_kq(n))));
      } else {
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          const int k = 4 * lk + h;
          fb[jj][h] = bs[4 * (k * (BN / 4) + ((n >> 2) ^ swz_nq(k))) + (n & 3)];
        }
      }
    }
    if (ktail != 0 && c == nchunks - 1 && 4 * lk >= ktail) {
      // this lane group's k (4 lk .. 4 lk + 3) lie past K
#pragma unroll
      for (int i = 0; i < FM; ++i) fa[i] = flt4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int jj = 0; jj < FN; ++jj) fb[jj] = flt4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int h = 0; h < 4; ++h)
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int jj = 0; jj < FN; ++jj)
          acc[i][jj] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[i][h], fb[jj][h], acc[i][jj], 0, 0, 0);
  }

  if constexpr (LC)
    lincomb_epilogue_f32<BM, BN, WM, WN>(acc, g, epi, Yb, YN, Cb, cbase, tc.z1,
                                         reinterpret_cast<double*>(lds), m0, n0, wave, tid);
  else
    store_acc_tile<FM, FN, TC>(acc, g, epi, Cb, cbase, tc.z1, m0 + wm, n0 + wn, lr, lk);
}

#ifndef PHIKS_F32DL_MIN_WAVES_LC
#define PHIKS_F32DL_MIN_WAVES_LC 3
#endif
template <class Epi>
constexpr int f32dl_min_waves() {
  return std::is_same<Epi, EpiLinComb>::value ? PHIKS_F32DL_MIN_WAVES_LC : PHIKS_F32DL_MIN_WAVES;
}

template <int BM, int BN, int WM, int WN, bool B_KCONTIG, class TA, class TC, class Epi>
__global__ void __launch_bounds__(256, f32dl_min_waves<Epi>()) gemm_f32_dl_kernel(GemmArgs g, Epi epi) {
  const int64_t rest = xcd_remap(blockIdx.x, g.total_tiles);
  if constexpr (std::is_same<Epi, EpiLinComb>::value)
    gemm_f32_dl_tile<BM, BN, WM, WN, B_KCONTIG, TA, TC, Epi>(g, epi, rest, epi.Y, epi.N);
  else
    gemm_f32_dl_tile<BM, BN, WM, WN, B_KCONTIG, TA, TC, Epi>(g, epi, rest, nullptr, 0);
}

// Grouped launch of the direct-to-LDS FP32 kernel (see gemm_f32_grouped).
template <int BM, int BN, int WM, int WN, bool B_KCONTIG, class TA, class TC, class Epi>
__global__ void __launch_bounds__(256, f32dl_min_waves<Epi>())
    gemm_f32_dl_grouped(const GroupItem* __restrict__ items, const int64_t* __restrict__ first,
                        int nitems, int64_t total, Epi epi) {
  const int64_t t = xcd_remap(blockIdx.x, total);
  const int i = find_group_item(first, nitems, t);
  const GroupItem& it = items[i];
  // the item's pre-step tensors go beside epi, not into a modified copy of it (a local
  // copy indexed by the tensor index lives in scratch memory)
  if constexpr (std::is_same<Epi, EpiLinComb>::value) {
    gemm_f32_dl_tile<BM, BN, WM, WN, B_KCONTIG, TA, TC, Epi>(it.g, epi, t - first[i], it.Y, it.YN);
  } else {
    gemm_f32_dl_tile<BM, BN, WM, WN, B_KCONTIG, TA, TC, Epi>(it.g, epi, t - first[i], nullptr, 0);
  }
}

}  // namespace phiks
