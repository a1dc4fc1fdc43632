// FP64 MFMA GEMM for gfx950 with direct-to-LDS operand loads: the mu-mode products of
// Section 2 at tile sizes 64 and 128, K a multiple of the chunk length.
//
// Same products, tile order and epilogues as gemm_f64_kernel (gemm_f64.hpp); what
// differs is how operands reach LDS.  Every operand load is a global_load_lds_dwordx4:
// each lane moves 16 bytes from global memory straight into LDS, lane l of a wave
// writing the l-th 16-byte slot after the wave's base (held in M0).  No registers hold
// staged operands and no instructions copy them, so chunks can be fetched ST - 1 ahead
// of the MFMAs through an ST-stage LDS ring, synchronised by the load counter (vmcnt)
// and one barrier per chunk.
//
// LDS layouts (16-byte slots; the lane -> slot map is fixed, so each lane fetches the
// global data that belongs in its slot):
//  * k-contiguous operand (A, and B of mode 1), rows r < R, k < BK: the slot of
//    (r, k pair kp) is r*KP + (kp ^ swz_kp(r)), KP = BK/2.  KP consecutive lanes fetch one
//    row's BK*8 contiguous bytes.  A fragment read takes one k pair per lane
//    (ds_read_b128) and feeds two MFMAs: lane group lk = l >> 4 of MFMA step 2j (2j+1)
//    holds k = 8j + 2lk (8j + 2lk + 1), the same k for both operands of each MFMA.
//  * n-contiguous operand (B of modes > 1), k < BK, columns c < BN: the slot of
//    (k, column pair cp) is k*BN/2 + (cp ^ swz_np(k)).  Fragment reads are 8 bytes.
// Both swizzles make every 16-lane (b128) or 32-lane (b64) group of a fragment read hit
// distinct banks; the DMA writes are contiguous.
//
// Ragged M and N: rows (columns) past the end are fetched from a clamped in-range
// address; they only reach output rows (columns) that are never stored.  K must be a
// multiple of BK (the launcher checks), so no zero fill is needed.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "gemm_f64.hpp"
// PHIKS_DL_BK: k per chunk; PHIKS_DL_MIN_WAVES: waves per SIMD the register budget must
// allow; PHIKS_DL_MIN_WAVES_LC: the same for the squaring epilogue (tuned values)
#include "kernel_tuning.inc"

namespace phiks {

#ifndef PHIKS_DL_ST
#define PHIKS_DL_ST 2   // LDS stages
#endif

template <int KP>
__device__ __forceinline__ int swz_kp(int r) { return (r / (16 / KP)) & (KP - 1); }
__device__ __forceinline__ int swz_np(int k) { return ((k >> 1) & 1) << 3; }

// s_waitcnt with only the vector-memory counter bounded (gfx9 encoding: vmcnt in bits
// 3:0 and 15:14, expcnt 6:4 and lgkmcnt 11:8 left at their no-wait maxima).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}
__device__ __forceinline__ void wait_lgkmcnt0() {
  __builtin_amdgcn_s_waitcnt(15 | (7 << 4) | (0 << 8) | (3 << 14));
}

// 16 bytes per lane from src into LDS: lane l writes bytes [16 l, 16 l + 16) after the
// wave-uniform LDS address lds_dst.  Issued from inline asm: the compiler would
// otherwise wait for every LDS-DMA load in flight before each LDS read it cannot prove
// disjoint from them, which serialises the stages.  The ordering is explicit instead:
// wait_vmcnt for this wave's loads of a chunk, then a barrier for everyone's.  The
// statement has no outputs; its inputs are read when it issues.
__device__ __forceinline__ void dma16(const PHIKS_GLOBAL double* src, double* lds_dst) {
  const uint32_t lds = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) double*)lds_dst;
  asm volatile("global_load_lds_dwordx4 %0, off" : : "v"(src), "{m0}"(lds) : "memory");
}

// The squaring epilogue (lincomb_wave_epilogue below) streams the pre-step tensors in
// 16-byte column pairs: even ldc, N, output strides and tensor stride, aligned Y
// (lincomb_dl_ok, checked by the launchers: launches that fail it take gemm_f64_kernel).
inline bool lincomb_dl_ok(const GemmArgs& g, const double* Y, int64_t YN) {
  return ((g.ldc | (int64_t)g.N | g.sC0 | g.sC1 | YN) & 1) == 0 && ((uintptr_t)Y & 15) == 0 &&
         (g.pC == nullptr);
}

// Squaring epilogue out = a_l acc + sum_{k <= l} c_lk Y_k with the pre-step tensors Y_k
// streamed through LDS by the same 16-byte DMA as the operands, instead of register loads
// whose latency each wave would wait out round after round.  Round r = k * FM + i brings
// fragment row i of Y_k for this wave only (16 rows of WN columns, stored as column pairs,
// slot row * WN/2 + (cp ^ (WN/4) (row & 1)) so the two row parities of a 32-lane read land
// on different bank halves) into one of the wave's YB buffers, YB - 1 rounds ahead.  A wave
// reads only what it fetched, so a round waits on the wave's own loads (vmcnt) and no
// work-group barrier follows the first: the waves do not wait for each other round after
// round, and the epilogue needs fewer registers than one with shared slices, so the
// squaring kernels run at 4 waves per SIMD.  Per element the arithmetic is acc *= a_l, then
// one fma per k in k order (every FP64 squaring kernel does exactly this).
template <int WM, int WN, int YB, int FM, int FN>
__device__ __forceinline__ void lincomb_wave_epilogue(dbl4 (&acc)[FM][FN], const GemmArgs& g,
                                                      const EpiLinComb& epi, const double* Yb,
                                                      int64_t YN, const TileOperands& t,
                                                      double* lds, int mw, int nw, int wave, int lane) {
  constexpr int CPW = WN / 2;                 // column pairs per row
  constexpr int SLICE = 16 * WN;              // doubles per wave slice
  constexpr int LW = 16 * CPW / 64;           // 16-byte loads per lane per round
  static_assert(CPW >= 2 && (16 * CPW) % 64 == 0, "whole waves of slots");
  const int lr = lane & 15, lk = lane >> 4;
  const int l = (int)t.z1;
  const int rounds = (l + 1) * FM;
  double* wbuf = lds + wave * YB * SLICE;
  const PHIKS_GLOBAL double* Y0 = gptr(Yb) + t.cbase - (int64_t)l * YN;   // Y_0 at this tile
  auto issue = [&](int r) {
    const int k = r / FM, i = r % FM;
    const PHIKS_GLOBAL double* Yk = Y0 + (int64_t)k * YN;
    double* buf = wbuf + (r % YB) * SLICE;
    // computed per round (not hoisted out of the k loop: held across it they would not fit)
    int64_t ldc = g.ldc;
    int M = g.M, N = g.N;
    int mr = __builtin_amdgcn_readfirstlane(mw), nc = __builtin_amdgcn_readfirstlane(nw);   // wave-uniform
    asm volatile("" : "+s"(ldc), "+s"(M), "+s"(N), "+s"(mr), "+s"(nc));
#pragma unroll
    for (int q = 0; q < LW; ++q) {
      const int s = q * 64 + lane;
      const int row = s / CPW, cp = (s % CPW) ^ ((row & 1) * (CPW / 2));
      const int grow = min(mr + i * 16 + row, M - 1), gcol = min(nc + 2 * cp, N - 2);
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
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] *= al;

  for (int k = 0; k <= l; ++k) {
    const double ck = epi.c[l][k];
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      const int r = k * FM + i;
      // round r has landed once at most the later rounds' loads are outstanding
      if (r + YB - 2 < rounds) wait_vmcnt<(YB - 2) * LW>();
      else wait_vmcnt<0>();
      asm volatile("" ::: "memory");
      // the buffer round r - 1 used is free: its reads fed the fmas above
      if (r + YB - 1 < rounds) issue(r + YB - 1);
      const double* buf = wbuf + (r % YB) * SLICE;
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int c = j * 16 + lr;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const int row = lk + 4 * rr;
          const double y = buf[2 * (row * CPW + ((c >> 1) ^ ((row & 1) * (CPW / 2)))) + (c & 1)];
          acc[i][j][rr] = __builtin_fma(ck, y, acc[i][j][rr]);
        }
      }
    }
  }

  const int ml = mw + lk, nl = nw + lr;
  const int64_t base = t.cbase + (int64_t)ml * g.ldc + nl;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr)
        if ((ml + i * 16 + 4 * rr < g.M) & (nl + j * 16 < g.N))
          t.Cb[base + (int64_t)(i * 16 + 4 * rr) * g.ldc + j * 16] = acc[i][j][rr];
}

template <int BM, int BN, int WM, int WN, bool B_KCONTIG, class Epi, int BK, int ST>
__device__ __forceinline__ void gemm_f64_dl_tile(const GemmArgs& g, const Epi& epi, int64_t rest,
                                                 const double* Yb, int64_t YN) {
  static_assert(BK == 8 || BK == 16, "chunk of 8 or 16 k");
  static_assert(ST >= 2, "at least two stages");
  constexpr int KP = BK / 2;
  constexpr int WGM = BM / WM, WGN = BN / WN;
  static_assert(WGM * WGN == 4, "4 waves per work-group");
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int A_SLOTS = BM * KP, B_SLOTS = BN * KP;
  // a tile of fewer than 256 slots is fetched by the first SLOTS/64 waves; the waves then
  // issue different load counts, which the per-chunk wait only allows with two stages
  // (every wait there is for all of a wave's loads)
  static_assert(A_SLOTS % 64 == 0 && B_SLOTS % 64 == 0, "whole waves of slots");
  static_assert(ST == 2 || (A_SLOTS % 256 == 0 && B_SLOTS % 256 == 0),
                "every wave fetches the same count");
  constexpr int LA = (A_SLOTS + 255) / 256, LB = (B_SLOTS + 255) / 256;
  static_assert(B_KCONTIG || BN / 2 >= 16, "column-pair swizzle needs BN >= 32");

  // LDS: the ST-stage operand ring; the squaring epilogue reuses the same memory for its
  // YB slice buffers per wave once the K loop is done (two: with three, a 128 x 64 tile
  // needs 48 KB and LDS holds only 3 work-groups per CU)
  constexpr bool LC = std::is_same<Epi, EpiLinComb>::value;
  constexpr int STAGE = 2 * (A_SLOTS + B_SLOTS);        // doubles per stage
  constexpr int YSLICE = WGM * 16 * BN, YB = 2;         // doubles per work-group slice round
  constexpr int LDS_DBL = (LC && YB * YSLICE > ST * STAGE) ? YB * YSLICE : ST * STAGE;
  __shared__ __align__(16) double lds[LDS_DBL];
  auto As = [&](int st) { return lds + st * STAGE; };
  auto Bs = [&](int st) { return lds + st * STAGE + 2 * A_SLOTS; };

  const TileOperands t = tile_operands<B_KCONTIG>(g, rest);
  const int m0 = t.tm * BM, n0 = t.tn * BN;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = (wave / WGN) * WM, wn = (wave % WGN) * WN;
  const int lr = lane & 15, lk = lane >> 4;

  // global sources of this thread's slots, chunk 0
  const PHIKS_GLOBAL double* asrc[LA];
  const PHIKS_GLOBAL double* bsrc[LB];
#pragma unroll
  for (int i = 0; i < LA; ++i) {
    const int s = min(i * 256 + tid, A_SLOTS - 1);   // (clamped slots are never issued)
    const int r = s / KP, kp = (s % KP) ^ swz_kp<KP>(s / KP);
    asrc[i] = t.A + (int64_t)min(m0 + r, g.M - 1) * g.lda + 2 * kp;
  }
#pragma unroll
  for (int i = 0; i < LB; ++i) {
    const int s = min(i * 256 + tid, B_SLOTS - 1);
    if constexpr (B_KCONTIG) {
      const int r = s / KP, kp = (s % KP) ^ swz_kp<KP>(s / KP);
      bsrc[i] = t.B + (int64_t)min(n0 + r, g.N - 1) * g.ldb + 2 * kp;
    } else {
      const int k = s / (BN / 2), cp = (s % (BN / 2)) ^ swz_np(s / (BN / 2));
      bsrc[i] = t.B + (int64_t)k * g.ldb + min(n0 + 2 * cp, g.N - 2);
    }
  }
  const int64_t bstep = B_KCONTIG ? BK : (int64_t)BK * g.ldb;   // source advance per chunk

  auto issue = [&](int c) {
    const int st = c % ST;
#pragma unroll
    for (int i = 0; i < LA; ++i)
      if (A_SLOTS % 256 == 0 || i * 256 + wave * 64 < A_SLOTS)
        dma16(asrc[i] + (int64_t)c * BK, As(st) + 2 * (i * 256 + wave * 64));
#pragma unroll
    for (int i = 0; i < LB; ++i)
      if (B_SLOTS % 256 == 0 || i * 256 + wave * 64 < B_SLOTS)
        dma16(bsrc[i] + (int64_t)c * bstep, Bs(st) + 2 * (i * 256 + wave * 64));
  };

  dbl4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};

  const int nchunks = g.K / BK;
#pragma unroll
  for (int c = 0; c < ST - 1; ++c)
    if (c < nchunks) issue(c);

  for (int c = 0; c < nchunks; ++c) {
    // chunk c has landed once no more than the later chunks' loads are outstanding
    if (c + ST - 2 < nchunks) wait_vmcnt<(ST - 2) * (LA + LB)>();
    else wait_vmcnt<0>();
    wait_lgkmcnt0();
    // chunk c visible; every wave is done with chunk c - 1.  The empty asm statements
    // keep the compiler from moving LDS accesses across the barrier (a fence would
    // also wait for the loads of the later chunks).
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    if (c + ST - 1 < nchunks) issue(c + ST - 1);   // into the stage chunk c - 1 used
    const double* as = As(c % ST);
    const double* bs = Bs(c % ST);
#pragma unroll
    for (int j = 0; j < BK / 8; ++j) {
      const int kp = 4 * j + lk;
      dbl2 fa[FM], fb[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        const int r = wm + i * 16 + lr;
        fa[i] = *reinterpret_cast<const dbl2*>(as + 2 * (r * KP + (kp ^ swz_kp<KP>(r))));
      }
#pragma unroll
      for (int jj = 0; jj < FN; ++jj) {
        const int n = wn + jj * 16 + lr;
        if constexpr (B_KCONTIG) {
          fb[jj] = *reinterpret_cast<const dbl2*>(bs + 2 * (n * KP + (kp ^ swz_kp<KP>(n))));
        } else {
          const int k = 8 * j + 2 * lk;
          fb[jj][0] = bs[2 * (k * (BN / 2) + ((n >> 1) ^ swz_np(k))) + (n & 1)];
          fb[jj][1] = bs[2 * ((k + 1) * (BN / 2) + ((n >> 1) ^ swz_np(k + 1))) + (n & 1)];
        }
      }
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int jj = 0; jj < FN; ++jj)
            acc[i][jj] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i][h], fb[jj][h], acc[i][jj], 0, 0, 0);
    }
  }

  if constexpr (LC) {
    lincomb_wave_epilogue<WM, WN, YB>(acc, g, epi, Yb, YN, t, lds, m0 + wm, n0 + wn, wave, lane);
  } else {
    store_tile_f64<FM, FN>(acc, g, epi, t.Cb, t.cbase, t.z1, m0 + wm, n0 + wn, lr, lk);
  }
}

template <class Epi>
constexpr int dl_min_waves() {
  return std::is_same<Epi, EpiLinComb>::value ? PHIKS_DL_MIN_WAVES_LC : PHIKS_DL_MIN_WAVES;
}

template <int BM, int BN, int WM, int WN, bool B_KCONTIG, class Epi>
__global__ void __launch_bounds__(256, dl_min_waves<Epi>()) gemm_f64_dl_kernel(GemmArgs g, Epi epi) {
  const int64_t rest = xcd_remap(blockIdx.x, g.total_tiles);
  if constexpr (std::is_same<Epi, EpiLinComb>::value)
    gemm_f64_dl_tile<BM, BN, WM, WN, B_KCONTIG, Epi, PHIKS_DL_BK, PHIKS_DL_ST>(g, epi, rest, epi.Y, epi.N);
  else
    gemm_f64_dl_tile<BM, BN, WM, WN, B_KCONTIG, Epi, PHIKS_DL_BK, PHIKS_DL_ST>(g, epi, rest, nullptr, 0);
}

// Grouped launch (many independent GEMMs of one kind in one grid; see gemm_f64_grouped).
template <int BM, int BN, int WM, int WN, bool B_KCONTIG, class Epi>
__global__ void __launch_bounds__(256, dl_min_waves<Epi>())
    gemm_f64_dl_grouped(const GroupItem* __restrict__ items, const int64_t* __restrict__ first,
                        int nitems, int64_t total, Epi epi) {
  const int64_t t = xcd_remap(blockIdx.x, total);
  const int i = find_group_item(first, nitems, t);
  const GroupItem& it = items[i];
  // the item's pre-step tensors are passed beside epi rather than through a modified
  // copy of it: a local copy indexed by the tensor index l lives in scratch memory
  if constexpr (std::is_same<Epi, EpiLinComb>::value) {
    gemm_f64_dl_tile<BM, BN, WM, WN, B_KCONTIG, Epi, PHIKS_DL_BK, PHIKS_DL_ST>(it.g, epi, t - first[i],
                                                                             it.Y, it.YN);
  } else {
    gemm_f64_dl_tile<BM, BN, WM, WN, B_KCONTIG, Epi, PHIKS_DL_BK, PHIKS_DL_ST>(it.g, epi, t - first[i],
                                                                             nullptr, 0);
  }
}

}  // namespace phiks
