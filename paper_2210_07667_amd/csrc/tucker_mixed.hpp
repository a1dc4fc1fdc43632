// Mixed-precision mu-mode products: launches of the FP32-MFMA kernels (gemm_f32_kernel,
// gemm_f32_dl_kernel) and of the BF16x3 kernels (three BF16 MFMA products per FP32
// product: gemm_bf16x3_kernel, gemm_bf16x3_dl_kernel), and the Tucker chain over either,
// including the BF16x3 pair chains.  Included once, by phiks.hip, after tucker_f64.hpp.
#pragma once
#include <vector>

#include "gemm_bf16x3.hpp"
#include "gemm_bf16x3_dl.hpp"
#include "gemm_f32.hpp"
#include "gemm_f32_dl.hpp"
#include "tucker_f64.hpp"

#ifndef PHIKS_BF_DL
#define PHIKS_BF_DL 1  // 1: BF16x3 products of modes > 1 on the direct-to-LDS kernel
#endif
#ifndef PHIKS_F32_DL_A64
#define PHIKS_F32_DL_A64 1  // 1: FP32 products with an FP64 A (first modes) on the direct-to-LDS kernel
#endif
#ifndef PHIKS_BF_PAIR
#define PHIKS_BF_PAIR 1  // 1: BF16x3 chains keep split pairs between modes where they can
#endif
#ifndef PHIKS_MIXED_LC_DL
#define PHIKS_MIXED_LC_DL 1  // 1: mixed-precision squaring launches on the direct-to-LDS kernels
#endif

namespace {

using namespace phiks;

// ------------------------------------------------- FP32 MFMA mu-mode launches
bool vec4_ok(const GemmArgs& g, bool kcontig) {
  if (g.K % 4 || g.lda % 4 || g.ldb % 4) return false;
  if (!kcontig && g.N % 4) return false;
  if (g.sA0 % 4 || g.sA1 % 4 || g.sB0 % 4 || g.sB1 % 4) return false;
  return aligned16(g.A) && aligned16(g.B);
}

// One launch of a mixed-precision mu-mode kernel over the whole tile grid, with the
// optional timing events of runtime.hpp.
template <int BM, int BN, class Epi>
int launch_grid(void (*kern)(GemmArgs, Epi), GemmArgs g, const Epi& epi, hipStream_t st) {
  g.tiles_m = (g.M + BM - 1) / BM;
  g.tiles_n = (g.N + BN - 1) / BN;
  g.total_tiles = (int64_t)g.tiles_m * g.tiles_n * g.nb0 * g.nb1;
  if (g.total_tiles <= 0) return PHIKS_OK;
  if (g.total_tiles > 0x7fffffffLL) {
    set_error("GEMM grid too large");
    return PHIKS_EINVAL;
  }
  return timed_launch(kern, (unsigned)g.total_tiles, st,
                      2.0 * g.M * (double)g.N * g.K * g.nb0 * (double)g.nb1, g, epi);
}

// The direct-to-LDS kernels' squaring epilogue needs lincomb_dl_ok; other epilogues pass.
template <class Epi>
bool lincomb_ok(const GemmArgs& g, const Epi& epi) {
  if constexpr (std::is_same<Epi, EpiLinComb>::value)
    return PHIKS_MIXED_LC_DL == 1 && lincomb_dl_ok(g, epi.Y, epi.N);
  else return true;
}

template <int BM, int BN, int WM, int WN, bool KC, bool VEC, class TA, class TC, class Epi>
int launch_cfg32(const GemmArgs& g, const Epi& epi, hipStream_t st) {
  if constexpr (PHIKS_DL == 1 && VEC && (PHIKS_F32_DL_A64 == 1 || std::is_same<TA, float>::value) &&
                BM >= 64 && BN >= 64) {
    // direct-to-LDS loads (16-k chunks, the last one partial when K is not a multiple
    // of 16; an FP64 A is converted at the fragment read); the squaring epilogue streams
    // its pre-step tensors through LDS too
    if (g.K % 4 == 0 && g.pA == nullptr && lincomb_ok(g, epi))
      return launch_grid<BM, BN>(&gemm_f32_dl_kernel<BM, BN, WM, WN, KC, TA, TC, Epi>, g, epi, st);
  }
  return launch_grid<BM, BN>(&gemm_f32_kernel<BM, BN, WM, WN, KC, VEC, TA, TC, Epi>, g, epi, st);
}

#ifndef PHIKS_F32_SKINNY64
#define PHIKS_F32_SKINNY64 1  // 1: skinny FP32 products on 64 x 64 direct-to-LDS tiles
#endif
#ifndef PHIKS_F32_SKINNY_LONG
#define PHIKS_F32_SKINNY_LONG 256  // the longer side from which a skinny product takes them
#endif
#ifndef PHIKS_F32_BIG_TILE
#define PHIKS_F32_BIG_TILE 1  // 1: 128 x 128 tiles (4 waves of 64 x 64) where they fill the GPU
#endif
// The configuration an FP32 product runs in (tile, load width, kernel): 128 x 128 tiles
// (4 waves of 64 x 64) where 256 of them fill the GPU, else 128 x 64 or 64 x 128 where those
// do, else 64 x 64 when both sides reach 48 (the direct-to-LDS kernel needs 64-wide tiles;
// a product too small to fill the GPU keeps that tile rather than splitting into 32 x 32
// ones, so grouped launches of many small products -- batches -- run it too), else 32 x 32.
// Skinny products (one side 16..47, the other >= 256: the small modes of mixed-size
// problems) take 64 x 64 tiles too when the direct-to-LDS kernel can run them (K a multiple
// of 4, its last chunk partial when K is not a multiple of 16): they move
// 2-3 flop per byte, so the tile's idle rows or columns cost no time, and their squaring
// steps get the LDS-streamed epilogue.
// launch_gemm32 runs exactly this; grouped launches of FP32 batches take it per item, so
// each item runs the tiles of its single call.  a_double: A is the FP64 input (mode 1);
// dl_epi_ok: the epilogue passes lincomb_ok.
struct Cfg32 {
  int bm, bn;
  bool vec, dl;
};
Cfg32 cfg32(const GemmArgs& g, bool kc, bool a_double, bool dl_epi_ok) {
  Cfg32 c{32, 32, vec4_ok(g, kc), false};
  if (PHIKS_F32_BIG_TILE == 1 && g.M >= 128 && g.N >= 128 && tiles_for(g, 128, 128) >= 256) {
    c.bm = c.bn = 128;
  } else {
    switch (pick_tile(g)) {
      case Tile::T128x128:
      case Tile::T128x64: c.bm = 128; c.bn = 64; break;
      case Tile::T64x128: c.bm = 64; c.bn = 128; break;
      case Tile::T64x64: c.bm = 64; c.bn = 64; break;
      default:
        if (g.M >= 48 && g.N >= 48) c.bm = c.bn = 64;
        break;
    }
  }
  auto dl_ok32 = [&](int bm, int bn) {
    return PHIKS_DL == 1 && c.vec && (PHIKS_F32_DL_A64 == 1 || !a_double) && bm >= 64 &&
           bn >= 64 && g.K % 4 == 0 && g.pA == nullptr && dl_epi_ok;
  };
  if (PHIKS_F32_SKINNY64 == 1 && c.bm == 32 && std::min(g.M, g.N) >= 16 &&
      std::max(g.M, g.N) >= PHIKS_F32_SKINNY_LONG && dl_ok32(64, 64))
    c.bm = c.bn = 64;
  c.dl = dl_ok32(c.bm, c.bn);
  return c;
}

template <bool KC, bool VEC, class TA, class TC, class Epi>
int launch_tile32(const GemmArgs& g, const Epi& epi, hipStream_t st) {
  const Cfg32 c = cfg32(g, KC, std::is_same<TA, double>::value, lincomb_ok(g, epi));
  if (c.bm == 128 && c.bn == 128) return launch_cfg32<128, 128, 64, 64, KC, VEC, TA, TC>(g, epi, st);
  if (c.bm == 128) return launch_cfg32<128, 64, 64, 32, KC, VEC, TA, TC>(g, epi, st);
  if (c.bn == 128) return launch_cfg32<64, 128, 32, 64, KC, VEC, TA, TC>(g, epi, st);
  if (c.bm == 64) return launch_cfg32<64, 64, 32, 32, KC, VEC, TA, TC>(g, epi, st);
  return launch_cfg32<32, 32, 16, 16, KC, VEC, TA, TC>(g, epi, st);
}

template <bool KC, class TA, class TC, class Epi>
int launch_gemm32(const GemmArgs& g, const Epi& epi, hipStream_t st) {
  if (vec4_ok(g, KC)) return launch_tile32<KC, true, TA, TC>(g, epi, st);
  return launch_tile32<KC, false, TA, TC>(g, epi, st);
}
// ---------------------------------------------- BF16x3 MFMA mu-mode launches
template <int BM, int BN, int WM, int WN, bool KC, bool VEC, class TA, class TC, class Epi>
int launch_cfg_bf(const GemmArgs& g, const Epi& epi, hipStream_t st) {
  if constexpr (PHIKS_DL == 1 && PHIKS_BF_DL == 1 && VEC && !KC && std::is_same<TA, float>::value &&
                BN >= 64) {
    // modes > 1 (FP32 operands, n-contiguous tensor): direct-to-LDS operand path
    if (g.K % 32 == 0 && g.N % 4 == 0 && g.ldb % 4 == 0 && g.pA == nullptr && lincomb_ok(g, epi))
      return launch_grid<BM, BN>(&gemm_bf16x3_dl_kernel<BM, BN, WM, WN, TC, Epi, false>, g, epi, st);
  }
  return launch_grid<BM, BN>(&gemm_bf16x3_kernel<BM, BN, WM, WN, KC, VEC, TA, TC, Epi>, g, epi,
                             st);
}

// 16-byte loads need K, the leading dimensions of the k-contiguous operands and the
// batch strides to be multiples of 4 floats, and 16-byte aligned bases.
bool vec_bf_ok(const GemmArgs& g, bool kcontig) {
  if (g.K % 4 || g.lda % 4 || (kcontig && g.ldb % 4)) return false;
  if (g.sA0 % 4 || g.sA1 % 4 || g.sB0 % 4 || g.sB1 % 4) return false;
  return aligned16(g.A) && aligned16(g.B);
}

#ifndef PHIKS_BF_BIG_TILE
#define PHIKS_BF_BIG_TILE 1  // 1: 128 x 128 tiles (4 waves of 64 x 64) where they fill the GPU
#endif
// Products too small for a 64 x 64 tile per compute unit go to the FP32 kernel.
template <bool KC, bool VEC, class TA, class TC, class Epi>
int launch_tile_bf(const GemmArgs& g, const Epi& epi, hipStream_t st) {
#if PHIKS_BF_BIG_TILE == 1
  if (g.M >= 128 && g.N >= 128 && tiles_for(g, 128, 128) >= 256)
    return launch_cfg_bf<128, 128, 64, 64, KC, VEC, TA, TC>(g, epi, st);
#endif
  switch (pick_tile(g)) {
    case Tile::T128x128:
    case Tile::T128x64: return launch_cfg_bf<128, 64, 64, 32, KC, VEC, TA, TC>(g, epi, st);
    case Tile::T64x128: return launch_cfg_bf<64, 128, 32, 64, KC, VEC, TA, TC>(g, epi, st);
    case Tile::T64x64: return launch_cfg_bf<64, 64, 32, 32, KC, VEC, TA, TC>(g, epi, st);
    default: return launch_gemm32<KC, TA, TC>(g, epi, st);
  }
}

template <bool KC, class TA, class TC, class Epi>
int launch_gemm_bf(const GemmArgs& g, const Epi& epi, hipStream_t st) {
  if (vec_bf_ok(g, KC)) return launch_tile_bf<KC, true, TA, TC>(g, epi, st);
  return launch_tile_bf<KC, false, TA, TC>(g, epi, st);
}

// ------------------------------------------------------- BF16x3 pair chains
// A product of modes > 1 whose operands are pair words (matrix and intermediate):
// only the direct-to-LDS kernel reads pairs, so a chain uses them only if every such
// product passes this test (the tile choice and the conditions of launch_tile_bf /
// launch_cfg_bf that lead there).
bool pair_dl_ok(const GemmArgs& g) {
  if (!vec_bf_ok(g, false)) return false;
  if (g.K % 32 || g.N % 4 || g.ldb % 4 || g.pA != nullptr) return false;
#if PHIKS_BF_BIG_TILE == 1
  if (g.M >= 128 && g.N >= 128 && tiles_for(g, 128, 128) >= 256) return true;
#endif
  return pick_tile(g) != Tile::T32x32;
}

template <int BM, int BN, int WM, int WN, class TC, class Epi>
int launch_pair_cfg(const GemmArgs& g, const Epi& epi, hipStream_t st) {
  return launch_grid<BM, BN>(&gemm_bf16x3_dl_kernel<BM, BN, WM, WN, TC, Epi, true>, g, epi, st);
}

// Same tiles as launch_tile_bf, pair operands.
template <class TC, class Epi>
int launch_pair(const GemmArgs& g, const Epi& epi, hipStream_t st) {
  if (!pair_dl_ok(g) || !lincomb_ok(g, epi)) {
    set_error("BF16x3 pair product outside the direct-to-LDS kernel's conditions");
    return PHIKS_EINVAL;
  }
#if PHIKS_BF_BIG_TILE == 1
  if (g.M >= 128 && g.N >= 128 && tiles_for(g, 128, 128) >= 256)
    return launch_pair_cfg<128, 128, 64, 64, TC>(g, epi, st);
#endif
  switch (pick_tile(g)) {
    case Tile::T128x128:
    case Tile::T128x64: return launch_pair_cfg<128, 64, 64, 32, TC>(g, epi, st);
    case Tile::T64x128: return launch_pair_cfg<64, 128, 32, 64, TC>(g, epi, st);
    default: return launch_pair_cfg<64, 64, 32, 32, TC>(g, epi, st);
  }
}

// mu-mode launch in the arithmetic PREC (PHIKS_FP32 or PHIKS_BF16X3)
template <int PREC, bool KC, class TA, class TC, class Epi>
int launch_mixed(const GemmArgs& g, const Epi& epi, hipStream_t st) {
  if constexpr (PREC == PHIKS_BF16X3) return launch_gemm_bf<KC, TA, TC>(g, epi, st);
  else return launch_gemm32<KC, TA, TC>(g, epi, st);
}

// Mixed-precision Tucker operator (FP32 or BF16x3 products): the chain input (FP64)
// is converted in the first mode, intermediate modes are FP32 (ta/tb hold floats), the
// last mode writes FP64 through the same epilogue as the FP64 chain.  L[mu] are FP32
// copies of the matrices.
// BF16x3 chains of d >= 2 whose products of modes > 1 all fit the direct-to-LDS kernel
// (pair_dl_ok) keep their intermediates as pair words and multiply the plan's pair
// copies of the matrices (pair_off): each value is split once, by the kernel that
// writes it, instead of by every work-group that reads it.  The MFMA operands are the
// same bfloat16 numbers either way, so the result is bitwise that of the FP32 form.
template <int PREC, class Epi>
int tucker_mixed(const phiks_plan_s& P, const double* in, int64_t in_stride,
                 float* const* L, const int64_t* l_stride, int nbatch, double* out,
                 double* ta, double* tb, const Epi& epi, hipStream_t st) {
  GemmArgs gs[PHIKS_MAX_D];
  double* Ld[PHIKS_MAX_D];
  for (int mu = 0; mu < P.d; ++mu) Ld[mu] = reinterpret_cast<double*>(L[mu]);
  tucker_args(P.d, P.n, P.N, in, in_stride, Ld, l_stride, nbatch, out, ta, tb, gs);
  if constexpr (PREC == PHIKS_BF16X3) {
    GemmArgs gp[PHIKS_MAX_D];
    bool pairs = PHIKS_BF_PAIR == 1 && PHIKS_BF_DL == 1 && PHIKS_DL == 1 && P.d >= 2;
    for (int mu = 2; mu <= P.d && pairs; ++mu) {
      gp[mu - 1] = gs[mu - 1];
      gp[mu - 1].A = reinterpret_cast<const double*>(L[mu - 1] + P.pair_off[mu - 1]);
      pairs = pair_dl_ok(gp[mu - 1]);
    }
    pairs = pairs && lincomb_ok(gp[P.d - 1], epi);
    if (pairs) {
      // first mode: FP64 input by the FP32 matrix as before, pair words out
      RET_IF((launch_mixed<PREC, true, double, unsigned>(gs[0], EpiStorePair{}, st)));
      for (int mu = 2; mu < P.d; ++mu) RET_IF((launch_pair<unsigned>(gp[mu - 1], EpiStorePair{}, st)));
      return launch_pair<double>(gp[P.d - 1], epi, st);
    }
  }
  for (int mu = 1; mu <= P.d; ++mu) {
    const bool last = (mu == P.d);
    const GemmArgs& g = gs[mu - 1];
    if (mu == 1) {
      // A: the FP64 input (converted on the way into LDS), B: the FP32 matrix
      if (last) RET_IF((launch_mixed<PREC, true, double, double>(g, epi, st)));
      else RET_IF((launch_mixed<PREC, true, double, float>(g, EpiStoreT<float>{1.0, 0.0}, st)));
    } else {
      // A: the FP32 matrix, B: the FP32 intermediate
      if (last) RET_IF((launch_mixed<PREC, false, float, double>(g, epi, st)));
      else RET_IF((launch_mixed<PREC, false, float, float>(g, EpiStoreT<float>{1.0, 0.0}, st)));
    }
  }
  return PHIKS_OK;
}

}  // namespace
