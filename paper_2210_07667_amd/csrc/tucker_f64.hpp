// FP64 mu-mode products: tile choice and launch of gemm_f64_kernel, and the Tucker
// operator as a chain of d such launches (Section 2, Lemma 1).  Included once, by
// phiks.hip, after runtime.hpp and plan.hpp.
#pragma once
#include <algorithm>
#include <type_traits>
#include <vector>

#include "gemm_f64.hpp"
#include "gemm_f64_dl.hpp"
#include "plan.hpp"
#include "runtime.hpp"

namespace {

using namespace phiks;

// ------------------------------------------------------------- GEMM launching
enum class Tile { T128x128, T128x64, T64x128, T64x64, T32x32 };

#ifndef PHIKS_DL
#define PHIKS_DL 1  // 1: products with 64- and 128-wide tiles load operands straight into LDS
#endif

int64_t tiles_for(const GemmArgs& g, int bm, int bn) {
  return (int64_t)((g.M + bm - 1) / bm) * ((g.N + bn - 1) / bn) * g.nb0 * g.nb1;
}

// Largest tile that still gives at least PHIKS_TILE_MIN_WG work-groups per compute unit;
// small products (the exponentials of the small matrices, 64^3 tensors) get small tiles and
// more groups.  One work-group per CU is one wave per SIMD, which leaves the MFMA pipes
// waiting on its loads: with two required, a 64^3 call (4-tensor products on 32 x 32
// instead of 64 x 64 tiles) took 0.116 instead of 0.127 ms, and 96^3-256^3 calls were
// unchanged; four gave no further gain.  The tile never changes results (one k order).
#ifndef PHIKS_BIG_TILE
#define PHIKS_BIG_TILE 0  // 0: 128 x 64, 1: 128 x 128
#endif
#ifndef PHIKS_TILE_MIN_WG
#define PHIKS_TILE_MIN_WG 2
#endif
Tile pick_tile(const GemmArgs& g) {
  constexpr int64_t kCUs = 256 * PHIKS_TILE_MIN_WG;
  if (PHIKS_BIG_TILE == 1 && g.M >= 128 && g.N >= 128 && tiles_for(g, 128, 128) >= kCUs)
    return Tile::T128x128;
  if (g.M >= 128 && g.N >= 64 && tiles_for(g, 128, 64) >= kCUs) return Tile::T128x64;
  if (g.M >= 64 && g.N >= 128 && tiles_for(g, 64, 128) >= kCUs) return Tile::T64x128;
  if (g.M >= 64 && g.N >= 64 && tiles_for(g, 64, 64) >= kCUs) return Tile::T64x64;
  // products too small to fill the chip take the smallest tiles: more work-groups in
  // flight (a work-group alone on its CU is bound by one wave per SIMD)
  return Tile::T32x32;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

// 16-byte loads need even contraction length, even leading dimensions and batch
// strides, 16-byte aligned bases, and (for n-contiguous B) an even N.
bool vec_ok(const GemmArgs& g, bool kcontig, const std::vector<const void*>& extra_ptrs) {
  if (g.K % 2 || g.lda % 2 || g.ldb % 2) return false;
  if (!kcontig && g.N % 2) return false;
  if (g.sA0 % 2 || g.sA1 % 2 || g.sB0 % 2 || g.sB1 % 2) return false;
  if (g.pA == nullptr && (!aligned16(g.A) || !aligned16(g.B))) return false;
  for (const void* q : extra_ptrs)
    if (!aligned16(q)) return false;
  return true;
}

template <int BM, int BN, int WM, int WN, bool KC, bool VEC, bool CPLX = false, class Epi>
int launch_cfg(GemmArgs g, const Epi& epi, hipStream_t st) {
  g.tiles_m = (g.M + BM - 1) / BM;
  g.tiles_n = (g.N + BN - 1) / BN;
  g.total_tiles = (int64_t)g.tiles_m * g.tiles_n * g.nb0 * g.nb1;
  if (g.total_tiles <= 0) return PHIKS_OK;
  if (g.total_tiles > 0x7fffffffLL) {
    set_error("GEMM grid too large");
    return PHIKS_EINVAL;
  }
  const double flops = 2.0 * g.M * (double)g.N * g.K * g.nb0 * (double)g.nb1;
  // batches whose small matrix differs per entry (node matrices, pointer arrays) run one
  // entry's tiles back to back; the squaring epilogue keeps the entries of one tile
  // together, since they read the same pre-step tensors
  if (!std::is_same<Epi, EpiLinComb>::value && g.nb1 > 1 &&
      (g.pA != nullptr || (KC ? g.sB1 != 0 : g.sA1 != 0)))
    g.order = 1;
  if constexpr (PHIKS_DL == 1 && VEC && !CPLX) {
    // direct-to-LDS operand loads: whole chunks of K only (and, for the squaring
    // epilogue, pre-step tensors it can stream in 16-byte pairs)
    bool ok = g.K % PHIKS_DL_BK == 0;
    if constexpr (std::is_same<Epi, EpiLinComb>::value) ok = ok && lincomb_dl_ok(g, epi.Y, epi.N);
    if (ok)
      return timed_launch(&gemm_f64_dl_kernel<BM, BN, WM, WN, KC, Epi>, (unsigned)g.total_tiles, st,
                          flops, g, epi);
  }
  return timed_launch(&gemm_f64_kernel<BM, BN, WM, WN, KC, VEC, Epi, CPLX>, (unsigned)g.total_tiles,
                      st, flops, g, epi);
}

template <bool KC, bool VEC, bool CPLX = false, class Epi>
int launch_tile(const GemmArgs& g, const Epi& epi, hipStream_t st) {
  Tile tile = pick_tile(g);
  // the squaring epilogue stages slices of 16 rows x BN of the pre-step tensors: 128
  // columns would take 96 KB of LDS, so it keeps 64-column tiles
  if (std::is_same<Epi, EpiLinComb>::value && tile == Tile::T64x128) tile = Tile::T64x64;
  switch (tile) {
#if PHIKS_BIG_TILE == 1
    case Tile::T128x128: return launch_cfg<128, 128, 64, 64, KC, VEC, CPLX>(g, epi, st);
#endif
    case Tile::T128x64: return launch_cfg<128, 64, 64, 32, KC, VEC, CPLX>(g, epi, st);
    case Tile::T64x128: return launch_cfg<64, 128, 32, 64, KC, VEC, CPLX>(g, epi, st);
    case Tile::T64x64: return launch_cfg<64, 64, 32, 32, KC, VEC, CPLX>(g, epi, st);
    default: return launch_cfg<32, 32, 16, 16, KC, VEC, CPLX>(g, epi, st);
  }
}

template <bool KC, class Epi>
int launch_gemm(const GemmArgs& g, const Epi& epi, hipStream_t st,
                const std::vector<const void*>& extra_ptrs = {}) {
  if (g.pA != nullptr && g.nb0 != 1) {
    set_error("pointer-array GEMM needs nb0 == 1");
    return PHIKS_EINVAL;
  }
  if (vec_ok(g, KC, extra_ptrs)) return launch_tile<KC, true>(g, epi, st);
  return launch_tile<KC, false>(g, epi, st);
}

// Complex mu-mode product of a mode > 1 (see CPLX in gemm_f64.hpp): A = [Re L | Im L]
// (M x K, K = 2n), B the interleaved tensor slab (n rows of N doubles); 16-byte loads.
template <class Epi>
int launch_gemm_cplx(const GemmArgs& g, const Epi& epi, hipStream_t st) {
  if (!vec_ok(g, false, {}) || g.K % 2) {
    set_error("complex mu-mode product needs even sizes and 16-byte aligned operands");
    return PHIKS_EINVAL;
  }
  return launch_tile<false, true, true>(g, epi, st);
}

// ---------------------------------------------------------- Tucker operator
// GEMM views of the d mu-mode products of one Tucker operator (Section 2, eq. tucker;
// Lemma 1 for the vec order) applied to nbatch tensors in_b = in + b*in_stride with
// the matrices L[mu] + b*l_stride[mu]; the last mode writes batch b at out + b*N.
// ta/tb: nbatch*N scratch; mode mu (< d) writes ta for odd mu and tb for even mu,
// so out must be the buffer the last mode does not read.  Pointers are copied, not
// dereferenced: the mixed-precision chains reuse these views with FP32 buffers.
// Every execution path (single, mixed, grouped over many problems) builds its
// launches from these views, so their per-element arithmetic is the same.
void tucker_args(int d, const int64_t* n, int64_t N, const double* in, int64_t in_stride,
                 double* const* L, const int64_t* l_stride, int nbatch, double* out,
                 double* ta, double* tb, GemmArgs* gs) {
  const double* cur = in;
  int64_t cur_stride = in_stride;
  for (int mu = 1; mu <= d; ++mu) {
    const int64_t nm = n[mu - 1];
    int64_t nlo = 1, nhi = 1;
    for (int k = 0; k < mu - 1; ++k) nlo *= n[k];
    for (int k = mu; k < d; ++k) nhi *= n[k];
    double* dst = (mu == d) ? out : ((mu % 2 == 1) ? ta : tb);
    GemmArgs& g = gs[mu - 1];
    g = empty_args();
    g.nb1 = nbatch;
    if (mu == 1) {
      // W[m][i] = sum_j X[m][j] L[i][j], rows m < n_>
      g.M = (int)nhi;
      g.N = (int)nm;
      g.K = (int)nm;
      g.A = cur;
      g.lda = nm;
      g.B = L[0];
      g.ldb = nm;
      g.C = dst;
      g.ldc = nm;
      g.sA1 = cur_stride;
      g.sB1 = l_stride[0];
      g.sC1 = N;
    } else {
      // W_b[i][a] = sum_j L[i][j] X_b[j][a], batch b < n_>
      g.M = (int)nm;
      g.N = (int)nlo;
      g.K = (int)nm;
      g.A = L[mu - 1];
      g.lda = nm;
      g.B = cur;
      g.ldb = nlo;
      g.C = dst;
      g.ldc = nlo;
      g.nb0 = (int)nhi;
      g.sA0 = 0;
      g.sB0 = nm * nlo;
      g.sC0 = nm * nlo;
      g.sA1 = l_stride[mu - 1];
      g.sB1 = cur_stride;
      g.sC1 = N;
    }
    cur = dst;
    cur_stride = N;
  }
}

// Applies the Tucker operator of tucker_args, the last mode through `epi`.
template <class Epi>
int tucker(const phiks_plan_s& P, const double* in, int64_t in_stride,
           double* const* L, const int64_t* l_stride, int nbatch, double* out,
           double* ta, double* tb, const Epi& epi, hipStream_t st) {
  GemmArgs gs[PHIKS_MAX_D];
  tucker_args(P.d, P.n, P.N, in, in_stride, L, l_stride, nbatch, out, ta, tb, gs);
  for (int mu = 1; mu <= P.d; ++mu) {
    const bool last = (mu == P.d);
    if (mu == 1) {
      if (last) RET_IF((launch_gemm<true>(gs[0], epi, st)));
      else RET_IF((launch_gemm<true>(gs[0], EpiStore{1.0, 0.0}, st)));
    } else {
      if (last) RET_IF((launch_gemm<false>(gs[mu - 1], epi, st)));
      else RET_IF((launch_gemm<false>(gs[mu - 1], EpiStore{1.0, 0.0}, st)));
    }
  }
  return PHIKS_OK;
}

// Complex Tucker operator on re/im interleaved tensors of N complex values (in_b = in
// + b*in_stride doubles, out batch b at out + 2bN).  Lr[mu]: real forms (2n x 2n,
// batch stride lr_stride[mu]) for mode 1; Ls[mu]: [Re | Im] forms (n x 2n, batch
// stride ls_stride[mu]) for the modes > 1.  Mode 1 is a real GEMM of the interleaved
// rows with the real form; the modes > 1 are the CPLX GEMMs.  ta/tb as tucker_args.
void tucker_args_complex(int d, const int64_t* n, int64_t N, const double* in,
                         int64_t in_stride, double* const* Lr, const int64_t* lr_stride,
                         double* const* Ls, const int64_t* ls_stride, int nbatch, double* out,
                         double* ta, double* tb, GemmArgs* gs) {
  const double* cur = in;
  int64_t cur_stride = in_stride;
  for (int mu = 1; mu <= d; ++mu) {
    const int64_t nm = n[mu - 1];
    int64_t nlo = 1, nhi = 1;
    for (int k = 0; k < mu - 1; ++k) nlo *= n[k];
    for (int k = mu; k < d; ++k) nhi *= n[k];
    double* dst = (mu == d) ? out : ((mu % 2 == 1) ? ta : tb);
    GemmArgs& g = gs[mu - 1];
    g = empty_args();
    g.nb1 = nbatch;
    if (mu == 1) {
      // W[m][(i,c)] = sum_(j,c') X[m][(j,c')] R[(i,c)][(j,c')]
      g.M = (int)nhi;
      g.N = (int)(2 * nm);
      g.K = (int)(2 * nm);
      g.A = cur;
      g.lda = 2 * nm;
      g.B = Lr[0];
      g.ldb = 2 * nm;
      g.C = dst;
      g.ldc = 2 * nm;
      g.sA1 = cur_stride;
      g.sB1 = lr_stride[0];
      g.sC1 = 2 * N;
    } else {
      // W_b = [Re L | Im L] [X_b ; X_b twisted], rows of 2 n_< doubles
      g.M = (int)nm;
      g.N = (int)(2 * nlo);
      g.K = (int)(2 * nm);
      g.A = Ls[mu - 1];
      g.lda = 2 * nm;
      g.B = cur;
      g.ldb = 2 * nlo;
      g.C = dst;
      g.ldc = 2 * nlo;
      g.nb0 = (int)nhi;
      g.sA0 = 0;
      g.sB0 = 2 * nm * nlo;
      g.sC0 = 2 * nm * nlo;
      g.sA1 = ls_stride[mu - 1];
      g.sB1 = cur_stride;
      g.sC1 = 2 * N;
    }
    cur = dst;
    cur_stride = 2 * N;
  }
}

template <class Epi>
int tucker_complex(const phiks_plan_s& P, const double* in, int64_t in_stride,
                   double* const* Lr, const int64_t* lr_stride, double* const* Ls,
                   const int64_t* ls_stride, int nbatch, double* out, double* ta, double* tb,
                   const Epi& epi, hipStream_t st) {
  GemmArgs gs[PHIKS_MAX_D];
  tucker_args_complex(P.d, P.n, P.N, in, in_stride, Lr, lr_stride, Ls, ls_stride, nbatch, out,
                      ta, tb, gs);
  for (int mu = 1; mu <= P.d; ++mu) {
    const bool last = (mu == P.d);
    if (mu == 1) {
      if (last) RET_IF((launch_gemm<true>(gs[0], epi, st)));
      else RET_IF((launch_gemm<true>(gs[0], EpiStore{1.0, 0.0}, st)));
    } else {
      if (last) RET_IF((launch_gemm_cplx(gs[mu - 1], epi, st)));
      else RET_IF((launch_gemm_cplx(gs[mu - 1], EpiStore{1.0, 0.0}, st)));
    }
  }
  return PHIKS_OK;
}

}  // namespace
