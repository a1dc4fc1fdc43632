// FP64 MFMA GEMM for gfx950, specialised for mu-mode products (Section 2 of the
// paper: each mu-mode product is one matrix-matrix product).
//
// A tensor V of shape n_1 x ... x n_d stored with i_1 fastest is, for mode mu, a
// batch of n_> = n_{mu+1}...n_d slabs X_b of shape n_mu x n_<  (n_< = n_1...n_{mu-1},
// contiguous along n_<).  The mu-mode product W = V x_mu L is
//   mode 1:        W[m][i] = sum_j X[m][j] L[i][j]           (rows m < n_>)
//   mode mu > 1:   W_b[i][a] = sum_j L[i][j] X_b[j][a]         (a < n_<, batch b)
// i.e. C = A B with A always contiguous along the contraction index k and B either
// contiguous along n (mode > 1) or along k (mode 1, B = L^T).  No permutation of the
// tensor is ever made; the tiles are staged through LDS in the layout the MFMA
// fragments read.
//
// MFMA: v_mfma_f64_16x16x4_f64.  Per lane l (64-wide wave), for the four k of one step
// (k_0..k_3; which k a step takes is the k order below):
//   A operand  A[m0 + (l & 15)][k_(l >> 4)]
//   B operand  B[k_(l >> 4)][n0 + (l & 15)]
//   C result   c[r] = C[m0 + (l >> 4) + 4 r][n0 + (l & 15)],  r = 0..3
//
// LDS: tiles are stored k-major (row k holds the BM (or BN) entries of that k) with
// an XOR swizzle of the column index so that both the transposing stores (lanes
// spread over k) and the fragment reads (16 columns x 2 rows per half-wave) hit
// distinct banks: column c of row k is stored at c ^ swz(k).
//
// Launch: 1-D grid, tile order 0 (order 1: GemmArgs::order).  Mode 1 (k-contiguous B):
// the n tile (along L) varies fastest, then the batch index z1, the m tile and z0, so
// that every work-group reading one row block of the tensor (shared by the nodes of a
// batch too) runs back to back.
// Modes > 1: z1 varies fastest (the p tensors of a squaring step share the epilogue
// operands), then the m tile (along L), the n tile and z0.  Ids are remapped so that
// consecutive logical tiles land on one XCD (work-groups are dealt round-robin over
// the 8 XCDs, each with its own L2).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "devptr.hpp"

namespace phiks {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef double dbl2 __attribute__((ext_vector_type(2)));

struct GemmArgs {
  int M, N, K;
  const double* A;
  int64_t lda;   // A(m, k) = A[m * lda + k]
  const double* B;
  int64_t ldb;   // B(k, n) = B[k * ldb + n] (n-contiguous) or B[n * ldb + k] (k-contiguous)
  double* C;
  int64_t ldc;   // C(m, n) = C[m * ldc + n]
  int nb0, nb1;  // batch z = (z0, z1)
  int64_t sA0, sA1, sB0, sB1, sC0, sC1;
  int tiles_m, tiles_n;
  int64_t total_tiles;
  // tile order: 0 as described above; 1 batch index z1 slowest (tiles of one z1 back to
  // back), for batches whose small-matrix operand differs per z1: with z1 fastest every
  // matrix of the batch is live in L2 at once and, past its capacity, refetched per tile
  int order;
  // pointer-array batch (used when pA != nullptr): operands of batch z1 are
  // pA[z1], pB[z1], pC[z1] (nb0 must be 1); the strides above are then ignored
  const double* const* pA;
  const double* const* pB;
  double* const* pC;
};

// C = alpha * acc (+ beta * C).  beta == 0 never reads C.
struct EpiStore {
  double alpha, beta;
  template <class P>
  __device__ __forceinline__ void operator()(P C, int64_t e, int64_t, double acc) const {
    C[e] = (beta == 0.0) ? alpha * acc : alpha * acc + beta * C[e];
  }
};

// Output tensor l = z1 (the batch index; tensors N apart from the C base pointer):
// out_l = a[l] * acc + sum_{k <= l} c[l][k] * Y_k   (Y_k = Y + k * N, same offset).
// This is the squaring step of eq. simul / eq. comb fused into the last mu-mode product.
struct EpiLinComb {
  const double* Y;
  int64_t N;
  int p;
  double a[8];
  double c[8][8];
  template <class P>
  __device__ __forceinline__ void operator()(P C, int64_t e, int64_t l, double acc) const {
    const int64_t off = e - l * N;
    const PHIKS_GLOBAL double* Yg = gptr(Y);
    double r = a[l] * acc;
    for (int k = 0; k <= (int)l; ++k) r += c[l][k] * Yg[k * N + off];
    C[e] = r;
  }
};

__device__ __forceinline__ int64_t xcd_remap(int64_t g, int64_t G) {
  const int64_t xcd = g & 7;
  const int64_t slot = g >> 3;
  const int64_t per = G >> 3;
  const int64_t rem = G & 7;
  return (xcd < rem) ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
}

// MFMA k order (shared by every FP64 kernel, so that a product gives the same bits
// whichever kernel or tile computes it): K is taken in groups of 8; within group j the
// first MFMA step takes k = 8j + 2 lk, the second k = 8j + 2 lk + 1 (lane group
// lk = l >> 4).  A 32-lane half of a fragment read then touches rows k and k + 2.
//
// swizzle of a transposed (k-major) tile, p = (k/2) mod 8: bit 4 from p's parity (rows
// k and k + 2 land on different bank halves), bits 2..3 from p/2, so the 8 even (odd)
// rows of a 16-k chunk written by one store instruction get distinct offsets
__device__ __forceinline__ int swz_t(int k) {
  const int p = (k >> 1) & 7;
  return ((p & 1) << 4) | ((p >> 1) << 2);
}
// swizzle of an n-contiguous tile: flips the 16-column half when bit 1 of k is set
__device__ __forceinline__ int swz_n(int k) { return ((k >> 1) & 1) << 4; }

// VEC: operands are loaded 2 doubles (16 bytes) at a time; requires even K, lda, ldb,
// batch strides and 16-byte aligned base pointers (checked by the launcher).
#ifndef PHIKS_GEMM_MIN_WAVES
#define PHIKS_GEMM_MIN_WAVES 3  // minimum waves per SIMD the register budget must allow
#endif

// Tile coordinates and operand bases of logical tile `rest` (tile order above).
struct TileOperands {
  const PHIKS_GLOBAL double* A;
  const PHIKS_GLOBAL double* B;
  PHIKS_GLOBAL double* Cb;
  int64_t cbase;   // offset of the output tensor within Cb
  int64_t z1;
  int tm, tn;
};

// Tile and batch coordinates of logical tile `rest` (tile order above).
struct TileCoords {
  int tm, tn;
  int64_t z0, z1;
};

template <bool B_KCONTIG>
__device__ __forceinline__ TileCoords tile_coords(const GemmArgs& g, int64_t rest) {
  TileCoords c;
  if (g.order == 1) {
    // the tiles sharing an operand block run back to back: mode 1 the n tiles of one
    // row block (one block of the tensor), modes > 1 the m tiles of one column block
    if constexpr (B_KCONTIG) {
      c.tn = (int)(rest % g.tiles_n);
      rest /= g.tiles_n;
      c.tm = (int)(rest % g.tiles_m);
      rest /= g.tiles_m;
    } else {
      c.tm = (int)(rest % g.tiles_m);
      rest /= g.tiles_m;
      c.tn = (int)(rest % g.tiles_n);
      rest /= g.tiles_n;
    }
    c.z0 = rest % g.nb0;
    c.z1 = rest / g.nb0;
  } else if constexpr (B_KCONTIG) {
    c.tn = (int)(rest % g.tiles_n);
    rest /= g.tiles_n;
    c.z1 = rest % g.nb1;
    rest /= g.nb1;
    c.tm = (int)(rest % g.tiles_m);
    c.z0 = rest / g.tiles_m;
  } else {
    c.z1 = rest % g.nb1;
    rest /= g.nb1;
    c.tm = (int)(rest % g.tiles_m);
    rest /= g.tiles_m;
    c.tn = (int)(rest % g.tiles_n);
    c.z0 = rest / g.tiles_n;
  }
  return c;
}

template <bool B_KCONTIG>
__device__ __forceinline__ TileOperands tile_operands(const GemmArgs& g, int64_t rest) {
  const TileCoords c = tile_coords<B_KCONTIG>(g, rest);
  TileOperands t;
  t.tm = c.tm;
  t.tn = c.tn;
  t.z1 = c.z1;
  if (g.pA != nullptr) {
    t.A = gptr(g.pA[c.z1]);
    t.B = gptr(g.pB[c.z1]);
    t.Cb = gptr(g.pC[c.z1]);
    t.cbase = 0;
  } else {
    t.A = gptr(g.A) + c.z0 * g.sA0 + c.z1 * g.sA1;
    t.B = gptr(g.B) + c.z0 * g.sB0 + c.z1 * g.sB1;
    t.Cb = gptr(g.C);
    t.cbase = c.z0 * g.sC0 + c.z1 * g.sC1;
  }
  return t;
}

// Writes a wave's FM x FN register tile (16 x 16 fragments, result row (l >> 4) + 4r) at
// rows mw.., columns nw.. of output tensor z1 through the epilogue.  Element (i, j, r)
// of a lane sits at the lane's base offset plus (16 i + 4 r) ldc + 16 j, a wave-uniform
// delta, so no per-element 64-bit addresses are held.
template <int FM, int FN, class Epi, class P>
__device__ __forceinline__ void store_tile_f64(dbl4 (&acc)[FM][FN], const GemmArgs& g, const Epi& epi,
                                               P Cb, int64_t cbase, int64_t z1, int mw, int nw,
                                               int lr, int lk, const double* Yb = nullptr,
                                               int64_t YN = 0) {
  const int ml = mw + lk, nl = nw + lr;                 // the lane's first row and column
  const int64_t base = cbase + (int64_t)ml * g.ldc + nl;
  auto delta = [&](int i, int j, int r) { return (int64_t)(i * 16 + 4 * r) * g.ldc + j * 16; };
  auto inside = [&](int i, int j, int r) { return (ml + i * 16 + 4 * r < g.M) & (nl + j * 16 < g.N); };
  if constexpr (std::is_same<Epi, EpiLinComb>::value) {
    // Squaring recurrence on the whole register tile: out = a_l acc + sum_k c_lk Y_k.
    // For each k and each pair of fragment rows, all loads are issued before their fused
    // multiply-adds (two rows at a time bounds the registers the loads hold).
    const int l = (int)z1;
    const double al = epi.a[l];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[i][j] *= al;
    constexpr int FI = FM < 2 ? FM : 2;
    static_assert(FM % FI == 0, "row pairs");
    for (int k = 0; k <= l; ++k) {
      const double ck = epi.c[l][k];
      const PHIKS_GLOBAL double* __restrict__ Yk = gptr(Yb ? Yb : epi.Y) + (int64_t)(k - l) * (Yb ? YN : epi.N) + base;
#pragma unroll
      for (int i0 = 0; i0 < FM; i0 += FI) {
        double y[FI][FN][4];
#pragma unroll
        for (int i = 0; i < FI; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              y[i][j][r] = inside(i0 + i, j, r) ? Yk[delta(i0 + i, j, r)] : 0.0;
#pragma unroll
        for (int i = 0; i < FI; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[i0 + i][j][r] = __builtin_fma(ck, y[i][j][r], acc[i0 + i][j][r]);
      }
    }
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (inside(i, j, r)) Cb[base + delta(i, j, r)] = acc[i][j][r];
  } else {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (inside(i, j, r)) epi(Cb, base + delta(i, j, r), z1, acc[i][j][r]);
  }
}

// One output tile of one GEMM: `rest` is the logical tile index in the tile order
// described above (0 .. g.total_tiles - 1).
//
// CPLX (n-contiguous B with 16-byte loads only): the complex mu-mode product of modes
// > 1 on re/im interleaved tensors.  With K = 2n, rows k < n of B are the tensor slab
// itself and rows k >= n are the same slab with every (re, im) pair replaced by
// (-im, re), so that C = [Re L | Im L] B is the interleaved complex product L X.
template <int BM, int BN, int WM, int WN, bool B_KCONTIG, bool VEC, class Epi, bool CPLX = false>
__device__ __forceinline__ void gemm_f64_tile(const GemmArgs& g, const Epi& epi, int64_t rest,
                                              const double* Yb = nullptr, int64_t YN = 0) {
  static_assert(!CPLX || (!B_KCONTIG && VEC), "the complex form needs an n-contiguous B, 16-byte loads");
  constexpr int BK = 16;
  constexpr int WGM = BM / WM;
  constexpr int WGN = BN / WN;
  static_assert(WGM * WGN == 4, "4 waves per work-group");
  static_assert(BM % 32 == 0 && BN % 32 == 0, "tiles are multiples of 32");
  constexpr int FM = WM / 16;
  constexpr int FN = WN / 16;
  constexpr int VW = VEC ? 2 : 1;                 // doubles per load
  constexpr int LA = BM * BK / (256 * VW);        // A loads per thread per chunk
  constexpr int LB = BN * BK / (256 * VW);

  __shared__ __align__(16) double As[2][BK][BM];
  __shared__ __align__(16) double Bs[2][BK][BN];

  const TileOperands t = tile_operands<B_KCONTIG>(g, rest);
  const PHIKS_GLOBAL double* __restrict__ A = t.A;
  const PHIKS_GLOBAL double* __restrict__ B = t.B;
  PHIKS_GLOBAL double* Cb = t.Cb;
  const int64_t cbase = t.cbase, z1 = t.z1;
  const int m0 = t.tm * BM;
  const int n0 = t.tn * BN;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave / WGN) * WM;
  const int wn = (wave % WGN) * WN;

  // Loads: A and k-contiguous B read VW consecutive k of one row per load; an
  // n-contiguous B reads VW consecutive n of one k.  Out-of-range elements read a
  // clamped in-range address; the zero fill is applied when the registers are
  // written to LDS, so that the loads of the next K chunk stay in flight while the
  // MFMAs of the current chunk run (no branches).
  typedef typename std::conditional<VEC, dbl2, double>::type vec_t;
  vec_t ra[LA], rb[LB];
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
      ra[i] = *reinterpret_cast<const PHIKS_GLOBAL vec_t*>(A + off);
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int e = tid + i * 256;
      int n, k;
      if constexpr (B_KCONTIG) { n = e / (BK / VW); k = VW * (e % (BK / VW)); }
      else { k = e / (BN / VW); n = VW * (e % (BN / VW)); }
      int gn = n0 + n, gk = k0 + k;
      const bool ok = b_ok(e, k0);
      if constexpr (!VEC) bmask |= (uint32_t)ok << i;
      if constexpr (CPLX) gk -= (gk >= (g.K >> 1)) ? (g.K >> 1) : 0;
      const int64_t off =
          ok ? (B_KCONTIG ? (int64_t)gn * g.ldb + gk : (int64_t)gk * g.ldb + gn) : 0;
      rb[i] = *reinterpret_cast<const PHIKS_GLOBAL vec_t*>(B + off);
    }
  };
  auto store_chunk = [&](int buf, int k0) {
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      const int e = tid + i * 256;
      const int m = e / (BK / VW), k = VW * (e % (BK / VW));
      const vec_t x = a_in(i, e, k0) ? ra[i] : vec_t(0.0);
      if constexpr (VEC) {
        As[buf][k][m ^ swz_t(k)] = x[0];
        As[buf][k + 1][m ^ swz_t(k + 1)] = x[1];
      } else {
        As[buf][k][m ^ swz_t(k)] = x;
      }
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int e = tid + i * 256;
      vec_t x = b_in(i, e, k0) ? rb[i] : vec_t(0.0);
      if constexpr (CPLX) {
        if (k0 + e / (BN / VW) >= (g.K >> 1)) x = vec_t{-x[1], x[0]};
      }
      if constexpr (B_KCONTIG) {
        const int n = e / (BK / VW), k = VW * (e % (BK / VW));
        if constexpr (VEC) {
          Bs[buf][k][n ^ swz_t(k)] = x[0];
          Bs[buf][k + 1][n ^ swz_t(k + 1)] = x[1];
        } else {
          Bs[buf][k][n ^ swz_t(k)] = x;
        }
      } else {
        const int k = e / (BN / VW), n = VW * (e % (BN / VW));
        if constexpr (VEC) *reinterpret_cast<dbl2*>(&Bs[buf][k][n ^ swz_n(k)]) = x;
        else Bs[buf][k][n ^ swz_n(k)] = x;
      }
    }
  };

  dbl4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};

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
      const int k = (kk & ~7) + 2 * lk + ((kk >> 2) & 1);   // the k order above
      double fa[FM], fb[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) fa[i] = As[buf][k][(wm + i * 16 + lr) ^ swz_t(k)];
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        if constexpr (B_KCONTIG) fb[j] = Bs[buf][k][(wn + j * 16 + lr) ^ swz_t(k)];
        else fb[j] = Bs[buf][k][(wn + j * 16 + lr) ^ swz_n(k)];
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i], fb[j], acc[i][j], 0, 0, 0);
    }
    if (c + 1 < nchunks) store_chunk(buf ^ 1, (c + 1) * BK);
    __syncthreads();
  }

  store_tile_f64<FM, FN>(acc, g, epi, Cb, cbase, z1, m0 + wm, n0 + wn, lr, lk, Yb, YN);
}

template <int BM, int BN, int WM, int WN, bool B_KCONTIG, bool VEC, class Epi, bool CPLX = false>
__global__ void __launch_bounds__(256, VEC ? PHIKS_GEMM_MIN_WAVES : 2) gemm_f64_kernel(GemmArgs g, Epi epi) {
  gemm_f64_tile<BM, BN, WM, WN, B_KCONTIG, VEC, Epi, CPLX>(g, epi, xcd_remap(blockIdx.x, g.total_tiles));
}

// Grouped launch: many independent GEMMs of one kind (same tile shape, operand layout
// and epilogue type) in one grid.  Item i owns the logical tiles first[i] ..
// first[i] + items[i].g.total_tiles - 1; a work-group finds its item by binary search
// over `first` (a few KB, served by the scalar cache).  The epilogue is shared by the
// launch except for the per-item output-side operands carried by GroupItem::Y / YN
// (used by EpiLinComb: the pre-step tensors of the item's problem).
struct GroupItem {
  GemmArgs g;
  const double* Y;
  int64_t YN;
};

// The item owning logical tile t: the last i with first[i] <= t (first[0] = 0).
__device__ __forceinline__ int find_group_item(const int64_t* __restrict__ first, int nitems, int64_t t) {
  int lo = 0, hi = nitems - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <int BM, int BN, int WM, int WN, bool B_KCONTIG, bool VEC, class Epi>
__global__ void __launch_bounds__(256, VEC ? PHIKS_GEMM_MIN_WAVES : 2)
    gemm_f64_grouped(const GroupItem* __restrict__ items, const int64_t* __restrict__ first,
                     int nitems, int64_t total, Epi epi) {
  const int64_t t = xcd_remap(blockIdx.x, total);
  const int lo = find_group_item(first, nitems, t);
  const GroupItem& it = items[lo];
  // the item's pre-step tensors go beside epi, not into a modified copy of it (a local
  // copy indexed by the tensor index lives in scratch memory)
  if constexpr (std::is_same<Epi, EpiLinComb>::value) {
    gemm_f64_tile<BM, BN, WM, WN, B_KCONTIG, VEC>(it.g, epi, t - first[lo], it.Y, it.YN);
  } else {
    gemm_f64_tile<BM, BN, WM, WN, B_KCONTIG, VEC>(it.g, epi, t - first[lo]);
  }
}

}  // namespace phiks
