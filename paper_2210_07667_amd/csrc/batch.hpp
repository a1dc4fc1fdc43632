// Many independent same-vector problems in one call: phiks_batch_plan / _apply.
//
// Every problem keeps its own plan (s, q, GLL rule, small exponentials) and its own
// recurrence (eqs. integrandsimul and simul, outputs as eq. scaldiffphi), exactly as
// phiks_plan / phiks_apply would run it alone.  What changes is the execution: the
// problems advance in lockstep, one step per mu-mode product, and each step runs the
// GEMMs of every problem that has one at that point as a few grouped launches (one
// per operand layout, tile class, load width, kernel and epilogue).  The GEMM views
// come from tucker_args, the node sums from the same CombineArgs as the single path,
// and every FP64 kernel takes K in the same order whatever its tile (gemm_f64.hpp), so
// every result is bitwise the one phiks_apply returns for that problem alone.
//
// Included once, at the end of phiks.hip.
#pragma once

#include <algorithm>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <thread>
#include <vector>

namespace {

// Launch tables of grouped executions: built per call in pinned host memory and
// uploaded once; grown when a call needs more.  A call waits on the host until the
// previous call's upload has read the staging buffer.
struct GroupTables {
  char* host = nullptr;
  void* dev = nullptr;
  size_t bytes = 0;
  hipEvent_t upload_done = nullptr;
  bool uploaded = false;
};

}  // namespace

struct phiks_batch_s {
  int count = 0;
  int p = 0, ns = 1, precision = PHIKS_FP64;
  int device = 0;
  hipStream_t stream = nullptr;           // stream the batch was built on
  std::vector<phiks_plan_s> plans;        // per problem; matrices inside dmem
  void* dmem = nullptr;
  std::vector<size_t> ws_off;             // per-problem workspace offsets, doubles
  size_t ws_doubles = 0;
  GroupTables tab;
  // The launches of the last pointer set (v, out, ws), captured into a graph the second
  // time that set is applied and replayed while it stays the same (phiks_batch_apply).
  std::vector<const void*> graph_key;
  hipGraphExec_t graph = nullptr;
  hipStream_t capture_stream = nullptr;   // capture only: nothing executes on it
  std::vector<hipStream_t> fork_streams;  // capture only: a step's partitions fork onto these
  hipStream_t graph_stream = nullptr;     // stream of the graph's last launch
};

namespace {

// Rules that pick the tile class of an FP64 grouped product (BatchSchedule::tile_class).
// The values in use come from batch_tuning.inc, written by tune_batch.py, which times the
// batched workload under every combination and keeps the fastest; phiks_batch_tuning
// reads or replaces them at run time (the tuner's own knob).
struct BatchTuning {
  int sq_min;    // 64 x 64 tiles when both sides reach this (else 32 x 32 or a skinny class)
  int skinny;    // 1: 32 x 128 / 128 x 32 tiles for one side <= 32 against the other >= 96
  int wide_m1;   // 1: 128 x 64 tiles for plain-store products of mode 1 with M >= 128
  int wide_mk;   // 1: 128 x 64 tiles for plain-store products of modes > 1 with M >= 128
  int wide_lc;   // 1: 128 x 64 tiles for the squaring epilogue's products with M >= 128
};
#include "batch_tuning.inc"
std::mutex g_tuning_mu;
BatchTuning g_batch_tuning = kBatchTuningTuned;
int64_t g_tuning_gen = 0;   // bumped on every change (captured graphs depend on the rules)

BatchTuning batch_tuning(int64_t* gen = nullptr) {
  std::lock_guard<std::mutex> lk(g_tuning_mu);
  if (gen) *gen = g_tuning_gen;
  return g_batch_tuning;
}

enum class StepKind { Gemm, Combine };

// One GEMM of a step: its views, its layout (mode 1: B k-contiguous), and whether it
// is the last mode of a squaring Tucker (squaring epilogue with Y = the problem's
// pre-step tensors).
struct StepGemm {
  GemmArgs g;
  bool kc;
  bool lincomb;
  const double* Y;
  int64_t YN;
  int p = 0;   // squaring epilogue: the problem's highest phi index (its coefficients)
  // arithmetic: PHIKS_FP64, or PHIKS_FP32 with f32_kind 0 (mode 1: FP64 input, FP32 out),
  // 1 (FP32 -> FP32), 2 (FP32 -> FP64 store), 3 (FP32 -> FP64 squaring epilogue)
  int prec = PHIKS_FP64;
  int f32_kind = 0;
};

#ifndef PHIKS_BATCH_FORK
#define PHIKS_BATCH_FORK 4  // streams a captured step's partitions fork onto (0: one chain)
#endif

struct GroupedLaunch {
  StepKind kind;
  bool kc = false, vec = false, lincomb = false;
  bool dl = false;       // direct-to-LDS kernel (16-byte operands, K a multiple of its chunk)
  int tile = 0;          // class (BM x BN): 0 64x64, 1 32x32, 2 32x128, 3 128x32, 4 128x64
  size_t items_off = 0;  // bytes into the table: GroupItem[n] or CombineArgs[n]
  size_t first_off = 0;  // bytes into the table: int64_t first[n] (GEMM)
  int n = 0;
  int64_t total = 0;     // GEMM: tiles; Combine: largest N
  double flops = 0.0;    // GEMM: algorithmic 2 M N K over all items and batches
  int step = 0;          // launches of one step touch disjoint problems
  int lin_p = 0;         // squaring epilogue: coefficients of BatchSchedule::lin[lin_p]
  // FP32 products: the single path's configuration (tile bm x bn, kernel), the kind of
  // product (StepGemm::f32_kind); single: one item, launched as the single path launches it
  int prec = PHIKS_FP64;
  int bm = 0, bn = 0, f32_kind = 0;
  bool single = false;
};

// Host builder of one call's launches and their tables.
struct BatchSchedule {
  std::vector<GroupedLaunch> launches;
  std::vector<char> buf;
  EpiLinComb lin[PHIKS_MAX_P + 1];   // squaring-epilogue coefficients by p (eq. simul)
  int steps = 0;

  // The coefficients of phiks_apply's squaring step for problems of highest index p:
  // out_l = 2^-l (acc + sum_{k<=l} Y_k / (l-k)!).
  void set_lin(int p) {
    EpiLinComb& e = lin[p];
    std::memset(&e, 0, sizeof(e));
    e.p = p;
    for (int ell = 1; ell <= p; ++ell) {
      const double sc = std::ldexp(1.0, -ell);
      e.a[ell - 1] = sc;
      for (int k = 1; k <= ell; ++k) e.c[ell - 1][k - 1] = sc / factorial(ell - k);
    }
  }

  size_t put(const void* src, size_t bytes) {
    const size_t off = (buf.size() + 15) & ~(size_t)15;
    buf.resize(off + bytes);
    if (src) std::memcpy(buf.data() + off, src, bytes);
    return off;
  }

  // Tile classes (BM x BN): 64 x 64 when both sides reach 48.  The direct-to-LDS kernel
  // also takes 128 x 64 tiles for the plain-store products of mode 1 (M >= 128), which
  // halve the operand reads per flop, and streams skinny products (one side at
  // most 32, the other long: the small modes of mixed-size problems, bound by HBM) through
  // 32 x 128 or 128 x 32 tiles.  Everything else takes 32 x 32.
  static constexpr int kClasses = 5;
  static constexpr int kBM[kClasses] = {64, 32, 32, 128, 128};
  static constexpr int kBN[kClasses] = {64, 32, 128, 32, 64};
  static bool dl_ok(const GemmArgs& g, bool kc) {
    return PHIKS_DL == 1 && g.K % PHIKS_DL_BK == 0 && vec_ok(g, kc, {});
  }
  BatchTuning tune = batch_tuning();
  int tile_class(const GemmArgs& g, bool kc, bool dl, bool lincomb) const {
    const bool wide = g.M >= 128 && g.N >= 64;
    if (dl && wide && !lincomb && (kc ? tune.wide_m1 : tune.wide_mk)) return 4;
    if (dl && wide && lincomb && tune.wide_lc) return 4;
    if (g.M >= tune.sq_min && g.N >= tune.sq_min) return 0;
    if (tune.skinny && dl && g.M <= 32 && g.N >= 96) return 2;
    if (tune.skinny && dl && g.N <= 32 && g.M >= 96) return 3;
    return 1;
  }

  // FP32 products of one step: partitioned by the configuration the single path gives
  // each item (cfg32), so every item runs the tiles and kernel of its single call.
  void add_gemm32(const std::vector<StepGemm>& items, int step) {
    struct Key {
      int kc, bm, bn, dl, kind, lp;
      bool operator<(const Key& o) const {
        return std::tie(kc, bm, bn, dl, kind, lp) < std::tie(o.kc, o.bm, o.bn, o.dl, o.kind, o.lp);
      }
    };
    std::map<Key, std::vector<const StepGemm*>> parts;
    for (const StepGemm& it : items) {
      const bool lc = it.f32_kind == 3;
      const bool dl_epi = !lc || (PHIKS_MIXED_LC_DL == 1 && lincomb_dl_ok(it.g, it.Y, it.YN));
      const Cfg32 c = cfg32(it.g, it.kc, it.f32_kind == 0, dl_epi);
      // grouped kernels exist for 16-byte loads, tiles up to 128 x 64 and mode 1 feeding
      // FP32 intermediates; anything else is launched alone, as its single call does
      const bool grouped = c.vec && !(c.bm == 128 && c.bn == 128) && (it.kc == (it.f32_kind == 0));
      if (!grouped) {
        GroupedLaunch L;
        L.kind = StepKind::Gemm;
        L.prec = PHIKS_FP32;
        L.single = true;
        L.kc = it.kc;
        L.f32_kind = it.f32_kind;
        L.lin_p = lc ? it.p : 0;
        L.lincomb = lc;
        GroupItem gi;
        gi.g = it.g;
        gi.Y = it.Y;
        gi.YN = it.YN;
        L.n = 1;
        L.total = 1;
        L.flops = 2.0 * it.g.M * (double)it.g.N * it.g.K * it.g.nb0 * (double)it.g.nb1;
        L.items_off = put(&gi, sizeof(gi));
        L.step = step;
        launches.push_back(L);
        continue;
      }
      parts[{it.kc ? 1 : 0, c.bm, c.bn, c.dl ? 1 : 0, it.f32_kind, lc ? it.p : 0}].push_back(&it);
    }
    for (auto& kv : parts) {
      const Key& k = kv.first;
      std::vector<GroupItem> part;
      std::vector<int64_t> first;
      int64_t total = 0;
      double flops = 0.0;
      for (const StepGemm* it : kv.second) {
        GroupItem gi;
        gi.g = it->g;
        gi.g.tiles_m = (gi.g.M + k.bm - 1) / k.bm;
        gi.g.tiles_n = (gi.g.N + k.bn - 1) / k.bn;
        gi.g.total_tiles = (int64_t)gi.g.tiles_m * gi.g.tiles_n * gi.g.nb0 * gi.g.nb1;
        if (gi.g.total_tiles <= 0) continue;
        gi.Y = it->Y;
        gi.YN = it->YN;
        flops += 2.0 * gi.g.M * (double)gi.g.N * gi.g.K * gi.g.nb0 * (double)gi.g.nb1;
        first.push_back(total);
        total += gi.g.total_tiles;
        part.push_back(gi);
      }
      if (part.empty()) continue;
      GroupedLaunch L;
      L.kind = StepKind::Gemm;
      L.prec = PHIKS_FP32;
      L.kc = k.kc == 1;
      L.bm = k.bm;
      L.bn = k.bn;
      L.dl = k.dl == 1;
      L.vec = true;
      L.f32_kind = k.kind;
      L.lincomb = k.kind == 3;
      L.lin_p = k.lp;
      L.n = (int)part.size();
      L.total = total;
      L.flops = flops;
      L.items_off = put(part.data(), part.size() * sizeof(GroupItem));
      L.first_off = put(first.data(), first.size() * sizeof(int64_t));
      L.step = step;
      launches.push_back(L);
    }
  }

  void add_gemm_step(const std::vector<StepGemm>& all) {
    const int step = steps++;
    std::vector<StepGemm> items, items32;
    for (const StepGemm& it : all) (it.prec == PHIKS_FP32 ? items32 : items).push_back(it);
    if (!items32.empty()) add_gemm32(items32, step);
    // the p values of the squaring-epilogue items (one launch per p: their coefficients)
    std::vector<int> lps;
    for (const StepGemm& it : items)
      if (it.lincomb && std::find(lps.begin(), lps.end(), it.p) == lps.end()) lps.push_back(it.p);
    if (lps.empty()) lps.push_back(0);
    // partition by (layout, tile class, 16-byte loads, direct-to-LDS, epilogue, its p)
    for (int kc = 0; kc < 2; ++kc)
      for (int tile = 0; tile < kClasses; ++tile)
        for (int vec = 0; vec < 2; ++vec)
          for (int dl = 0; dl < 2; ++dl)
            for (int lc = 0; lc < 2; ++lc)
            for (size_t pi = 0; pi < (lc == 1 ? lps.size() : 1); ++pi) {
              const int lp = (lc == 1) ? lps[pi] : 0;
              std::vector<GroupItem> part;
              std::vector<int64_t> first;
              int64_t total = 0;
              double flops = 0.0;
              for (const StepGemm& it : items) {
                if (it.kc != (kc == 1) || it.lincomb != (lc == 1)) continue;
                if (it.lincomb && it.p != lp) continue;
                if (vec_ok(it.g, it.kc, {}) != (vec == 1)) continue;
                const bool idl = dl_ok(it.g, it.kc) && (!it.lincomb || lincomb_dl_ok(it.g, it.Y, it.YN));
                if (idl != (dl == 1) || tile_class(it.g, it.kc, idl, it.lincomb) != tile) continue;
                GroupItem gi;
                gi.g = it.g;
                const int bm = kBM[tile], bn = kBN[tile];
                gi.g.tiles_m = (gi.g.M + bm - 1) / bm;
                gi.g.tiles_n = (gi.g.N + bn - 1) / bn;
                gi.g.total_tiles = (int64_t)gi.g.tiles_m * gi.g.tiles_n * gi.g.nb0 * gi.g.nb1;
                if (gi.g.total_tiles <= 0) continue;
                gi.Y = it.Y;
                gi.YN = it.YN;
                flops += 2.0 * gi.g.M * (double)gi.g.N * gi.g.K * gi.g.nb0 * (double)gi.g.nb1;
                first.push_back(total);
                total += gi.g.total_tiles;
                part.push_back(gi);
              }
              if (part.empty()) continue;
              GroupedLaunch L;
              L.kind = StepKind::Gemm;
              L.kc = kc == 1;
              L.tile = tile;
              L.vec = vec == 1;
              L.dl = dl == 1;
              L.lincomb = lc == 1;
              L.n = (int)part.size();
              L.total = total;
              L.flops = flops;
              L.items_off = put(part.data(), part.size() * sizeof(GroupItem));
              L.first_off = put(first.data(), first.size() * sizeof(int64_t));
              L.step = step;
              L.lin_p = lp;
              launches.push_back(L);
            }
  }

  void add_combine_step(const std::vector<CombineArgs>& items) {
    if (items.empty()) return;
    GroupedLaunch L;
    L.kind = StepKind::Combine;
    L.n = (int)items.size();
    for (const CombineArgs& a : items) L.total = std::max(L.total, a.N);
    L.items_off = put(items.data(), items.size() * sizeof(CombineArgs));
    L.step = steps++;
    launches.push_back(L);
  }
};

template <int BM, int BN, int WM, int WN, bool KC, bool VEC, class Epi>
int launch_grouped_cfg(const GroupedLaunch& L, const char* dev, const Epi& epi, hipStream_t st) {
  if (L.total > 0x7fffffffLL) {
    set_error("grouped GEMM grid too large");
    return PHIKS_EINVAL;
  }
  return timed_launch(&gemm_f64_grouped<BM, BN, WM, WN, KC, VEC, Epi>, (unsigned)L.total, st, L.flops,
                      (const GroupItem*)(dev + L.items_off), (const int64_t*)(dev + L.first_off),
                      L.n, L.total, epi);
}

template <int BM, int BN, int WM, int WN, bool KC, class Epi>
int launch_grouped_dl(const GroupedLaunch& L, const char* dev, const Epi& epi, hipStream_t st) {
  if (L.total > 0x7fffffffLL) {
    set_error("grouped GEMM grid too large");
    return PHIKS_EINVAL;
  }
  return timed_launch(&gemm_f64_dl_grouped<BM, BN, WM, WN, KC, Epi>, (unsigned)L.total, st, L.flops,
                      (const GroupItem*)(dev + L.items_off), (const int64_t*)(dev + L.first_off),
                      L.n, L.total, epi);
}

template <bool KC, bool VEC, class Epi>
int launch_grouped_tile(const GroupedLaunch& L, const char* dev, const Epi& epi, hipStream_t st) {
  if constexpr (VEC && PHIKS_DL == 1) {
    if (L.dl) {
      switch (L.tile) {
        case 0: return launch_grouped_dl<64, 64, 32, 32, KC>(L, dev, epi, st);
        case 2: return launch_grouped_dl<32, 128, 32, 32, KC>(L, dev, epi, st);
        case 3: return launch_grouped_dl<128, 32, 32, 32, KC>(L, dev, epi, st);
        case 4: return launch_grouped_dl<128, 64, 64, 32, KC>(L, dev, epi, st);
        default: return launch_grouped_dl<32, 32, 16, 16, KC>(L, dev, epi, st);
      }
    }
  }
  if (L.tile == 0) return launch_grouped_cfg<64, 64, 32, 32, KC, VEC>(L, dev, epi, st);
  if (L.tile != 1) {
    set_error("grouped GEMM tile class needs the direct-to-LDS kernel");
    return PHIKS_EINVAL;
  }
  return launch_grouped_cfg<32, 32, 16, 16, KC, VEC>(L, dev, epi, st);
}

template <class Epi>
int launch_grouped(const GroupedLaunch& L, const char* dev, const Epi& epi, hipStream_t st) {
  if (L.kc) {
    return L.vec ? launch_grouped_tile<true, true>(L, dev, epi, st)
                 : launch_grouped_tile<true, false>(L, dev, epi, st);
  }
  return L.vec ? launch_grouped_tile<false, true>(L, dev, epi, st)
               : launch_grouped_tile<false, false>(L, dev, epi, st);
}

// One grouped execution: problem i runs plan *plans[i] (all with the same p and
// n_scales) on v[i] into out[i] (laid out as phiks_apply's out), with ws[i] a
// workspace of workspace_doubles(*plans[i]) doubles, 16-byte aligned.
struct GroupWork {
  std::vector<const phiks_plan_s*> plans;
  std::vector<const double*> v;
  std::vector<double*> out;
  std::vector<double*> ws;
  int p = 0, ns = 1;
};

// Matrices of a plan's Tucker operator in its arithmetic: the node matrices (level false,
// from node idx) or exp(B/2^idx) (level true); FP32 plans use their FP32 copies (views
// hold them as double pointers, as the single path's mixed chains do).
void plan_mats(const phiks_plan_s& P, bool level, int idx, double** L) {
  for (int mu = 0; mu < P.d; ++mu) {
    const size_t off = (size_t)idx * P.n[mu] * P.n[mu];
    if (P.precision == PHIKS_FP32)
      L[mu] = reinterpret_cast<double*>((level ? P.E32[mu] : P.Lnode32[mu]) + off);
    else
      L[mu] = (level ? P.E[mu] : P.Lnode[mu]) + off;
  }
}

// A step item of mode mu (1-based) of a plan's Tucker operator, tagged with its arithmetic.
StepGemm step_item(const phiks_plan_s& P, const GemmArgs& g, int mu, bool lincomb,
                   const double* Y, int p) {
  const bool last = (mu == P.d);
  StepGemm it{g, mu == 1, last && lincomb, (last && lincomb) ? Y : nullptr, P.N, p};
  if (P.precision == PHIKS_FP32) {
    it.prec = PHIKS_FP32;
    it.f32_kind = !last ? (mu == 1 ? 0 : 1) : (lincomb ? 3 : 2);
  }
  return it;
}

// Builds the launches of one grouped execution (the same order of operations as
// phiks_apply for every problem).
void build_group_schedule(const GroupWork& W, BatchSchedule& S) {
  const int p = W.p, ns = W.ns;
  const int count = (int)W.plans.size();
  const double* const* v = W.v.data();
  double* const* out = W.out.data();
  struct Bufs { double *ta, *tb, *pa, *pb, *cur; };
  std::vector<Bufs> bf(count);
  int dmax = 0, smax = 0;
  for (int i = 0; i < count; ++i) {
    const phiks_plan_s& P = (*W.plans[i]);
    const int64_t N = P.N;
    const int64_t t = std::max<int64_t>({(int64_t)P.q - 1, (int64_t)p, 1});
    bf[i].ta = W.ws[i];
    bf[i].tb = bf[i].ta + t * N;
    bf[i].pa = bf[i].tb + t * N;
    bf[i].pb = bf[i].pa + (int64_t)p * N;
    dmax = std::max(dmax, P.d);
    smax = std::max(smax, P.s);
  }
  auto slot = [&](int i, int level, int ell) {
    return out[i] + ((int64_t)level * (p + 1) + ell) * (*W.plans[i]).N;
  };
  // squaring-epilogue coefficients (the same for every problem: they depend on p only)
  S.set_lin(p);
  if (p > 0) {
    // eq. integrandsimul: the node Tuckers of every problem, mode by mode
    std::vector<std::vector<GemmArgs>> views(count, std::vector<GemmArgs>(PHIKS_MAX_D));
    for (int i = 0; i < count; ++i) {
      const phiks_plan_s& P = (*W.plans[i]);
      int64_t stride[PHIKS_MAX_D];
      for (int mu = 0; mu < P.d; ++mu) stride[mu] = P.n[mu] * P.n[mu];
      double* wbuf = tucker_free_buffer(P.d, bf[i].ta, bf[i].tb);
      double* Ln[PHIKS_MAX_D];
      plan_mats(P, false, 0, Ln);
      tucker_args(P.d, P.n, P.N, v[i], 0, Ln, stride, plan_nodes(P), wbuf, bf[i].ta,
                  bf[i].tb, views[i].data());
    }
    for (int mu = 1; mu <= dmax; ++mu) {
      std::vector<StepGemm> items;
      for (int i = 0; i < count; ++i)
        if ((*W.plans[i]).d >= mu)
          items.push_back(step_item(*W.plans[i], views[i][mu - 1], mu, false, nullptr, p));
      S.add_gemm_step(items);
    }
    // node sums
    std::vector<CombineArgs> comb;
    for (int i = 0; i < count; ++i) {
      const phiks_plan_s& P = (*W.plans[i]);
      const int nodes = plan_nodes(P);
      double* wbuf = tucker_free_buffer(P.d, bf[i].ta, bf[i].tb);
      bf[i].cur = (P.s < ns) ? slot(i, P.s, 1) : bf[i].pa;
      CombineArgs ca;
      std::memset(&ca, 0, sizeof(ca));
      ca.nin = nodes + 1;
      for (int k = 0; k < nodes; ++k) ca.in[k] = wbuf + (int64_t)k * P.N;
      ca.in[nodes] = v[i];
      ca.out = bf[i].cur;
      ca.out_stride = P.N;
      ca.nout = p;
      ca.beta = 0.0;
      ca.N = P.N;
      for (int ell = 1; ell <= p; ++ell)
        for (int k = 0; k < P.q; ++k)
          ca.coef[ell - 1][k] = P.w[k] * std::pow(P.theta[k], ell - 1) / factorial(ell - 1);
      ca.vec = combine_vec_ok(ca) ? 1 : 0;
      comb.push_back(ca);
    }
    S.add_combine_step(comb);
    // eq. simul: iteration t runs level j = s_i - t of every problem with s_i > t
    for (int t = 0; t < smax; ++t) {
      std::vector<std::vector<GemmArgs>> lv(count, std::vector<GemmArgs>(PHIKS_MAX_D));
      std::vector<double*> dst(count, nullptr);
      for (int i = 0; i < count; ++i) {
        const phiks_plan_s& P = (*W.plans[i]);
        if (P.s <= t) continue;
        const int j = P.s - t;
        dst[i] = (j - 1 < ns) ? slot(i, j - 1, 1) : ((bf[i].cur == bf[i].pa) ? bf[i].pb : bf[i].pa);
        double* L[PHIKS_MAX_D];
        int64_t stride[PHIKS_MAX_D] = {0};
        plan_mats(P, true, j, L);
        tucker_args(P.d, P.n, P.N, bf[i].cur, P.N, L, stride, p, dst[i], bf[i].ta, bf[i].tb,
                    lv[i].data());
      }
      for (int mu = 1; mu <= dmax; ++mu) {
        std::vector<StepGemm> items;
        for (int i = 0; i < count; ++i) {
          const phiks_plan_s& P = (*W.plans[i]);
          if (P.s <= t || P.d < mu) continue;
          const bool last = (mu == P.d);
          items.push_back(step_item(P, lv[i][mu - 1], mu, last, bf[i].cur, p));
        }
        S.add_gemm_step(items);
      }
      for (int i = 0; i < count; ++i)
        if ((*W.plans[i]).s > t) bf[i].cur = dst[i];
    }
  }
  // exponential outputs exp(2^-j tau K) v
  for (int lev = 0; lev < ns; ++lev) {
    std::vector<std::vector<GemmArgs>> ev(count, std::vector<GemmArgs>(PHIKS_MAX_D));
    for (int i = 0; i < count; ++i) {
      const phiks_plan_s& P = (*W.plans[i]);
      double* L[PHIKS_MAX_D];
      int64_t stride[PHIKS_MAX_D] = {0};
      plan_mats(P, true, lev, L);
      tucker_args(P.d, P.n, P.N, v[i], 0, L, stride, 1, slot(i, lev, 0), bf[i].ta, bf[i].tb,
                  ev[i].data());
    }
    for (int mu = 1; mu <= dmax; ++mu) {
      std::vector<StepGemm> items;
      for (int i = 0; i < count; ++i)
        if ((*W.plans[i]).d >= mu)
          items.push_back(step_item(*W.plans[i], ev[i][mu - 1], mu, false, nullptr, p));
      S.add_gemm_step(items);
    }
  }
}

// Uploads S's tables (growing them if needed) on st.
int upload_group(GroupTables& T, const BatchSchedule& S, hipStream_t st) {
  // the previous call's upload must have read the staging buffer before it is rewritten
  if (T.uploaded) HIP_OK(hipEventSynchronize(T.upload_done));
  if (!T.upload_done) HIP_OK(hipEventCreateWithFlags(&T.upload_done, hipEventDisableTiming));
  const size_t need = std::max<size_t>(S.buf.size(), 16);
  if (need > T.bytes) {
    // the old device table is released in stream order
    const size_t bytes = need + need / 4;
    char* h = nullptr;
    void* d = nullptr;
    if (hipHostMalloc((void**)&h, bytes, hipHostMallocDefault) != hipSuccess) {
      set_error("hipHostMalloc of the launch tables failed");
      return PHIKS_ENOMEM;
    }
    if (hipMallocAsync(&d, bytes, st) != hipSuccess) {
      (void)hipHostFree(h);
      set_error("hipMallocAsync of the launch tables failed");
      return PHIKS_ENOMEM;
    }
    if (T.dev) HIP_OK(hipFreeAsync(T.dev, st));
    if (T.host) (void)hipHostFree(T.host);
    T.host = h;
    T.dev = d;
    T.bytes = bytes;
  }
  if (!S.buf.empty()) std::memcpy(T.host, S.buf.data(), S.buf.size());
  HIP_OK(hipMemcpyAsync(T.dev, T.host, need, hipMemcpyHostToDevice, st));
  HIP_OK(hipEventRecord(T.upload_done, st));
  T.uploaded = true;
  return PHIKS_OK;
}

// ------------------------------------------------ FP32 grouped launches
template <int BM, int BN, int WM, int WN, bool KC, class TA, class TC, class Epi>
int launch_grouped32_cfg(const GroupedLaunch& L, const char* dev, const Epi& epi, hipStream_t st) {
  if (L.total > 0x7fffffffLL) {
    set_error("grouped GEMM grid too large");
    return PHIKS_EINVAL;
  }
  const GroupItem* items = (const GroupItem*)(dev + L.items_off);
  const int64_t* first = (const int64_t*)(dev + L.first_off);
  if constexpr (BM >= 64 && BN >= 64) {
    if (L.dl)
      return timed_launch(&gemm_f32_dl_grouped<BM, BN, WM, WN, KC, TA, TC, Epi>, (unsigned)L.total, st,
                          L.flops, items, first, L.n, L.total, epi);
  }
  return timed_launch(&gemm_f32_grouped<BM, BN, WM, WN, KC, true, TA, TC, Epi>, (unsigned)L.total, st,
                      L.flops, items, first, L.n, L.total, epi);
}

template <bool KC, class TA, class TC, class Epi>
int launch_grouped32(const GroupedLaunch& L, const char* dev, const Epi& epi, hipStream_t st) {
  if (L.bm == 128 && L.bn == 64) return launch_grouped32_cfg<128, 64, 64, 32, KC, TA, TC>(L, dev, epi, st);
  if (L.bm == 64 && L.bn == 128) return launch_grouped32_cfg<64, 128, 32, 64, KC, TA, TC>(L, dev, epi, st);
  if (L.bm == 64 && L.bn == 64) return launch_grouped32_cfg<64, 64, 32, 32, KC, TA, TC>(L, dev, epi, st);
  return launch_grouped32_cfg<32, 32, 16, 16, KC, TA, TC>(L, dev, epi, st);
}

// An FP32 product of a batch: grouped, or (L.single) launched as its single call does.
int issue_one32(const GroupedLaunch& L, const char* dev, const BatchSchedule& S, hipStream_t st) {
  const EpiStoreT<float> to32{1.0, 0.0};
  const EpiStore to64{1.0, 0.0};
  if (L.single) {
    const GroupItem& it = *(const GroupItem*)(S.buf.data() + L.items_off);   // host copy
    switch (L.f32_kind) {
      case 0:
        return L.kc ? launch_gemm32<true, double, float>(it.g, to32, st)
                    : launch_gemm32<false, double, float>(it.g, to32, st);
      case 1: return launch_gemm32<false, float, float>(it.g, to32, st);
      case 2: return L.kc ? launch_gemm32<true, double, double>(it.g, to64, st)
                          : launch_gemm32<false, float, double>(it.g, to64, st);
      default: {
        EpiLinComb e = S.lin[L.lin_p];
        e.Y = it.Y;
        e.N = it.YN;
        return L.kc ? launch_gemm32<true, double, double>(it.g, e, st)
                    : launch_gemm32<false, float, double>(it.g, e, st);
      }
    }
  }
  switch (L.f32_kind) {
    case 0: return launch_grouped32<true, double, float>(L, dev, to32, st);
    case 1: return launch_grouped32<false, float, float>(L, dev, to32, st);
    case 2: return launch_grouped32<false, float, double>(L, dev, to64, st);
    default: return launch_grouped32<false, float, double>(L, dev, S.lin[L.lin_p], st);
  }
}

int issue_one(const GroupedLaunch& L, const char* dev, const BatchSchedule& S, hipStream_t st) {
  if (L.kind == StepKind::Gemm && L.prec == PHIKS_FP32) return issue_one32(L, dev, S, st);
  if (L.kind == StepKind::Combine) {
    const int64_t blocks = std::min<int64_t>((L.total + 255) / 256, 1024);
    (void)hipGetLastError();
    hipLaunchKernelGGL(combine_grouped_kernel, dim3((unsigned)blocks, (unsigned)L.n), dim3(256),
                       0, st, (const CombineArgs*)(dev + L.items_off));
    CHECK_LAUNCH();
    return PHIKS_OK;
  }
  if (L.lincomb) return launch_grouped(L, dev, S.lin[L.lin_p], st);
  return launch_grouped(L, dev, EpiStore{1.0, 0.0}, st);
}

// Issues S's launches on st (their tables uploaded by upload_group).  Kernel launches
// only, so the sequence can be captured into a graph.
int issue_group(const GroupTables& T, const BatchSchedule& S, hipStream_t st) {
  const char* dev = (const char*)T.dev;
  for (const GroupedLaunch& L : S.launches) RET_IF(issue_one(L, dev, S, st));
  return PHIKS_OK;
}

// Fork and join of a captured call: the launches of one step (disjoint problems) are
// forked over the aux streams and joined back before the next step, so the graph may
// run a step's small partitions beside its large one.  The plan is host data only (so
// it can be checked without a device): a step with one launch, or no aux stream, runs on
// the main stream; otherwise the main stream records a fork event that `used` aux
// streams wait for, the step's launches go round-robin over them, and each aux stream
// records a join event the main stream waits for.  Events are numbered in order of use;
// a call needs at most launches + steps of them.
struct ForkOp {
  enum Kind { Record = 0, Wait = 1, Launch = 2 } kind;
  int stream;   // -1: the main stream, else an aux stream
  int event;    // Record / Wait
  int launch;   // Launch: index into BatchSchedule::launches
};

std::vector<ForkOp> fork_plan(const BatchSchedule& S, int naux) {
  std::vector<ForkOp> ops;
  const std::vector<GroupedLaunch>& Ls = S.launches;
  int e = 0;
  for (size_t i = 0; i < Ls.size();) {
    size_t j = i;
    while (j < Ls.size() && Ls[j].step == Ls[i].step) ++j;
    if (j - i == 1 || naux <= 0) {
      for (size_t k = i; k < j; ++k) ops.push_back({ForkOp::Launch, -1, -1, (int)k});
      i = j;
      continue;
    }
    const int fork = e++;
    ops.push_back({ForkOp::Record, -1, fork, -1});
    const int used = (int)std::min<size_t>((size_t)naux, j - i);
    for (int a = 0; a < used; ++a) ops.push_back({ForkOp::Wait, a, fork, -1});
    for (size_t k = i; k < j; ++k) ops.push_back({ForkOp::Launch, (int)((k - i) % used), -1, (int)k});
    for (int a = 0; a < used; ++a) {
      const int join = e++;
      ops.push_back({ForkOp::Record, a, join, -1});
      ops.push_back({ForkOp::Wait, -1, join, -1});
    }
    i = j;
  }
  return ops;
}

// As issue_group, for capture on st, following fork_plan over the aux streams.  ev:
// events for the fork and join points (hipEventDisableTiming), launches + steps of them.
int issue_group_forked(const GroupTables& T, const BatchSchedule& S, hipStream_t st,
                       const std::vector<hipStream_t>& aux, const std::vector<hipEvent_t>& ev) {
  const char* dev = (const char*)T.dev;
  for (const ForkOp& op : fork_plan(S, (int)aux.size())) {
    hipStream_t s = op.stream < 0 ? st : aux[op.stream];
    if (op.kind == ForkOp::Record) HIP_OK(hipEventRecord(ev[op.event], s));
    else if (op.kind == ForkOp::Wait) HIP_OK(hipStreamWaitEvent(s, ev[op.event], 0));
    else RET_IF(issue_one(S.launches[op.launch], dev, S, s));
  }
  return PHIKS_OK;
}

int run_group(GroupTables& T, const BatchSchedule& S, hipStream_t st) {
  RET_IF(upload_group(T, S, st));
  return issue_group(T, S, st);
}

// Releases a batch's captured graph once its last launch has finished.
void drop_graph(phiks_batch_s& B) {
  if (!B.graph) return;
  (void)hipStreamSynchronize(B.graph_stream);
  (void)hipGraphExecDestroy(B.graph);
  B.graph = nullptr;
}

// Captures S's launches (tables already uploaded) into B.graph on B's capture stream.
int capture_group(phiks_batch_s& B, const BatchSchedule& S) {
  if (!B.capture_stream) HIP_OK(hipStreamCreateWithFlags(&B.capture_stream, hipStreamNonBlocking));
  while ((int)B.fork_streams.size() < PHIKS_BATCH_FORK) {
    hipStream_t a = nullptr;
    HIP_OK(hipStreamCreateWithFlags(&a, hipStreamNonBlocking));
    B.fork_streams.push_back(a);
  }
  // fork and join points: one per step with several launches, plus one per joined stream
  std::vector<hipEvent_t> ev(S.launches.size() + (size_t)S.steps);
  for (hipEvent_t& e : ev) {
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      for (hipEvent_t& x : ev)
        if (x) (void)hipEventDestroy(x);
      set_error("hipEventCreate failed");
      return PHIKS_EDEVICE;
    }
  }
  HIP_OK(hipStreamBeginCapture(B.capture_stream, hipStreamCaptureModeThreadLocal));
  const int rc = issue_group_forked(B.tab, S, B.capture_stream, B.fork_streams, ev);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(B.capture_stream, &g);
  for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  if (rc != PHIKS_OK || ec != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    set_error("capture of the batched launches failed");
    return PHIKS_EDEVICE;
  }
  const hipError_t ei = hipGraphInstantiate(&B.graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) {
    B.graph = nullptr;
    (void)hipGetLastError();
    set_error("instantiation of the batched launch graph failed");
    return PHIKS_EDEVICE;
  }
  return PHIKS_OK;
}

// Frees the tables; the caller has synchronised the stream that used them.
void free_group_tables(GroupTables& T) {
  if (T.dev) (void)hipFree(T.dev);
  if (T.host) (void)hipHostFree(T.host);
  if (T.upload_done) (void)hipEventDestroy(T.upload_done);
  T = GroupTables();
}

// ---------------------------------------------------------------- host dry run
// phiks_batch_dryrun: builds a call's schedule and fork plan for given shapes and plans
// with synthetic device addresses (nothing is dereferenced or launched) and checks them.
// Each buffer of a problem (plan matrices, v, out, workspace) is a region of a synthetic
// address space with a gap after it; every operand range a launch table names must lie
// inside one region, all ranges of one item inside the same problem's regions.
struct DryRunSpace {
  uintptr_t next = (uintptr_t)1 << 44;
  struct Region { uintptr_t lo, hi; int owner; };
  std::vector<Region> regions;
  double* take(size_t doubles, int owner) {
    const uintptr_t lo = next, hi = lo + std::max<size_t>(doubles, 1) * sizeof(double);
    regions.push_back({lo, hi, owner});
    next = (hi + ((uintptr_t)1 << 20) + 255) & ~(uintptr_t)255;
    return reinterpret_cast<double*>(lo);
  }
  int owner(uintptr_t lo, uintptr_t hi) const {
    for (const Region& r : regions)
      if (lo >= r.lo && hi <= r.hi) return r.owner;
    return -1;
  }
};

struct DryRunCheck {
  int64_t violations = 0;
  std::string first;
  void fail(const std::string& what) {
    if (violations++ == 0) first = what;
  }
};

// Owner of the byte range [base + lo_el, base + hi_el) in doubles, or -1.
int dry_owner(const DryRunSpace& sp, const double* base, int64_t lo_el, int64_t hi_el) {
  const uintptr_t b = reinterpret_cast<uintptr_t>(base);
  return sp.owner(b + (uintptr_t)(lo_el * 8), b + (uintptr_t)(hi_el * 8));
}

void dry_check_schedule(const BatchSchedule& S, const DryRunSpace& sp, int count,
                        const std::vector<int64_t>& want_gemms, int naux, DryRunCheck& ck) {
  std::vector<int64_t> gemms(count, 0), combs(count, 0);
  for (size_t li = 0; li < S.launches.size(); ++li) {
    const GroupedLaunch& L = S.launches[li];
    const std::string at = "launch " + std::to_string(li) + ": ";
    if (L.n < 1) ck.fail(at + "empty launch");
    if (L.kind == StepKind::Combine) {
      const CombineArgs* items = (const CombineArgs*)(S.buf.data() + L.items_off);
      for (int k = 0; k < L.n; ++k) {
        const CombineArgs& a = items[k];
        if (a.nin < 1 || a.nin > kMaxIn || a.nout < 1 || a.nout > 8 || a.N < 1 ||
            a.N > L.total) {
          ck.fail(at + "combine item sizes");
          continue;
        }
        const int own = dry_owner(sp, a.out, 0, (int64_t)(a.nout - 1) * a.out_stride + a.N);
        if (own < 0) ck.fail(at + "combine output outside its buffer");
        for (int t = 0; t < a.nin; ++t)
          if (dry_owner(sp, a.in[t], 0, a.N) != own) ck.fail(at + "combine input outside the problem");
        if (own >= 0) ++combs[own];
      }
      continue;
    }
    const GroupItem* items = (const GroupItem*)(S.buf.data() + L.items_off);
    const int64_t* first = (const int64_t*)(S.buf.data() + L.first_off);
    const int bm = BatchSchedule::kBM[L.tile], bn = BatchSchedule::kBN[L.tile];
    int64_t tiles = 0;
    for (int k = 0; k < L.n; ++k) {
      const GemmArgs& g = items[k].g;
      if (first[k] != tiles) ck.fail(at + "first[] is not the prefix sum of the item tiles");
      if (g.M < 1 || g.N < 1 || g.K < 1 || g.nb0 < 1 || g.nb1 < 1 || g.pA != nullptr) {
        ck.fail(at + "item view sizes");
        continue;
      }
      if (g.tiles_m != (g.M + bm - 1) / bm || g.tiles_n != (g.N + bn - 1) / bn ||
          g.total_tiles != (int64_t)g.tiles_m * g.tiles_n * g.nb0 * g.nb1)
        ck.fail(at + "tile counts do not match the tile class");
      if (L.dl && g.K % PHIKS_DL_BK != 0) ck.fail(at + "direct-to-LDS item with a partial K chunk");
      tiles += g.total_tiles;
      const int64_t bz = (int64_t)(g.nb0 - 1), b1 = (int64_t)(g.nb1 - 1);
      const int64_t a_hi = bz * g.sA0 + b1 * g.sA1 + (int64_t)(g.M - 1) * g.lda + g.K;
      const int64_t b_hi = bz * g.sB0 + b1 * g.sB1 +
                           (L.kc ? (int64_t)(g.N - 1) * g.ldb + g.K : (int64_t)(g.K - 1) * g.ldb + g.N);
      const int64_t c_hi = bz * g.sC0 + b1 * g.sC1 + (int64_t)(g.M - 1) * g.ldc + g.N;
      const int oa = dry_owner(sp, g.A, 0, a_hi), ob = dry_owner(sp, g.B, 0, b_hi),
                oc = dry_owner(sp, g.C, 0, c_hi);
      if (oa < 0 || ob < 0 || oc < 0) ck.fail(at + "operand range outside its buffer");
      else if (oa != ob || ob != oc) ck.fail(at + "operands of one item in different problems");
      if (L.lincomb) {
        const int64_t y_hi = b1 * items[k].YN + bz * g.sC0 + (int64_t)(g.M - 1) * g.ldc + g.N;
        if (dry_owner(sp, items[k].Y, 0, y_hi) != oc) ck.fail(at + "squaring-epilogue tensors outside the problem");
        if (b1 + 1 != S.lin[L.lin_p].p) ck.fail(at + "squaring epilogue batch is not p");
      }
      if (oc >= 0) ++gemms[oc];
    }
    if (tiles != L.total) ck.fail(at + "launch total is not the sum of its item tiles");
  }
  for (int i = 0; i < count; ++i)
    if (gemms[i] != want_gemms[i])
      ck.fail("problem " + std::to_string(i) + ": " + std::to_string(gemms[i]) +
              " mu-mode products scheduled, " + std::to_string(want_gemms[i]) + " expected");
  // fork and join of the captured form
  const std::vector<ForkOp> ops = fork_plan(S, naux);
  const int nev = (int)(S.launches.size() + S.steps);
  std::vector<char> recorded(nev, 0);
  std::vector<int> launched(S.launches.size(), 0);
  int last_step = -1;
  for (const ForkOp& op : ops) {
    if (op.stream < -1 || op.stream >= std::max(naux, 0)) ck.fail("fork plan: stream index out of range");
    if (op.kind == ForkOp::Launch) {
      if (op.launch < 0 || op.launch >= (int)S.launches.size()) {
        ck.fail("fork plan: launch index out of range");
        continue;
      }
      ++launched[op.launch];
      if (S.launches[op.launch].step < last_step) ck.fail("fork plan: steps out of order");
      last_step = S.launches[op.launch].step;
      continue;
    }
    if (op.event < 0 || op.event >= nev) {
      ck.fail("fork plan: event index out of range");
      continue;
    }
    if (op.kind == ForkOp::Record) recorded[op.event] = 1;
    else if (!recorded[op.event]) ck.fail("fork plan: wait on an event not yet recorded");
  }
  for (int c : launched)
    if (c != 1) ck.fail("fork plan: a launch issued other than once");
}

}  // namespace

extern "C" {

int phiks_batch_tuning(int set, int* params) {
  if (!params) return PHIKS_EINVAL;
  std::lock_guard<std::mutex> lk(g_tuning_mu);
  if (set) {
    if (params[0] < 1 || params[0] > 128) return PHIKS_EINVAL;
    for (int k = 1; k < 5; ++k)
      if (params[k] != 0 && params[k] != 1) return PHIKS_EINVAL;
    g_batch_tuning = BatchTuning{params[0], params[1], params[2], params[3], params[4]};
    ++g_tuning_gen;
  }
  params[0] = g_batch_tuning.sq_min;
  params[1] = g_batch_tuning.skinny;
  params[2] = g_batch_tuning.wide_m1;
  params[3] = g_batch_tuning.wide_mk;
  params[4] = g_batch_tuning.wide_lc;
  return PHIKS_OK;
}

int phiks_batch_dryrun(int count, const int* d, const int64_t* const* n, const int* s,
                       const int* q, int p, int n_scales, int fork_streams, int64_t* launches,
                       int64_t* table_bytes, int64_t* violations) {
  if (count < 1 || !d || !n || !s || !q || !launches || !table_bytes || !violations)
    return PHIKS_EINVAL;
  if (p < 0 || p > PHIKS_MAX_P || n_scales < 1 || n_scales > 16 || fork_streams < 0)
    return PHIKS_EINVAL;
  std::vector<phiks_plan_s> plans(count);
  DryRunSpace sp;
  GroupWork W;
  W.p = p;
  W.ns = n_scales;
  std::vector<int64_t> want(count, 0);
  for (int i = 0; i < count; ++i) {
    if (d[i] < 1 || d[i] > PHIKS_MAX_D || !n[i] || s[i] < std::max(0, n_scales - 1) || s[i] > kSMax)
      return PHIKS_EINVAL;
    if (p > 0 && (q[i] < kQMin || q[i] > kQMax)) return PHIKS_EINVAL;
    phiks_plan_s& P = plans[i];
    P.d = d[i];
    P.N = 1;
    for (int mu = 0; mu < d[i]; ++mu) {
      if (n[i][mu] < 1 || n[i][mu] > PHIKS_MAX_N) return PHIKS_EINVAL;
      P.n[mu] = n[i][mu];
      P.N *= n[i][mu];
    }
    if (!views_fit_int32(P.d, P.n, 1)) return PHIKS_EINVAL;
    P.p = p;
    P.ns = n_scales;
    P.task = PHIKS_SAME_VECTOR;
    P.precision = PHIKS_FP64;
    P.s = s[i];
    P.q = p > 0 ? q[i] : 0;
    if (p > 0) gll_rule(P.q, P.theta, P.w);
    plan_assign(P, sp.take(plan_device_doubles(P), i));
    W.plans.push_back(&P);
    W.v.push_back(sp.take(P.N, i));
    W.out.push_back(sp.take((size_t)n_scales * (p + 1) * P.N, i));
    W.ws.push_back(sp.take(workspace_doubles(P), i));
    want[i] = (int64_t)P.d * ((p > 0 ? 1 + P.s : 0) + n_scales);
  }
  BatchSchedule S;
  build_group_schedule(W, S);
  DryRunCheck ck;
  dry_check_schedule(S, sp, count, want, fork_streams, ck);
  *launches = (int64_t)S.launches.size();
  *table_bytes = (int64_t)S.buf.size();
  *violations = ck.violations;
  if (ck.violations) set_error(ck.first);
  return PHIKS_OK;
}



void phiks_batch_destroy(phiks_batch_t batch) {
  if (!batch) return;
  int cur = 0;
  const bool switched = (hipGetDevice(&cur) == hipSuccess) && cur != batch->device;
  if (switched) (void)hipSetDevice(batch->device);
  // Waits for the batch's stream, then frees.  (A host function queued on the stream
  // may not call the HIP API, and the pinned tables need hipHostFree.)
  (void)hipStreamSynchronize(batch->stream);
  drop_graph(*batch);
  if (batch->capture_stream) (void)hipStreamDestroy(batch->capture_stream);
  for (hipStream_t a : batch->fork_streams) (void)hipStreamDestroy(a);
  if (batch->dmem) (void)hipFree(batch->dmem);
  free_group_tables(batch->tab);
  delete batch;
  if (switched) (void)hipSetDevice(cur);
}

int phiks_batch_plan(int count, const int* d, const int64_t* const* n,
                     const double* const* const* A, const double* tau, int p, int n_scales,
                     double tol, const double* vnorms, int precision, void* hip_stream,
                     phiks_batch_t* out) {
  if (!out) return PHIKS_EINVAL;
  *out = nullptr;
  if (count < 1 || !d || !n || !A || !tau) return PHIKS_EINVAL;
  if (precision != PHIKS_FP64 && precision != PHIKS_FP32) {
    set_error("batched problems run in FP64 or FP32");
    return PHIKS_EINVAL;
  }
  phiks_batch_s* B = new (std::nothrow) phiks_batch_s;
  if (!B) return PHIKS_ENOMEM;
  B->count = count;
  B->p = p;
  B->ns = n_scales;
  B->precision = precision;
  B->plans.resize(count);
  // host planning of the problems on a few threads (the planner keeps no shared
  // mutable state; its kernel table is built once under call_once)
  std::vector<int> rcs(count, PHIKS_OK);
  std::vector<std::string> errs(count);
  {
    const int nt = std::max(1, std::min<int>({count, 16, (int)std::thread::hardware_concurrency()}));
    std::vector<std::thread> pool;
    for (int t = 0; t < nt; ++t)
      pool.emplace_back([&, t]() {
        for (int i = t; i < count; i += nt) {
          rcs[i] = plan_init_host(B->plans[i], d[i], n[i], A[i], tau[i], p, n_scales, tol,
                                  PHIKS_SAME_VECTOR, vnorms ? vnorms + i : nullptr, precision);
          if (rcs[i] != PHIKS_OK) errs[i] = g_last_error;
        }
      });
    for (std::thread& th : pool) th.join();
  }
  for (int i = 0; i < count; ++i) {
    if (rcs[i] != PHIKS_OK) {
      set_error("problem " + std::to_string(i) + ": " + phiks_status_string(rcs[i]) +
                (errs[i].empty() ? "" : " (" + errs[i] + ")"));
      delete B;
      return rcs[i];
    }
  }
  hipStream_t st = (hipStream_t)hip_stream;
  B->stream = st;
  auto fail = [&](int code) {
    phiks_batch_destroy(B);
    return code;
  };
  if (hipGetDevice(&B->device) != hipSuccess) { set_error("hipGetDevice failed"); return fail(PHIKS_EDEVICE); }
  // one allocation for every problem's matrices (each slice 16-byte aligned)
  std::vector<size_t> moff(count);
  size_t total = 0;
  for (int i = 0; i < count; ++i) {
    moff[i] = total;
    total += (plan_device_doubles(B->plans[i]) + 1) & ~(size_t)1;
  }
  if (hipMallocAsync(&B->dmem, std::max<size_t>(total, 1) * sizeof(double), st) != hipSuccess) {
    B->dmem = nullptr;
    set_error("hipMallocAsync of batch matrices failed");
    return fail(PHIKS_ENOMEM);
  }
  std::vector<phiks_plan_s*> ptrs(count);
  std::vector<const double* const*> mats(count);
  for (int i = 0; i < count; ++i) {
    plan_assign(B->plans[i], (double*)B->dmem + moff[i]);
    B->plans[i].device = B->device;
    B->plans[i].stream = st;
    ptrs[i] = &B->plans[i];
    mats[i] = A[i];
  }
  int rc = build_plan_matrices(ptrs, mats, st);
  if (rc != PHIKS_OK) return fail(rc);
  // workspace: each problem's single-call workspace, 16-byte aligned slices
  B->ws_off.resize(count);
  for (int i = 0; i < count; ++i) {
    B->ws_off[i] = B->ws_doubles;
    B->ws_doubles += (workspace_doubles(B->plans[i]) + 1) & ~(size_t)1;
  }
  *out = B;
  return PHIKS_OK;
}

int phiks_batch_workspace_size(phiks_batch_t batch, size_t* bytes) {
  if (!batch || !bytes) return PHIKS_EINVAL;
  *bytes = batch->ws_doubles * sizeof(double);
  return PHIKS_OK;
}

int phiks_batch_info(phiks_batch_t batch, int i, int* s, int* q, int* tucker_paper,
                     int* tucker_exec) {
  if (!batch || i < 0 || i >= batch->count) return PHIKS_EINVAL;
  const phiks_plan_s& P = batch->plans[i];
  if (s) *s = P.s;
  if (q) *q = P.q;
  if (tucker_paper) *tucker_paper = P.t_paper;
  if (tucker_exec) *tucker_exec = P.t_exec;
  return PHIKS_OK;
}

int phiks_batch_apply(phiks_batch_t batch, const double* const* v, double* const* out, void* ws,
                      size_t ws_bytes, void* hip_stream) {
  if (!batch || !v || !out) return PHIKS_EINVAL;
  phiks_batch_s& B = *batch;
  for (int i = 0; i < B.count; ++i)
    if (!v[i] || !out[i]) return PHIKS_EINVAL;
  if (!ws || ws_bytes < B.ws_doubles * sizeof(double)) return PHIKS_EWORKSPACE;
  if ((uintptr_t)ws % 16) {
    set_error("batch workspace must be 16-byte aligned");
    return PHIKS_EINVAL;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  // The launches depend only on the batch and the pointers: the second call with one
  // pointer set captures them into a graph, later calls with that set replay it (no
  // schedule, no upload, one launch).  Calls with kernel timing on stay eager.
  std::vector<const void*> key(v, v + B.count);
  key.insert(key.end(), out, out + B.count);
  key.push_back(ws);
  int64_t gen = 0;
  (void)batch_tuning(&gen);
  key.push_back((const void*)(uintptr_t)gen);   // the rules the captured launches used
  const bool timing = kernel_timing_on();
  if (!timing && B.graph && key == B.graph_key) {
    HIP_OK(hipGraphLaunch(B.graph, st));
    B.graph_stream = st;
    return PHIKS_OK;
  }
  GroupWork W;
  W.p = B.p;
  W.ns = B.ns;
  for (int i = 0; i < B.count; ++i) {
    W.plans.push_back(&B.plans[i]);
    W.v.push_back(v[i]);
    W.out.push_back(out[i]);
    W.ws.push_back((double*)ws + B.ws_off[i]);
  }
  BatchSchedule S;
  build_group_schedule(W, S);
  drop_graph(B);   // the upload below rewrites the tables a graph reads
  const bool repeat = (key == B.graph_key);
  B.graph_key.swap(key);
  RET_IF(upload_group(B.tab, S, st));
  if (timing || !repeat || capture_group(B, S) != PHIKS_OK) return issue_group(B.tab, S, st);
  HIP_OK(hipGraphLaunch(B.graph, st));
  B.graph_stream = st;
  return PHIKS_OK;
}

}  // extern "C"
