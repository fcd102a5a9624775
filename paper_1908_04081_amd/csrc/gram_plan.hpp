// Compile-time plans of the Gram products, shared by the fused last sweep.
#pragma once

#include <utility>

#include "device.hpp"

namespace assg {

template <int NC>
__host__ __device__ constexpr int pair_index(int a, int b) {   // a <= b, row-major upper triangle
  return a * NC - (a * (a - 1)) / 2 + (b - a);
}

// Compile-time work split of the Gram matrix G = Y^T Y (Section 2) over the
// W waves of a workgroup.  Columns come in levels (2L, 2L+1), which one
// 16-byte LDS read delivers together; the unique entries (a <= b) are
// grouped by level pairs, and each wave takes level pairs greedily -- the
// one adding the fewest new levels to what it already reads -- up to its
// share of the entries, so every wave keeps few columns in registers.
template <int NC, int W>
struct GramPlan {
  static constexpr int NP = NC * (NC + 1) / 2;
  static constexpr int NL = (NC + 1) / 2;
  static constexpr int NLP = NL * (NL + 1) / 2;
  int a[NP];
  int b[NP];
  int start[W + 1];
  bool need[W][NC];
  static constexpr int count(int la, int lb) {   // entries (a <= b) of level pair (la, lb)
    int n = 0;
    for (int x = 2 * la; x < 2 * la + 2 && x < NC; ++x)
      for (int y = 2 * lb; y < 2 * lb + 2 && y < NC; ++y)
        if (x <= y) ++n;
    return n;
  }
  constexpr GramPlan() : a{}, b{}, start{}, need{} {
    int pla[NLP] = {}, plb[NLP] = {};
    bool used[NLP] = {};
    int k = 0;
    for (int la = 0; la < NL; ++la)
      for (int lb = la; lb < NL; ++lb) {
        pla[k] = la;
        plb[k] = lb;
        ++k;
      }
    int q = 0, rem = NP;
    for (int w = 0; w < W; ++w) {
      start[w] = q;
      const int target = (w == W - 1) ? rem : (rem + (W - w) - 1) / (W - w);
      bool lev[NL] = {};
      int cnt = 0;
      while (cnt < target) {
        int best = -1, bnew = 0, bn = 0;
        for (int i = 0; i < NLP; ++i) {
          if (used[i]) continue;
          const int nw = (lev[pla[i]] ? 0 : 1) + (lev[plb[i]] || pla[i] == plb[i] ? 0 : 1);
          const int n = count(pla[i], plb[i]);
          // fewest new levels; then the largest block that still fits
          const bool fits = cnt + n <= target, bfits = cnt + bn <= target;
          bool better = best < 0 || nw < bnew;
          if (!better && nw == bnew) better = (fits && !bfits) || (fits && bfits && n > bn) ||
                                              (!fits && !bfits && n < bn);
          if (better) {
            best = i;
            bnew = nw;
            bn = n;
          }
        }
        if (best < 0) break;
        used[best] = true;
        lev[pla[best]] = lev[plb[best]] = true;
        for (int x = 2 * pla[best]; x < 2 * pla[best] + 2 && x < NC; ++x)
          for (int y = 2 * plb[best]; y < 2 * plb[best] + 2 && y < NC; ++y)
            if (x <= y) {
              a[q] = x;
              b[q] = y;
              ++q;
            }
        cnt += bn;
      }
      rem -= cnt;
    }
    start[W] = q;
    for (int w = 0; w < W; ++w) {
      for (int c = 0; c < NC; ++c) need[w][c] = false;
      for (int qq = start[w]; qq < start[w + 1]; ++qq) {
        need[w][a[qq]] = true;
        need[w][b[qq]] = true;
      }
    }
  }
};

template <int NC, int W>
struct GramPlanHolder {
  static constexpr GramPlan<NC, W> P{};
  static constexpr int qmax() {
    int m = 0;
    for (int w = 0; w < W; ++w)
      if (P.start[w + 1] - P.start[w] > m) m = P.start[w + 1] - P.start[w];
    return m;
  }
  static constexpr int QMAX = qmax();
};

template <int NC, int W>
__host__ __device__ constexpr bool gram_need(int w, int c) {
  return c < NC && GramPlanHolder<NC, W>::P.need[w][c];
}

// Per-wave accumulation over 64 rows of a pair-major tile in LDS: entry
// tile[L*TS + row] holds columns 2L and 2L+1 of the row (one 16-byte read
// gives both); every index is a compile-time constant.
template <int NC, int W, int WID, int TS, int L>
__device__ __forceinline__ void gram_load_pair(double* v, const double2* tile, int lane) {
  constexpr bool n0 = gram_need<NC, W>(WID, 2 * L);
  constexpr bool n1 = gram_need<NC, W>(WID, 2 * L + 1);
  if constexpr (n0 || n1) {
    const double2 t = tile[L * TS + lane];
    if constexpr (n0) v[2 * L] = t.x;
    if constexpr (n1) v[2 * L + 1] = t.y;
  }
}
template <int NC, int W, int WID, int TS, int... L>
__device__ __forceinline__ void gram_load(double* v, const double2* tile, int lane,
                                          std::integer_sequence<int, L...>) {
  (gram_load_pair<NC, W, WID, TS, L>(v, tile, lane), ...);
}
template <int NC, int W, int WID, int Q>
__device__ __forceinline__ void gram_fma_one(double* acc, const double* v) {
  constexpr int q = GramPlanHolder<NC, W>::P.start[WID] + Q;
  if constexpr (q < GramPlanHolder<NC, W>::P.start[WID + 1]) {
    constexpr int ia = GramPlanHolder<NC, W>::P.a[q];
    constexpr int ib = GramPlanHolder<NC, W>::P.b[q];
    acc[Q] = fma(v[ia], v[ib], acc[Q]);
  }
}
template <int NC, int W, int WID, int... Q>
__device__ __forceinline__ void gram_fma(double* acc, const double* v,
                                         std::integer_sequence<int, Q...>) {
  (gram_fma_one<NC, W, WID, Q>(acc, v), ...);
}

template <int NC, int W, int WID, int TS>
__device__ __forceinline__ void gram_accum_wave(double* acc, const double2* tile, int lane) {
  double v[NC + 1];
  gram_load<NC, W, WID, TS>(v, tile, lane, std::make_integer_sequence<int, (NC + 1) / 2>{});
  gram_fma<NC, W, WID>(acc, v, std::make_integer_sequence<int, GramPlanHolder<NC, W>::QMAX>{});
}

// Wave ``wave`` (uniform) runs its own compile-time plan.
template <int NC, int W, int TS, int I = 0>
__device__ __forceinline__ void gram_accum(int wave, double* acc, const double2* tile, int lane) {
  if constexpr (I < W) {
    if (wave == I)
      gram_accum_wave<NC, W, I, TS>(acc, tile, lane);
    else
      gram_accum<NC, W, TS, I + 1>(wave, acc, tile, lane);
  }
}

// Lane sums of the per-wave accumulators, written as this workgroup's
// partial of each unique entry: partials[pair * nparts + part].
template <int NC, int W, int WID, int Q>
__device__ __forceinline__ void gram_flush_one(const double* acc, int lane, double* partials,
                                               int nparts, int part) {
  constexpr int q = GramPlanHolder<NC, W>::P.start[WID] + Q;
  if constexpr (q < GramPlanHolder<NC, W>::P.start[WID + 1]) {
    constexpr int ia = GramPlanHolder<NC, W>::P.a[q];
    constexpr int ib = GramPlanHolder<NC, W>::P.b[q];
    const double s = wave_sum_dpp(acc[Q]);
    if (lane == 0) partials[(size_t)pair_index<NC>(ia, ib) * nparts + part] = s;
  }
}
template <int NC, int W, int WID, int... Q>
__device__ __forceinline__ void gram_flush(const double* acc, int lane, double* partials,
                                           int nparts, int part,
                                           std::integer_sequence<int, Q...>) {
  (gram_flush_one<NC, W, WID, Q>(acc, lane, partials, nparts, part), ...);
}

}  // namespace assg

namespace assg {
template <int NC, int W, int I = 0>
__device__ __forceinline__ void gram_flush_all(int wave, const double* acc, int lane,
                                               double* partials, int nparts, int part) {
  if constexpr (I < W) {
    if (wave == I)
      gram_flush<NC, W, I>(acc, lane, partials, nparts, part,
                           std::make_integer_sequence<int, GramPlanHolder<NC, W>::QMAX>{});
    else
      gram_flush_all<NC, W, I + 1>(wave, acc, lane, partials, nparts, part);
  }
}
}  // namespace assg
