// Compile-time work split of the Gram matrix G = Y^T Y (Section 2) over the
// W waves of a workgroup.  The NC(NC+1)/2 unique entries (a <= b) are
// ordered by 4x4 column blocks and cut into W contiguous chunks, so each
// wave touches few distinct columns and keeps its partial sums in registers.
#pragma once

#include <utility>

namespace assg {

template <int NC>
__host__ __device__ constexpr int pair_index(int a, int b) {   // a <= b, row-major upper triangle
  return a * NC - (a * (a - 1)) / 2 + (b - a);
}

template <int NC, int W>
struct GramPlan {
  static constexpr int NP = NC * (NC + 1) / 2;
  static constexpr int BS = 4;
  int a[NP];
  int b[NP];
  int start[W + 1];
  bool need[W][NC];
  constexpr GramPlan() : a{}, b{}, start{}, need{} {
    int q = 0;
    const int nbk = (NC + BS - 1) / BS;
    for (int ba = 0; ba < nbk; ++ba)
      for (int bb = ba; bb < nbk; ++bb)
        for (int i = ba * BS; i < (ba + 1) * BS && i < NC; ++i)
          for (int j = bb * BS; j < (bb + 1) * BS && j < NC; ++j)
            if (i <= j) {
              a[q] = i;
              b[q] = j;
              ++q;
            }
    for (int w = 0; w <= W; ++w) start[w] = (NP * w) / W;
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
  static constexpr int QMAX = (GramPlan<NC, W>::NP + W - 1) / W;
};

// Per-wave accumulation over 64 rows of a tile held column-major in LDS
// (tile[c*TS + row]); every index is a compile-time constant.
template <int NC, int W, int WID, int TS, int C>
__device__ __forceinline__ void gram_load_one(double* v, const double* tile, int lane) {
  if constexpr (GramPlanHolder<NC, W>::P.need[WID][C]) v[C] = tile[C * TS + lane];
}
template <int NC, int W, int WID, int TS, int... C>
__device__ __forceinline__ void gram_load(double* v, const double* tile, int lane,
                                          std::integer_sequence<int, C...>) {
  (gram_load_one<NC, W, WID, TS, C>(v, tile, lane), ...);
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
__device__ __forceinline__ void gram_accum_wave(double* acc, const double* tile, int lane) {
  double v[NC];
  gram_load<NC, W, WID, TS>(v, tile, lane, std::make_integer_sequence<int, NC>{});
  gram_fma<NC, W, WID>(acc, v, std::make_integer_sequence<int, GramPlanHolder<NC, W>::QMAX>{});
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
    double s = acc[Q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
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
