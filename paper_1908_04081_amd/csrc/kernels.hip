// Row kernels of the adaptive s-step CG hot path for gfx950 (wave64).
//
//  k_spmv        y = A x                                   (CSR, LPR lanes/row)
//  k_setup       r0 = b - A x0, Y level 0 = (r0, r0), ||b||  (Algorithm 5 start)
//  k_sweep       one matrix-powers level of both chains (2.3) from one read of A
//  k_last_gram   last P-chain level fused with the Gram partial sums of G = Y^T Y
//  k_gram_reduce fixed-order sum of the Gram partials (the single reduction)
//  k_recover     x += Y x', (p, r) = (Y p', Y r') into basis level 0 (2.6)
//  k_check       true residual ||b - A x|| when the updated residual reached tol,
//                and the end-of-loop commit of the outcome
//  k_h_*         Hestenes-Stiefel CG (Algorithm 1) comparator
//
// The basis Y_{k,s} is stored as s "pair" vectors (P_l[i], R_l[i]) (16 bytes
// per row, l = 0..s-1) plus one vector P_s: interleaved column order
// [p0, r0, p1, r1, ..., p_s].  A gather of x[col] fetches both chains at once.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "gram_plan.hpp"
#include "launch.hpp"

namespace assg {

#define ASSG_LPR_SWITCH(lpr, CALL) \
  switch (lpr) {                   \
    case 2: { constexpr int LPR = 2; CALL; } break;   \
    case 4: { constexpr int LPR = 4; CALL; } break;   \
    case 8: { constexpr int LPR = 8; CALL; } break;   \
    case 16: { constexpr int LPR = 16; CALL; } break; \
    case 32: { constexpr int LPR = 32; CALL; } break; \
    default: { constexpr int LPR = 64; CALL; } break; \
  }

int row_blocks(int64_t n) {
  const int64_t ntiles = (n + TILE_ROWS - 1) / TILE_ROWS;
  int64_t nb = ((ntiles + NXCD - 1) / NXCD) * NXCD;
  if (nb > MAX_ROW_BLOCKS) nb = MAX_ROW_BLOCKS;
  if (nb < NXCD) nb = NXCD;
  return (int)nb;
}

int pick_lpr(int64_t n, int64_t nnz) {
  const int64_t avg = (nnz + n - 1) / (n > 0 ? n : 1);
  int l = 2;
  while (l < 64 && l < avg) l <<= 1;
  return l;
}

// Rows owned by this workgroup: tiles [t0, t1) of TILE_ROWS rows.
struct RowIter {
  int64_t t0, t1;
  __device__ RowIter(int64_t n) {
    const int L = xcd_logical(blockIdx.x, gridDim.x);
    tile_range(L, gridDim.x, (n + TILE_ROWS - 1) / TILE_ROWS, t0, t1);
  }
};

// ------------------------------------------------------------------ SpMV
template <int LPR>
__global__ __launch_bounds__(ROW_THREADS) void k_spmv(CsrView A, const double* __restrict__ x,
                                                      double* __restrict__ y) {
  constexpr int RPP = ROW_THREADS / LPR;
  const int g = threadIdx.x / LPR, sub = threadIdx.x % LPR;
  RowIter it(A.n);
  for (int64_t t = it.t0; t < it.t1; ++t)
    for (int r = 0; r < TILE_ROWS; r += RPP) {
      const int64_t row = t * TILE_ROWS + r + g;
      const bool act = row < A.n;
      const double v = csr_dot<LPR>(A.rp, A.ci, A.va, x, row, sub, act);
      if (act && sub == 0) y[row] = v;
    }
}

void launch_spmv(hipStream_t s, const CsrView& A, int lpr, const double* x, double* y) {
  const int nb = row_blocks(A.n);
  ASSG_LPR_SWITCH(lpr, hipLaunchKernelGGL(k_spmv<LPR>, dim3(nb), dim3(ROW_THREADS), 0, s, A, x, y));
}

// ----------------------------------------------------------------- setup
template <int LPR>
__global__ __launch_bounds__(ROW_THREADS) void k_setup(Ctl* ctl, CsrView A,
                                                       const double* __restrict__ b,
                                                       const double* __restrict__ x,
                                                       double2* __restrict__ pairs,
                                                       double* __restrict__ partials) {
  __shared__ double sh[ROW_THREADS / WAVE];
  constexpr int RPP = ROW_THREADS / LPR;
  const int g = threadIdx.x / LPR, sub = threadIdx.x % LPR;
  double part = 0.0;
  RowIter it(A.n);
  for (int64_t t = it.t0; t < it.t1; ++t)
    for (int r = 0; r < TILE_ROWS; r += RPP) {
      const int64_t row = t * TILE_ROWS + r + g;
      const bool act = row < A.n;
      const double ax = csr_dot<LPR>(A.rp, A.ci, A.va, x, row, sub, act);
      if (act && sub == 0) {
        const double bi = b[row];
        const double ri = bi - ax;
        pairs[row] = make_double2(ri, ri);
        part = fma(bi, bi, part);
      }
    }
  part = block_sum<ROW_THREADS>(part, sh);
  double tot;
  if (last_block_total(part, partials, ctl, &tot, sh)) ctl->nb = sqrt(tot);
}

void launch_setup(hipStream_t s, Ctl* ctl, const CsrView& A, int lpr, const double* b,
                  const double* x, double2* pairs, double* partials) {
  const int nb = row_blocks(A.n);
  ASSG_LPR_SWITCH(lpr, hipLaunchKernelGGL(k_setup<LPR>, dim3(nb), dim3(ROW_THREADS), 0, s, ctl,
                                          A, b, x, pairs, partials));
}

// ------------------------------------------------ matrix powers: one level
// y_l = (A y_{l-1} - theta_{l-1} y_{l-1} - mu_{l-2} y_{l-2}) / gamma_{l-1}
// for both chains (2.3); levels beyond the loop's s-bar exit at once.
template <int LPR>
__global__ __launch_bounds__(ROW_THREADS) void k_sweep(const Ctl* __restrict__ ctl, int level,
                                                       CsrView A, double2* __restrict__ pairs,
                                                       int64_t ld) {
  if (ctl->status != ST_RUNNING || level >= ctl->sbar) return;
  const double th = ctl->theta[level - 1];
  const double ga = ctl->gamma[level - 1];
  const double mu = (level >= 2) ? ctl->mu[level - 2] : 0.0;
  const double2* __restrict__ X = pairs + (size_t)(level - 1) * ld;
  const double2* __restrict__ X2 = pairs + (size_t)(level >= 2 ? level - 2 : 0) * ld;
  double2* __restrict__ Yo = pairs + (size_t)level * ld;
  constexpr int RPP = ROW_THREADS / LPR;
  const int g = threadIdx.x / LPR, sub = threadIdx.x % LPR;
  RowIter it(A.n);
  for (int64_t t = it.t0; t < it.t1; ++t)
    for (int r = 0; r < TILE_ROWS; r += RPP) {
      const int64_t row = t * TILE_ROWS + r + g;
      const bool act = row < A.n;
      const double2 a = csr_dot2<LPR>(A.rp, A.ci, A.va, X, row, sub, act);
      if (act && sub == 0) {
        const double2 xo = X[row];
        double yx = a.x - th * xo.x;
        double yy = a.y - th * xo.y;
        if (mu != 0.0) {
          const double2 x2 = X2[row];
          yx -= mu * x2.x;
          yy -= mu * x2.y;
        }
        Yo[row] = make_double2(yx / ga, yy / ga);
      }
    }
}

void launch_sweep(hipStream_t s, const Ctl* ctl, int level, const CsrView& A, int lpr,
                  double2* pairs, int64_t ld) {
  const int nb = row_blocks(A.n);
  ASSG_LPR_SWITCH(lpr, hipLaunchKernelGGL(k_sweep<LPR>, dim3(nb), dim3(ROW_THREADS), 0, s, ctl,
                                          level, A, pairs, ld));
}

// --------------------------------- last level fused with the Gram partials
// For each 64-row tile: stage Y's 2 sbar columns in LDS (column-major),
// compute P_sbar for the tile (its theta/mu terms read the staged columns),
// then every wave adds its share of the unique products Y_a * Y_b to
// register accumulators.  Columns past 2 sbar + 1 stay zero.
template <int NC, int W>
__global__ __launch_bounds__(64 * W) void k_last_gram(const Ctl* __restrict__ ctl, CsrView A,
                                                      int lpr, const double2* __restrict__ pairs,
                                                      double* __restrict__ plast, int64_t ld,
                                                      double* __restrict__ partials) {
  if (ctl->status != ST_RUNNING) return;
  constexpr int NT = 64 * W;
  constexpr int QMAX = GramPlanHolder<NC, W>::QMAX;
  __shared__ double tile[NC * 64];
  const int s = ctl->sbar;
  const double th = ctl->theta[s - 1];
  const double ga = ctl->gamma[s - 1];
  const double mu = (s >= 2) ? ctl->mu[s - 2] : 0.0;
  const double* __restrict__ xsrc = reinterpret_cast<const double*>(pairs + (size_t)(s - 1) * ld);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int i = tid; i < (NC - 2 * s - 1) * 64; i += NT) tile[(2 * s + 1) * 64 + i] = 0.0;
  double acc[QMAX];
#pragma unroll
  for (int q = 0; q < QMAX; ++q) acc[q] = 0.0;

  const int L = xcd_logical(blockIdx.x, gridDim.x);
  int64_t t0, t1;
  tile_range(L, gridDim.x, (A.n + 63) / 64, t0, t1);
  const int rpp = NT / lpr;
  const int g = tid / lpr, sub = tid % lpr;
  for (int64_t t = t0; t < t1; ++t) {
    const int64_t base = t * 64;
    for (int i = tid; i < s * 64; i += NT) {
      const int l = i >> 6, rl = i & 63;
      const int64_t row = base + rl;
      double2 v = make_double2(0.0, 0.0);
      if (row < A.n) v = pairs[(size_t)l * ld + row];
      tile[(2 * l) * 64 + rl] = v.x;
      tile[(2 * l + 1) * 64 + rl] = v.y;
    }
    __syncthreads();
    for (int r = 0; r < 64; r += rpp) {
      const int rl = r + g;
      const int64_t row = base + rl;
      const bool act = (rl < 64) && (row < A.n);
      double a = 0.0;
      if (act) {
        const int32_t e0 = A.rp[row], e1 = A.rp[row + 1];
        for (int32_t k = e0 + sub; k < e1; k += lpr)
          a = fma(ldnt(A.va + k), xsrc[2 * (int64_t)ldnt(A.ci + k)], a);
      }
      for (int off = lpr >> 1; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
      if (sub == 0 && rl < 64) {
        double y = 0.0;
        if (act) {
          y = a - th * tile[(2 * s - 2) * 64 + rl];
          if (mu != 0.0) y -= mu * tile[(2 * s - 4) * 64 + rl];
          y = y / ga;
          plast[row] = y;
        }
        tile[(2 * s) * 64 + rl] = y;
      }
    }
    __syncthreads();
    switch (wave) {
      case 0: gram_accum_wave<NC, W, 0>(acc, tile, lane); break;
      case 1: gram_accum_wave<NC, W, 1>(acc, tile, lane); break;
      case 2: gram_accum_wave<NC, W, 2>(acc, tile, lane); break;
      case 3: gram_accum_wave<NC, W, 3>(acc, tile, lane); break;
      default:
        if constexpr (W > 4) {
          switch (wave) {
            case 4: gram_accum_wave<NC, W, (W > 4 ? 4 : 0)>(acc, tile, lane); break;
            case 5: gram_accum_wave<NC, W, (W > 5 ? 5 : 0)>(acc, tile, lane); break;
            case 6: gram_accum_wave<NC, W, (W > 6 ? 6 : 0)>(acc, tile, lane); break;
            case 7: gram_accum_wave<NC, W, (W > 7 ? 7 : 0)>(acc, tile, lane); break;
          }
        }
        break;
    }
    __syncthreads();
  }
  const auto qs = std::make_integer_sequence<int, QMAX>{};
  switch (wave) {
    case 0: gram_flush<NC, W, 0>(acc, lane, partials, gridDim.x, blockIdx.x, qs); break;
    case 1: gram_flush<NC, W, 1>(acc, lane, partials, gridDim.x, blockIdx.x, qs); break;
    case 2: gram_flush<NC, W, 2>(acc, lane, partials, gridDim.x, blockIdx.x, qs); break;
    case 3: gram_flush<NC, W, 3>(acc, lane, partials, gridDim.x, blockIdx.x, qs); break;
    default:
      if constexpr (W > 4) {
        switch (wave) {
          case 4: gram_flush<NC, W, (W > 4 ? 4 : 0)>(acc, lane, partials, gridDim.x, blockIdx.x, qs); break;
          case 5: gram_flush<NC, W, (W > 5 ? 5 : 0)>(acc, lane, partials, gridDim.x, blockIdx.x, qs); break;
          case 6: gram_flush<NC, W, (W > 6 ? 6 : 0)>(acc, lane, partials, gridDim.x, blockIdx.x, qs); break;
          case 7: gram_flush<NC, W, (W > 7 ? 7 : 0)>(acc, lane, partials, gridDim.x, blockIdx.x, qs); break;
        }
      }
      break;
  }
}

template <int NC>
constexpr int gram_waves() { return NC <= 21 ? 4 : 8; }

template <int NC>
static int last_gram_blocks_nc(int cus) {
  constexpr int W = gram_waves<NC>();
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_last_gram<NC, W>, 64 * W, 0) !=
          hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  int nb = cus * per_cu;
  nb = ((nb + NXCD - 1) / NXCD) * NXCD;
  return nb < 4096 ? nb : 4096;   // partials are sized for 4096 workgroups
}

#define ASSG_SIGMA_SWITCH(sigma, CALL)                    \
  switch (sigma) {                                         \
    case 1: { constexpr int NC = 3; CALL; } break;         \
    case 2: { constexpr int NC = 5; CALL; } break;         \
    case 3: { constexpr int NC = 7; CALL; } break;         \
    case 4: { constexpr int NC = 9; CALL; } break;         \
    case 5: { constexpr int NC = 11; CALL; } break;        \
    case 6: { constexpr int NC = 13; CALL; } break;        \
    case 7: { constexpr int NC = 15; CALL; } break;        \
    case 8: { constexpr int NC = 17; CALL; } break;        \
    case 9: { constexpr int NC = 19; CALL; } break;        \
    case 10: { constexpr int NC = 21; CALL; } break;       \
    case 11: { constexpr int NC = 23; CALL; } break;       \
    case 12: { constexpr int NC = 25; CALL; } break;       \
    case 13: { constexpr int NC = 27; CALL; } break;       \
    case 14: { constexpr int NC = 29; CALL; } break;       \
    case 15: { constexpr int NC = 31; CALL; } break;       \
    default: { constexpr int NC = 33; CALL; } break;       \
  }

int last_gram_blocks(int sigma, int cus) {
  int nb = NXCD;
  ASSG_SIGMA_SWITCH(sigma, nb = last_gram_blocks_nc<NC>(cus));
  return nb;
}

void launch_last_gram(hipStream_t s, const Ctl* ctl, int sigma, const CsrView& A, int lpr,
                      int nblocks, const double2* pairs, double* plast, int64_t ld,
                      double* partials) {
  ASSG_SIGMA_SWITCH(sigma, {
    constexpr int W = gram_waves<NC>();
    hipLaunchKernelGGL((k_last_gram<NC, W>), dim3(nblocks), dim3(64 * W), 0, s, ctl, A, lpr,
                       pairs, plast, ld, partials);
  });
}

// G[a][b] = G[b][a] = sum over workgroups of the partials, fixed order.
template <int NC>
__global__ __launch_bounds__(256) void k_gram_reduce(Ctl* __restrict__ ctl, int nparts,
                                                     const double* __restrict__ partials) {
  if (ctl->status != ST_RUNNING) return;
  __shared__ double sh[4];
  const int p = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 256) s += partials[(size_t)p * nparts + i];
  s = block_sum<256>(s, sh);
  if (threadIdx.x == 0) {
    int a = 0, q = p;
    while (q >= NC - a) {
      q -= NC - a;
      ++a;
    }
    const int b = a + q;
    ctl->G[a * MAXC + b] = s;
    ctl->G[b * MAXC + a] = s;
  }
}

void launch_gram_reduce(hipStream_t s, Ctl* ctl, int sigma, int nparts, const double* partials) {
  ASSG_SIGMA_SWITCH(sigma, hipLaunchKernelGGL(k_gram_reduce<NC>, dim3(NC * (NC + 1) / 2),
                                              dim3(256), 0, s, ctl, nparts, partials));
}

// -------------------------------------------------------------- recovery
// (2.6): x += Y x', p = Y p', r = Y r' over the 2 s_k + 1 columns that carry
// coordinates after s_k inner steps ((2.1): P_0..P_{s_k}, R_0..R_{s_k-1});
// (p, r) overwrite basis level 0 row by row (each row is read before it is
// written by the same thread).
__global__ __launch_bounds__(ROW_THREADS) void k_recover(const Ctl* __restrict__ ctl, int64_t n,
                                                         double2* __restrict__ pairs,
                                                         const double* __restrict__ plast,
                                                         int64_t ld, double* __restrict__ x) {
  if (ctl->status != ST_RUNNING || ctl->skip_recover) return;
  const int sk = ctl->sk, sbar = ctl->sbar;
  const double* __restrict__ plevel =
      (sk == sbar) ? plast : reinterpret_cast<const double*>(pairs + (size_t)sk * ld);
  const int pstride = (sk == sbar) ? 1 : 2;
  RowIter it(n);
  for (int64_t t = it.t0; t < it.t1; ++t) {
    const int64_t row = t * TILE_ROWS + threadIdx.x;
    if (row >= n) continue;
    double xs = 0.0, ps = 0.0, rs = 0.0;
    for (int l = 0; l < sk; ++l) {
      const double2 y = pairs[(size_t)l * ld + row];
      xs = fma(ctl->cx[2 * l], y.x, xs);
      xs = fma(ctl->cx[2 * l + 1], y.y, xs);
      ps = fma(ctl->cp[2 * l], y.x, ps);
      ps = fma(ctl->cp[2 * l + 1], y.y, ps);
      rs = fma(ctl->cr[2 * l], y.x, rs);
      rs = fma(ctl->cr[2 * l + 1], y.y, rs);
    }
    const double yl = plevel[pstride * row];
    xs = fma(ctl->cx[2 * sk], yl, xs);
    ps = fma(ctl->cp[2 * sk], yl, ps);
    rs = fma(ctl->cr[2 * sk], yl, rs);
    x[row] += xs;
    pairs[row] = make_double2(ps, rs);
  }
}

void launch_recover(hipStream_t s, const Ctl* ctl, int64_t n, double2* pairs,
                    const double* plast, int64_t ld, double* x) {
  hipLaunchKernelGGL(k_recover, dim3(row_blocks(n)), dim3(ROW_THREADS), 0, s, ctl, n, pairs,
                     plast, ld, x);
}

// ------------------------------------------------ end of an outer loop
// Applies the stopping reading: the true relative residual decides when the
// updated one reached tol; 5 failed confirmations in a row without a 10%
// improvement of the best one stop the solve (STAGNATED); caps give MAX_ITER.
__device__ void commit_loop(Ctl* ctl, assg_trace_t* trace, bool checked, double rel) {
  int st = ctl->pending;
  const int64_t k = ctl->k;
  if (checked) {
    ctl->relres_true = rel;
    if (ctl->record_trace && k < ctl->trace_cap) trace[k].relres_true = rel;
    if (st == ST_RUNNING) {
      if (rel <= ctl->tol) {
        st = ASSG_CONVERGED;
      } else if (rel < 0.9 * ctl->best_true) {
        ctl->best_true = rel;
        ctl->fail_streak = 0;
      } else if (++ctl->fail_streak >= 5) {
        st = ASSG_STAGNATED;
      }
      if (st == ST_RUNNING && (ctl->m >= ctl->max_iters || k + 1 >= ctl->max_outer))
        st = ASSG_MAX_ITER;
    }
  }
  ctl->k = (int32_t)(k + 1);
  ctl->sbar = ctl->sbar_next;
  ctl->candidate = 0;
  ctl->skip_recover = 0;
  ctl->pending = ST_RUNNING;
  ctl->status = st;
}

template <int LPR>
__global__ __launch_bounds__(ROW_THREADS) void k_check(Ctl* ctl, assg_trace_t* trace, CsrView A,
                                                       const double* __restrict__ b,
                                                       const double* __restrict__ x,
                                                       double* __restrict__ partials,
                                                       int measure_only) {
  __shared__ double sh[ROW_THREADS / WAVE];
  if (!measure_only) {
    if (ctl->status != ST_RUNNING) return;
    if (!ctl->candidate) {
      if (blockIdx.x == 0 && threadIdx.x == 0) commit_loop(ctl, trace, false, -1.0);
      return;
    }
  }
  constexpr int RPP = ROW_THREADS / LPR;
  const int g = threadIdx.x / LPR, sub = threadIdx.x % LPR;
  double part = 0.0;
  RowIter it(A.n);
  for (int64_t t = it.t0; t < it.t1; ++t)
    for (int r = 0; r < TILE_ROWS; r += RPP) {
      const int64_t row = t * TILE_ROWS + r + g;
      const bool act = row < A.n;
      const double ax = csr_dot<LPR>(A.rp, A.ci, A.va, x, row, sub, act);
      if (act && sub == 0) {
        const double ri = b[row] - ax;
        part = fma(ri, ri, part);
      }
    }
  part = block_sum<ROW_THREADS>(part, sh);
  double tot;
  if (last_block_total(part, partials, ctl, &tot, sh)) {
    const double rel = sqrt(tot) / ctl->nb;
    if (measure_only)
      ctl->relres_true = rel;
    else
      commit_loop(ctl, trace, true, rel);
  }
}

void launch_check(hipStream_t s, Ctl* ctl, assg_trace_t* trace, const CsrView& A, int lpr,
                  const double* b, const double* x, double* partials, int measure_only) {
  const int nb = row_blocks(A.n);
  ASSG_LPR_SWITCH(lpr, hipLaunchKernelGGL(k_check<LPR>, dim3(nb), dim3(ROW_THREADS), 0, s, ctl,
                                          trace, A, b, x, partials, measure_only));
}

// ------------------------------------------------------------------ HSCG
template <int LPR>
__global__ __launch_bounds__(ROW_THREADS) void k_h_init(Ctl* ctl, CsrView A,
                                                        const double* __restrict__ b,
                                                        const double* __restrict__ x,
                                                        double* __restrict__ r,
                                                        double* __restrict__ p,
                                                        double* __restrict__ partials) {
  __shared__ double sh[ROW_THREADS / WAVE];
  constexpr int RPP = ROW_THREADS / LPR;
  const int g = threadIdx.x / LPR, sub = threadIdx.x % LPR;
  double pb = 0.0, pr = 0.0;
  RowIter it(A.n);
  for (int64_t t = it.t0; t < it.t1; ++t)
    for (int rr = 0; rr < TILE_ROWS; rr += RPP) {
      const int64_t row = t * TILE_ROWS + rr + g;
      const bool act = row < A.n;
      const double ax = csr_dot<LPR>(A.rp, A.ci, A.va, x, row, sub, act);
      if (act && sub == 0) {
        const double bi = b[row];
        const double ri = bi - ax;
        r[row] = ri;
        p[row] = ri;
        pb = fma(bi, bi, pb);
        pr = fma(ri, ri, pr);
      }
    }
  // two sums: partials[0..nb) and partials[nb..2nb)
  pb = block_sum<ROW_THREADS>(pb, sh);
  pr = block_sum<ROW_THREADS>(pr, sh);
  double tot;
  if (threadIdx.x == 0) partials[gridDim.x + blockIdx.x] = pr;
  if (last_block_total(pb, partials, ctl, &tot, sh)) {
    double rr = 0.0;
    for (int i = 0; i < (int)gridDim.x; ++i)
      rr += __hip_atomic_load(partials + gridDim.x + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    ctl->nb = sqrt(tot);
    ctl->h_rho = rr;
  }
}

void launch_h_init(hipStream_t s, Ctl* ctl, const CsrView& A, int lpr, const double* b,
                   const double* x, double* r, double* p, double* partials) {
  const int nb = row_blocks(A.n);
  ASSG_LPR_SWITCH(lpr, hipLaunchKernelGGL(k_h_init<LPR>, dim3(nb), dim3(ROW_THREADS), 0, s, ctl,
                                          A, b, x, r, p, partials));
}

// w = A p with the p^T w partial sum; the last workgroup forms alpha.
template <int LPR>
__global__ __launch_bounds__(ROW_THREADS) void k_h_spmv(Ctl* ctl, CsrView A,
                                                        const double* __restrict__ p,
                                                        double* __restrict__ w,
                                                        double* __restrict__ partials) {
  if (ctl->status != ST_RUNNING || ctl->pending != ST_RUNNING) return;
  __shared__ double sh[ROW_THREADS / WAVE];
  constexpr int RPP = ROW_THREADS / LPR;
  const int g = threadIdx.x / LPR, sub = threadIdx.x % LPR;
  double part = 0.0;
  RowIter it(A.n);
  for (int64_t t = it.t0; t < it.t1; ++t)
    for (int r = 0; r < TILE_ROWS; r += RPP) {
      const int64_t row = t * TILE_ROWS + r + g;
      const bool act = row < A.n;
      const double v = csr_dot<LPR>(A.rp, A.ci, A.va, p, row, sub, act);
      if (act && sub == 0) {
        w[row] = v;
        part = fma(p[row], v, part);
      }
    }
  part = block_sum<ROW_THREADS>(part, sh);
  double pw;
  if (last_block_total(part, partials, ctl, &pw, sh)) {
    if (!(pw > 0.0) || !isfinite(pw)) {
      ctl->pending = isfinite(pw) ? ASSG_BREAKDOWN : ASSG_DIVERGED;
    } else {
      ctl->h_alpha = ctl->h_rho / pw;
    }
  }
}

void launch_h_spmv(hipStream_t s, Ctl* ctl, const CsrView& A, int lpr, const double* p,
                   double* w, double* partials) {
  const int nb = row_blocks(A.n);
  ASSG_LPR_SWITCH(lpr, hipLaunchKernelGGL(k_h_spmv<LPR>, dim3(nb), dim3(ROW_THREADS), 0, s, ctl,
                                          A, p, w, partials));
}

// x += alpha p; r -= alpha w; r^T r partial; the last workgroup forms beta
// and the updated relative residual.
__global__ __launch_bounds__(ROW_THREADS) void k_h_update(Ctl* ctl, int64_t n,
                                                          double* __restrict__ x,
                                                          double* __restrict__ r,
                                                          const double* __restrict__ p,
                                                          const double* __restrict__ w,
                                                          double* __restrict__ partials) {
  if (ctl->status != ST_RUNNING || ctl->pending != ST_RUNNING) return;
  __shared__ double sh[ROW_THREADS / WAVE];
  const double alpha = ctl->h_alpha;
  double part = 0.0;
  RowIter it(n);
  for (int64_t t = it.t0; t < it.t1; ++t) {
    const int64_t row = t * TILE_ROWS + threadIdx.x;
    if (row >= n) continue;
    const double q = alpha * p[row];
    x[row] += q;
    const double ri = r[row] - alpha * w[row];
    r[row] = ri;
    part = fma(ri, ri, part);
  }
  part = block_sum<ROW_THREADS>(part, sh);
  double rr;
  if (last_block_total(part, partials, ctl, &rr, sh)) {
    const double beta = rr / ctl->h_rho;
    ctl->h_rho = rr;
    ctl->h_beta = beta;
    ctl->m += 1;
    const double rel = sqrt(rr) / ctl->nb;
    ctl->relres_upd = rel;
    if (!isfinite(rel))
      ctl->pending = ASSG_DIVERGED;
    else if (rel <= ctl->tol)
      ctl->candidate = 1;
    else if (ctl->m >= ctl->max_iters)
      ctl->pending = ASSG_MAX_ITER;
  }
}

void launch_h_update(hipStream_t s, Ctl* ctl, int64_t n, double* x, double* r, const double* p,
                     const double* w, double* partials) {
  hipLaunchKernelGGL(k_h_update, dim3(row_blocks(n)), dim3(ROW_THREADS), 0, s, ctl, n, x, r, p,
                     w, partials);
}

__global__ __launch_bounds__(ROW_THREADS) void k_h_dir(const Ctl* ctl, int64_t n,
                                                       const double* __restrict__ r,
                                                       double* __restrict__ p) {
  if (ctl->status != ST_RUNNING || ctl->pending != ST_RUNNING) return;
  const double beta = ctl->h_beta;
  RowIter it(n);
  for (int64_t t = it.t0; t < it.t1; ++t) {
    const int64_t row = t * TILE_ROWS + threadIdx.x;
    if (row < n) p[row] = r[row] + beta * p[row];
  }
}

void launch_h_dir(hipStream_t s, const Ctl* ctl, int64_t n, const double* r, double* p) {
  hipLaunchKernelGGL(k_h_dir, dim3(row_blocks(n)), dim3(ROW_THREADS), 0, s, ctl, n, r, p);
}

// ----------------------------------------------------- basis/Gram helpers
__global__ void k_pair_init(int64_t n, const double* __restrict__ p, const double* __restrict__ r,
                            double2* __restrict__ pairs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) pairs[i] = make_double2(p[i], r[i]);
}

void launch_pair_init(hipStream_t s, int64_t n, const double* p, const double* r,
                      double2* pairs) {
  const int64_t nb = (n + 255) / 256;
  hipLaunchKernelGGL(k_pair_init, dim3((unsigned)nb), dim3(256), 0, s, n, p, r, pairs);
}

__global__ void k_export_Y(int64_t n, int sbar, const double2* __restrict__ pairs,
                           const double* __restrict__ plast, int64_t ld, double* __restrict__ Y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int l = 0; l < sbar; ++l) {
    const double2 v = pairs[(size_t)l * ld + i];
    Y[(size_t)(2 * l) * n + i] = v.x;
    Y[(size_t)(2 * l + 1) * n + i] = v.y;
  }
  Y[(size_t)(2 * sbar) * n + i] = plast[i];
}

void launch_export_Y(hipStream_t s, int64_t n, int sbar, const double2* pairs,
                     const double* plast, int64_t ld, double* Y) {
  const int64_t nb = (n + 255) / 256;
  hipLaunchKernelGGL(k_export_Y, dim3((unsigned)nb), dim3(256), 0, s, n, sbar, pairs, plast, ld,
                     Y);
}

}  // namespace assg
