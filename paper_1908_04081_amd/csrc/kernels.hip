// Row kernels of the adaptive s-step CG hot path for gfx950 (wave64).
//
//  k_spmv        y = A x                                   (CSR-stream row blocks)
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
#include "launch.hpp"

namespace assg {


// Grid of a row-block kernel: one workgroup per block (rounded up to a
// multiple of 8), or at most ``cap`` workgroups each looping over a
// contiguous range of blocks.
static int block_grid(const CsrView& A, int cap) {
  int64_t g = ((int64_t)A.nblk + NXCD - 1) / NXCD * NXCD;
  if (g > cap) g = cap;
  if (g < NXCD) g = NXCD;
  return (int)g;
}

// Bounds of row block b and of the calling thread's own row.
struct BlockRows {
  int32_t r0, nr, e0, ne, rs, re;
  bool own;
  int64_t row;
  __device__ __forceinline__ BlockRows(const CsrView& A, int32_t b) {
    ASSG_DCHECK(b >= 0 && b < A.nblk, 1);
    r0 = A.blk[b];
    nr = A.blk[b + 1] - r0;
    e0 = A.blke[b];
    ne = A.blke[b + 1] - e0;
    ASSG_DCHECK(r0 >= 0 && nr >= 1 && (int64_t)r0 + nr <= A.n, 2);
    ASSG_DCHECK(e0 >= 0 && ne >= 0 && (int64_t)e0 + ne <= A.nnz, 3);
    ASSG_DCHECK(nr <= SB_ROWS && (ne <= SB_CAP || nr == 1), 4);
    own = (int)threadIdx.x < nr;
    row = (int64_t)r0 + threadIdx.x;
    rs = re = 0;
    if (own) {
      rs = A.rp[row] - e0;
      re = A.rp[row + 1] - e0;
      ASSG_DCHECK(rs >= 0 && rs <= re && re <= ne, 5);
    }
  }
};


// Local row i of system R's part of A x from the diagonal storage: the
// products in column order (offsets ascending), each rounded before it is
// added, as a sequential CSR product adds them; a diagonal position without
// an entry of A holds 0 and adds +0, which leaves the sum unchanged.  Eight
// diagonals' loads are issued before their products are added.  src is
// indexed by the batch row (R.row0 + column).  The record is read through
// the constant address space, so its fields come through the scalar cache
// (the same for every lane) and no vector load stands between a row and its
// diagonals' addresses.  With SHIFT, within a run of consecutive offsets
// (off_d = off_{d-1} + 1, as the x-neighbours of a stencil) row i's source
// entry for diagonal d is row i + 1's for diagonal d - 1: lane l takes it
// from lane l + 1 by a wave shift instead of a gather, and lane 63, whose
// neighbour row lies in the next wave, loads it.  Then every lane of the
// wave calls this; a lane whose row lies past its block (row_ok false)
// gathers for its neighbour but loads no values, and its sums are not used.
typedef const __attribute__((address_space(4))) DiaSys kDiaSys;
template <int CH, bool SHIFT, class S>
__device__ __forceinline__ void dia_row(const DiaSys* Rp, const double* __restrict__ val,
                                        const S& src, int64_t i, bool row_ok, double& sx,
                                        double& sy) {
#pragma clang fp contract(off)
  const kDiaSys& R = *(const kDiaSys*)Rp;
  sx = 0.0;
  sy = 0.0;
  const int32_t nd = R.nd;
  const int64_t n = R.n;
  const double* __restrict__ v0 = val + R.val0 + i;
  const bool lane63 = (threadIdx.x & 63) == 63;
  int32_t prev = 0;                           // offset of the previous diagonal
  double2 xprev = make_double2(0.0, 0.0);     // and this lane's source entry for it
  static_assert(DIA_MAX % 8 == 0, "diagonals are taken eight at a time");
  for (int d0 = 0; d0 < nd; d0 += 8) {
    int32_t off[8];                           // one batch of scalar loads
#pragma unroll
    for (int k = 0; k < 8; ++k) off[k] = R.off[d0 + k];
    bool run[8];                              // continues the previous diagonal's run
#pragma unroll
    for (int k = 0; k < 8; ++k)
      run[k] = SHIFT && d0 + k < nd && d0 + k > 0 && off[k] == (k == 0 ? prev : off[k - 1]) + 1;
    double v[8];
    double2 x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int d = d0 + k;
      const int64_t j = i + off[k];
      const bool ok = d < nd && j >= 0 && j < n;
      v[k] = (ok && row_ok) ? ldnt(v0 + (int64_t)d * n) : 0.0;
      x[k] = (ok && (!run[k] || lane63)) ? src.get((int32_t)(R.row0 + j)) : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (run[k]) {
        const double2 pv = (k == 0) ? xprev : x[k - 1];
        const double sxv = wave_shl1_d(pv.x);
        const double syv = (CH == 2) ? wave_shl1_d(pv.y) : 0.0;
        if (!lane63) x[k] = make_double2(sxv, syv);
      }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      sx += v[k] * x[k].x;
      if constexpr (CH == 2) sy += v[k] * x[k].y;
    }
    xprev = x[7];
    prev = off[7];
  }
}

// The block of this workgroup in a diagonal-storage kernel (one row per
// thread, XCD-aware), or -1, and its system.
__device__ __forceinline__ int32_t dia_block(const CsrView& A, int32_t& sys) {
  const int32_t bb = xcd_logical(blockIdx.x, gridDim.x);
  if (bb >= A.dia.nblk) return -1;
  sys = A.dia.bsys ? A.dia.bsys[bb] : 0;
  return bb;
}

static int dia_grid(const CsrView& A) {
  return (A.dia.nblk + NXCD - 1) / NXCD * NXCD;
}

// ------------------------------------------------------------------ SpMV
__global__ __launch_bounds__(256) void k_spmv(CsrView A, const double* __restrict__ x,
                                              double* __restrict__ y) {
  __shared__ double prod[SB_CAP];
  __shared__ double red[4];
  int32_t b0, b1;
  block_range(A.nblk, b0, b1);
  for (int32_t b = b0; b < b1; ++b) {
    const BlockRows br(A, b);
    double sx, sy;
    stream_rows<1, 256, SB_CAP>(A.ci, A.va, Src1{x}, br.e0, br.ne, br.rs, br.re, br.own, prod,
                                red, sx, sy);
    if (br.own) y[br.row] = sx;
    __syncthreads();
  }
}

void launch_spmv(hipStream_t s, const CsrView& A, const double* x, double* y) {
  hipLaunchKernelGGL(k_spmv, dim3(block_grid(A, 1 << 30)), dim3(256), 0, s, A, x, y);
}

// ----------------------------------------------------------------- setup
// One chunk of row blocks per workgroup (chunks never straddle systems);
// the partial ||b||^2 of each chunk, summed per system by k_fin_setup.
__global__ __launch_bounds__(256) void k_setup(Ctl* ctl, CsrView A, const double* __restrict__ b,
                                               const double* __restrict__ x,
                                               double2* __restrict__ pairs,
                                               double* __restrict__ part) {
  __shared__ double prod[SB_CAP];
  __shared__ double red[4];
  int32_t b0, b1, sys;
  const int32_t c = chunk_of(A, b0, b1, sys);
  double my = 0.0;
  for (int32_t bb = b0; bb < b1; ++bb) {
    const BlockRows br(A, bb);
    double bi = 0.0;
    if (br.own) bi = b[br.row];
    double ax, unused;
    stream_rows<1, 256, SB_CAP>(A.ci, A.va, Src1{x}, br.e0, br.ne, br.rs, br.re, br.own, prod,
                                red, ax, unused);
    if (br.own) {
      const double ri = bi - ax;
      pairs[br.row] = make_double2(ri, ri);
      my = fma(bi, bi, my);
    }
    __syncthreads();
  }
  my = block_sum<256>(my, red);
  if (threadIdx.x == 0) part[c] = my;
}

// System blockIdx.x: the sum of its chunks' partials, in chunk order.
__global__ __launch_bounds__(1024) void k_fin_setup(Ctl* ctl, CsrView A,
                                                    const double* __restrict__ part) {
  __shared__ double sh[16];
  const int i = blockIdx.x;
  const int32_t c0 = A.sys_chunk[i], c1 = A.sys_chunk[i + 1];
  const double t = finish_sum<1024>(part + c0, c1 - c0, sh);
  if (threadIdx.x == 0) ctl[i].nb = sqrt(t);
}

void launch_setup(hipStream_t s, Ctl* ctl, const CsrView& A, const double* b, const double* x,
                  double2* pairs, double* part) {
  hipLaunchKernelGGL(k_setup, dim3(A.nchunk), dim3(256), 0, s, ctl, A, b, x, pairs, part);
  hipLaunchKernelGGL(k_fin_setup, dim3(A.nsys), dim3(1024), 0, s, ctl, A, part);
}

// ------------------------------------------------ matrix powers: one level
// y_l = (A y_{l-1} - theta_{l-1} y_{l-1} - mu_{l-2} y_{l-2}) / gamma_{l-1}
// for both chains (2.3) from one read of A and one 16-byte gather per
// nonzero; levels beyond the loop's s-bar exit at once.
__global__ __launch_bounds__(256) void k_sweep(const Ctl* __restrict__ ctls, int level, CsrView A,
                                               double2* __restrict__ pairs, int64_t ld) {
  __shared__ __align__(16) double prod[2 * SB_CAP];   // read as double2
  __shared__ double red[4];
  const double2* __restrict__ X = pairs + (size_t)(level - 1) * ld;
  const double2* __restrict__ X2 = pairs + (size_t)(level >= 2 ? level - 2 : 0) * ld;
  double2* __restrict__ Yo = pairs + (size_t)level * ld;
  int32_t b0, b1;
  block_range(A.nblk, b0, b1);
  for (int32_t b = b0; b < b1; ++b) {
    const Ctl* ctl = ctls + block_sys(A, b);
    if (ctl->status != ST_RUNNING || level >= ctl->sbar) continue;
    const double th = ctl->theta[level - 1];
    const double ga = ctl->gamma[level - 1];
    const double mu = (level >= 2) ? ctl->mu[level - 2] : 0.0;
    const BlockRows br(A, b);
    double2 xo = make_double2(0.0, 0.0), x2 = make_double2(0.0, 0.0);
    if (br.own) {
      xo = X[br.row];
      if (mu != 0.0) x2 = ldnt2(X2 + br.row);
    }
    double ax, ay;
    stream_rows<2, 256, SB_CAP>(A.ci, A.va, Src2{X}, br.e0, br.ne, br.rs, br.re, br.own, prod,
                                red, ax, ay);
    if (br.own) {
      double yx = ax - th * xo.x;
      double yy = ay - th * xo.y;
      if (mu != 0.0) {
        yx -= mu * x2.x;
        yy -= mu * x2.y;
      }
      stnt2(Yo + br.row, make_double2(yx / ga, yy / ga));
    }
    __syncthreads();
  }
}

// The same level from the diagonal storage: one row per thread, every load
// coalesced, no product buffer and no barrier.
__global__ __launch_bounds__(256) void k_sweep_dia(const Ctl* __restrict__ ctls, int level,
                                                   CsrView A, double2* __restrict__ pairs,
                                                   int64_t ld) {
  int32_t sys;
  const int32_t bb = dia_block(A, sys);
  if (bb < 0) return;
  const Ctl* ctl = ctls + sys;
  if (ctl->status != ST_RUNNING || level >= ctl->sbar) return;
  // every lane takes part in the row products (rows past the block only
  // gather for their neighbours)
  const int64_t i = (int64_t)A.dia.blk[bb] + threadIdx.x;
  const bool own = i < A.dia.blk[bb + 1];
  const kDiaSys& R = *(const kDiaSys*)(A.dia.sys + sys);
  const double th = ctl->theta[level - 1];
  const double ga = ctl->gamma[level - 1];
  const double mu = (level >= 2) ? ctl->mu[level - 2] : 0.0;
  const double2* __restrict__ X = pairs + (size_t)(level - 1) * ld;
  const double2* __restrict__ X2 = pairs + (size_t)(level >= 2 ? level - 2 : 0) * ld;
  double2* __restrict__ Yo = pairs + (size_t)level * ld;
  double ax, ay;
  dia_row<2, true>(A.dia.sys + sys, A.dia.val, Src2{X}, i - R.row0, own, ax, ay);
  if (!own) return;
  const double2 xo = X[i];
  double2 x2 = make_double2(0.0, 0.0);
  if (mu != 0.0) x2 = ldnt2(X2 + i);
  double yx = ax - th * xo.x;
  double yy = ay - th * xo.y;
  if (mu != 0.0) {
    yx -= mu * x2.x;
    yy -= mu * x2.y;
  }
  stnt2(Yo + i, make_double2(yx / ga, yy / ga));
}

void launch_sweep(hipStream_t s, const Ctl* ctl, int level, const CsrView& A, double2* pairs,
                  int64_t ld) {
  if (A.dia.nd > 0)
    hipLaunchKernelGGL(k_sweep_dia, dim3(dia_grid(A)), dim3(256), 0, s, ctl, level, A, pairs, ld);
  else
    hipLaunchKernelGGL(k_sweep, dim3(block_grid(A, 1 << 30)), dim3(256), 0, s, ctl, level, A,
                       pairs, ld);
}

// --------------------------------- last level fused with the Gram partials
// Zero source of the direct-to-LDS basis loads for rows past a block.
__device__ double2 g_zero_rows[64];

// For each row block (<= 256 rows): first the block's CSR-stream products
// (gathers of P_{sbar-1}, products into an LDS buffer that is the start of
// the tile, row sums), then its s-bar basis pairs go from HBM straight into
// a pair-major LDS tile (direct-to-LDS loads, no registers) and P_sbar
// becomes the tile's level s-bar.  Sharing the buffer keeps the workgroup
// at 45 KB of LDS (three per CU at s-bar = 10, which the register budget
// is held to).  G = Y^T Y is then accumulated on the matrix cores, four
// rows per v_mfma_f64_16x16x4_f64, the block's 4-row groups dealt to the
// waves in turn (so a block of few long rows still keeps every wave busy),
// for the 16 x 16 blocks (I, J), I <= J, of the columns padded to NG * 16
// (columns past 2 sbar + 1 and rows past the block are zero).  The next
// block's nonzeros and row ranges are fetched before the Gram, and its
// bounds one block earlier still.  At the end the waves' accumulators are
// added in wave order and the unique entries written as this chunk's
// partials.  From the diagonal storage (DIA) the products need no LDS, so
// the tile loads are issued first and stream in while each thread forms its
// row of A P_{sbar-1}.
typedef double mfma_d4 __attribute__((ext_vector_type(4)));

template <int NC, int W, bool DIA>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(NC <= 23 ? 3 : 2)))
void k_last_gram(const Ctl* __restrict__ ctls, CsrView A, const double2* __restrict__ pairs,
                 double* __restrict__ plast, int64_t ld, double* __restrict__ partials) {
  int32_t b0, b1, sys;
  int32_t chunk;
  if constexpr (DIA) {
    chunk = xcd_logical(blockIdx.x, gridDim.x);
    ASSG_DCHECK(chunk >= 0 && chunk < A.dia.nchunk, 14);
    b0 = A.dia.cblk[chunk];
    b1 = A.dia.cblk[chunk + 1];
    sys = A.dia.csys ? A.dia.csys[chunk] : 0;
  } else {
    chunk = chunk_of(A, b0, b1, sys);
  }
  const Ctl* ctl = ctls + sys;
  if (ctl->status != ST_RUNNING) return;
  constexpr int NT = 64 * W;
  constexpr int TS = SB_ROWS;
  constexpr int TP = TS + 2;                 // padded level stride (LDS banks)
  constexpr int NL = (NC + 1) / 2;           // pair levels (the last holds P_sbar, 0)
  constexpr int NG = (NC + 15) / 16;         // 16-column groups
  constexpr int NB = NG * (NG + 1) / 2;      // accumulated 16 x 16 blocks
  constexpr int TILE_D = 2 * NL * TP;        // tile doubles
  constexpr int LDS_D = TILE_D > SB_CAP ? TILE_D : SB_CAP;   // products alias the tile
  // the waves' accumulators are added WR waves at a time through the LDS
  constexpr int WR = (W * NB * 256 <= LDS_D) ? W : (W / 2 * NB * 256 <= LDS_D) ? W / 2
                     : (W / 4 * NB * 256 <= LDS_D) ? W / 4 : 1;
  static_assert(WR * NB * 256 <= LDS_D, "accumulator staging exceeds the tile");
  __shared__ __align__(16) double lds[LDS_D];   // read as double2 (16-byte LDS reads)
  __shared__ double red[W];
  double2* const tile = reinterpret_cast<double2*>(lds);
  double* const prod = lds;
  const double* const tcol = lds;            // column c of row r: tcol[2 (c/2 TP + r) + c%2]
  const int s = ctl->sbar;
  const double th = ctl->theta[s - 1];
  const double ga = ctl->gamma[s - 1];
  const double mu = (s >= 2) ? ctl->mu[s - 2] : 0.0;
  const double* __restrict__ xsrc = reinterpret_cast<const double*>(pairs + (size_t)(s - 1) * ld);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  mfma_d4 acc[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) acc[q] = mfma_d4{0.0, 0.0, 0.0, 0.0};
  // this lane's column within each 16-column group, and its tile offsets
  int coff[NG];
  bool cin[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    const int c = 16 * g + (lane & 15);
    cin[g] = c < 2 * NL;
    coff[g] = cin[g] ? 2 * ((c >> 1) * TP) + (c & 1) : 0;
  }
  const int krow = lane >> 4;                // row within a group of four
  constexpr int RPW = TS / W;                // rows per wave in a full block

  // Row-block bounds come through the scalar cache one block ahead (the
  // partition is read-only), so a block's fetch never waits for them.
  typedef const __attribute__((address_space(4))) int32_t kint;
  kint* const kblk = (kint*)(DIA ? A.dia.blk : A.blk);
  kint* const kblke = (kint*)A.blke;
  struct Rows {
    int32_t r0, nr, e0, ne, rs, re;
  };
  auto bounds = [&](int32_t b, Rows& r) {
    r.r0 = kblk[b];
    r.nr = kblk[b + 1] - r.r0;
    if constexpr (DIA) {
      r.e0 = r.ne = 0;
      ASSG_DCHECK(b >= 0 && b < A.dia.nblk && r.nr >= 1 && r.nr <= TS &&
                      (int64_t)r.r0 + r.nr <= A.n, 24);
      return;
    }
    r.e0 = kblke[b];
    r.ne = kblke[b + 1] - r.e0;
    ASSG_DCHECK(b >= 0 && b < A.nblk, 21);
    ASSG_DCHECK(r.r0 >= 0 && r.nr >= 1 && r.nr <= TS && (int64_t)r.r0 + r.nr <= A.n, 22);
    ASSG_DCHECK(r.e0 >= 0 && r.ne >= 0 && (int64_t)r.e0 + r.ne <= A.nnz &&
                    (r.ne <= SB_CAP || r.nr == 1), 23);
  };
  auto own_range = [&](Rows& r) {   // vector loads, consumed after the next drain
    r.rs = r.re = 0;
    if (!DIA && tid < r.nr) {
      r.rs = A.rp[(int64_t)r.r0 + tid] - r.e0;
      r.re = A.rp[(int64_t)r.r0 + tid + 1] - r.e0;
    }
  };
  constexpr int SMAX = (NC - 1) / 2;   // basis levels in the tile (sbar <= SMAX)
  constexpr int ND = 4 * SMAX;        // 64-row loads per block
  constexpr int NDW = (ND + W - 1) / W;
  constexpr int K = SB_CAP / NT;
  RowFetch<NT, SB_CAP> f;
  Rows cur{}, nxt{};
  if (b0 < b1) {
    bounds(b0, cur);
    own_range(cur);
    if (!DIA && cur.ne <= SB_CAP && cur.ne > 0) f.issue(A.ci, A.va, cur.e0, cur.ne);
    if (b0 + 1 < b1) bounds(b0 + 1, nxt);
  }
  for (int32_t b = b0; b < b1; ++b) {
    // CSR: the products first (their LDS buffer is the start of the tile),
    // then the block's basis pairs into the tile in 64-row loads; DIA: the
    // tile loads, then each thread's row of A P_{sbar-1}.  Levels past sbar
    // and lanes past the block read zeros; 64-row chunks past the block are
    // not loaded (the Gram stops at the block's last 4-row group, which lies
    // in a loaded chunk).  Every wave waits for its own loads before the
    // barrier, so the tile is complete after it.
    const bool own = tid < cur.nr;
    double a = 0.0, unused;
    if constexpr (DIA) {
#pragma unroll
      for (int j = 0; j < NDW; ++j) {
        const int i = wave + j * W;
        if ((ND % W == 0 || i < ND) && ((i & 3) << 6) < cur.nr) {
          const int l = i >> 2, row = ((i & 3) << 6) + lane;
          const double2* src =
              (l < s && row < cur.nr) ? pairs + (size_t)l * ld + cur.r0 + row : g_zero_rows + lane;
          __builtin_amdgcn_global_load_lds(
              (const void*)src,
              (void __attribute__((address_space(3)))*)(tile + l * TP + ((i & 3) << 6)), 16, 0,
              2);   // nt: streamed once
        }
      }
      if (own) {   // plain gathers: the wave shift measured slower here
        const kDiaSys& R = *(const kDiaSys*)(A.dia.sys + sys);
        dia_row<1, false>(A.dia.sys + sys, A.dia.val, SrcP{xsrc}, (int64_t)cur.r0 + tid - R.row0,
                          true, a, unused);
      }
    } else {
      if (cur.ne <= SB_CAP) {
        if (cur.ne > 0) {
          double gx[K];
#pragma unroll
          for (int k = 0; k < K; ++k) gx[k] = xsrc[2 * (int64_t)f.c[k]];
#pragma unroll
          for (int k = 0; k < K; ++k) {
            const int32_t e = tid + NT * k;
            if (e < cur.ne) prod[e] = f.a[k] * gx[k];
          }
        }
        __syncthreads();
        if (own)
          for (int32_t e = cur.rs; e < cur.re; ++e) a += prod[e];
      } else {
        long_row<1, NT>(A.ci, A.va, SrcP{xsrc}, cur.e0, cur.ne, red, a, unused);
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < NDW; ++j) {
        const int i = wave + j * W;
        if ((ND % W == 0 || i < ND) && ((i & 3) << 6) < cur.nr) {
          const int l = i >> 2, row = ((i & 3) << 6) + lane;
          const double2* src =
              (l < s && row < cur.nr) ? pairs + (size_t)l * ld + cur.r0 + row : g_zero_rows + lane;
          __builtin_amdgcn_global_load_lds(
              (const void*)src,
              (void __attribute__((address_space(3)))*)(tile + l * TP + ((i & 3) << 6)), 16, 0,
              2);   // nt: streamed once
        }
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid < TS) {
      double y = 0.0;
      if (own) {
        y = a - th * tile[(s - 1) * TP + tid].x;
        if (mu != 0.0) y -= mu * tile[(s - 2) * TP + tid].x;
        y = y / ga;
        stnt(plast + (int64_t)cur.r0 + tid, y);
      }
      tile[s * TP + tid] = make_double2(y, 0.0);
      // the top level is not loaded; the products may have left values in it
      if (s < SMAX) tile[SMAX * TP + tid] = make_double2(0.0, 0.0);
    }
    const int nrb = cur.nr;
    if (b + 1 < b1) {
      cur = nxt;
      own_range(cur);
      if (!DIA && cur.ne <= SB_CAP && cur.ne > 0) f.issue(A.ci, A.va, cur.e0, cur.ne);
      if (b + 2 < b1) bounds(b + 2, nxt);
    }
    __syncthreads();
    // Gram on the matrix cores, four rows per step: the block's 4-row groups
    // are dealt to the waves in turn, up to its last group (rows past the
    // block within it are zero in the tile), so a short block (many
    // nonzeros per row) keeps every wave busy
#pragma unroll
    for (int k = 0; k < RPW / 4; ++k) {
      const int r = 4 * (wave + k * W);
      if (r < nrb) {
        double v[NG];
#pragma unroll
        for (int g = 0; g < NG; ++g) v[g] = cin[g] ? tcol[coff[g] + 2 * (r + krow)] : 0.0;
        int q = 0;
#pragma unroll
        for (int gi = 0; gi < NG; ++gi)
#pragma unroll
          for (int gj = gi; gj < NG; ++gj, ++q)
            acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[gi], v[gj], acc[q], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // the waves' accumulators through the LDS, added in wave order, then the
  // unique entries (a <= b, row-major upper triangle) as this chunk's partials
  constexpr int NP = NC * (NC + 1) / 2;
  constexpr int NPT = (NP + NT - 1) / NT;
  int at[NPT];
  double sum[NPT];
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    sum[k] = 0.0;
    at[k] = -1;
    const int p = tid + k * NT;
    if (p < NP) {
      int ia = 0, qq = p;
      while (qq >= NC - ia) {
        qq -= NC - ia;
        ++ia;
      }
      const int ib = ia + qq;
      const int gi = ia >> 4, gj = ib >> 4, i = ia & 15, j = ib & 15;
      const int q = gi * NG - (gi * (gi - 1)) / 2 + (gj - gi);
      at[k] = (q * 4 + (i >> 2)) * 64 + j + 16 * (i & 3);   // D[i][j]: lane j + 16 (i % 4), reg i / 4
    }
  }
  for (int w0 = 0; w0 < W; w0 += WR) {
    if (wave >= w0 && wave < w0 + WR) {
#pragma unroll
      for (int q = 0; q < NB; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) lds[(((wave - w0) * NB + q) * 4 + e) * 64 + lane] = acc[q][e];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NPT; ++k)
      if (at[k] >= 0)
        for (int w = 0; w < WR; ++w) sum[k] += lds[w * NB * 256 + at[k]];
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < NPT; ++k)
    if (at[k] >= 0)
      partials[(size_t)(tid + k * NT) * (DIA ? A.dia.nchunk : A.nchunk) + chunk] = sum[k];
}

template <int NC>
constexpr int gram_waves() { return 4; }

template <int NC>
static int last_gram_blocks_nc(int cus) {
  constexpr int W = gram_waves<NC>();
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_last_gram<NC, W, false>, 64 * W, 0) !=
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

void launch_last_gram(hipStream_t s, const Ctl* ctl, int sigma, const CsrView& A,
                      const double2* pairs, double* plast, int64_t ld, double* partials) {
  ASSG_SIGMA_SWITCH(sigma, {
    constexpr int W = gram_waves<NC>();
    if (A.dia.nd > 0)
      hipLaunchKernelGGL((k_last_gram<NC, W, true>), dim3(A.dia.nchunk), dim3(64 * W), 0, s, ctl,
                         A, pairs, plast, ld, partials);
    else
      hipLaunchKernelGGL((k_last_gram<NC, W, false>), dim3(A.nchunk), dim3(64 * W), 0, s, ctl, A,
                         pairs, plast, ld, partials);
  });
}

// G[a][b] = G[b][a] of system blockIdx.y = the sum of its chunks' partials
// of entry blockIdx.x, fixed order.
template <int NC>
__global__ __launch_bounds__(256) void k_gram_reduce(Ctl* __restrict__ ctls, CsrView A,
                                                     const double* __restrict__ partials) {
  Ctl* ctl = ctls + blockIdx.y;
  if (ctl->status != ST_RUNNING) return;
  __shared__ double sh[4];
  const int p = blockIdx.x;
  const int32_t c0 = A.sys_chunk[blockIdx.y], c1 = A.sys_chunk[blockIdx.y + 1];
  const double* __restrict__ src = partials + (size_t)p * A.nchunk;
  double s = 0.0;
  for (int32_t i = c0 + threadIdx.x; i < c1; i += 256) s += src[i];
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

void launch_gram_reduce(hipStream_t s, Ctl* ctl, int sigma, const CsrView& A,
                        const double* partials) {
  // the partials are laid out over the chunks of the storage the last sweep read
  CsrView v = A;
  if (A.dia.nd > 0) {
    v.nchunk = A.dia.nchunk;
    v.cblk = A.dia.cblk;
    v.csys = A.dia.csys;
    v.sys_chunk = A.dia.sys_chunk;
  }
  ASSG_SIGMA_SWITCH(sigma, hipLaunchKernelGGL(k_gram_reduce<NC>, dim3(NC * (NC + 1) / 2, v.nsys),
                                              dim3(256), 0, s, ctl, v, partials));
}

// -------------------------------------------------------------- recovery
// (2.6): x += Y x', p = Y p', r = Y r' over the 2 s_k + 1 columns that carry
// coordinates after s_k inner steps ((2.1): P_0..P_{s_k}, R_0..R_{s_k-1});
// (p, r) overwrite basis level 0 row by row (each row is read before it is
// written by the same thread).  One workgroup per row block, one row per
// thread, all basis loads of a row issued together.
__global__ __launch_bounds__(256) void k_recover(const Ctl* __restrict__ ctls, CsrView A,
                                                 double2* __restrict__ pairs,
                                                 const double* __restrict__ plast, int64_t ld,
                                                 double* __restrict__ x) {
  const int32_t bb = xcd_logical(blockIdx.x, gridDim.x);
  if (bb >= A.nblk) return;
  const Ctl* ctl = ctls + block_sys(A, bb);
  if (ctl->status != ST_RUNNING || ctl->skip_recover) return;
  const int32_t r0 = A.blk[bb], nr = A.blk[bb + 1] - r0;
  if ((int)threadIdx.x >= nr) return;
  const int64_t row = (int64_t)r0 + threadIdx.x;
  const int sk = ctl->sk, sbar = ctl->sbar;
  const double* __restrict__ plevel =
      (sk == sbar) ? plast : reinterpret_cast<const double*>(pairs + (size_t)sk * ld);
  const int pstride = (sk == sbar) ? 1 : 2;
  const double yl = ldnt(plevel + pstride * row);
  const double x0 = ldnt(x + row);
  double xs = 0.0, ps = 0.0, rs = 0.0;
  for (int l = 0; l < sk; ++l) {
    const double2 y = ldnt2(pairs + (size_t)l * ld + row);
    xs = fma(ctl->cx[2 * l], y.x, xs);
    xs = fma(ctl->cx[2 * l + 1], y.y, xs);
    ps = fma(ctl->cp[2 * l], y.x, ps);
    ps = fma(ctl->cp[2 * l + 1], y.y, ps);
    rs = fma(ctl->cr[2 * l], y.x, rs);
    rs = fma(ctl->cr[2 * l + 1], y.y, rs);
  }
  xs = fma(ctl->cx[2 * sk], yl, xs);
  ps = fma(ctl->cp[2 * sk], yl, ps);
  rs = fma(ctl->cr[2 * sk], yl, rs);
  stnt(x + row, x0 + xs);
  stnt2(pairs + row, make_double2(ps, rs));
}

void launch_recover(hipStream_t s, const Ctl* ctl, const CsrView& A, double2* pairs,
                    const double* plast, int64_t ld, double* x) {
  hipLaunchKernelGGL(k_recover, dim3(block_grid(A, 1 << 30)), dim3(256), 0, s, ctl, A, pairs,
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
    if (trace && ctl->record_trace && k < ctl->trace_cap) trace[k].relres_true = rel;
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

// One chunk per workgroup (a small grid: this kernel usually exits at once,
// and an empty launch of one workgroup per row block costs ~15 us).
__global__ __launch_bounds__(256) void k_check(const Ctl* ctls, CsrView A,
                                               const double* __restrict__ b,
                                               const double* __restrict__ x,
                                               double* __restrict__ part, int measure_only) {
  __shared__ double prod[SB_CAP];
  __shared__ double red[4];
  int32_t b0, b1, sys;
  const int32_t c = chunk_of(A, b0, b1, sys);
  const Ctl* ctl = ctls + sys;
  if (!measure_only && (ctl->status != ST_RUNNING || !ctl->candidate)) return;
  double my = 0.0;
  for (int32_t bb = b0; bb < b1; ++bb) {
    const BlockRows br(A, bb);
    double bi = 0.0;
    if (br.own) bi = b[br.row];
    double ax, unused;
    stream_rows<1, 256, SB_CAP>(A.ci, A.va, Src1{x}, br.e0, br.ne, br.rs, br.re, br.own, prod,
                                red, ax, unused);
    if (br.own) {
      const double ri = bi - ax;
      my = fma(ri, ri, my);
    }
    __syncthreads();
  }
  my = block_sum<256>(my, red);
  if (threadIdx.x == 0) part[c] = my;
}

// End of an outer loop (or HSCG iteration) of system blockIdx.x: the true
// relative residual when a candidate was flagged, then the commit.
__global__ __launch_bounds__(1024) void k_fin_check(Ctl* ctls, assg_trace_t* trace, CsrView A,
                                                    const double* __restrict__ part,
                                                    int measure_only) {
  __shared__ double sh[16];
  const int i = blockIdx.x;
  Ctl* ctl = ctls + i;
  if (!measure_only && ctl->status != ST_RUNNING) return;
  const bool checked = measure_only || ctl->candidate;
  const int32_t c0 = A.sys_chunk[i], c1 = A.sys_chunk[i + 1];
  double t = 0.0;
  if (checked) t = finish_sum<1024>(part + c0, c1 - c0, sh);
  if (threadIdx.x == 0) {
    // b = 0 (x = 0, nothing iterated): the residual is exactly 0
    const double rel = !checked ? -1.0 : (ctl->nb > 0.0 ? sqrt(t) / ctl->nb : (t == 0.0 ? 0.0 : INFINITY));
    if (measure_only)
      ctl->relres_true = rel;
    else
      commit_loop(ctl, trace, checked, rel);
  }
}

void launch_check(hipStream_t s, Ctl* ctl, assg_trace_t* trace, const CsrView& A,
                  const double* b, const double* x, double* part, int measure_only) {
  hipLaunchKernelGGL(k_check, dim3(A.nchunk), dim3(256), 0, s, ctl, A, b, x, part, measure_only);
  hipLaunchKernelGGL(k_fin_check, dim3(A.nsys), dim3(1024), 0, s, ctl, A.nsys == 1 ? trace : nullptr,
                     A, part, measure_only);
}

// ------------------------------------------------------------------ HSCG
// Algorithm 1, one iteration = seven launches over the row blocks (each
// grid sum finished by a one-workgroup kernel in index order):
//  k_h_spmv + k_fin_alpha    w = A p and the p^T w sum -> alpha;
//  k_h_update + k_fin_beta   x += alpha p, r -= alpha w and the r^T r sum
//                            -> beta;
//  k_h_dir                   p = r + beta p;
//  k_check + k_fin_check     the stopping test (the true residual when the
//                            updated one reached tol).
__global__ __launch_bounds__(256) void k_h_init(Ctl* ctl, CsrView A, const double* __restrict__ b,
                                                const double* __restrict__ x,
                                                double* __restrict__ r, double* __restrict__ p,
                                                double* __restrict__ part) {
  __shared__ double prod[SB_CAP];
  __shared__ double red[4];
  const int32_t bb = xcd_logical(blockIdx.x, gridDim.x);
  double mb = 0.0, mr = 0.0;
  if (bb < A.nblk) {
    const BlockRows br(A, bb);
    double bi = 0.0;
    if (br.own) bi = b[br.row];
    double ax, unused;
    stream_rows<1, 256, SB_CAP>(A.ci, A.va, Src1{x}, br.e0, br.ne, br.rs, br.re, br.own, prod,
                                red, ax, unused);
    if (br.own) {
      const double ri = bi - ax;
      r[br.row] = ri;
      p[br.row] = ri;
      mb = bi * bi;
      mr = ri * ri;
    }
  }
  mb = block_sum<256>(mb, red);
  mr = block_sum<256>(mr, red);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = mb;
    part[gridDim.x + blockIdx.x] = mr;
  }
}

__global__ __launch_bounds__(1024) void k_fin_h_init(Ctl* ctl, const double* __restrict__ part,
                                                     int n) {
  __shared__ double sh[16];
  const double tb = finish_sum<1024>(part, n, sh);
  const double tr = finish_sum<1024>(part + n, n, sh);
  if (threadIdx.x == 0) {
    ctl->nb = sqrt(tb);
    ctl->h_rho = tr;
    ctl->h_beta = 0.0;
  }
}

void launch_h_init(hipStream_t s, Ctl* ctl, const CsrView& A, const double* b, const double* x,
                   double* r, double* p, double* part) {
  const int g = block_grid(A, 1 << 30);
  hipLaunchKernelGGL(k_h_init, dim3(g), dim3(256), 0, s, ctl, A, b, x, r, p, part);
  hipLaunchKernelGGL(k_fin_h_init, dim3(1), dim3(1024), 0, s, ctl, part, g);
}

__global__ __launch_bounds__(256) void k_h_spmv(const Ctl* ctl, CsrView A,
                                                const double* __restrict__ p,
                                                double* __restrict__ w,
                                                double* __restrict__ part) {
  if (ctl->status != ST_RUNNING || ctl->pending != ST_RUNNING) return;
  __shared__ double prod[SB_CAP];
  __shared__ double red[4];
  const int32_t bb = xcd_logical(blockIdx.x, gridDim.x);
  double my = 0.0;
  if (bb < A.nblk) {
    const BlockRows br(A, bb);
    double pi = 0.0;
    if (br.own) pi = p[br.row];
    double v, unused;
    stream_rows<1, 256, SB_CAP>(A.ci, A.va, Src1{p}, br.e0, br.ne, br.rs, br.re, br.own, prod,
                                red, v, unused);
    if (br.own) {
      stnt(w + br.row, v);
      my = pi * v;
    }
  }
  my = block_sum<256>(my, red);
  if (threadIdx.x == 0) part[blockIdx.x] = my;
}

__global__ __launch_bounds__(1024) void k_fin_alpha(Ctl* ctl, const double* __restrict__ part,
                                                    int n) {
  if (ctl->status != ST_RUNNING || ctl->pending != ST_RUNNING) return;
  __shared__ double sh[16];
  const double pw = finish_sum<1024>(part, n, sh);
  if (threadIdx.x == 0) {
    if (!(pw > 0.0) || !isfinite(pw))
      ctl->pending = isfinite(pw) ? ASSG_BREAKDOWN : ASSG_DIVERGED;
    else
      ctl->h_alpha = ctl->h_rho / pw;
  }
}

// w = A p and the p^T w partials from the diagonal storage.
__global__ __launch_bounds__(256) void k_h_spmv_dia(const Ctl* ctl, CsrView A,
                                                    const double* __restrict__ p,
                                                    double* __restrict__ w,
                                                    double* __restrict__ part) {
  if (ctl->status != ST_RUNNING || ctl->pending != ST_RUNNING) return;
  __shared__ double red[4];
  int32_t sys;
  const int32_t bb = dia_block(A, sys);
  const int64_t i = bb < 0 ? -1 : (int64_t)A.dia.blk[bb] + threadIdx.x;
  double my = 0.0;
  if (bb >= 0) {   // every lane: rows past the block gather for their neighbours
    const bool own = i < A.dia.blk[bb + 1];
    const kDiaSys& R = *(const kDiaSys*)(A.dia.sys + sys);
    double v, unused;
    dia_row<1, true>(A.dia.sys + sys, A.dia.val, Src1{p}, i - R.row0, own, v, unused);
    if (own) {
      stnt(w + i, v);
      my = p[i] * v;
    }
  }
  my = block_sum<256>(my, red);
  if (threadIdx.x == 0) part[blockIdx.x] = my;
}

void launch_h_spmv(hipStream_t s, Ctl* ctl, const CsrView& A, const double* p, double* w,
                   double* part) {
  if (A.dia.nd > 0) {
    const int g = dia_grid(A);
    hipLaunchKernelGGL(k_h_spmv_dia, dim3(g), dim3(256), 0, s, ctl, A, p, w, part);
    hipLaunchKernelGGL(k_fin_alpha, dim3(1), dim3(1024), 0, s, ctl, part, g);
    return;
  }
  const int g = block_grid(A, 1 << 30);
  hipLaunchKernelGGL(k_h_spmv, dim3(g), dim3(256), 0, s, ctl, A, p, w, part);
  hipLaunchKernelGGL(k_fin_alpha, dim3(1), dim3(1024), 0, s, ctl, part, g);
}

// p = r + beta p, one row per thread.
__global__ __launch_bounds__(256) void k_h_dir(const Ctl* ctl, CsrView A,
                                               const double* __restrict__ r,
                                               double* __restrict__ p) {
  if (ctl->status != ST_RUNNING || ctl->pending != ST_RUNNING) return;
  const int32_t bb = xcd_logical(blockIdx.x, gridDim.x);
  if (bb >= A.nblk) return;
  const int32_t r0 = A.blk[bb], nr = A.blk[bb + 1] - r0;
  if ((int)threadIdx.x >= nr) return;
  const int64_t row = (int64_t)r0 + threadIdx.x;
  stnt(p + row, ldnt(r + row) + ctl->h_beta * ldnt(p + row));
}

void launch_h_dir(hipStream_t s, const Ctl* ctl, const CsrView& A, const double* r, double* p) {
  hipLaunchKernelGGL(k_h_dir, dim3(block_grid(A, 1 << 30)), dim3(256), 0, s, ctl, A, r, p);
}

__global__ __launch_bounds__(256) void k_h_update(const Ctl* ctl, CsrView A,
                                                  double* __restrict__ x, double* __restrict__ r,
                                                  const double* __restrict__ p,
                                                  const double* __restrict__ w,
                                                  double* __restrict__ part) {
  if (ctl->status != ST_RUNNING || ctl->pending != ST_RUNNING) return;
  __shared__ double red[4];
  const double alpha = ctl->h_alpha;
  const int32_t bb = xcd_logical(blockIdx.x, gridDim.x);
  double my = 0.0;
  if (bb < A.nblk) {
    const int32_t r0 = A.blk[bb], nr = A.blk[bb + 1] - r0;
    if ((int)threadIdx.x < nr) {
      const int64_t row = (int64_t)r0 + threadIdx.x;
      const double pi = ldnt(p + row), wi = ldnt(w + row), xi = ldnt(x + row), ri = ldnt(r + row);
      stnt(x + row, xi + alpha * pi);
      const double rn = ri - alpha * wi;
      stnt(r + row, rn);
      my = rn * rn;
    }
  }
  my = block_sum<256>(my, red);
  if (threadIdx.x == 0) part[blockIdx.x] = my;
}

__global__ __launch_bounds__(1024) void k_fin_beta(Ctl* ctl, const double* __restrict__ part,
                                                   int n) {
  if (ctl->status != ST_RUNNING || ctl->pending != ST_RUNNING) return;
  __shared__ double sh[16];
  const double rr = finish_sum<1024>(part, n, sh);
  if (threadIdx.x == 0) {
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

void launch_h_update(hipStream_t s, Ctl* ctl, const CsrView& A, double* x, double* r,
                     const double* p, const double* w, double* part) {
  const int g = block_grid(A, 1 << 30);
  hipLaunchKernelGGL(k_h_update, dim3(g), dim3(256), 0, s, ctl, A, x, r, p, w, part);
  hipLaunchKernelGGL(k_fin_beta, dim3(1), dim3(1024), 0, s, ctl, part, g);
}

// ----------------------------------------------------- basis/Gram helpers
// ------------------------------------------- differentiation: alpha u v^T
// One row block per workgroup: the owner of each row writes its (local) row
// number for the row's nonzeros into LDS, then the nonzeros are visited in
// order with coalesced column loads and stores.
__global__ __launch_bounds__(256) void k_outer_pattern(CsrView A, const double* __restrict__ u,
                                                       const double* __restrict__ v, double alpha,
                                                       double* __restrict__ out) {
  __shared__ uint8_t rowof[SB_CAP];
  __shared__ double su[SB_ROWS];
  int32_t b0, b1;
  block_range(A.nblk, b0, b1);
  for (int32_t b = b0; b < b1; ++b) {
    const BlockRows br(A, b);
    const int t = threadIdx.x;
    if (br.ne <= SB_CAP) {
      if (br.own) {
        su[t] = alpha * u[br.row];
        for (int32_t e = br.rs; e < br.re; ++e) rowof[e] = (uint8_t)t;
      }
      __syncthreads();
      for (int32_t e = t; e < br.ne; e += 256)
        out[br.e0 + e] = su[rowof[e]] * v[A.ci[br.e0 + e]];
    } else {
      const double ui = alpha * u[br.r0];
      for (int32_t e = t; e < br.ne; e += 256)
        out[br.e0 + e] = ui * v[A.ci[br.e0 + e]];
    }
    __syncthreads();
  }
}

void launch_outer_pattern(hipStream_t s, const CsrView& A, const double* u, const double* v,
                          double alpha, double* out) {
  hipLaunchKernelGGL(k_outer_pattern, dim3(block_grid(A, 1 << 30)), dim3(256), 0, s, A, u, v,
                     alpha, out);
}

// ---------------------------------------------------- diagonal storage
// *flag = 1 (every offending thread stores the same value) unless each
// row's column offsets c - i are a strictly increasing subsequence of the
// ascending R.off (sorted, duplicate-free rows whose entries all lie on the
// diagonals).
__global__ __launch_bounds__(256) void k_dia_probe(const int32_t* __restrict__ rp,
                                                   const int32_t* __restrict__ ci, DiaSys R,
                                                   int32_t* __restrict__ flag) {
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < R.n && !bad;
       i += (int64_t)gridDim.x * 256) {
    int d = 0;
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
      const int64_t off = (int64_t)ci[e] - i;
      while (d < R.nd && R.off[d] < off) ++d;
      if (d >= R.nd || R.off[d] != off) {
        bad = true;
        break;
      }
      ++d;
    }
  }
  if (bad) flag[0] = 1;
}

void launch_dia_probe(hipStream_t s, const int32_t* rp, const int32_t* ci, const DiaSys& R,
                      int32_t* flag) {
  const int64_t g = ((int64_t)R.n + 255) / 256;
  if (g > 0)
    hipLaunchKernelGGL(k_dia_probe, dim3((unsigned)(g < 4096 ? g : 4096)), dim3(256), 0, s, rp,
                       ci, R, flag);
}

// val[d * n + i] = A[i][i + off[d]], or 0.  One workgroup per 64 rows:
// their CSR entries (at most 32 per row, which the probe has checked) come
// into the LDS in coalesced loads, then four threads per row walk the row's
// entries against the diagonals in order, each writing every fourth
// diagonal (sixteen consecutive rows per wave and diagonal).
__global__ __launch_bounds__(256) void k_dia_fill(const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ ci,
                                                  const double* __restrict__ va, DiaSys R,
                                                  double* __restrict__ val) {
  constexpr int RB = 64;
  __shared__ int32_t sc[RB * DIA_MAX];
  __shared__ double sv[RB * DIA_MAX];
  const int64_t n = R.n;
  const int64_t r0 = (int64_t)blockIdx.x * RB;
  if (r0 >= n) return;
  const int64_t r1 = r0 + RB < n ? r0 + RB : n;
  const int32_t e0 = rp[r0];
  const int32_t ne = rp[r1] - e0;
  ASSG_DCHECK(ne >= 0 && ne <= RB * DIA_MAX, 41);
  for (int32_t e = threadIdx.x; e < ne; e += 256) {
    sc[e] = ldnt(ci + e0 + e);
    sv[e] = ldnt(va + e0 + e);
  }
  __syncthreads();
  const int q = threadIdx.x & 3;
  const int64_t i = r0 + (threadIdx.x >> 2);
  if (i >= r1) return;
  int32_t e = rp[i] - e0;
  const int32_t e1 = rp[i + 1] - e0;
  for (int d = 0; d < R.nd; ++d) {
    double v = 0.0;
    if (e < e1 && (int64_t)sc[e] - i == R.off[d]) v = sv[e++];
    if ((d & 3) == q) stnt(val + (int64_t)d * n + i, v);
  }
}

void launch_dia_fill(hipStream_t s, const int32_t* rp, const int32_t* ci, const double* va,
                     const DiaSys& R, double* val) {
  const int64_t g = ((int64_t)R.n + 63) / 64;
  if (g > 0)
    hipLaunchKernelGGL(k_dia_fill, dim3((unsigned)g), dim3(256), 0, s, rp, ci, va, R, val);
}

// *flag = 1 when a column index of ci[0, nnz) lies outside [0, n) (every
// offending thread stores the same value).
__global__ __launch_bounds__(256) void k_check_cols(const int32_t* __restrict__ ci, int64_t nnz,
                                                    int32_t n, int32_t* __restrict__ flag) {
  bool bad = false;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * 256) {
    const int32_t c = ldnt(ci + e);
    bad |= (c < 0) | (c >= n);
  }
  if (bad) flag[0] = 1;
}

void launch_check_cols(hipStream_t s, const int32_t* ci, int64_t nnz, int32_t n, int32_t* flag) {
  const int64_t g = (nnz + 255) / 256;
  if (g > 0)
    hipLaunchKernelGGL(k_check_cols, dim3((unsigned)(g < 4096 ? g : 4096)), dim3(256), 0, s, ci,
                       nnz, n, flag);
}

// dst[i] = src[i] + add (column indices of a system placed in a batch).
__global__ void k_offset_copy(const int32_t* __restrict__ src, int32_t* __restrict__ dst,
                              int64_t n, int32_t add) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = src[i] + add;
}

void launch_offset_copy(hipStream_t s, const int32_t* src, int32_t* dst, int64_t n, int32_t add) {
  const int64_t g = (n + 255) / 256;
  if (g > 0)
    hipLaunchKernelGGL(k_offset_copy, dim3((unsigned)g), dim3(256), 0, s, src, dst, n, add);
}

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

// The first failed check of a debug build since the last call (0: none, or
// a release build), cleared.
int debug_code_take_kernels(hipStream_t s) {
#ifdef ASSG_DEBUG
  int v = 0;
  if (hipMemcpyFromSymbolAsync(&v, HIP_SYMBOL(g_debug_code), sizeof(int), 0,
                               hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return -1;
  if (v != 0) {
    const int z = 0;
    if (hipMemcpyToSymbolAsync(HIP_SYMBOL(g_debug_code), &z, sizeof(int), 0,
                               hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return -1;
  }
  return v;
#else
  (void)s;
  return 0;
#endif
}

}  // namespace assg
