// Host-side launchers of the device kernels (kernels.hip, controller.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "assg.h"
#include "ctl.hpp"
#include "partition.hpp"

namespace assg {

// Diagonal storage of stencil matrices: every entry of a system lies on one
// of at most DIA_MAX diagonals (i, i + off[d]), offsets ascending, and the
// system's values are val[val0 + d * n + i] for its local row i (0 where A
// has no entry), so a row's products are added in column order as in the
// CSR kernels, and no column index or row pointer is read.  The row kernels
// take blocks of at most SB_ROWS rows that never straddle systems (blk,
// bsys), and the reduction chunks run over those blocks (cblk, csys,
// sys_chunk).  nd = 0: the matrix is read as CSR.  DIA_MAX: partition.hpp.
struct DiaSys {
  int64_t val0;              // first value of the system in the storage
  int64_t row0;              // first row of the system (0 for a single system)
  int32_t n;                 // rows
  int32_t nd;                // diagonals
  int32_t off[DIA_MAX];
};
struct DiaView {
  int32_t nd;                // the most diagonals of any system; 0: CSR
  const DiaSys* sys;         // one record per system
  const double* val;
  const int32_t* blk;        // nblk + 1 row starts
  const int32_t* bsys;       // nblk: system of each block (null: one system)
  int32_t nblk;
  const int32_t* cblk;       // nchunk + 1 first blocks
  const int32_t* csys;       // nchunk: system of each chunk (null: one system)
  const int32_t* sys_chunk;  // nsys + 1 first chunks
  int32_t nchunk;
};

// A matrix with its row-block partition.  A batch of independent systems
// is one block-diagonal matrix (systems' rows and columns concatenated);
// row blocks never straddle systems, and neither do the "chunks" (runs of
// consecutive row blocks) that the reduction kernels give one workgroup
// each.  A single solve is a batch of one: bsys and csys are null.
struct CsrView {
  int64_t n, nnz;
  const int32_t* rp;
  const int32_t* ci;
  const double* va;
  const int32_t* blk;        // nblk + 1 row starts of the row blocks
  const int32_t* blke;       // nblk + 1 nonzero starts (row_ptr[blk[b]])
  int32_t nblk;
  const int32_t* bsys;       // nblk: system of each row block (null: system 0)
  const int32_t* cblk;       // nchunk + 1: first row block of each chunk
  const int32_t* csys;       // nchunk: system of each chunk (null: system 0)
  const int32_t* sys_chunk;  // nsys + 1: first chunk of each system
  int32_t nchunk;            // a multiple of 8 (trailing chunks may be empty)
  int32_t nsys;
  DiaView dia;               // diagonal storage (dia.nd = 0: none)
};

void launch_spmv(hipStream_t s, const CsrView& A, const double* x, double* y);


// Kernels of the s-step path take the control blocks of all systems
// (ctl[i] for system i) and run every system of the batch.

// r = b - A x, pairs[0] = (r, r), ctl[i].nb = ||b_i||.
void launch_setup(hipStream_t s, Ctl* ctl, const CsrView& A, const double* b, const double* x,
                  double2* pairs, double* part);

// Two-chain sweep producing basis level ``level`` (1 <= level < sbar).
void launch_sweep(hipStream_t s, const Ctl* ctl, int level, const CsrView& A, double2* pairs,
                  int64_t ld);

// Last sweep (P chain, level sbar) fused with the Gram partial sums.
int last_gram_blocks(int sigma, int cus);
// One workgroup per chunk; partials[pair * nchunk + chunk].
void launch_last_gram(hipStream_t s, const Ctl* ctl, int sigma, const CsrView& A,
                      const double2* pairs, double* plast, int64_t ld, double* partials);
void launch_gram_reduce(hipStream_t s, Ctl* ctl, int sigma, const CsrView& A,
                        const double* partials);

// One workgroup per system; the trace is recorded for a batch of one only.
void launch_controller(hipStream_t s, Ctl* ctl, assg_trace_t* trace, int sigma, int nsys);

void launch_recover(hipStream_t s, const Ctl* ctl, const CsrView& A, double2* pairs,
                    const double* plast, int64_t ld, double* x);

// True relative residual when the loop's updated residual reached tol, then
// commit of the loop's outcome.  With ``measure_only`` it only stores
// ||b - A x|| / ||b|| in ctl->relres_true.
void launch_check(hipStream_t s, Ctl* ctl, assg_trace_t* trace, const CsrView& A,
                  const double* b, const double* x, double* part, int measure_only);

// HSCG (Algorithm 1): k_h_spmv forms w = A p and p^T w (-> alpha),
// k_h_update x += alpha p, r -= alpha w and r^T r (-> beta), k_h_dir
// p = r + beta p.
void launch_h_init(hipStream_t s, Ctl* ctl, const CsrView& A, const double* b, const double* x,
                   double* r, double* p, double* part);
void launch_h_spmv(hipStream_t s, Ctl* ctl, const CsrView& A, const double* p, double* w,
                   double* part);
void launch_h_dir(hipStream_t s, const Ctl* ctl, const CsrView& A, const double* r, double* p);
void launch_h_update(hipStream_t s, Ctl* ctl, const CsrView& A, double* x, double* r,
                     const double* p, const double* w, double* part);

// out[k] = alpha u[row(k)] v[col(k)] on A's pattern.
void launch_outer_pattern(hipStream_t s, const CsrView& A, const double* u, const double* v,
                          double alpha, double* out);

// Diagonal storage of one system R (rows of its own CSR arrays): *flag = 1
// unless every row's column offsets form a strictly increasing subsequence
// of R.off (flag cleared by the caller); the fill writes the system's values
// val[d * R.n + i] (val: the storage at R.val0; every position, 0 where A
// has no entry) from the CSR values.
void launch_dia_probe(hipStream_t s, const int32_t* rp, const int32_t* ci, const DiaSys& R,
                      int32_t* flag);
void launch_dia_fill(hipStream_t s, const int32_t* rp, const int32_t* ci, const double* va,
                     const DiaSys& R, double* val);

// *flag = 1 if some ci[e], e < nnz, is outside [0, n) (flag cleared by the caller).
void launch_check_cols(hipStream_t s, const int32_t* ci, int64_t nnz, int32_t n, int32_t* flag);

// dst[i] = src[i] + add, i < n (batch assembly).
void launch_offset_copy(hipStream_t s, const int32_t* src, int32_t* dst, int64_t n, int32_t add);

// Helpers of assg_basis_gram.
void launch_pair_init(hipStream_t s, int64_t n, const double* p, const double* r, double2* pairs);
void launch_export_Y(hipStream_t s, int64_t n, int sbar, const double2* pairs,
                     const double* plast, int64_t ld, double* Y);

// Debug builds (-DASSG_DEBUG): the code of the first failed kernel check
// since the last call, per translation unit (0: none; always 0 in release
// builds; -1: reading it failed), cleared.
int debug_code_take_kernels(hipStream_t s);
int debug_code_take_controller(hipStream_t s);

}  // namespace assg
