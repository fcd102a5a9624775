// Row-block and reduction-chunk partitions of a CSR matrix (host code, no
// HIP): the work units of the CSR-stream kernels and of the grid
// reductions.  Plain C++ so that it can also be built and checked on its own.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace assg {

constexpr int NXCD = 8;          // MI355X: 8 XCDs, workgroups dispatched round-robin

// Row blocks of the CSR-stream kernels: at most SB_ROWS rows and SB_CAP
// nonzeros each, except single rows longer than SB_CAP.
constexpr int SB_ROWS = 256;
constexpr int SB_CAP = 2048;

// Greedy row-block partition of rows [0, n) of the CSR row pointers
// ``row_ptr`` (n + 1 entries): rows are appended while a block has fewer
// than ``rows`` rows and at most ``cap`` (<= SB_CAP) nonzeros; a row longer
// than ``cap`` is a block of its own.  blk receives nblk + 1 row starts.
void make_blocks(const int32_t* row_ptr, int64_t n, std::vector<int32_t>& blk,
                 int rows = SB_ROWS, int cap = SB_CAP);

// Chunks over the row blocks of each system (sys_blk: nsys + 1 block
// starts): about ``target`` chunks in all, in proportion to each system's
// blocks, at least one per system, padded with empty chunks to a multiple
// of NXCD.  cblk: first block of each chunk (+ the end), csys: system of
// each chunk, sys_chunk: first chunk of each system (+ the end).
void make_chunks(const std::vector<int32_t>& sys_blk, int target, std::vector<int32_t>& cblk,
                 std::vector<int32_t>& csys, std::vector<int32_t>& sys_chunk);

// Per-workgroup partial sums of the grid reductions over the row-block grid
// (two sums for the HSCG start).
size_t reduce_doubles(int32_t nblk);

// Diagonal storage: at most DIA_MAX diagonals per system.
constexpr int DIA_MAX = 32;
constexpr int DIA_SAMPLE = 64;

// The DIA_SAMPLE rows of [0, n) whose column offsets are the candidate
// diagonals: fractions of n spread by the golden-ratio sequence (evenly
// spaced fractions land on the boundary planes of power-of-two grids, whose
// rows lack some diagonals).  n >= 1.
void dia_sample_rows(int64_t n, std::vector<int64_t>& rows);

// The candidate diagonals from the column offsets (column - row) of the
// sampled rows' entries: sorted and duplicate-free in ``offs``.  Returns
// nullptr when they qualify, else the reason: a sampled row with more than
// DIA_MAX entries (``max_row`` is the longest sampled row), no entries, more
// than DIA_MAX diagonals, or, with ``check_fill``, diagonals whose n
// positions each exceed the nnz entries of A by more than 15%.  Whether every
// row's entries lie on them is checked on the device afterwards.
const char* dia_offsets(std::vector<int64_t>& offs, int64_t max_row, int64_t n, int64_t nnz,
                        bool check_fill);

}  // namespace assg
