// Row-block and reduction-chunk partitions (see partition.hpp).
#include "partition.hpp"

#include <algorithm>
#include <cmath>

namespace assg {

void make_blocks(const int32_t* rp, int64_t n, std::vector<int32_t>& blk, int rows, int cap) {
  blk.clear();
  blk.push_back(0);
  int64_t r = 0;
  while (r < n) {
    const int64_t r0 = r;
    ++r;                                    // a block always takes its first row
    if ((int64_t)rp[r] - rp[r0] <= cap)
      while (r < n && r - r0 < rows && (int64_t)rp[r + 1] - rp[r0] <= cap) ++r;
    blk.push_back((int32_t)r);
  }
}

void make_chunks(const std::vector<int32_t>& sys_blk, int target, std::vector<int32_t>& cblk,
                 std::vector<int32_t>& csys, std::vector<int32_t>& sys_chunk) {
  const int nsys = (int)sys_blk.size() - 1;
  const int64_t nblk = sys_blk[nsys];
  cblk.clear();
  csys.clear();
  sys_chunk.assign(1, 0);
  for (int i = 0; i < nsys; ++i) {
    const int64_t b0 = sys_blk[i], nb = sys_blk[i + 1] - b0;
    int64_t k = (nblk > 0) ? (nb * target + nblk / 2) / nblk : 1;
    if (k < 1) k = 1;
    if (k > nb && nb > 0) k = nb;
    for (int64_t c = 0; c < k; ++c) {
      cblk.push_back((int32_t)(b0 + nb * c / k));
      csys.push_back(i);
    }
    sys_chunk.push_back((int32_t)cblk.size());
  }
  while (cblk.size() % NXCD) {
    cblk.push_back((int32_t)nblk);
    csys.push_back(nsys - 1);
  }
  cblk.push_back((int32_t)nblk);
}

void dia_sample_rows(int64_t n, std::vector<int64_t>& rows) {
  rows.clear();
  for (int k = 0; k < DIA_SAMPLE; ++k) {
    const double f = std::fmod(0.5 + 0.6180339887498949 * k, 1.0);
    const int64_t i = (int64_t)(f * (double)n);
    rows.push_back(i < n - 1 ? i : n - 1);
  }
}

const char* dia_offsets(std::vector<int64_t>& offs, int64_t max_row, int64_t n, int64_t nnz,
                        bool check_fill) {
  if (max_row > DIA_MAX) return "a row has more than 32 entries";
  std::sort(offs.begin(), offs.end());
  offs.erase(std::unique(offs.begin(), offs.end()), offs.end());
  if (offs.empty() || (int64_t)offs.size() > DIA_MAX) return "more than 32 diagonals";
  if (check_fill && (double)offs.size() * (double)n > 1.15 * (double)nnz)
    return "the diagonals hold more than 15% more positions than A has entries";
  return nullptr;
}

size_t reduce_doubles(int32_t nblk) {
  const size_t g = ((size_t)nblk + NXCD - 1) / NXCD * NXCD;
  return 2 * g + 64;
}

}  // namespace assg
