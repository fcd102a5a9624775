// Row-block and reduction-chunk partitions (see partition.hpp).
#include "partition.hpp"

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

size_t reduce_doubles(int32_t nblk) {
  const size_t g = ((size_t)nblk + NXCD - 1) / NXCD * NXCD;
  return 2 * g + 64;
}

}  // namespace assg
