// Host driver for the row-block and chunk partitions (tests/test_partition.py
// builds it with g++ and the address and undefined-behaviour sanitizers).
// stdin: "B n rows cap" then n+1 row pointers  -> prints the block starts;
//        "C nsys target" then nsys+1 block starts -> prints cblk | csys | sys_chunk;
//        "D n nnz check_fill" then n+1 row pointers and nnz column indices
//          -> prints the sampled rows, then "ok" and the candidate diagonals
//             or "no" and the reason.
#include <cstdio>
#include <vector>

#include "partition.hpp"

int main() {
  char mode;
  while (std::scanf(" %c", &mode) == 1) {
    if (mode == 'B') {
      long long n;
      int rows, cap;
      if (std::scanf("%lld %d %d", &n, &rows, &cap) != 3) return 2;
      std::vector<int32_t> rp((size_t)n + 1);
      for (auto& v : rp)
        if (std::scanf("%d", &v) != 1) return 2;
      std::vector<int32_t> blk;
      assg::make_blocks(rp.data(), n, blk, rows, cap);
      for (int32_t v : blk) std::printf("%d ", v);
      std::printf("\n");
    } else if (mode == 'C') {
      int nsys, target;
      if (std::scanf("%d %d", &nsys, &target) != 2) return 2;
      std::vector<int32_t> sys_blk((size_t)nsys + 1);
      for (auto& v : sys_blk)
        if (std::scanf("%d", &v) != 1) return 2;
      std::vector<int32_t> cblk, csys, sys_chunk;
      assg::make_chunks(sys_blk, target, cblk, csys, sys_chunk);
      for (int32_t v : cblk) std::printf("%d ", v);
      std::printf("|");
      for (int32_t v : csys) std::printf(" %d", v);
      std::printf(" |");
      for (int32_t v : sys_chunk) std::printf(" %d", v);
      std::printf("\n");
    } else if (mode == 'D') {
      long long n, nnz;
      int check;
      if (std::scanf("%lld %lld %d", &n, &nnz, &check) != 3 || n < 1) return 2;
      std::vector<int32_t> rp((size_t)n + 1), ci((size_t)nnz);
      for (auto& v : rp)
        if (std::scanf("%d", &v) != 1) return 2;
      for (auto& v : ci)
        if (std::scanf("%d", &v) != 1) return 2;
      std::vector<int64_t> rows, offs;
      assg::dia_sample_rows(n, rows);
      long long max_row = 0;
      for (int64_t i : rows) {
        std::printf("%lld ", (long long)i);
        const long long len = (long long)rp[i + 1] - rp[i];
        if (len > max_row) max_row = len;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) offs.push_back((int64_t)ci[e] - i);
      }
      std::printf("|");
      const char* no = assg::dia_offsets(offs, max_row, n, nnz, check != 0);
      if (no) {
        std::printf(" no %s\n", no);
      } else {
        std::printf(" ok");
        for (int64_t o : offs) std::printf(" %lld", (long long)o);
        std::printf("\n");
      }
    } else {
      return 2;
    }
  }
  return 0;
}
