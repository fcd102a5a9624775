// Host driver for the row-block and chunk partitions (tests/test_partition.py
// builds it with g++ and the address and undefined-behaviour sanitizers).
// stdin: "B n rows cap" then n+1 row pointers  -> prints the block starts;
//        "C nsys target" then nsys+1 block starts -> prints cblk | csys | sys_chunk.
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
    } else {
      return 2;
    }
  }
  return 0;
}
