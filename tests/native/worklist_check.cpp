// Host check of the batched launch's work list (csrc/work_list.h), built
// with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_batch_worklist_cpu.py. Reads scenarios from stdin, one per
// line: "<n> <tiles_0> ... <tiles_{n-1}>". For each it builds the list,
// checks it, then walks every item of the grid as the kernels do
// (work_list_slot) and asserts that each (solve, tile < tiles) pair is
// visited exactly once, that padding items lie at the end of their solve's
// range and number fewer than 8, and that every item0 entry is a multiple
// of 8. Prints "ok <items>" or "rejected <reason>" per scenario; exits 1 on
// a violated property.
#define __host__
#define __device__
#include "work_list.h"

#include <cstdio>
#include <iostream>
#include <string>
#include <vector>

int main() {
  size_t n;
  while (std::cin >> n) {
    std::vector<uint32_t> tiles(n);
    for (auto &t : tiles) std::cin >> t;
    std::vector<uint32_t> item0;
    std::string why;
    if (!hd::build_work_list(tiles, &item0, &why)) {
      std::printf("rejected %s\n", why.c_str());
      continue;
    }
    if (!hd::check_work_list(tiles, item0, &why)) {
      std::printf("FAIL check %s\n", why.c_str());
      return 1;
    }
    const uint32_t nitems = item0.back();
    std::vector<std::vector<unsigned char>> seen(n);
    for (size_t i = 0; i < n; ++i) seen[i].assign(tiles[i], 0);
    size_t padding = 0;
    for (uint32_t item = 0; item < nitems; ++item) {
      const int slot = hd::work_list_slot(item0.data(), (int)n, item);
      if (slot < 0 || (size_t)slot >= n || item < item0[slot] || item >= item0[slot + 1]) {
        std::printf("FAIL slot %d for item %u\n", slot, item);
        return 1;
      }
      const uint32_t tile = item - item0[slot];
      if (tile >= tiles[slot]) {
        ++padding;
        continue;
      }
      if (seen[slot][tile]++) {
        std::printf("FAIL item %u repeats tile %u of solve %d\n", item, tile, slot);
        return 1;
      }
    }
    for (size_t i = 0; i < n; ++i) {
      if (item0[i] % hd::kListAlign) {
        std::printf("FAIL item0[%zu] = %u not a multiple of 8\n", i, item0[i]);
        return 1;
      }
      for (uint32_t t = 0; t < tiles[i]; ++t)
        if (seen[i][t] != 1) {
          std::printf("FAIL tile %u of solve %zu not visited once\n", t, i);
          return 1;
        }
    }
    if (padding >= hd::kListAlign * n) {
      std::printf("FAIL padding %zu\n", padding);
      return 1;
    }
    std::printf("ok %u\n", nitems);
  }
  return 0;
}
