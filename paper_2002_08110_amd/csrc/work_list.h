// Work list of a batched stage launch: the solves of one launch group share
// one grid, solve i owning the work items item0[i] <= item < item0[i + 1].
// Item `item` is tile item - item0[i] of solve i; tiles at or beyond the
// solve's tile count are padding, which the kernel skips. Every item0[i] is
// a multiple of kListAlign (8, the XCD count), so that the workgroup of an
// item runs on the XCD that the solve's own launch gives the same tile: the
// hardware hands workgroup ids to the XCDs in turn.
//
// Plain C++ (host and device): the host builds and checks the list, the
// kernels look items up with work_list_slot.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace hd {

constexpr uint32_t kListAlign = 8;
// Largest grid of one launch (the x dimension of a HIP grid).
constexpr uint64_t kListMaxItems = 0x7fffffffull;

// The slot that owns `item`: the last i with item0[i] <= item, found by
// bisection over the nslots + 1 non-decreasing entries (item < item0[nslots]).
__host__ __device__ inline int work_list_slot(const uint32_t *item0, int nslots, uint32_t item) {
  int lo = 0, hi = nslots;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (item0[mid] <= item) lo = mid;
    else hi = mid;
  }
  return lo;
}

// item0 for solves of tiles[i] tiles each (every count >= 1): solve i's range
// is its tile count rounded up to a multiple of 8. Returns false, with the
// reason, for an empty list, a solve without tiles, or more items than one
// grid holds.
inline bool build_work_list(const std::vector<uint32_t> &tiles, std::vector<uint32_t> *item0,
                            std::string *why) {
  item0->assign(1, 0);
  if (tiles.empty()) {
    *why = "empty work list";
    return false;
  }
  uint64_t at = 0;
  for (size_t i = 0; i < tiles.size(); ++i) {
    if (tiles[i] == 0) {
      *why = "solve " + std::to_string(i) + " has no tile";
      return false;
    }
    at += ((uint64_t)tiles[i] + kListAlign - 1) / kListAlign * kListAlign;
    if (at > kListMaxItems) {
      *why = "work list exceeds one grid (2^31 - 1 items)";
      return false;
    }
    item0->push_back((uint32_t)at);
  }
  return true;
}

// The properties the kernels rely on: item0[0] = 0, every entry a multiple of
// 8, each range holding its solve's tiles and fewer than 8 padding items
// (so it is strictly increasing), the total within one grid.
inline bool check_work_list(const std::vector<uint32_t> &tiles, const std::vector<uint32_t> &item0,
                            std::string *why) {
  if (tiles.empty() || item0.size() != tiles.size() + 1 || item0[0] != 0) {
    *why = "work list shape";
    return false;
  }
  for (size_t i = 0; i < tiles.size(); ++i) {
    const uint64_t span = (uint64_t)item0[i + 1] - item0[i];
    if (item0[i + 1] < item0[i] || item0[i + 1] % kListAlign != 0 || tiles[i] == 0 ||
        span < tiles[i] || span >= (uint64_t)tiles[i] + kListAlign) {
      *why = "work list range of solve " + std::to_string(i);
      return false;
    }
  }
  if (item0.back() > kListMaxItems) {
    *why = "work list exceeds one grid";
    return false;
  }
  return true;
}

}  // namespace hd
