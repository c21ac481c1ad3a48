// dimp_pack.hpp -- packing of patch-set lines into 64-lane work items
// (host code, no HIP types, so that it can be checked by a plain C++ build).
//
// A line is one interior row (x sweep) or one chunk of tile columns (y sweep)
// of a patch.  Lines are cut into segments of at most SEG_MAX cells; each
// segment occupies its cells plus SEG_HALO lanes on both sides of a wave (the
// stencil halo, clamped into the patch by the kernels), so short lines of
// several patches share one work item.
#pragma once
#include <algorithm>
#include <cstdint>
#include <vector>

namespace dimp {

constexpr int SEG_LANES = 64, SEG_HALO = 3, SEG_MAX = SEG_LANES - 2 * SEG_HALO;

// {patch, line (row j, or first column x0), first cell along the sweep,
//  lane0 | ncells << 8}; the device reads it as an int4
struct Seg {
  int32_t patch, line, first, lanes;
};

struct Line {
  int32_t patch, line, len;
};

// Greedy packing: every segment takes its cells plus the halo lanes on both
// sides; a line longer than the free lanes continues in the next item.  Item
// k holds segments [beg[k], beg[k+1]).  With per_patch every patch starts a
// new item and pwork[p] is the first item of patch p (npatch + 1 entries).
// Lines must come grouped by patch in increasing patch order.
inline void pack_lines(const std::vector<Line>& lines, int64_t npatch, bool per_patch, std::vector<Seg>& seg,
                       std::vector<int64_t>& beg, std::vector<int64_t>& pwork) {
  constexpr int H2 = 2 * SEG_HALO;
  int free = 0, lane = 0;
  int64_t next_patch = 0;
  seg.clear();
  beg.clear();
  pwork.assign(npatch + 1, 0);
  for (const Line& L : lines) {
    if (per_patch && L.patch >= next_patch) {
      free = 0;  // close the open item
      for (int64_t p = next_patch; p <= L.patch; ++p) pwork[p] = (int64_t)beg.size();
      next_patch = L.patch + 1;
    }
    int pos = 0, rem = L.len;
    while (rem > 0) {
      if (free < H2 + 1) {
        beg.push_back((int64_t)seg.size());
        free = SEG_LANES;
        lane = 0;
      }
      const int n = std::min(rem, std::min(free - H2, SEG_MAX));
      seg.push_back(Seg{L.patch, L.line, pos, lane | (n << 8)});
      lane += n + H2;
      free -= n + H2;
      pos += n;
      rem -= n;
    }
  }
  for (int64_t p = per_patch ? next_patch : 0; p <= npatch; ++p) pwork[p] = (int64_t)beg.size();
  beg.push_back((int64_t)seg.size());
}

}  // namespace dimp
