// Host check of the patch-set work-list packing and of the lane decoding the
// sweep kernels apply to it: every interior cell of every line is written by
// exactly one writer lane, segments fit their 64-lane item, each writer's
// stencil lanes (within SEG_HALO) stay inside its own segment, and per-patch
// lists never mix patches.  Prints "OK <items> <lane utilisation>" per list.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <tuple>
#include <vector>

#include "dimp_pack.hpp"

using namespace dimp;

static int fails = 0;
#define CHECK(c, ...)                       \
  do {                                      \
    if (!(c)) {                             \
      if (fails++ < 10) {                   \
        std::printf("FAIL %s: ", #c);       \
        std::printf(__VA_ARGS__);           \
        std::printf("\n");                  \
      }                                     \
    }                                       \
  } while (0)

// the segment a lane belongs to: the last one whose first lane is <= lane
static int seg_of(const std::vector<Seg>& seg, int64_t sb, int64_t se, int lane) {
  int64_t k = sb;
  for (int64_t i = sb + 1; i < se; ++i)
    if (lane >= (seg[i].lanes & 255)) k = i;
  return (int)k;
}

static void check_list(const char* name, const std::vector<Line>& lines, int64_t npatch, bool per_patch) {
  std::vector<Seg> seg;
  std::vector<int64_t> beg, pwork;
  pack_lines(lines, npatch, per_patch, seg, beg, pwork);
  std::map<std::pair<int, int>, int> len;
  int64_t cells = 0;
  for (const Line& L : lines) {
    len[{L.patch, L.line}] = L.len;
    cells += L.len;
  }
  std::map<std::tuple<int, int, int>, int> hits;
  const int64_t nwork = (int64_t)beg.size() - 1;
  CHECK(nwork >= 1, "%s: no work", name);
  CHECK(beg.back() == (int64_t)seg.size(), "%s: sentinel", name);
  for (int64_t w = 0; w < nwork; ++w) {
    const int64_t sb = beg[w], se = beg[w + 1];
    CHECK(se > sb, "%s: empty item %lld", name, (long long)w);
    CHECK((seg[sb].lanes & 255) == 0, "%s: item %lld does not start at lane 0", name, (long long)w);
    int end = 0;
    for (int64_t k = sb; k < se; ++k) {
      const int l0 = seg[k].lanes & 255, n = seg[k].lanes >> 8;
      CHECK(l0 >= end, "%s: overlapping segments", name);
      CHECK(n >= 1 && n <= SEG_MAX, "%s: segment of %d cells", name, n);
      end = l0 + n + 2 * SEG_HALO;
      CHECK(end <= SEG_LANES, "%s: segment past lane 63", name);
    }
    for (int lane = 0; lane < SEG_LANES; ++lane) {
      const int k = seg_of(seg, sb, se, lane);
      const Seg& s = seg[k];
      const int q = lane - (s.lanes & 255), n = s.lanes >> 8;
      const bool writer = q >= SEG_HALO && q < n + SEG_HALO;
      if (!writer) continue;
      const int cell = s.first + q - SEG_HALO;
      auto it = len.find({s.patch, s.line});
      CHECK(it != len.end(), "%s: unknown line", name);
      if (it == len.end()) continue;
      CHECK(cell >= 0 && cell < it->second, "%s: cell %d outside line of %d", name, cell, it->second);
      hits[{s.patch, s.line, cell}] += 1;
      for (int d = -SEG_HALO; d <= SEG_HALO; ++d) {
        const int nb = lane + d;
        CHECK(nb >= 0 && nb < SEG_LANES, "%s: stencil lane %d", name, nb);
        if (nb >= 0 && nb < SEG_LANES) CHECK(seg_of(seg, sb, se, nb) == k, "%s: stencil leaves its segment", name);
      }
      if (per_patch) {
        CHECK(w >= pwork[s.patch] && w < pwork[s.patch + 1], "%s: patch %d outside its items", name, s.patch);
      }
    }
  }
  CHECK((int64_t)hits.size() == cells, "%s: %zu cells written of %lld", name, hits.size(), (long long)cells);
  for (auto& kv : hits) CHECK(kv.second == 1, "%s: a cell written %d times", name, kv.second);
  if (per_patch) {
    CHECK(pwork[0] == 0 && pwork[npatch] == nwork, "%s: pwork ends", name);
    for (int64_t p = 0; p < npatch; ++p) CHECK(pwork[p + 1] >= pwork[p], "%s: pwork order", name);
  }
  std::printf("OK %s items %lld utilisation %.3f\n", name, (long long)nwork, double(cells) / (64.0 * nwork));
}

int main() {
  std::mt19937_64 rng(12345);
  std::vector<std::pair<int, int>> sizes = {{1, 1}, {57, 3}, {58, 58}, {59, 59}, {116, 2}, {117, 117}, {64, 5},
                                            {7, 200}, {300, 1}};
  std::uniform_real_distribution<double> U(0.0, 1.0);
  for (int i = 0; i < 300; ++i) sizes.push_back({(int)(1 + 200 * U(rng) * U(rng)), (int)(1 + 150 * U(rng))});
  const int64_t np = (int64_t)sizes.size();
  std::vector<Line> rows, cols4, cols8;
  for (int64_t p = 0; p < np; ++p) {
    for (int j = 0; j < sizes[p].second; ++j) rows.push_back({(int32_t)p, j, sizes[p].first});
    for (int x0 = 0; x0 < sizes[p].first; x0 += 4) cols4.push_back({(int32_t)p, x0, sizes[p].second});
    for (int x0 = 0; x0 < sizes[p].first; x0 += 8) cols8.push_back({(int32_t)p, x0, sizes[p].second});
  }
  check_list("rows", rows, np, false);
  check_list("rows_per_patch", rows, np, true);
  check_list("cols4", cols4, np, false);
  check_list("cols4_per_patch", cols4, np, true);
  check_list("cols8_per_patch", cols8, np, true);
  // patches with no line at all between others keep empty item ranges
  std::vector<Line> sparse = {{0, 0, 10}, {3, 0, 70}, {3, 1, 5}};
  check_list("sparse_per_patch", sparse, 5, true);
  if (fails) {
    std::printf("%d failures\n", fails);
    return 1;
  }
  return 0;
}
