// Host harness for the uneven batch's work planner (r1plan::plan_work, the
// library's own header), built by the CPU tests with the host compiler, under
// AddressSanitizer and UndefinedBehaviorSanitizer.  For random tables (depth 1
// and 2, a few layout variants) and random per-point indices, including empty
// batches and variants with no points, it checks what the persistent kernels
// rely on:
//   - per variant, the point items, then the outer items, in one contiguous run
//     of the item list, variant after variant, covering it exactly;
//   - point items name 1 to 4 order entries, in bounds; kind 0 for depth-1 points
//     and kind 2 for depth-2 points, depth-1 items first; every point in exactly
//     one point item, in the variant of its table entry;
//   - each list largest cost first, ties in point order;
//   - a depth-2 point has one outer item per outer direction, 0 .. n_dir0 - 1,
//     and its outer-result slots pbase .. pbase + n_dir0 tile [0, n_outer);
//   - the final range lists the variant's depth-2 points in their item order.
// Prints "ok <trials>" or the first violated property (exit status 1).
#include <cstdint>
#include <cstdio>
#include <vector>

#include "r1_batched_plan.hpp"

namespace {

uint64_t rs = 0x9E3779B97F4A7C15ull;
int rnd(int n) {  // uniform in [0, n)
  rs ^= rs << 13;
  rs ^= rs >> 7;
  rs ^= rs << 17;
  return int((rs >> 33) % uint64_t(n));
}

#define REQUIRE(c)                                                          \
  do {                                                                      \
    if (!(c)) {                                                             \
      std::printf("trial %d: %s (line %d)\n", trial, #c, __LINE__);         \
      return false;                                                         \
    }                                                                       \
  } while (0)

bool check(int trial, const std::vector<r1plan::Entry>& table, const std::vector<int32_t>& idx, int n_var) {
  using namespace r1plan;
  const Plan pl = plan_work(table, idx, n_var);
  const int64_t n = int64_t(idx.size());
  REQUIRE(int64_t(pl.first.size()) == 3 * n_var && int64_t(pl.count.size()) == 3 * n_var);
  REQUIRE(int64_t(pl.pbase.size()) == n);
  std::vector<int> seen(static_cast<size_t>(n), 0);
  std::vector<int> slot(size_t(pl.n_outer), 0);
  int64_t next_item = 0, n_depth2 = 0;
  for (int c = 0; c < n_var; ++c) {
    const int64_t* first = &pl.first[size_t(c) * 3];
    const int64_t* count = &pl.count[size_t(c) * 3];
    REQUIRE(first[kPoint] == next_item && count[kPoint] >= 0);
    REQUIRE(first[kOuter] == first[kPoint] + count[kPoint] && count[kOuter] >= 0);
    next_item = first[kOuter] + count[kOuter];
    REQUIRE(next_item <= int64_t(pl.items.size()));
    // point items: order entries, kinds, sizes
    std::vector<int32_t> lists[2];
    int last_kind = 0;
    for (int64_t i = first[kPoint]; i < first[kPoint] + count[kPoint]; ++i) {
      const Item& it = pl.items[size_t(i)];
      REQUIRE(it.x == 0 || it.x == 2);
      REQUIRE(it.x >= last_kind);
      last_kind = it.x;
      REQUIRE(it.y >= 0 && it.z >= 1 && it.z <= 4 && int64_t(it.y) + it.z <= int64_t(pl.order.size()));
      for (int k = 0; k < it.z; ++k) {
        const int32_t p = pl.order[size_t(it.y + k)];
        REQUIRE(p >= 0 && p < n);
        const Entry& e = table[size_t(idx[size_t(p)])];
        REQUIRE(e.var == c);
        REQUIRE((e.depth == 1) == (it.x == 0));
        seen[size_t(p)] += 1;
        lists[it.x / 2].push_back(p);
      }
    }
    for (int k = 0; k < 2; ++k)
      for (size_t j = 1; j < lists[k].size(); ++j) {
        const double c0 = point_cost(table[size_t(idx[size_t(lists[k][j - 1])])]);
        const double c1 = point_cost(table[size_t(idx[size_t(lists[k][j])])]);
        REQUIRE(c0 > c1 || (c0 == c1 && lists[k][j - 1] < lists[k][j]));
      }
    // outer items: one per outer direction of each depth-2 point, in point order
    int64_t i = first[kOuter];
    for (int32_t p : lists[1]) {
      const Entry& e = table[size_t(idx[size_t(p)])];
      REQUIRE(pl.pbase[size_t(p)] >= 0 && pl.pbase[size_t(p)] + e.n_dir0 <= pl.n_outer);
      for (int mo = 0; mo < e.n_dir0; ++mo, ++i) {
        REQUIRE(i < first[kOuter] + count[kOuter]);
        const Item& it = pl.items[size_t(i)];
        REQUIRE(it.x == kOuter && it.y == p && it.z == mo);
        slot[size_t(pl.pbase[size_t(p)] + mo)] += 1;
      }
    }
    REQUIRE(i == first[kOuter] + count[kOuter]);
    // final pass: the depth-2 points again, same order
    REQUIRE(count[kFinal] == int64_t(lists[1].size()));
    REQUIRE(first[kFinal] >= 0 && first[kFinal] + count[kFinal] <= int64_t(pl.order.size()));
    for (size_t j = 0; j < lists[1].size(); ++j) REQUIRE(pl.order[size_t(first[kFinal]) + j] == lists[1][j]);
    n_depth2 += int64_t(lists[1].size());
  }
  REQUIRE(next_item == int64_t(pl.items.size()));
  for (int64_t p = 0; p < n; ++p) REQUIRE(seen[size_t(p)] == 1);
  for (int64_t s = 0; s < pl.n_outer; ++s) REQUIRE(slot[size_t(s)] == 1);
  REQUIRE(int64_t(pl.order.size()) == n + n_depth2);
  return true;
}

}  // namespace

int main() {
  const int nt[] = {257, 513, 1025, 2049};
  const int nd[] = {1, 3, 32, 64, 128};
  int trials = 0;
  for (int trial = 0; trial < 300; ++trial, ++trials) {
    const int n_var = 1 + rnd(4);
    const int n_entries = 1 + rnd(8);
    std::vector<r1plan::Entry> table;
    for (int k = 0; k < n_entries; ++k) {
      r1plan::Entry e{};
      e.depth = 1 + rnd(2);
      e.n_dir0 = nd[rnd(5)];
      e.n_t0 = nt[rnd(4)];
      e.n_dir1 = e.depth == 2 ? nd[rnd(5)] : 0;
      e.n_t1 = e.depth == 2 ? nt[rnd(4)] : 0;
      e.var = rnd(n_var);
      table.push_back(e);
    }
    // empty batches, batches below one item, and a few thousand points
    const int n = trial % 10 == 0 ? 0 : (trial % 3 == 0 ? 1 + rnd(5) : rnd(3000));
    std::vector<int32_t> idx(static_cast<size_t>(n));
    for (auto& v : idx) v = rnd(n_entries);
    if (!check(trial, table, idx, n_var)) return 1;
  }
  std::printf("ok %d\n", trials);
  return 0;
}
