// Work planner of the uneven batch: turns the per-point table indices into the
// ordered work lists of the persistent launches.  Plain host C++ with no HIP
// dependency, so the CPU test harness can build and check it on its own.
#pragma once
#include <algorithm>
#include <cstdint>
#include <vector>

namespace r1plan {

// Work item of the persistent kernels: {kind, a, b, 0}.  Point items (kind 0:
// depth-1 points, full result; kind 2: depth-2 points, W^1 at the point) name
// the points order[a .. a + b); outer items (kind 1) name point a, outer
// direction b.
struct Item {
  int x, y, z, w;
};

// What the planner needs of a table entry.
struct Entry {
  int depth;
  int n_dir0, n_t0;   // outermost level
  int n_dir1, n_t1;   // inner level (depth 2)
  int var;            // layout variant of the innermost level, in [0, n_var)
};

constexpr int kPoint = 0, kOuter = 1, kFinal = 2;

struct Plan {
  std::vector<Item> items;
  std::vector<int32_t> order;
  std::vector<int64_t> pbase;          // per point: first outer-result slot (depth-2 points)
  int64_t n_outer = 0;                 // outer-result slots
  // per variant and kind: first item (first order entry for kFinal) and count
  std::vector<int64_t> first, count;   // [var * 3 + kind]
};

// Point cost in W samples, the key of the largest-first order.
inline double point_cost(const Entry& e) {
  if (e.depth == 1) return double(e.n_dir0) * double(e.n_t0 - 1);
  return double(e.n_t0 - 1) * (double(e.n_dir1) * double(e.n_t1 - 1) + 1.0);
}

// idx[p] in [0, table.size()) for every point (checked by the caller).  Per
// variant: point items (groups of up to 4 points, depth 1 first, each list
// largest first), then the outer lines of its depth-2 points, then those points
// again for the final pass.
inline Plan plan_work(const std::vector<Entry>& table, const std::vector<int32_t>& idx, int n_var) {
  Plan pl;
  const int64_t n = int64_t(idx.size());
  pl.pbase.assign(size_t(n), 0);
  pl.first.assign(size_t(n_var) * 3, 0);
  pl.count.assign(size_t(n_var) * 3, 0);
  std::vector<std::vector<int64_t>> d1(static_cast<size_t>(n_var)), d2(static_cast<size_t>(n_var));
  for (int64_t p = 0; p < n; ++p) {
    const Entry& e = table[size_t(idx[size_t(p)])];
    (e.depth == 2 ? d2 : d1)[size_t(e.var)].push_back(p);
  }
  auto larger = [&](int64_t x, int64_t y) {
    return point_cost(table[size_t(idx[size_t(x)])]) > point_cost(table[size_t(idx[size_t(y)])]);
  };
  for (int c = 0; c < n_var; ++c) {
    std::stable_sort(d1[size_t(c)].begin(), d1[size_t(c)].end(), larger);
    std::stable_sort(d2[size_t(c)].begin(), d2[size_t(c)].end(), larger);
    int64_t* first = &pl.first[size_t(c) * 3];
    int64_t* count = &pl.count[size_t(c) * 3];
    first[kPoint] = int64_t(pl.items.size());
    for (int kind = 0; kind < 2; ++kind) {
      const std::vector<int64_t>& pts = kind == 0 ? d1[size_t(c)] : d2[size_t(c)];
      const int64_t o0 = int64_t(pl.order.size());
      for (int64_t p : pts) pl.order.push_back(int32_t(p));
      for (int64_t g = 0; 4 * g < int64_t(pts.size()); ++g) {
        const int cnt = int(std::min<int64_t>(4, int64_t(pts.size()) - 4 * g));
        pl.items.push_back(Item{kind == 0 ? 0 : 2, int(o0 + 4 * g), cnt, 0});
      }
    }
    count[kPoint] = int64_t(pl.items.size()) - first[kPoint];
    first[kOuter] = int64_t(pl.items.size());
    for (int64_t p : d2[size_t(c)]) {
      const Entry& e = table[size_t(idx[size_t(p)])];
      pl.pbase[size_t(p)] = pl.n_outer;
      pl.n_outer += e.n_dir0;
      for (int mo = 0; mo < e.n_dir0; ++mo) pl.items.push_back(Item{1, int(p), mo, 0});
    }
    count[kOuter] = int64_t(pl.items.size()) - first[kOuter];
    first[kFinal] = int64_t(pl.order.size());
    for (int64_t p : d2[size_t(c)]) pl.order.push_back(int32_t(p));
    count[kFinal] = int64_t(d2[size_t(c)].size());
  }
  return pl;
}

}  // namespace r1plan
