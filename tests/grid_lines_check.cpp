// Host harness for the line-start decoding of the grid variant: reads a mesh
// (dim, node counts), integer steps and a minimum line length from stdin and
// prints, per step, the
// line count, longest line, index step and every decoded start with its line
// length and whether stepping (line_advance by 1 and by 5) reaches it.  Built with the host compiler against the library's own header; the
// test compares the output with a brute-force enumeration.
#include <cstdio>
#include <vector>

#include "r1_grid_lines.hpp"

int main() {
  r1_grid grid{};
  int n_dir = 0;
  if (std::scanf("%d", &grid.dim) != 1) return 2;
  const int dd = grid.dim * grid.dim;
  for (int c = 0; c < dd; ++c)
    if (std::scanf("%d", &grid.n[c]) != 1) return 2;
  grid.delta = 1.0;
  r1g::GridArgs g;
  if (r1g::grid_args(&grid, &g) != R1_OK) return 3;
  if (std::scanf("%d", &n_dir) != 1) return 2;
  int min_len = 1;
  if (std::scanf("%d", &min_len) != 1) return 2;
  for (int m = 0; m < n_dir; ++m) {
    r1g::Step s{};
    for (int c = 0; c < dd; ++c)
      if (std::scanf("%d", &s.s[c]) != 1) return 2;
    r1g::step_slabs(g, &s, min_len);
    std::printf("%lld %d %lld\n", static_cast<long long>(s.count), s.len, static_cast<long long>(s.ds));
    // decoded one by one; and reached by stepping (line_advance) from the previous
    // start (delta 1) and from the start 5 before (delta 5), decoding afresh only
    // where the step leaves the slab
    const int64_t cnt = s.count;
    std::vector<int> ok(size_t(cnt), 1);
    for (int delta : {1, 5}) {
      for (int64_t r0 = 0; r0 < delta && r0 < cnt; ++r0) {
        int J[9] = {0};
        int64_t q = 0;
        int slab = 0;
        for (int64_t t = r0; t < cnt; t += delta) {
          if (t == r0 || !r1g::line_advance(g, s, slab, J, &q, uint32_t(delta))) q = r1g::line_start(g, s, t, J, &slab);
          int I[9];
          int c = 0;
          const int64_t p = r1g::line_start(g, s, t, I, &c);
          bool same = q == p && slab == c;
          for (int k = 0; k < dd; ++k) same = same && J[k] == I[k];
          if (!same) ok[size_t(t)] = 0;
        }
      }
    }
    for (int64_t t = 0; t < cnt; ++t) {
      int I[9];
      const int64_t p = r1g::line_start(g, s, t, I);
      std::printf("%lld %d %d\n", static_cast<long long>(p), r1g::line_length(g, s, I), ok[size_t(t)]);
    }
  }
  return 0;
}
