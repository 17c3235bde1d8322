// Row ranges of the pruned darkfield FFT passes (host code).  A range is a
// cyclic run of rows of an N-row grid in FFT order: rows y0, y0 + 1, ... mod N,
// n of them.  Row passes run whole workgroups of `group` rows, so every range
// is rounded up to a multiple of `group` (at least one group) and capped at N.
#pragma once

#include <algorithm>

namespace apic {

struct RowRange {
  int y0 = 0, n = 0;
};

inline int round_rows(int rows, int n_grid, int group) {
  return std::min(n_grid, std::max(group, (rows + group - 1) / group * group));
}

// The signed rows lo .. hi (an empty span has hi < lo) as a range from lo's
// FFT-order row.
inline RowRange rows_of_span(int lo, int hi, int n_grid, int group) {
  RowRange r;
  r.y0 = lo & (n_grid - 1);
  r.n = round_rows(hi - lo + 1, n_grid, group);
  return r;
}

// The shortest range that holds ranges a and b.  The shortest cyclic cover of
// two arcs starts where one of them starts: from a's start it must reach b's
// end, and from b's start a's end.
inline RowRange cyclic_hull(RowRange a, RowRange b, int n_grid, int group) {
  const int off_b = (b.y0 - a.y0) & (n_grid - 1), off_a = (a.y0 - b.y0) & (n_grid - 1);
  const int len_a = std::max(a.n, off_b + b.n), len_b = std::max(b.n, off_a + a.n);
  RowRange r;
  r.y0 = len_a <= len_b ? a.y0 : b.y0;
  r.n = round_rows(std::min(len_a, len_b), n_grid, group);
  return r;
}

}  // namespace apic
