// Reads cases from stdin and prints the row ranges the darkfield passes use:
//   "s N group lo hi"          -> "y0 n" of rows_of_span
//   "h N group a0 an b0 bn"    -> "y0 n" of cyclic_hull
#include <cstdio>

#include "../../paper_2407_20469_amd/csrc/rowspan.hpp"

int main() {
  char op;
  while (std::scanf(" %c", &op) == 1) {
    int n, g;
    if (std::scanf("%d %d", &n, &g) != 2) return 1;
    apic::RowRange r;
    if (op == 's') {
      int lo, hi;
      if (std::scanf("%d %d", &lo, &hi) != 2) return 1;
      r = apic::rows_of_span(lo, hi, n, g);
    } else {
      apic::RowRange a, b;
      if (std::scanf("%d %d %d %d", &a.y0, &a.n, &b.y0, &b.n) != 4) return 1;
      r = apic::cyclic_hull(a, b, n, g);
    }
    std::printf("%d %d\n", r.y0, r.n);
  }
  return 0;
}
