// Host-side panel plans of the transient integral-sized workspaces (plain
// C++, no HIP: the CPU tests compile it on its own).
//
// The gradient with respect to L stores, for a panel of whole block rows
// A0 .. A1 - 1 of the block-pair triangle (row A holds the nbv - A pairs
// (A, B), B >= A), one tile per (block pair of the panel, block pair of the
// whole triangle).  The plan sizes the workspace from the first panel,
// which starts at the longest row, and then grows every later panel only
// while it still fits in that same workspace: rows get shorter down the
// triangle, so a later panel holds more rows, never more bytes.
#pragma once

#include <algorithm>
#include <cstddef>
#include <utility>
#include <vector>

namespace lrcc {

struct PanelPlan {
  size_t bytes = 0;                       // workspace the largest panel needs
  std::vector<std::pair<int, int>> rows;  // [A0, A1) of each panel, in order
};

// Block pairs of the rows A0 .. A1 - 1.
inline long panel_pairs(int nbv, int A0, int A1) {
  long n = 0;
  for (int A = A0; A < A1; ++A) n += nbv - A;
  return n;
}

// Panels of whole block rows, each pair costing `pair_bytes` (one tile per
// block pair of the triangle), within `cap` bytes and at least one row.
inline PanelPlan plan_row_panels(int nbv, size_t pair_bytes, size_t cap) {
  PanelPlan p;
  if (nbv <= 0) return p;
  const size_t first = (size_t)panel_pairs(nbv, 0, 1) * pair_bytes;
  const size_t lim = std::max(cap, first);
  int maxrows = 1;
  while (maxrows < nbv && (size_t)panel_pairs(nbv, 0, maxrows + 1) * pair_bytes <= lim) ++maxrows;
  p.bytes = (size_t)panel_pairs(nbv, 0, maxrows) * pair_bytes;
  for (int A0 = 0; A0 < nbv;) {
    int A1 = A0 + 1;
    while (A1 < nbv && (size_t)panel_pairs(nbv, A0, A1 + 1) * pair_bytes <= p.bytes) ++A1;
    p.rows.emplace_back(A0, A1);
    A0 = A1;
  }
  return p;
}

}  // namespace lrcc
