// Subdomain boxes of the Schwarz preconditioner, 2D: the i + 2j wavefront order of
// a box and the map from box cells to grid cells.  Device functions only.
#pragma once

#include "common.h"

namespace acch {

// Row of thread t on wavefront w (rows j = t mod T, 0 <= w - 2j < bw), or -1.
template <int T>
ACCH_DEV int row_on_level(int w, int t, int bw, int bh) {
  const int jmax = w >> 1;
  if (jmax < t) return -1;
  const int j = jmax - ((jmax - t) & (T - 1));
  if (j >= bh || w - 2 * j >= bw) return -1;
  return j;
}

// Global cell of box cell (i, j) of subdomain si, or -1 if it is padding or outside
// a Neumann domain.
ACCH_DEV long box_to_global(const SubInfo &si, int i, int j, int nx, int ny, int periodic) {
  if (i >= si.ex || j >= si.ey) return -1;
  int gx = si.ox + i, gy = si.oy + j;
  if (periodic) {
    gx = gx < 0 ? gx + nx : (gx >= nx ? gx - nx : gx);
    gy = gy < 0 ? gy + ny : (gy >= ny ? gy - ny : gy);
  } else if (gx < 0 || gx >= nx || gy < 0 || gy >= ny) {
    return -1;
  }
  return (long)gy * nx + gx;
}

}  // namespace acch
