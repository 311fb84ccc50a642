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

// Calls f(k, lx, ly) for every box k that holds grid cell (gx, gy), with the cell's
// box coordinates, in a fixed order.  Such boxes belong to the cell's owner
// subdomain (own_x / own_y: owner index of each grid column / row) or to one of its
// neighbours, since the overlap is at most one subdomain wide.
template <class Fn>
ACCH_DEV void for_boxes_of(const SubInfo *subs, int nx, int ny, int periodic, int px, int py, const int *own_x,
                           const int *own_y, int gx, int gy, Fn &&f) {
  int cx[3], cy[3], ncx = 0, ncy = 0;
  for (int d = -1; d <= 1; ++d) {
    int sx = own_x[gx] + d, sy = own_y[gy] + d;
    if (periodic) {
      sx = (sx + px) % px;
      sy = (sy + py) % py;
    }
    bool newx = sx >= 0 && sx < px, newy = sy >= 0 && sy < py;
    for (int q = 0; q < ncx; ++q) newx = newx && cx[q] != sx;
    for (int q = 0; q < ncy; ++q) newy = newy && cy[q] != sy;
    if (newx) cx[ncx++] = sx;
    if (newy) cy[ncy++] = sy;
  }
  for (int b = 0; b < ncy; ++b)
    for (int a = 0; a < ncx; ++a) {
      const int k = cy[b] * px + cx[a];
      const SubInfo si = subs[k];
      int lx = gx - si.ox, ly = gy - si.oy;
      if (periodic) {
        lx = ((lx % nx) + nx) % nx;
        ly = ((ly % ny) + ny) % ny;
      }
      if (lx >= 0 && lx < si.ex && ly >= 0 && ly < si.ey) f(k, lx, ly);
    }
}

}  // namespace acch
