// Geometry of the box-pattern ILU(0) subdomain solver (2D).  Host and device.
//
// A padded box of bw x bh cells is swept by wavefronts w = i + 3 j (0 <= w < bw + 3 (bh - 1)):
// every cell within 2 of cell (i, j) along both axes that precedes it in the natural order
// (x fastest) lies on an earlier wavefront, and every one that follows it on a later one.
// The records of the cells of one wavefront are stored together, rows j in increasing
// order: cell (w - 3 j, j) at lvoff[w] + j - level_jlo(w, bw).
#pragma once

#include <vector>

namespace acch {

constexpr int kBoxIluRec = 52;       // record slots per cell (L and U records each)
constexpr int kBoxIluThreads = 256;  // one box row per thread
constexpr int kBoxIluMaxW = 144;     // widest padded box: at most 48 cells per wavefront
constexpr int kBoxIluMaxH = 160;     // tallest padded box (rows of the LDS value ring)

struct BoxIluGeom {
  int bw, bh;       // padded box (cells)
  int nlev;         // wavefronts, bw + 3 (bh - 1)
  int ncell;        // bw bh
  int maxcount;     // most cells on one wavefront
};

// First row of wavefront w: the smallest j with w - 3 j < bw.
__host__ __device__ inline int level_jlo(int w, int bw) {
  const int d = w - bw + 1;
  return d > 0 ? (d + 2) / 3 : 0;
}

// Wavefront offsets (nlev + 1 entries), the box cell (j << 16 | i) of each record
// position (cellof, optional) and the geometry of a bw x bh box.
inline BoxIluGeom make_boxilu_geom(int bw, int bh, std::vector<int> *lvoff, std::vector<int> *cellof = nullptr) {
  BoxIluGeom X{};
  X.bw = bw;
  X.bh = bh;
  X.nlev = bw + 3 * (bh - 1);
  X.ncell = bw * bh;
  if (lvoff) lvoff->assign(X.nlev + 1, 0);
  if (cellof) cellof->clear();
  for (int w = 0; w < X.nlev; ++w) {
    int cnt = 0;
    for (int j = level_jlo(w, bw); j < bh && 3 * j <= w; ++j) {
      if (cellof) cellof->push_back(j << 16 | (w - 3 * j));
      ++cnt;
    }
    X.maxcount = cnt > X.maxcount ? cnt : X.maxcount;
    if (lvoff) (*lvoff)[w + 1] = (*lvoff)[w] + cnt;
  }
  return X;
}

}  // namespace acch
