// Band storage of the 2D subdomain matrices for the exact-LU and ILU(k) subdomain
// solvers (Table 2).  Host and device.
//
// The unknowns of a padded box (bw x bh cells) are numbered cell by cell, x fastest,
// u before v: row R = 2 (j bw + i) + t.  Every coupling of the Jacobian stencil lies
// within kl = 4 bw of the diagonal (the u-row reaches u at (0, +-2)), and so does all
// fill of the LU factorisation in this order.  The box base pattern of ILU(k) (all
// couplings of cells up to 2 apart along each axis) reaches (+-2, +-2), i.e. 4 bw + 5
// unknowns, and its band is that much wider.  A box matrix is stored as the nd = 2 kl + 1
// diagonals of its band, in 64-row chunks with the diagonal index in the middle:
// entry (R, C = R + d - kl) at [(R / 64) nd + d] * 64 + R % 64, so the 64 rows of a
// chunk are contiguous for every d.  The factors overwrite the matrix in place: L below
// the diagonal (unit diagonal not stored), U on and above it with 1/u_RR in place of
// the diagonal.
#pragma once

namespace acch {

struct BandGeom {
  int bw, bh;       // padded box (cells)
  int n;            // rows of a box matrix, 2 bw bh
  int kl;           // half bandwidth: 4 bw, or 4 bw + 5 for the box base pattern
  int nd;           // stored diagonals, 2 kl + 1
  int nchunk;       // 64-row chunks, ceil(n / 64)
  int nr;           // register tiles per thread and direction of the factorisation
  int mwords;       // 32-bit mask words per row of an ILU(k) pattern, ceil(nd / 32)
  long box_elems;   // stored values per box, nchunk nd 64
};

// Window tiles of the factorisation (16 nr window rows and columns >= kl + 1).
constexpr int kBandTiles[] = {4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14};
constexpr int kBandMaxWidth = (16 * 14 - 1) / 4;          // widest padded box: 55 cells
constexpr int kBandMaxWidthBox = (16 * 14 - 1 - 5) / 4;   // with the box base pattern: 54

inline BandGeom make_band_geom(int bw, int bh, bool box_pattern = false) {
  BandGeom B{};
  B.bw = bw;
  B.bh = bh;
  B.n = 2 * bw * bh;
  B.kl = 4 * bw + (box_pattern ? 5 : 0);
  B.nd = 2 * B.kl + 1;
  B.nchunk = (B.n + 63) / 64;
  B.nr = 0;
  for (int t : kBandTiles)
    if (B.nr == 0 && 16 * t >= B.kl + 1) B.nr = t;
  B.mwords = (B.nd + 31) / 32;
  B.box_elems = (long)B.nchunk * B.nd * 64;
  return B;
}

}  // namespace acch
