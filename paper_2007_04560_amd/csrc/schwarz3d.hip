// Restricted additive Schwarz with subdomain ILU(0), 3D (Section 3.1), and its exact
// transpose for the adjoint.
//
// Unknowns of a box are ordered cell by cell (x fastest, then y, then z), u before v
// at a cell; the ILU(0) pattern is the structural Jacobian stencil (u-row: u on the
// 25-point set, v on the 7-point star; v-row: v on the star, u at the cell).  Every
// earlier neighbour in that order lies on an earlier level w = i + 2j + 3k, so the
// factorisation and the sweeps walk the levels in order, one workgroup per box and
// a host-built list of each level's cells, a barrier separating levels.  The
// general kernels keep a box's values in a device-memory box buffer (a box of 34^3
// cells does not fit in LDS); the windowed apply keeps only the levels a sweep still
// reads in LDS (see k_ras_apply3d_win).
//
// Factor storage: 40 values per box cell (box-local index i + bw (j + bh k)): the
// u-row's 32 pattern entries in column order (15 multipliers of L, then U with the
// diagonal stored inverted) and the v-row's 8 (4 multipliers, inverted diagonal,
// 3 of U).
#include <utility>

#include "../../include/acch.h"
#include "bufio.h"
#include "kernels.h"
#include "stencil3d.h"

namespace acch {
namespace {

struct Col3 {
  int t, dx, dy, dz;   // column type (0 = u, 1 = v) and cell offset
};

__host__ __device__ constexpr Col3 ucol3(int k) {
  constexpr Col3 tab[32] = {
      {0, 0, 0, -2},                                                                    // lower
      {0, 0, -1, -1}, {0, -1, 0, -1}, {0, 0, 0, -1}, {1, 0, 0, -1}, {0, 1, 0, -1}, {0, 0, 1, -1},
      {0, 0, -2, 0},  {0, -1, -1, 0}, {0, 0, -1, 0}, {1, 0, -1, 0}, {0, 1, -1, 0},
      {0, -2, 0, 0},  {0, -1, 0, 0},  {1, -1, 0, 0},
      {0, 0, 0, 0},                                                                     // diagonal (15)
      {1, 0, 0, 0},   {0, 1, 0, 0},   {1, 1, 0, 0},  {0, 2, 0, 0},                     // upper
      {0, -1, 1, 0},  {0, 0, 1, 0},   {1, 0, 1, 0},  {0, 1, 1, 0},  {0, 0, 2, 0},
      {0, 0, -1, 1},  {0, -1, 0, 1},  {0, 0, 0, 1},  {1, 0, 0, 1},  {0, 1, 0, 1},  {0, 0, 1, 1},
      {0, 0, 0, 2}};
  return tab[k];
}
__host__ __device__ constexpr Col3 vcol3(int k) {
  constexpr Col3 tab[8] = {{1, 0, 0, -1}, {1, 0, -1, 0}, {1, -1, 0, 0}, {0, 0, 0, 0},
                           {1, 0, 0, 0},  {1, 1, 0, 0},  {1, 0, 1, 0},  {1, 0, 0, 1}};
  return tab[k];
}
constexpr int kUL = 15, kUD = 15, kUN = 32;   // u-row: lower count, diagonal index, entries
constexpr int kVL = 4, kVD = 4, kVN = 8;      // v-row

__host__ __device__ constexpr int find_u3(int t, int dx, int dy, int dz) {
  for (int k = 0; k < kUN; ++k) {
    const Col3 c = ucol3(k);
    if (c.t == t && c.dx == dx && c.dy == dy && c.dz == dz) return k;
  }
  return -1;
}
__host__ __device__ constexpr int find_v3(int t, int dx, int dy, int dz) {
  for (int k = 0; k < kVN; ++k) {
    const Col3 c = vcol3(k);
    if (c.t == t && c.dx == dx && c.dy == dy && c.dz == dz) return k;
  }
  return -1;
}
// Jacobian slot (include/acch.h) of a column of a u-row (rt = 0) or v-row (rt = 1).
__host__ __device__ constexpr int jslot3(int rt, Col3 c) {
  if (rt == 0 && c.t == 0) {
    for (int k = 0; k < 25; ++k)
      if (uu3(k).dx == c.dx && uu3(k).dy == c.dy && uu3(k).dz == c.dz) return k;
    return -1;
  }
  if (rt == 1 && c.t == 0) return (c.dx == 0 && c.dy == 0 && c.dz == 0) ? 39 : -1;
  for (int k = 0; k < 7; ++k)
    if (star3(k).dx == c.dx && star3(k).dy == c.dy && star3(k).dz == c.dz) return (rt == 0 ? 25 : 32) + k;
  return -1;
}
__host__ __device__ constexpr bool tables3_consistent() {
  for (int k = 0; k < kUN; ++k)
    if (jslot3(0, ucol3(k)) < 0) return false;
  for (int k = 0; k < kVN; ++k)
    if (jslot3(1, vcol3(k)) < 0) return false;
  // strictly increasing unknown order, diagonal where claimed
  for (int k = 1; k < kUN; ++k) {
    const Col3 a = ucol3(k - 1), b = ucol3(k);
    const long ka = ((long)a.dz * 64 + a.dy) * 64 * 2 + a.dx * 2 + a.t, kb = ((long)b.dz * 64 + b.dy) * 64 * 2 + b.dx * 2 + b.t;
    if (!(ka < kb)) return false;
  }
  const Col3 d = ucol3(kUD), dv = vcol3(kVD);
  return d.t == 0 && d.dx == 0 && d.dy == 0 && d.dz == 0 && dv.t == 1 && dv.dx == 0 && dv.dy == 0 && dv.dz == 0;
}
static_assert(tables3_consistent(), "3D ILU pattern tables");

// Slots of a cell's factor record.
constexpr int kFA = 0;     // u-row entries 0..31
constexpr int kFB = 32;    // v-row entries 32..39

struct Box3 {
  int bw, bh, bd;
  ACCH_DEV bool in(int i, int j, int k) const { return i >= 0 && i < bw && j >= 0 && j < bh && k >= 0 && k < bd; }
  ACCH_DEV int at(int i, int j, int k) const { return i + bw * (j + bh * k); }
};

ACCH_DEV long box3_to_global(const SubInfo &si, int i, int j, int k, const Phys &P) {
  if (i >= si.ex || j >= si.ey || k >= si.ez) return -1;
  int gx = si.ox + i, gy = si.oy + j, gz = si.oz + k;
  if (P.periodic) {
    gx = gx < 0 ? gx + P.nx : (gx >= P.nx ? gx - P.nx : gx);
    gy = gy < 0 ? gy + P.ny : (gy >= P.ny ? gy - P.ny : gy);
    gz = gz < 0 ? gz + P.nz : (gz >= P.nz ? gz - P.nz : gz);
  } else if (gx < 0 || gx >= P.nx || gy < 0 || gy >= P.ny || gz < 0 || gz >= P.nz) {
    return -1;
  }
  return ((long)gz * P.ny + gy) * P.nx + gx;
}

ACCH_DEV bool owned3(const SubInfo &si, int i, int j, int k) {
  return i >= si.own_x0 && i < si.own_x1 && j >= si.own_y0 && j < si.own_y1 && k >= si.own_z0 && k < si.own_z1;
}

// Index of box cell (i+dx, j+dy, k+dz), or `self` when it lies outside the box (the
// caller masks the term), so every load of a sweep is unconditional and the loads of
// a cell can all be in flight together.
ACCH_DEV int nb_or(const Box3 &B, int i, int j, int k, int dx, int dy, int dz, int self, bool &in) {
  in = B.in(i + dx, j + dy, k + dz);
  return in ? B.at(i + dx, j + dy, k + dz) : self;
}

// Level lists hold box coordinates packed as i | j << 10 | k << 20.
ACCH_DEV void unpack(int c, int &i, int &j, int &k) {
  i = c & 1023;
  j = (c >> 10) & 1023;
  k = c >> 20;
}

ACCH_DEV void decode(int e, const Box3 &B, int &i, int &j, int &k) {
  i = e % B.bw;
  const int r = e / B.bw;
  j = r % B.bh;
  k = r / B.bh;
}

// ---- ILU(0) of A_k + shift diag(A_k) ------------------------------------------
template <int P, int E>
ACCH_DEV void elim3_u(double (&a)[kUN], double l, const double *prow) {
  constexpr Col3 pc = ucol3(P);
  constexpr Col3 e = (pc.t == 0) ? ucol3(kUD + E) : vcol3(kVD + E);
  constexpr int tgt = find_u3(e.t, pc.dx + e.dx, pc.dy + e.dy, pc.dz + e.dz);
  if constexpr (tgt > P) a[tgt] -= l * prow[E];
}
template <int P, int... Es>
ACCH_DEV void elim3_u_row(double (&a)[kUN], double l, const double *prow, std::integer_sequence<int, Es...>) {
  (elim3_u<P, Es + 1>(a, l, prow), ...);
}
template <int P, int E>
ACCH_DEV void elim3_v(double (&b)[kVN], double l, const double *prow) {
  constexpr Col3 pc = vcol3(P);
  constexpr Col3 e = (pc.t == 0) ? ucol3(kUD + E) : vcol3(kVD + E);
  constexpr int tgt = find_v3(e.t, pc.dx + e.dx, pc.dy + e.dy, pc.dz + e.dz);
  if constexpr (tgt > P) b[tgt] -= l * prow[E];
}
template <int P, int... Es>
ACCH_DEV void elim3_v_row(double (&b)[kVN], double l, const double *prow, std::integer_sequence<int, Es...>) {
  (elim3_v<P, Es + 1>(b, l, prow), ...);
}

// Loads the U part of the pivot row of column P (a u-row: 17 values, v-row: 4) of
// cell q, first value the inverted diagonal.
template <typename FT, int NE>
ACCH_DEV void load_urow(const FT *rec, int first, double (&prow)[NE]) {
#pragma unroll
  for (int e = 0; e < NE; ++e) prow[e] = (double)rec[first + e];
}

// A pivot column outside the box reads the record of box cell 0, whatever it holds,
// and masks it to zero, so the loads carry no branch.
template <int P, typename FT>
ACCH_DEV void pivot_u(double (&a)[kUN], const FT *fk, const Box3 &B, int i, int j, int k) {
  constexpr Col3 pc = ucol3(P);
  bool in;
  const int q = nb_or(B, i, j, k, pc.dx, pc.dy, pc.dz, 0, in);
  const FT *rec = fk + (long)q * kNSlot3D;
  constexpr int ne = (pc.t == 0) ? kUN - kUD : kVN - kVD;
  double prow[ne];
  load_urow<FT, ne>(rec, pc.t == 0 ? kFA + kUD : kFB + kVD, prow);
#pragma unroll
  for (int e = 0; e < ne; ++e) prow[e] = in ? prow[e] : 0.0;
  const double l = a[P] * prow[0];
  a[P] = l;
  elim3_u_row<P>(a, l, prow, std::make_integer_sequence<int, ne - 1>{});
}

template <int P, typename FT>
ACCH_DEV void pivot_v(double (&b)[kVN], const FT *fk, const Box3 &B, int i, int j, int k) {
  constexpr Col3 pc = vcol3(P);
  bool in;
  const int q = nb_or(B, i, j, k, pc.dx, pc.dy, pc.dz, 0, in);
  const FT *rec = fk + (long)q * kNSlot3D;
  double prow[kVN - kVD];
  load_urow<FT, kVN - kVD>(rec, kFB + kVD, prow);
#pragma unroll
  for (int e = 0; e < kVN - kVD; ++e) prow[e] = in ? prow[e] : 0.0;
  const double l = b[P] * prow[0];
  b[P] = l;
  elim3_v_row<P>(b, l, prow, std::make_integer_sequence<int, kVN - kVD - 1>{});
}

template <int... Ps, typename FT>
ACCH_DEV void pivots_u(std::integer_sequence<int, Ps...>, double (&a)[kUN], const FT *fk, const Box3 &B, int i,
                       int j, int k) {
  (pivot_u<Ps>(a, fk, B, i, j, k), ...);
}
template <int... Ps, typename FT>
ACCH_DEV void pivots_v(std::integer_sequence<int, Ps...>, double (&b)[kVN], const FT *fk, const Box3 &B, int i,
                       int j, int k) {
  (pivot_v<Ps>(b, fk, B, i, j, k), ...);
}

// A_k = R_k J R_k^T plus the shift on its diagonal, written as each box cell's record
// in the factor storage (pattern order; entries coupling to cells outside the box or
// the domain are zero, padding cells are decoupled identity rows).  A block takes 128
// consecutive box cells: one thread per cell reads its Jacobian row (a wave's reads
// of one slot are contiguous), the records go through LDS and leave as one contiguous
// run.
constexpr int kExtractCells = 128;

template <typename FT>
__global__ __launch_bounds__(kExtractCells) void k_extract3d(Phys P, BoxGeom G, const SubInfo *__restrict__ subs,
                                                             const double *__restrict__ J, double shift,
                                                             FT *__restrict__ fac) {
  __shared__ FT tile[kExtractCells * kNSlot3D];
  const long n = (long)P.nx * P.ny * P.nz;
  const long total = (long)G.nsub * G.ncb;
  const long x0 = (long)blockIdx.x * kExtractCells;
  const long x = x0 + threadIdx.x;
  FT *rec = tile + threadIdx.x * kNSlot3D;
  if (x < total) {
    const Box3 B{G.bw, G.bh, G.bd};
    const int sub = (int)(x / G.ncb), e = (int)(x - (long)sub * G.ncb);
    const SubInfo si = subs[sub];
    int i, j, k;
    decode(e, B, i, j, k);
    const long g = box3_to_global(si, i, j, k, P);
    // the neighbour at offset d along an axis is a real cell of the box and of the domain
    auto axis_ok = [&](int c, int d, int ext, int org, int nn) {
      const int cc = c + d;
      return cc >= 0 && cc < ext && (P.periodic || (org + cc >= 0 && org + cc < nn));
    };
    bool okx[5], oky[5], okz[5];
#pragma unroll
    for (int d = -2; d <= 2; ++d) {
      okx[d + 2] = axis_ok(i, d, si.ex, si.ox, P.nx);
      oky[d + 2] = axis_ok(j, d, si.ey, si.oy, P.ny);
      okz[d + 2] = axis_ok(k, d, si.ez, si.oz, P.nz);
    }
    if (g >= 0) {
#pragma unroll
      for (int c = 0; c < kUN; ++c) {
        const Col3 cc = ucol3(c);
        const bool in = okx[cc.dx + 2] && oky[cc.dy + 2] && okz[cc.dz + 2];
        const double a = in ? J[(long)jslot3(0, cc) * n + g] : 0.0;
        rec[kFA + c] = (FT)(c == kUD ? a * (1.0 + shift) : a);
      }
#pragma unroll
      for (int c = 0; c < kVN; ++c) {
        const Col3 cc = vcol3(c);
        const bool in = okx[cc.dx + 2] && oky[cc.dy + 2] && okz[cc.dz + 2];
        const double b = in ? J[(long)jslot3(1, cc) * n + g] : 0.0;
        rec[kFB + c] = (FT)(c == kVD ? b * (1.0 + shift) : b);
      }
    } else {
#pragma unroll
      for (int c = 0; c < kUN; ++c) rec[kFA + c] = (FT)(c == kUD ? 1.0 : 0.0);
#pragma unroll
      for (int c = 0; c < kVN; ++c) rec[kFB + c] = (FT)(c == kVD ? 1.0 : 0.0);
    }
  }
  __syncthreads();
  const long cells = total - x0 < kExtractCells ? total - x0 : kExtractCells;
  FT *dst = fac + x0 * kNSlot3D;
  for (long q = threadIdx.x; q < cells * kNSlot3D; q += kExtractCells) dst[q] = tile[q];
}

// ILU(0) of the extracted records in place, level by level; with wfac, each record
// also goes to the level-major pair copy of the windowed apply ([sub][w][pair][W][2],
// at the thread owning the cell's column).
template <typename FT>
__global__ __launch_bounds__(256) void k_ilu_factor3d(BoxGeom G, const int *__restrict__ lvl,
                                                      const int *__restrict__ cells, const int *__restrict__ owner,
                                                      FT *__restrict__ fac, FT *__restrict__ wfac) {
  const Box3 B{G.bw, G.bh, G.bd};
  FT *fk = fac + (long)blockIdx.x * G.ncb * kNSlot3D;
  const int W = win3d_row(G);
  for (int w = 0; w < G.nlev; ++w) {
    for (int q = lvl[w] + threadIdx.x; q < lvl[w + 1]; q += blockDim.x) {
      int i, j, k;
      unpack(cells[q], i, j, k);
      const int e = B.at(i, j, k);
      double a[kUN], b[kVN];
      {
        const FT *own = fk + (long)e * kNSlot3D;
#pragma unroll
        for (int c = 0; c < kUN; ++c) a[c] = (double)own[kFA + c];
#pragma unroll
        for (int c = 0; c < kVN; ++c) b[c] = (double)own[kFB + c];
      }
      pivots_u(std::make_integer_sequence<int, kUL>{}, a, fk, B, i, j, k);
      a[kUD] = 1.0 / a[kUD];
      // v-row: v pivots of earlier cells, then the u-row of this cell
      pivots_v(std::make_integer_sequence<int, kVL - 1>{}, b, fk, B, i, j, k);
      {
        const double l = b[kVL - 1] * a[kUD];
        b[kVL - 1] = l;
        elim3_v_row<kVL - 1>(b, l, &a[kUD], std::make_integer_sequence<int, kUN - kUD - 1>{});
      }
      b[kVD] = 1.0 / b[kVD];
      FT *rec = fk + (long)e * kNSlot3D;
#pragma unroll
      for (int c = 0; c < kUN; ++c) rec[kFA + c] = (FT)a[c];
#pragma unroll
      for (int c = 0; c < kVN; ++c) rec[kFB + c] = (FT)b[c];
      if (wfac) {
        FT *dst = wfac + (((long)blockIdx.x * G.nlev + w) * kNSlot3D) * W + 2 * owner[j + G.bh * k];
#pragma unroll
        for (int c = 0; c < kUN; ++c) dst[(long)((kFA + c) / 2) * 2 * W + ((kFA + c) & 1)] = (FT)a[c];
#pragma unroll
        for (int c = 0; c < kVN; ++c) dst[(long)((kFB + c) / 2) * 2 * W + ((kFB + c) & 1)] = (FT)b[c];
      }
    }
    __syncthreads();
  }
}

// ---- z = M^{-1} r (left-restricted) ---------------------------------------------
template <typename FT>
__global__ __launch_bounds__(256) void k_ras_apply3d(Phys P, BoxGeom G, const SubInfo *__restrict__ subs,
                                                     const int *__restrict__ lvl, const int *__restrict__ cells,
                                                     const FT *__restrict__ fac, double2 *__restrict__ ybuf,
                                                     const double *__restrict__ r, double *__restrict__ z,
                                                     const GmresState *st, long vstride, int kind) {
  double sc = 1.0;
  if (st) {
    if (st->done) return;
    const int jj = st->j;
    r += (long)jj * vstride;
    z += (long)jj * vstride;
    sc = st->inv_norm[jj];
  }
  const SubInfo si = subs[blockIdx.x];
  const Box3 B{G.bw, G.bh, G.bd};
  const long n = (long)P.nx * P.ny * P.nz;
  const FT *fk = fac + (long)blockIdx.x * G.ncb * kNSlot3D;
  double2 *yb = ybuf + (long)blockIdx.x * G.ncb;
  for (int e = threadIdx.x; e < G.ncb; e += blockDim.x) {
    int i, j, k;
    decode(e, B, i, j, k);
    const long g = box3_to_global(si, i, j, k, P);
    // the right-restricted variant restricts the input to the owned cells
    const bool take = g >= 0 && (kind != ACCH_RAS_RIGHT || owned3(si, i, j, k));
    yb[e] = take ? make_double2(sc * r[g], sc * r[n + g]) : make_double2(0.0, 0.0);
  }
  __syncthreads();
  // L y = R r
  for (int w = 0; w < G.nlev; ++w) {
    for (int q = lvl[w] + threadIdx.x; q < lvl[w + 1]; q += blockDim.x) {
      int i, j, k;
      unpack(cells[q], i, j, k);
      const int e = B.at(i, j, k);
      const FT *rec = fk + (long)e * kNSlot3D;
      const double2 y0 = yb[e];
      double yu = y0.x, yv = y0.y;
#pragma unroll
      for (int c = 0; c < kUL; ++c) {
        const Col3 cc = ucol3(c);
        bool in;
        const double2 v = yb[nb_or(B, i, j, k, cc.dx, cc.dy, cc.dz, e, in)];
        const double l = in ? (double)rec[kFA + c] : 0.0;
        yu = fma(-l, cc.t == 0 ? v.x : v.y, yu);
      }
#pragma unroll
      for (int c = 0; c < kVL - 1; ++c) {
        const Col3 cc = vcol3(c);
        bool in;
        const double2 v = yb[nb_or(B, i, j, k, cc.dx, cc.dy, cc.dz, e, in)];
        const double l = in ? (double)rec[kFB + c] : 0.0;
        yv = fma(-l, cc.t == 0 ? v.x : v.y, yv);
      }
      yv -= (double)rec[kFB + kVL - 1] * yu;
      yb[e] = make_double2(yu, yv);
    }
    __syncthreads();
  }
  // U x = y
  for (int w = G.nlev - 1; w >= 0; --w) {
    for (int q = lvl[w] + threadIdx.x; q < lvl[w + 1]; q += blockDim.x) {
      int i, j, k;
      unpack(cells[q], i, j, k);
      const int e = B.at(i, j, k);
      const FT *rec = fk + (long)e * kNSlot3D;
      const double2 y0 = yb[e];
      double xv = y0.y;
#pragma unroll
      for (int c = kVD + 1; c < kVN; ++c) {
        const Col3 cc = vcol3(c);
        bool in;
        const double2 v = yb[nb_or(B, i, j, k, cc.dx, cc.dy, cc.dz, e, in)];
        const double u = in ? (double)rec[kFB + c] : 0.0;
        xv = fma(-u, cc.t == 0 ? v.x : v.y, xv);
      }
      xv *= (double)rec[kFB + kVD];
      double xu = y0.x - (double)rec[kFA + kUD + 1] * xv;   // column (0,0,0,v)
#pragma unroll
      for (int c = kUD + 2; c < kUN; ++c) {
        const Col3 cc = ucol3(c);
        bool in;
        const double2 v = yb[nb_or(B, i, j, k, cc.dx, cc.dy, cc.dz, e, in)];
        const double u = in ? (double)rec[kFA + c] : 0.0;
        xu = fma(-u, cc.t == 0 ? v.x : v.y, xu);
      }
      xu *= (double)rec[kFA + kUD];
      yb[e] = make_double2(xu, xv);
    }
    __syncthreads();
  }
  // right-restricted / classical: the whole box stays in the box buffer and is summed
  // over the boxes of each cell by k_ras_t_gather3d
  if (kind != ACCH_RAS_LEFT) return;
  for (int e = threadIdx.x; e < G.ncb; e += blockDim.x) {
    int i, j, k;
    decode(e, B, i, j, k);
    const long g = box3_to_global(si, i, j, k, P);
    if (g >= 0 && owned3(si, i, j, k)) {
      z[g] = yb[e].x;
      z[n + g] = yb[e].y;
    }
  }
}

// ---- z = M^{-1} r through a rolling LDS window (left-restricted) ------------------
// A sweep at level w reads neighbours at most 6 levels away (offset (0,0,-2) forward,
// (0,0,+2) backward), and the cells of one level differ in (j, k).  LDS slot
// (i mod 8, j, k) therefore holds every value a level reads: a cell's slot is next
// written 8 levels later, by (i + 8, j, k) forward or (i - 8, j, k) backward.  The
// window starts zeroed and only ever holds finite values, and a factor entry of a
// column outside the box is exactly zero (factorisation above), so a neighbour read
// needs no mask, only an address kept inside the window.
//
// Threads own box columns (j, k) (host-built lists, columns of one thread busy on
// disjoint level ranges), so a thread finds its cell of a level from a column cursor.
// Factor entries and forward results sit in level-major arrays (the entry of thread t
// on level w at w * W + t; the factorisation fills the factor copy), so a wave's
// accesses to them are contiguous.  The operands of a level (right-hand side or
// forward result, factor entries) are loaded two levels ahead, and the barrier
// between levels waits for LDS only, so those loads stay in flight across it.  Every
// device-memory access of the sweeps is unconditional, so the count of outstanding
// accesses is the same on every path and the compiler waits for exactly the level it
// needs: an idle thread's buffer accesses fall past the end of the buffer (no memory
// access), its right-hand-side load reads cell 0 and its z values go to a spare pair
// after the box buffers.
constexpr int kWinSpan = 8;   // window depth in i: more than the 6 levels a sweep reaches back
static_assert(kWin3DSlots == kNSlot3D, "level-major factor copy holds whole records");

struct WinCell {
  int i, j, k;
  bool act;   // the thread has a cell on this level
};
// Factor entries travel in pairs of consecutive slots (one 16-byte load in FP64): the
// forward sweep reads pairs 0..7 (u-row multipliers, slot 15 unused) and 16..17
// (v-row), the backward sweep pairs 7..15 (u-row U part, slot 14 unused) and 18..19.
constexpr int kPairs = kNSlot3D / 2;
constexpr int kFwdPairsU = 8, kBwdPair0U = 7, kBwdPairsU = 9;

struct WinFwd {
  WinCell c;
  bool dom;                  // inside the domain (else a decoupled identity row with rhs 0)
  double ru, rv;             // right-hand side as loaded
  double lu[2 * kFwdPairsU]; // u-row multipliers in 0..14
  double lv[kVL];            // v-row multipliers, the last one for column (0,0,0,u)
};
struct WinBwd {
  WinCell c;
  double yu, yv;             // forward-sweep result
  double uu[2 * kBwdPairsU]; // u-row: slot 14 (unused), inverted diagonal, then U
  double uv[kVN - kVD];      // v-row: inverted diagonal, then U
};

// Barrier for values exchanged through LDS only: device-memory loads issued before it
// stay in flight (__syncthreads would also wait for them).
ACCH_DEV void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// A thread's columns, packed j | k << 10 (-1: none), the current one first.
struct ColCursor {
  int col[kWin3DCols];
  ACCH_DEV static int first_level(int c) { return c < 0 ? (1 << 29) : 2 * (c & 1023) + 3 * (c >> 10); }
  // Cell of level w (levels visited one by one, upward if `up`, else downward).
  ACCH_DEV WinCell at(int w, int bw, bool up) {
    const int o = first_level(col[0]);
    const bool next = up ? w >= o + bw : w < o;
#pragma unroll
    for (int m = 0; m + 1 < kWin3DCols; ++m) col[m] = next ? col[m + 1] : col[m];
    col[kWin3DCols - 1] = next ? -1 : col[kWin3DCols - 1];
    const int c = col[0], o2 = first_level(c), i = w - o2;
    const bool act = c >= 0 && i >= 0 && i < bw;
    return act ? WinCell{i, c & 1023, c >> 10, true} : WinCell{0, 0, 0, false};
  }
};

// one pair of factor entries
ACCH_DEV void pair_load(__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff, const double *, double &a,
                        double &b) {
  const double_pair d = __builtin_bit_cast(double_pair, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0));
  a = d.x;
  b = d.y;
}
ACCH_DEV void pair_load(__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff, const float *, double &a,
                        double &b) {
  const float_pair f = __builtin_bit_cast(float_pair, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0));
  a = (double)f.x;
  b = (double)f.y;
}

// Operands are loaded D levels ahead: D + 1 operand sets rotate by name through a
// loop unrolled D + 1 times (copying a set still being loaded would wait for it).
template <typename FT, int D>
__global__ __launch_bounds__(kWin3DThreads) void k_ras_apply3d_win(
    Phys P, BoxGeom G, const SubInfo *__restrict__ subs, const int *__restrict__ wcols, const FT *__restrict__ wfac,
    double2 *__restrict__ ybuf, double *__restrict__ spare, const double *__restrict__ r, double *__restrict__ z,
    const GmresState *st, long vstride) {
  extern __shared__ double2 win[];   // kWinSpan * bh * bd values
  double sc = 1.0;
  if (st) {
    if (st->done) return;
    const int jj = st->j;
    r += (long)jj * vstride;
    z += (long)jj * vstride;
    sc = st->inv_norm[jj];
  }
  const SubInfo si = subs[blockIdx.x];
  const long n = (long)P.nx * P.ny * P.nz;
  const int W = blockDim.x;   // row width of the level-major arrays
  const unsigned tid = threadIdx.x;
  // this box's level-major factor pairs [level][pair][W] and forward results [level][W]
  const long fbox = (long)G.nlev * kNSlot3D * W;
  const __amdgpu_buffer_rsrc_t rsF = buffer_rsrc(wfac + blockIdx.x * fbox, (unsigned)(fbox * sizeof(FT)));
  const __amdgpu_buffer_rsrc_t rsY =
      buffer_rsrc(ybuf + (long)blockIdx.x * G.nlev * W, (unsigned)((long)G.nlev * W * sizeof(double2)));
  // (uniform: kept in a scalar register, as the loads' scalar offsets need)
  const unsigned pair_bytes = __builtin_amdgcn_readfirstlane((unsigned)W * 2 * sizeof(FT));
  const int plane = G.bh * G.bd;
  const unsigned last_slot = (unsigned)(kWinSpan * plane - 1);
  const int top = G.nlev - 1;
  for (int e = threadIdx.x; e <= (int)last_slot; e += W) win[e] = make_double2(0.0, 0.0);
  ColCursor cur;
#pragma unroll
  for (int m = 0; m < kWin3DCols; ++m) cur.col[m] = wcols[m * kWin3DThreads + threadIdx.x];
  __syncthreads();

  // byte offset of this thread's pair 0 on level w (past the end when idle)
  auto foff = [&](const WinCell &c, int w) -> unsigned {
    return c.act ? ((unsigned)w * kPairs * W + tid) * (unsigned)(2 * sizeof(FT)) : kPastEnd;
  };
  auto yoff = [&](const WinCell &c, int w) -> unsigned {
    return c.act ? ((unsigned)w * W + tid) * (unsigned)sizeof(double2) : kPastEnd;
  };
  // value pair of the neighbour at offset cc of cell c (any finite pair outside the box)
  auto nb = [&](const WinCell &c, const Col3 cc) -> double2 {
    const int s = ((c.i + cc.dx) & (kWinSpan - 1)) * plane + (c.j + cc.dy) * G.bd + (c.k + cc.dz);
    return win[min((unsigned)s, last_slot)];
  };
  auto fetch_fwd = [&](int w, WinFwd &d) {
    d.c = cur.at(w, G.bw, true);
    const long g = box3_to_global(si, d.c.i, d.c.j, d.c.k, P);
    d.dom = g >= 0;
    const long gs = g >= 0 ? g : 0;
    d.ru = r[gs];
    d.rv = r[n + gs];
    const unsigned o = foff(d.c, w);
#pragma unroll
    for (int q = 0; q < kFwdPairsU; ++q) pair_load(rsF, o, q * pair_bytes, wfac, d.lu[2 * q], d.lu[2 * q + 1]);
#pragma unroll
    for (int q = 0; q < kVL / 2; ++q)
      pair_load(rsF, o, (kFB / 2 + q) * pair_bytes, wfac, d.lv[2 * q], d.lv[2 * q + 1]);
  };
  auto fetch_bwd = [&](int w, WinBwd &d) {
    d.c = cur.at(w, G.bw, false);
    const double_pair y =
        __builtin_bit_cast(double_pair, __builtin_amdgcn_raw_buffer_load_b128(rsY, yoff(d.c, w), 0, 0));
    d.yu = y.x;
    d.yv = y.y;
    const unsigned o = foff(d.c, w);
#pragma unroll
    for (int q = 0; q < kBwdPairsU; ++q)
      pair_load(rsF, o, (kBwdPair0U + q) * pair_bytes, wfac, d.uu[2 * q], d.uu[2 * q + 1]);
#pragma unroll
    for (int q = 0; q < (kVN - kVD) / 2; ++q)
      pair_load(rsF, o, ((kFB + kVD) / 2 + q) * pair_bytes, wfac, d.uv[2 * q], d.uv[2 * q + 1]);
  };
  auto slot = [&](const WinCell &c) { return (c.i & (kWinSpan - 1)) * plane + c.j * G.bd + c.k; };

  // L y = R r
  {
    auto level = [&](const WinFwd &d, int w) {
      const WinCell &c = d.c;
      double yu = d.dom ? sc * d.ru : 0.0, yv = d.dom ? sc * d.rv : 0.0;
#pragma unroll
      for (int q = 0; q < kUL; ++q) {
        const Col3 cc = ucol3(q);
        const double2 v = nb(c, cc);
        yu = fma(-d.lu[q], cc.t == 0 ? v.x : v.y, yu);
      }
#pragma unroll
      for (int q = 0; q < kVL - 1; ++q) {
        const Col3 cc = vcol3(q);
        const double2 v = nb(c, cc);
        yv = fma(-d.lv[q], cc.t == 0 ? v.x : v.y, yv);
      }
      yv = fma(-d.lv[kVL - 1], yu, yv);
      if (c.act) win[slot(c)] = make_double2(yu, yv);
      const double_pair y{yu, yv};
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(word4, y), rsY, yoff(c, w), 0, 0);
      lds_barrier();
    };
    WinFwd s[D + 1];
#pragma unroll
    for (int m = 0; m < D; ++m) fetch_fwd(m, s[m]);
    for (int w = 0; w <= top; w += D + 1) {
#pragma unroll
      for (int m = 0; m <= D; ++m) {
        fetch_fwd(w + m + D, s[(m + D) % (D + 1)]);
        level(s[m], w + m);
      }
    }
  }
#pragma unroll
  for (int m = 0; m < kWin3DCols; ++m) cur.col[m] = wcols[(kWin3DCols + m) * kWin3DThreads + threadIdx.x];
  __syncthreads();   // the forward results in the box buffer are read below
  // U x = y, owned cells straight to z
  {
    auto level = [&](const WinBwd &d) {
      const WinCell &c = d.c;
      double xv = d.yv;
#pragma unroll
      for (int q = kVD + 1; q < kVN; ++q) {
        const Col3 cc = vcol3(q);
        const double2 v = nb(c, cc);
        xv = fma(-d.uv[q - kVD], cc.t == 0 ? v.x : v.y, xv);
      }
      xv *= d.uv[0];
      double xu = fma(-d.uu[2], xv, d.yu);   // column (0,0,0,v)
#pragma unroll
      for (int q = kUD + 2; q < kUN; ++q) {
        const Col3 cc = ucol3(q);
        const double2 v = nb(c, cc);
        xu = fma(-d.uu[q - kUD + 1], cc.t == 0 ? v.x : v.y, xu);
      }
      xu *= d.uu[1];
      if (c.act) win[slot(c)] = make_double2(xu, xv);
      const long g = box3_to_global(si, c.i, c.j, c.k, P);
      const bool out = c.act && g >= 0 && owned3(si, c.i, c.j, c.k);
      *(out ? z + g : spare) = xu;
      *(out ? z + n + g : spare + 1) = xv;
      lds_barrier();
    };
    WinBwd t[D + 1];
#pragma unroll
    for (int m = 0; m < D; ++m) fetch_bwd(top - m, t[m]);
    for (int w = top; w >= 0; w -= D + 1) {
#pragma unroll
      for (int m = 0; m <= D; ++m) {
        fetch_bwd(w - m - D, t[(m + D) % (D + 1)]);
        level(t[m]);
      }
    }
  }
}

// ---- z = M^{-T} r through the LDS window (adjoint) --------------------------------
// M^{-T} = sum_k (R_k^delta)^T (L_k U_k)^{-T} R_k^0: restrict r to the owned cells,
// solve U^T y = R r (lower triangular: levels upward) and L^T x = y (levels
// downward), then add every box's x into z (k_ras_t_gather3d).  Row p of U^T / L^T
// holds the coefficients of column p of U / L, which sit in the rows of the cells
// q = p - o for the pattern offsets o of those rows; a transposed record gathers them
// per cell (k_pack_window3d_t), so the sweeps have the shape of the forward apply:
// own-record loads, neighbour values from the window (q lies at most 6 levels away).
//
// Transposed record slots (value of row q at column p, zero when q is outside the box):
//   0..11  U[u_q][u_p], q = p - o over the u-row's U columns of type u
//   12     1 / U[u_p][u_p]
//   13..16 U[u_q][v_p] over the u-row's U columns of type v (the first: q = p)
//   17..19 U[v_q][v_p] over the v-row's U columns
//   20     1 / U[v_p][v_p]
//   21..32 L[u_q][u_p] over the u-row's L columns of type u
//   33     L[v_p][u_p]
//   34..36 L[u_q][v_p] over the u-row's L columns of type v
//   37..39 L[v_q][v_p] over the v-row's L columns
// The forward sweep reads pairs 0..10 (slot 21 unused), the backward pairs 10..19
// (slot 20 unused).
__host__ __device__ constexpr int nth_ucol(int lo, int hi, int t, int m) {
  for (int c = lo; c < hi; ++c)
    if (ucol3(c).t == t && m-- == 0) return c;
  return -1;
}
constexpr int kTUU = 0, kTUI = 12, kTVU = 13, kTVV = 17, kTVI = 20, kTLUU = 21, kTLUV = 33, kTLVU = 34, kTLVV = 37;
constexpr int kTFwdPairs = 11, kTBwdPair0 = 10, kTBwdPairs = 10;
// pattern column of transposed slot m: (is_u_row_of_q, column index in that row)
__host__ __device__ constexpr Col3 tcol(int m, bool &urow, int &slot) {
  if (m < kTUI) { slot = kFA + nth_ucol(kUD + 1, kUN, 0, m - kTUU); urow = true; return ucol3(slot - kFA); }
  if (m == kTUI) { slot = kFA + kUD; urow = true; return ucol3(kUD); }
  if (m < kTVV) { slot = kFA + nth_ucol(kUD + 1, kUN, 1, m - kTVU); urow = true; return ucol3(slot - kFA); }
  if (m < kTVI) { slot = kFB + kVD + 1 + (m - kTVV); urow = false; return vcol3(slot - kFB); }
  if (m == kTVI) { slot = kFB + kVD; urow = false; return vcol3(kVD); }
  if (m < kTLUV) { slot = kFA + nth_ucol(0, kUL, 0, m - kTLUU); urow = true; return ucol3(slot - kFA); }
  if (m == kTLUV) { slot = kFB + kVL - 1; urow = false; return vcol3(kVL - 1); }
  if (m < kTLVV) { slot = kFA + nth_ucol(0, kUL, 1, m - kTLVU); urow = true; return ucol3(slot - kFA); }
  slot = kFB + (m - kTLVV);
  urow = false;
  return vcol3(m - kTLVV);
}
__host__ __device__ constexpr bool tcols_consistent() {
  // 12 + 4 u-row U columns, 12 + 3 u-row L columns, the first v-type U column at p itself
  bool ok = nth_ucol(kUD + 1, kUN, 0, 11) >= 0 && nth_ucol(kUD + 1, kUN, 0, 12) < 0 &&
            nth_ucol(kUD + 1, kUN, 1, 3) >= 0 && nth_ucol(kUD + 1, kUN, 1, 4) < 0 &&
            nth_ucol(0, kUL, 0, 11) >= 0 && nth_ucol(0, kUL, 0, 12) < 0 && nth_ucol(0, kUL, 1, 2) >= 0 &&
            nth_ucol(0, kUL, 1, 3) < 0;
  const Col3 own = ucol3(nth_ucol(kUD + 1, kUN, 1, 0));
  return ok && own.dx == 0 && own.dy == 0 && own.dz == 0;
}
static_assert(tcols_consistent(), "transposed record layout");

template <typename FT>
__global__ __launch_bounds__(kWin3DThreads) void k_pack_window3d_t(BoxGeom G, const int *__restrict__ wcols,
                                                                   const FT *__restrict__ fac,
                                                                   FT *__restrict__ wfact) {
  const int w = blockIdx.x, sub = blockIdx.y, W = blockDim.x, t = threadIdx.x;
  int i = 0, j = 0, k = 0;
  bool found = false;
#pragma unroll
  for (int m = 0; m < kWin3DCols; ++m) {
    const int c = wcols[m * kWin3DThreads + t];
    const int jj = c & 1023, kk = c >> 10, ii = w - 2 * jj - 3 * kk;
    if (c >= 0 && ii >= 0 && ii < G.bw) {
      i = ii;
      j = jj;
      k = kk;
      found = true;
    }
  }
  if (!found) return;
  const Box3 B{G.bw, G.bh, G.bd};
  const FT *fk = fac + (long)sub * G.ncb * kNSlot3D;
  FT *dst = wfact + (((long)sub * G.nlev + w) * kNSlot3D) * W + 2 * t;
#pragma unroll
  for (int m = 0; m < kNSlot3D; ++m) {
    bool urow = false;
    int slot = 0;
    const Col3 cc = tcol(m, urow, slot);
    const int qi = i - cc.dx, qj = j - cc.dy, qk = k - cc.dz;   // the row holding column p
    const FT v = B.in(qi, qj, qk) ? fk[(long)B.at(qi, qj, qk) * kNSlot3D + slot] : (FT)0;
    dst[(long)(m / 2) * 2 * W + (m & 1)] = v;
  }
}

template <typename FT, int D>
__global__ __launch_bounds__(kWin3DThreads) void k_ras_t_apply3d_win(
    Phys P, BoxGeom G, const SubInfo *__restrict__ subs, const int *__restrict__ wcols, const FT *__restrict__ wfact,
    double2 *__restrict__ ybuf, double2 *__restrict__ tbox, const double *__restrict__ r, const GmresState *st,
    long vstride) {
  extern __shared__ double2 win[];   // kWinSpan * bh * bd values
  double sc = 1.0;
  if (st) {
    if (st->done) return;
    r += (long)st->j * vstride;
    sc = st->inv_norm[st->j];
  }
  const SubInfo si = subs[blockIdx.x];
  const Box3 B{G.bw, G.bh, G.bd};
  const long n = (long)P.nx * P.ny * P.nz;
  const int W = blockDim.x;
  const unsigned tid = threadIdx.x;
  const long fbox = (long)G.nlev * kNSlot3D * W;
  const __amdgpu_buffer_rsrc_t rsF = buffer_rsrc(wfact + blockIdx.x * fbox, (unsigned)(fbox * sizeof(FT)));
  const __amdgpu_buffer_rsrc_t rsY =
      buffer_rsrc(ybuf + (long)blockIdx.x * G.nlev * W, (unsigned)((long)G.nlev * W * sizeof(double2)));
  const __amdgpu_buffer_rsrc_t rsX =
      buffer_rsrc(tbox + (long)blockIdx.x * G.ncb, (unsigned)((long)G.ncb * sizeof(double2)));
  const unsigned pair_bytes = __builtin_amdgcn_readfirstlane((unsigned)W * 2 * sizeof(FT));
  const int plane = G.bh * G.bd;
  const unsigned last_slot = (unsigned)(kWinSpan * plane - 1);
  const int top = G.nlev - 1;
  for (int e = threadIdx.x; e <= (int)last_slot; e += W) win[e] = make_double2(0.0, 0.0);
  ColCursor cur;
#pragma unroll
  for (int m = 0; m < kWin3DCols; ++m) cur.col[m] = wcols[m * kWin3DThreads + threadIdx.x];
  __syncthreads();

  auto foff = [&](const WinCell &c, int w) -> unsigned {
    return c.act ? ((unsigned)w * kPairs * W + tid) * (unsigned)(2 * sizeof(FT)) : kPastEnd;
  };
  auto yoff = [&](const WinCell &c, int w) -> unsigned {
    return c.act ? ((unsigned)w * W + tid) * (unsigned)sizeof(double2) : kPastEnd;
  };
  // value pair at cell c - o (the row q of a transposed entry; any finite pair outside the box)
  auto nbm = [&](const WinCell &c, const Col3 o) -> double2 {
    const int s = ((c.i - o.dx) & (kWinSpan - 1)) * plane + (c.j - o.dy) * G.bd + (c.k - o.dz);
    return win[min((unsigned)s, last_slot)];
  };
  auto slot = [&](const WinCell &c) { return (c.i & (kWinSpan - 1)) * plane + c.j * G.bd + c.k; };
  struct TF {
    WinCell c;
    bool own;
    double ru, rv;
    double e[2 * kTFwdPairs];
  };
  struct TB {
    WinCell c;
    double yu, yv;
    double e[2 * kTBwdPairs];
  };
  auto fetch_f = [&](int w, TF &d) {
    d.c = cur.at(w, G.bw, true);
    const long g = box3_to_global(si, d.c.i, d.c.j, d.c.k, P);
    d.own = g >= 0 && owned3(si, d.c.i, d.c.j, d.c.k);
    const long gs = g >= 0 ? g : 0;
    d.ru = r[gs];
    d.rv = r[n + gs];
    const unsigned o = foff(d.c, w);
#pragma unroll
    for (int q = 0; q < kTFwdPairs; ++q) pair_load(rsF, o, q * pair_bytes, wfact, d.e[2 * q], d.e[2 * q + 1]);
  };
  auto fetch_b = [&](int w, TB &d) {
    d.c = cur.at(w, G.bw, false);
    const double_pair y =
        __builtin_bit_cast(double_pair, __builtin_amdgcn_raw_buffer_load_b128(rsY, yoff(d.c, w), 0, 0));
    d.yu = y.x;
    d.yv = y.y;
    const unsigned o = foff(d.c, w);
#pragma unroll
    for (int q = 0; q < kTBwdPairs; ++q)
      pair_load(rsF, o, (kTBwdPair0 + q) * pair_bytes, wfact, d.e[2 * q], d.e[2 * q + 1]);
  };
  // U^T y = R^0 r
  {
    auto level = [&](const TF &d, int w) {
      const WinCell &c = d.c;
      double yu = d.own ? sc * d.ru : 0.0, yv = d.own ? sc * d.rv : 0.0;
#pragma unroll
      for (int m = kTUU; m < kTUI; ++m) {
        bool urow = false;
        int sl = 0;
        yu = fma(-d.e[m], nbm(c, tcol(m, urow, sl)).x, yu);
      }
      yu *= d.e[kTUI];
      yv = fma(-d.e[kTVU], yu, yv);   // q = p
#pragma unroll
      for (int m = kTVU + 1; m < kTVV; ++m) {
        bool urow = false;
        int sl = 0;
        yv = fma(-d.e[m], nbm(c, tcol(m, urow, sl)).x, yv);
      }
#pragma unroll
      for (int m = kTVV; m < kTVI; ++m) {
        bool urow = false;
        int sl = 0;
        yv = fma(-d.e[m], nbm(c, tcol(m, urow, sl)).y, yv);
      }
      yv *= d.e[kTVI];
      if (c.act) win[slot(c)] = make_double2(yu, yv);
      const double_pair y{yu, yv};
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(word4, y), rsY, yoff(c, w), 0, 0);
      lds_barrier();
    };
    TF s[D + 1];
#pragma unroll
    for (int m = 0; m < D; ++m) fetch_f(m, s[m]);
    for (int w = 0; w <= top; w += D + 1) {
#pragma unroll
      for (int m = 0; m <= D; ++m) {
        fetch_f(w + m + D, s[(m + D) % (D + 1)]);
        level(s[m], w + m);
      }
    }
  }
#pragma unroll
  for (int m = 0; m < kWin3DCols; ++m) cur.col[m] = wcols[(kWin3DCols + m) * kWin3DThreads + threadIdx.x];
  __syncthreads();   // the forward results are read below
  // L^T x = y; the whole box's x to tbox (cell order)
  {
    auto level = [&](const TB &d) {
      const WinCell &c = d.c;
      constexpr int o = kTBwdPair0 * 2;   // slot of d.e[0]
      double xv = d.yv;
#pragma unroll
      for (int m = kTLVU; m < kTLVV; ++m) {
        bool urow = false;
        int sl = 0;
        xv = fma(-d.e[m - o], nbm(c, tcol(m, urow, sl)).x, xv);
      }
#pragma unroll
      for (int m = kTLVV; m < kNSlot3D; ++m) {
        bool urow = false;
        int sl = 0;
        xv = fma(-d.e[m - o], nbm(c, tcol(m, urow, sl)).y, xv);
      }
      double xu = fma(-d.e[kTLUV - o], xv, d.yu);   // L[v_p][u_p]
#pragma unroll
      for (int m = kTLUU; m < kTLUV; ++m) {
        bool urow = false;
        int sl = 0;
        xu = fma(-d.e[m - o], nbm(c, tcol(m, urow, sl)).x, xu);
      }
      if (c.act) win[slot(c)] = make_double2(xu, xv);
      const double_pair x{xu, xv};
      const unsigned xo = c.act ? (unsigned)B.at(c.i, c.j, c.k) * (unsigned)sizeof(double2) : kPastEnd;
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(word4, x), rsX, xo, 0, 0);
      lds_barrier();
    };
    TB t[D + 1];
#pragma unroll
    for (int m = 0; m < D; ++m) fetch_b(top - m, t[m]);
    for (int w = top; w >= 0; w -= D + 1) {
#pragma unroll
      for (int m = 0; m <= D; ++m) {
        fetch_b(w - m - D, t[(m + D) % (D + 1)]);
        level(t[m]);
      }
    }
  }
}

// ---- z = M^{-T} r: restrict to owned cells, U^T then L^T sweeps (coefficients of
// the neighbour rows), add whole boxes (k_ras_t_gather3d) ---------------------------
template <typename FT>
__global__ __launch_bounds__(256) void k_ras_t_sweep3d(Phys P, BoxGeom G, const SubInfo *__restrict__ subs,
                                                       const int *__restrict__ lvl, const int *__restrict__ cells,
                                                       const FT *__restrict__ fac, double2 *__restrict__ ybuf,
                                                       const double *__restrict__ r, const GmresState *st,
                                                       long vstride) {
  double sc = 1.0;
  if (st) {
    if (st->done) return;
    const int jj = st->j;
    r += (long)jj * vstride;
    sc = st->inv_norm[jj];
  }
  const SubInfo si = subs[blockIdx.x];
  const Box3 B{G.bw, G.bh, G.bd};
  const long n = (long)P.nx * P.ny * P.nz;
  const FT *fk = fac + (long)blockIdx.x * G.ncb * kNSlot3D;
  double2 *yb = ybuf + (long)blockIdx.x * G.ncb;
  for (int e = threadIdx.x; e < G.ncb; e += blockDim.x) {
    int i, j, k;
    decode(e, B, i, j, k);
    const long g = box3_to_global(si, i, j, k, P);
    const bool own = g >= 0 && owned3(si, i, j, k);
    yb[e] = own ? make_double2(sc * r[g], sc * r[n + g]) : make_double2(0.0, 0.0);
  }
  __syncthreads();
  auto coefq = [&](int q, int slot) -> double { return (double)fk[(long)q * kNSlot3D + slot]; };
  // U^T y = R r: column p receives the U entries of the earlier rows q = p - o
  for (int w = 0; w < G.nlev; ++w) {
    for (int q = lvl[w] + threadIdx.x; q < lvl[w + 1]; q += blockDim.x) {
      int i, j, k;
      unpack(cells[q], i, j, k);
      const int e = B.at(i, j, k);
      const double2 y0 = yb[e];
      double yu = y0.x, yv = y0.y;
#pragma unroll
      for (int c = kUD + 1; c < kUN; ++c) {   // u-rows q with a u column at p
        const Col3 cc = ucol3(c);
        if (cc.t != 0) continue;
        bool in;
        const int nq = nb_or(B, i, j, k, -cc.dx, -cc.dy, -cc.dz, e, in);
        const double u = in ? coefq(nq, kFA + c) : 0.0;
        yu = fma(-u, yb[nq].x, yu);
      }
      yu *= coefq(e, kFA + kUD);
#pragma unroll
      for (int c = kUD + 1; c < kUN; ++c) {   // u-rows q with a v column at p (q = p for (0,0,0,v))
        const Col3 cc = ucol3(c);
        if (cc.t != 1) continue;
        bool in;
        const int nq = nb_or(B, i, j, k, -cc.dx, -cc.dy, -cc.dz, e, in);
        const double u = in ? coefq(nq, kFA + c) : 0.0;
        const double yq = (cc.dx == 0 && cc.dy == 0 && cc.dz == 0) ? yu : yb[nq].x;
        yv = fma(-u, yq, yv);
      }
#pragma unroll
      for (int c = kVD + 1; c < kVN; ++c) {   // v-rows q with a v column at p
        const Col3 cc = vcol3(c);
        bool in;
        const int nq = nb_or(B, i, j, k, -cc.dx, -cc.dy, -cc.dz, e, in);
        const double u = in ? coefq(nq, kFB + c) : 0.0;
        yv = fma(-u, yb[nq].y, yv);
      }
      yv *= coefq(e, kFB + kVD);
      yb[e] = make_double2(yu, yv);
    }
    __syncthreads();
  }
  // L^T x = y (unit diagonal): column p receives the L entries of the later rows
  for (int w = G.nlev - 1; w >= 0; --w) {
    for (int q = lvl[w] + threadIdx.x; q < lvl[w + 1]; q += blockDim.x) {
      int i, j, k;
      unpack(cells[q], i, j, k);
      const int e = B.at(i, j, k);
      const double2 y0 = yb[e];
      double xu = y0.x, xv = y0.y;
#pragma unroll
      for (int c = 0; c < kUL; ++c) {   // u-rows q with a v column at p
        const Col3 cc = ucol3(c);
        if (cc.t != 1) continue;
        bool in;
        const int nq = nb_or(B, i, j, k, -cc.dx, -cc.dy, -cc.dz, e, in);
        const double l = in ? coefq(nq, kFA + c) : 0.0;
        xv = fma(-l, yb[nq].x, xv);
      }
#pragma unroll
      for (int c = 0; c < kVL - 1; ++c) {   // v-rows q with a v column at p
        const Col3 cc = vcol3(c);
        bool in;
        const int nq = nb_or(B, i, j, k, -cc.dx, -cc.dy, -cc.dz, e, in);
        const double l = in ? coefq(nq, kFB + c) : 0.0;
        xv = fma(-l, yb[nq].y, xv);
      }
#pragma unroll
      for (int c = 0; c < kUL; ++c) {   // u-rows q with a u column at p
        const Col3 cc = ucol3(c);
        if (cc.t != 0) continue;
        bool in;
        const int nq = nb_or(B, i, j, k, -cc.dx, -cc.dy, -cc.dz, e, in);
        const double l = in ? coefq(nq, kFA + c) : 0.0;
        xu = fma(-l, yb[nq].x, xu);
      }
      xu -= coefq(e, kFB + kVL - 1) * xv;   // the v-row of this cell, column (0,0,0,u)
      yb[e] = make_double2(xu, xv);
    }
    __syncthreads();
  }
}

// z = sum over the boxes holding a cell (owner and neighbour subdomains per axis).
__global__ __launch_bounds__(256) void k_ras_t_gather3d(Phys P, BoxGeom G, const SubInfo *__restrict__ subs, int px,
                                                        int py, int pz, const int *__restrict__ own,
                                                        const double2 *__restrict__ ybuf, double *__restrict__ z,
                                                        const GmresState *st, long vstride) {
  if (st && st->done) return;
  const int jj = st ? st->j : 0;
  const long n = (long)P.nx * P.ny * P.nz;
  double *zu = z + (long)jj * vstride, *zv = zu + n;
  const int *own_x = own, *own_y = own + P.nx, *own_z = own + P.nx + P.ny;
  const Box3 B{G.bw, G.bh, G.bd};
  for (long g = blockIdx.x * 256L + threadIdx.x; g < n; g += (long)gridDim.x * 256) {
    const int gx = (int)(g % P.nx), gy = (int)((g / P.nx) % P.ny), gz = (int)(g / ((long)P.nx * P.ny));
    int cs[3][3], nc[3] = {0, 0, 0};
    const int o3[3] = {own_x[gx], own_y[gy], own_z[gz]}, p3[3] = {px, py, pz};
    for (int a = 0; a < 3; ++a)
      for (int d = -1; d <= 1; ++d) {
        int s = o3[a] + d;
        if (P.periodic) s = (s + p3[a]) % p3[a];
        bool fresh = s >= 0 && s < p3[a];
        for (int q = 0; q < nc[a]; ++q) fresh = fresh && cs[a][q] != s;
        if (fresh) cs[a][nc[a]++] = s;
      }
    double su = 0.0, sv = 0.0;
    for (int c = 0; c < nc[2]; ++c)
      for (int b = 0; b < nc[1]; ++b)
        for (int a = 0; a < nc[0]; ++a) {
          const int kb = (cs[2][c] * py + cs[1][b]) * px + cs[0][a];
          const SubInfo si = subs[kb];
          int lx = gx - si.ox, ly = gy - si.oy, lz = gz - si.oz;
          if (P.periodic) {
            lx = ((lx % P.nx) + P.nx) % P.nx;
            ly = ((ly % P.ny) + P.ny) % P.ny;
            lz = ((lz % P.nz) + P.nz) % P.nz;
          }
          if (lx >= 0 && lx < si.ex && ly >= 0 && ly < si.ey && lz >= 0 && lz < si.ez) {
            const double2 v = ybuf[(long)kb * G.ncb + B.at(lx, ly, lz)];
            su += v.x;
            sv += v.y;
          }
        }
    zu[g] = su;
    zv[g] = sv;
  }
}

// Factors of box cells -> FP64 [sub][slot][cell] (the 40-slot record of each cell).
template <typename FT>
__global__ void k_export_factors3d(BoxGeom G, const FT *__restrict__ fac, double *__restrict__ out) {
  const long total = (long)G.nsub * kNSlot3D * G.ncb;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < total; e += (long)gridDim.x * 256) {
    const long cell = e % G.ncb;
    const long ss = e / G.ncb;
    const long sub = ss / kNSlot3D;
    const int k = (int)(ss - sub * kNSlot3D);
    out[e] = (double)fac[(sub * G.ncb + cell) * kNSlot3D + k];
  }
}

}  // namespace

hipError_t launch_ilu_factor3d(const Phys &P, const BoxGeom &G, const SubInfo *subs, const int *lvl, const int *cells,
                               const double *J, double shift, void *fac, void *wfac, int fp32, hipStream_t s) {
  const long total = (long)G.nsub * G.ncb;
  const int nb = (int)((total + kExtractCells - 1) / kExtractCells);
  const bool win = wfac && G.wmax > 0;
  const int *owner = win ? cells + G.ncb + 2 * kWin3DCols * kWin3DThreads : nullptr;
  if (fp32) {
    hipLaunchKernelGGL(k_extract3d<float>, dim3(nb), dim3(kExtractCells), 0, s, P, G, subs, J, shift, (float *)fac);
    hipLaunchKernelGGL(k_ilu_factor3d<float>, dim3(G.nsub), dim3(256), 0, s, G, lvl, cells, owner, (float *)fac,
                       win ? (float *)wfac : nullptr);
  } else {
    hipLaunchKernelGGL(k_extract3d<double>, dim3(nb), dim3(kExtractCells), 0, s, P, G, subs, J, shift,
                       (double *)fac);
    hipLaunchKernelGGL(k_ilu_factor3d<double>, dim3(G.nsub), dim3(256), 0, s, G, lvl, cells, owner, (double *)fac,
                       win ? (double *)wfac : nullptr);
  }
  return hipGetLastError();
}

namespace {
bool g_ras3d_window = true;
constexpr int kWinDepth = 3;   // levels the windowed apply loads ahead
constexpr size_t kLdsDefault3 = 64 * 1024;
constexpr size_t kLdsMax3 = 160 * 1024;   // LDS per CU on gfx950

// Launches the windowed apply when the box allows it; false: use the general kernel.
template <typename FT>
bool ras_apply3d_win(const Phys &P, const BoxGeom &G, const SubInfo *subs, const int *cells, const void *wfac,
                     void *ybuf, const double *r, double *z, const GmresState *st, long vstride, hipStream_t s) {
  const size_t lds = (size_t)kWinSpan * G.bh * G.bd * sizeof(double2);
  if (!g_ras3d_window || !wfac || G.wmax <= 0 || G.wmax > kWin3DThreads || lds > kLdsMax3) return false;
  static size_t allowed = kLdsDefault3;   // per instantiation
  if (lds > allowed) {
    if (hipFuncSetAttribute((const void *)k_ras_apply3d_win<FT, kWinDepth>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax3) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    allowed = kLdsMax3;
  }
  double *spare = (double *)((double2 *)ybuf + box3_ypairs(G));
  hipLaunchKernelGGL((k_ras_apply3d_win<FT, kWinDepth>), dim3(G.nsub), dim3(win3d_row(G)), lds, s, P, G, subs,
                     cells + G.ncb, (const FT *)wfac, (double2 *)ybuf, spare, r, z, st, vstride);
  return true;
}
}  // namespace

void set_ras3d_window(bool on) { g_ras3d_window = on; }

hipError_t launch_ras_apply3d(const Phys &P, const BoxGeom &G, const SubInfo *subs, const int *lvl, const int *cells,
                              const void *fac, const void *wfac, void *ybuf, const double *r, double *z,
                              const GmresState *st, long vstride, int fp32, hipStream_t s, const RasVariant &rv) {
  const int kind = rv.kind;
  if (kind != ACCH_RAS_LEFT && !rv.own_x) return hipErrorInvalidValue;
  if (kind == ACCH_RAS_LEFT && (fp32 ? ras_apply3d_win<float>(P, G, subs, cells, wfac, ybuf, r, z, st, vstride, s)
                                     : ras_apply3d_win<double>(P, G, subs, cells, wfac, ybuf, r, z, st, vstride, s)))
    return hipGetLastError();
  if (fp32)
    hipLaunchKernelGGL(k_ras_apply3d<float>, dim3(G.nsub), dim3(256), 0, s, P, G, subs, lvl, cells,
                       (const float *)fac, (double2 *)ybuf, r, z, st, vstride, kind);
  else
    hipLaunchKernelGGL(k_ras_apply3d<double>, dim3(G.nsub), dim3(256), 0, s, P, G, subs, lvl, cells,
                       (const double *)fac, (double2 *)ybuf, r, z, st, vstride, kind);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || kind == ACCH_RAS_LEFT) return e;
  const int nb = reduce_blocks((long)P.nx * P.ny * P.nz);
  hipLaunchKernelGGL(k_ras_t_gather3d, dim3(nb), dim3(256), 0, s, P, G, subs, rv.px, rv.py, rv.pz, rv.own_x,
                     (const double2 *)ybuf, z, st, vstride);
  return hipGetLastError();
}

namespace {
// Windowed transposed apply when the box allows it (packs the transposed records first
// unless *packed); false: use the box-buffer kernels.
template <typename FT>
bool ras_t_apply3d_win(const Phys &P, const BoxGeom &G, const SubInfo *subs, const int *cells, int px, int py,
                       int pz, const int *own, const void *fac, void *wfact, bool *packed, void *ybuf, double *tbox,
                       const double *r, double *z, const GmresState *st, long vstride, hipStream_t s) {
  const size_t lds = (size_t)kWinSpan * G.bh * G.bd * sizeof(double2);
  if (!g_ras3d_window || !wfact || G.wmax <= 0 || G.wmax > kWin3DThreads || lds > kLdsMax3) return false;
  static size_t allowed = kLdsDefault3;   // per instantiation
  if (lds > allowed) {
    if (hipFuncSetAttribute((const void *)k_ras_t_apply3d_win<FT, kWinDepth>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax3) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    allowed = kLdsMax3;
  }
  const int *wcols = cells + G.ncb;
  if (!*packed) {
    hipLaunchKernelGGL(k_pack_window3d_t<FT>, dim3(G.nlev, G.nsub), dim3(win3d_row(G)), 0, s, G, wcols,
                       (const FT *)fac, (FT *)wfact);
    *packed = true;
  }
  hipLaunchKernelGGL((k_ras_t_apply3d_win<FT, kWinDepth>), dim3(G.nsub), dim3(win3d_row(G)), lds, s, P, G, subs,
                     wcols, (const FT *)wfact, (double2 *)ybuf, (double2 *)tbox, r, st, vstride);
  const int nb = reduce_blocks((long)P.nx * P.ny * P.nz);
  hipLaunchKernelGGL(k_ras_t_gather3d, dim3(nb), dim3(256), 0, s, P, G, subs, px, py, pz, own,
                     (const double2 *)tbox, z, st, vstride);
  return true;
}
}  // namespace

hipError_t launch_ras_t_apply3d(const Phys &P, const BoxGeom &G, const SubInfo *subs, const int *lvl,
                                const int *cells, int px, int py, int pz, const int *own, const void *fac,
                                void *wfact, bool *packed, void *ybuf, double *tbox, const double *r, double *z,
                                const GmresState *st, long vstride, int fp32, hipStream_t s) {
  if (fp32 ? ras_t_apply3d_win<float>(P, G, subs, cells, px, py, pz, own, fac, wfact, packed, ybuf, tbox, r, z, st,
                                      vstride, s)
           : ras_t_apply3d_win<double>(P, G, subs, cells, px, py, pz, own, fac, wfact, packed, ybuf, tbox, r, z, st,
                                       vstride, s))
    return hipGetLastError();
  if (fp32)
    hipLaunchKernelGGL(k_ras_t_sweep3d<float>, dim3(G.nsub), dim3(256), 0, s, P, G, subs, lvl, cells,
                       (const float *)fac, (double2 *)ybuf, r, st, vstride);
  else
    hipLaunchKernelGGL(k_ras_t_sweep3d<double>, dim3(G.nsub), dim3(256), 0, s, P, G, subs, lvl, cells,
                       (const double *)fac, (double2 *)ybuf, r, st, vstride);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nb = reduce_blocks((long)P.nx * P.ny * P.nz);
  hipLaunchKernelGGL(k_ras_t_gather3d, dim3(nb), dim3(256), 0, s, P, G, subs, px, py, pz, own,
                     (const double2 *)ybuf, z, st, vstride);
  return hipGetLastError();
}

hipError_t launch_export_factors3d(const BoxGeom &G, const void *fac, int fp32, double *out, hipStream_t s) {
  const long total = (long)G.nsub * kNSlot3D * G.ncb;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  if (fp32)
    hipLaunchKernelGGL(k_export_factors3d<float>, dim3(blocks), dim3(256), 0, s, G, (const float *)fac, out);
  else
    hipLaunchKernelGGL(k_export_factors3d<double>, dim3(blocks), dim3(256), 0, s, G, (const double *)fac, out);
  return hipGetLastError();
}

}  // namespace acch
