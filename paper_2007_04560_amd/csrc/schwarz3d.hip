// Restricted additive Schwarz with subdomain ILU(0), 3D (Section 3.1), and its exact
// transpose for the adjoint.
//
// Unknowns of a box are ordered cell by cell (x fastest, then y, then z), u before v
// at a cell; the ILU(0) pattern is the structural Jacobian stencil (u-row: u on the
// 25-point set, v on the 7-point star; v-row: v on the star, u at the cell).  Every
// earlier neighbour in that order lies on an earlier level w = i + 2j + 3k, so the
// factorisation and the sweeps walk the levels in order, one workgroup per box and
// a host-built list of each level's cells; values of a box live in a global box
// buffer (a box of 34^3 cells does not fit in LDS) and a barrier separates levels.
//
// Factor storage: 40 values per box cell (box-local index i + bw (j + bh k)): the
// u-row's 32 pattern entries in column order (15 multipliers of L, then U with the
// diagonal stored inverted) and the v-row's 8 (4 multipliers, inverted diagonal,
// 3 of U).
#include <utility>

#include "../../include/acch.h"
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

template <int P, typename FT>
ACCH_DEV void pivot_u(double (&a)[kUN], const FT *fk, const Box3 &B, int i, int j, int k) {
  constexpr Col3 pc = ucol3(P);
  const int qi = i + pc.dx, qj = j + pc.dy, qk = k + pc.dz;
  if (!B.in(qi, qj, qk)) {
    a[P] = 0.0;
    return;
  }
  const FT *rec = fk + (long)B.at(qi, qj, qk) * kNSlot3D;
  constexpr int ne = (pc.t == 0) ? kUN - kUD : kVN - kVD;
  double prow[ne];
  load_urow<FT, ne>(rec, pc.t == 0 ? kFA + kUD : kFB + kVD, prow);
  const double l = a[P] * prow[0];
  a[P] = l;
  elim3_u_row<P>(a, l, prow, std::make_integer_sequence<int, ne - 1>{});
}

template <int P, typename FT>
ACCH_DEV void pivot_v(double (&b)[kVN], const FT *fk, const Box3 &B, int i, int j, int k) {
  constexpr Col3 pc = vcol3(P);
  const int qi = i + pc.dx, qj = j + pc.dy, qk = k + pc.dz;
  if (!B.in(qi, qj, qk)) {
    b[P] = 0.0;
    return;
  }
  const FT *rec = fk + (long)B.at(qi, qj, qk) * kNSlot3D;
  double prow[kVN - kVD];
  load_urow<FT, kVN - kVD>(rec, kFB + kVD, prow);
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

template <typename FT>
__global__ __launch_bounds__(256) void k_ilu_factor3d(Phys P, BoxGeom G, const SubInfo *__restrict__ subs,
                                                      const int *__restrict__ lvl, const int *__restrict__ cells,
                                                      const double *__restrict__ J, double shift,
                                                      FT *__restrict__ fac) {
  const SubInfo si = subs[blockIdx.x];
  const Box3 B{G.bw, G.bh, G.bd};
  const long n = (long)P.nx * P.ny * P.nz;
  FT *fk = fac + (long)blockIdx.x * G.ncb * kNSlot3D;
  for (int w = 0; w < G.nlev; ++w) {
    for (int q = lvl[w] + threadIdx.x; q < lvl[w + 1]; q += blockDim.x) {
      const int e = cells[q];
      int i, j, k;
      decode(e, B, i, j, k);
      const long g = box3_to_global(si, i, j, k, P);
      double a[kUN], b[kVN];
      if (g >= 0) {
#pragma unroll
        for (int c = 0; c < kUN; ++c) {
          const Col3 cc = ucol3(c);
          const int ii = i + cc.dx, jj = j + cc.dy, kk = k + cc.dz;
          const bool in = B.in(ii, jj, kk) && box3_to_global(si, ii, jj, kk, P) >= 0;
          a[c] = in ? J[(long)jslot3(0, cc) * n + g] : 0.0;
        }
#pragma unroll
        for (int c = 0; c < kVN; ++c) {
          const Col3 cc = vcol3(c);
          const int ii = i + cc.dx, jj = j + cc.dy, kk = k + cc.dz;
          const bool in = B.in(ii, jj, kk) && box3_to_global(si, ii, jj, kk, P) >= 0;
          b[c] = in ? J[(long)jslot3(1, cc) * n + g] : 0.0;
        }
        a[kUD] *= 1.0 + shift;
        b[kVD] *= 1.0 + shift;
      } else {  // padding / outside the domain: a decoupled identity row pair
#pragma unroll
        for (int c = 0; c < kUN; ++c) a[c] = c == kUD ? 1.0 : 0.0;
#pragma unroll
        for (int c = 0; c < kVN; ++c) b[c] = c == kVD ? 1.0 : 0.0;
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
                                                     const GmresState *st, long vstride) {
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
    yb[e] = g >= 0 ? make_double2(sc * r[g], sc * r[n + g]) : make_double2(0.0, 0.0);
  }
  __syncthreads();
  auto val = [&](int i, int j, int k, int t) -> double {
    const double2 v = yb[B.at(i, j, k)];
    return t == 0 ? v.x : v.y;
  };
  // L y = R r
  for (int w = 0; w < G.nlev; ++w) {
    for (int q = lvl[w] + threadIdx.x; q < lvl[w + 1]; q += blockDim.x) {
      const int e = cells[q];
      int i, j, k;
      decode(e, B, i, j, k);
      const FT *rec = fk + (long)e * kNSlot3D;
      double yu = yb[e].x, yv = yb[e].y;
#pragma unroll
      for (int c = 0; c < kUL; ++c) {
        const Col3 cc = ucol3(c);
        const int ii = i + cc.dx, jj = j + cc.dy, kk = k + cc.dz;
        if (B.in(ii, jj, kk)) yu -= (double)rec[kFA + c] * val(ii, jj, kk, cc.t);
      }
#pragma unroll
      for (int c = 0; c < kVL - 1; ++c) {
        const Col3 cc = vcol3(c);
        const int ii = i + cc.dx, jj = j + cc.dy, kk = k + cc.dz;
        if (B.in(ii, jj, kk)) yv -= (double)rec[kFB + c] * val(ii, jj, kk, cc.t);
      }
      yv -= (double)rec[kFB + kVL - 1] * yu;
      yb[e] = make_double2(yu, yv);
    }
    __syncthreads();
  }
  // U x = y
  for (int w = G.nlev - 1; w >= 0; --w) {
    for (int q = lvl[w] + threadIdx.x; q < lvl[w + 1]; q += blockDim.x) {
      const int e = cells[q];
      int i, j, k;
      decode(e, B, i, j, k);
      const FT *rec = fk + (long)e * kNSlot3D;
      double xv = yb[e].y;
#pragma unroll
      for (int c = kVD + 1; c < kVN; ++c) {
        const Col3 cc = vcol3(c);
        const int ii = i + cc.dx, jj = j + cc.dy, kk = k + cc.dz;
        if (B.in(ii, jj, kk)) xv -= (double)rec[kFB + c] * val(ii, jj, kk, cc.t);
      }
      xv *= (double)rec[kFB + kVD];
      double xu = yb[e].x - (double)rec[kFA + kUD + 1] * xv;   // column (0,0,0,v)
#pragma unroll
      for (int c = kUD + 2; c < kUN; ++c) {
        const Col3 cc = ucol3(c);
        const int ii = i + cc.dx, jj = j + cc.dy, kk = k + cc.dz;
        if (B.in(ii, jj, kk)) xu -= (double)rec[kFA + c] * val(ii, jj, kk, cc.t);
      }
      xu *= (double)rec[kFA + kUD];
      yb[e] = make_double2(xu, xv);
    }
    __syncthreads();
  }
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
  auto coef = [&](int i, int j, int k, int slot) -> double {
    return (double)fk[(long)B.at(i, j, k) * kNSlot3D + slot];
  };
  auto val = [&](int i, int j, int k, int t) -> double {
    const double2 v = yb[B.at(i, j, k)];
    return t == 0 ? v.x : v.y;
  };
  // U^T y = R r: column p receives the U entries of the earlier rows q = p - o
  for (int w = 0; w < G.nlev; ++w) {
    for (int q = lvl[w] + threadIdx.x; q < lvl[w + 1]; q += blockDim.x) {
      const int e = cells[q];
      int i, j, k;
      decode(e, B, i, j, k);
      double yu = yb[e].x, yv = yb[e].y;
#pragma unroll
      for (int c = kUD + 1; c < kUN; ++c) {   // u-rows q with a u column at p
        const Col3 cc = ucol3(c);
        if (cc.t != 0) continue;
        const int ii = i - cc.dx, jj = j - cc.dy, kk = k - cc.dz;
        if (B.in(ii, jj, kk)) yu -= coef(ii, jj, kk, kFA + c) * val(ii, jj, kk, 0);
      }
      yu *= coef(i, j, k, kFA + kUD);
#pragma unroll
      for (int c = kUD + 1; c < kUN; ++c) {   // u-rows q with a v column at p (q = p for (0,0,0,v))
        const Col3 cc = ucol3(c);
        if (cc.t != 1) continue;
        const int ii = i - cc.dx, jj = j - cc.dy, kk = k - cc.dz;
        if (!B.in(ii, jj, kk)) continue;
        const double yq = (cc.dx == 0 && cc.dy == 0 && cc.dz == 0) ? yu : val(ii, jj, kk, 0);
        yv -= coef(ii, jj, kk, kFA + c) * yq;
      }
#pragma unroll
      for (int c = kVD + 1; c < kVN; ++c) {   // v-rows q with a v column at p
        const Col3 cc = vcol3(c);
        const int ii = i - cc.dx, jj = j - cc.dy, kk = k - cc.dz;
        if (B.in(ii, jj, kk)) yv -= coef(ii, jj, kk, kFB + c) * val(ii, jj, kk, 1);
      }
      yv *= coef(i, j, k, kFB + kVD);
      yb[e] = make_double2(yu, yv);
    }
    __syncthreads();
  }
  // L^T x = y (unit diagonal): column p receives the L entries of the later rows
  for (int w = G.nlev - 1; w >= 0; --w) {
    for (int q = lvl[w] + threadIdx.x; q < lvl[w + 1]; q += blockDim.x) {
      const int e = cells[q];
      int i, j, k;
      decode(e, B, i, j, k);
      double xu = yb[e].x, xv = yb[e].y;
#pragma unroll
      for (int c = 0; c < kUL; ++c) {   // u-rows q with a v column at p
        const Col3 cc = ucol3(c);
        if (cc.t != 1) continue;
        const int ii = i - cc.dx, jj = j - cc.dy, kk = k - cc.dz;
        if (B.in(ii, jj, kk)) xv -= coef(ii, jj, kk, kFA + c) * val(ii, jj, kk, 0);
      }
#pragma unroll
      for (int c = 0; c < kVL - 1; ++c) {   // v-rows q with a v column at p
        const Col3 cc = vcol3(c);
        const int ii = i - cc.dx, jj = j - cc.dy, kk = k - cc.dz;
        if (B.in(ii, jj, kk)) xv -= coef(ii, jj, kk, kFB + c) * val(ii, jj, kk, 1);
      }
#pragma unroll
      for (int c = 0; c < kUL; ++c) {   // u-rows q with a u column at p
        const Col3 cc = ucol3(c);
        if (cc.t != 0) continue;
        const int ii = i - cc.dx, jj = j - cc.dy, kk = k - cc.dz;
        if (B.in(ii, jj, kk)) xu -= coef(ii, jj, kk, kFA + c) * val(ii, jj, kk, 0);
      }
      xu -= coef(i, j, k, kFB + kVL - 1) * xv;   // the v-row of this cell, column (0,0,0,u)
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
                               const double *J, double shift, void *fac, int fp32, hipStream_t s) {
  if (fp32)
    hipLaunchKernelGGL(k_ilu_factor3d<float>, dim3(G.nsub), dim3(256), 0, s, P, G, subs, lvl, cells, J, shift,
                       (float *)fac);
  else
    hipLaunchKernelGGL(k_ilu_factor3d<double>, dim3(G.nsub), dim3(256), 0, s, P, G, subs, lvl, cells, J, shift,
                       (double *)fac);
  return hipGetLastError();
}

hipError_t launch_ras_apply3d(const Phys &P, const BoxGeom &G, const SubInfo *subs, const int *lvl, const int *cells,
                              const void *fac, void *ybuf, const double *r, double *z, const GmresState *st,
                              long vstride, int fp32, hipStream_t s) {
  if (fp32)
    hipLaunchKernelGGL(k_ras_apply3d<float>, dim3(G.nsub), dim3(256), 0, s, P, G, subs, lvl, cells,
                       (const float *)fac, (double2 *)ybuf, r, z, st, vstride);
  else
    hipLaunchKernelGGL(k_ras_apply3d<double>, dim3(G.nsub), dim3(256), 0, s, P, G, subs, lvl, cells,
                       (const double *)fac, (double2 *)ybuf, r, z, st, vstride);
  return hipGetLastError();
}

hipError_t launch_ras_t_apply3d(const Phys &P, const BoxGeom &G, const SubInfo *subs, const int *lvl,
                                const int *cells, int px, int py, int pz, const int *own, const void *fac, void *ybuf,
                                const double *r, double *z, const GmresState *st, long vstride, int fp32,
                                hipStream_t s) {
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
