// Restricted additive Schwarz preconditioner with subdomain ILU(0), 2D (Section 3.1).
//
// Each subdomain box Omega_k^delta (padded to bw x bh cells) is handled by one
// workgroup.  Unknowns inside a box are ordered cell by cell, x fastest, with u
// before v at each cell; the ILU(0) pattern is the structural Jacobian stencil
// (u-row: u on the radius-2 diamond, v on the star; v-row: v on the star, u at the
// cell).  With that order every lower neighbour of cell (i, j) lies on an earlier
// wavefront w = i + 2j, so both the factorisation and the triangular solves sweep
// the bw + 2(bh - 1) wavefronts in order.  Thread t owns the box rows j = t (mod T);
// a wavefront meets each row at most once because bw < 2T.
//
// Factors are stored per subdomain as 24 slot arrays in wavefront order (cells of
// one wavefront are contiguous, so a wavefront's loads coalesce).
#include <utility>

#include "kernels.h"

namespace acch {
namespace {

// ---- static description of the u-row and v-row patterns ----------------------
struct Col {
  int t, dx, dy;  // column type (0 = u, 1 = v) and cell offset
};

// u-row columns: 8 lower ones in elimination order, then the diagonal and the 9
// upper ones in increasing unknown order.
__host__ __device__ constexpr Col ucol(int k) {
  constexpr Col tab[18] = {{0, 0, -2}, {0, -1, -1}, {0, 0, -1}, {1, 0, -1}, {0, 1, -1}, {0, -2, 0},
                           {0, -1, 0}, {1, -1, 0},  {0, 0, 0},  {1, 0, 0},  {0, 1, 0},  {1, 1, 0},
                           {0, 2, 0},  {0, -1, 1},  {0, 0, 1},  {1, 0, 1},  {0, 1, 1},  {0, 0, 2}};
  return tab[k];
}
// v-row columns: 3 lower, the diagonal, 2 upper.
__host__ __device__ constexpr Col vcol(int k) {
  constexpr Col tab[6] = {{1, 0, -1}, {1, -1, 0}, {0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {1, 0, 1}};
  return tab[k];
}
__host__ __device__ constexpr int find_ucol(int t, int dx, int dy) {
  for (int k = 0; k < 18; ++k) {
    const Col c = ucol(k);
    if (c.t == t && c.dx == dx && c.dy == dy) return k;
  }
  return -1;
}
__host__ __device__ constexpr int find_vcol(int t, int dx, int dy) {
  for (int k = 0; k < 6; ++k) {
    const Col c = vcol(k);
    if (c.t == t && c.dx == dx && c.dy == dy) return k;
  }
  return -1;
}
// Jacobian slot of (row type, column) in the 24-slot layout of include/acch.h.
__host__ __device__ constexpr int jslot(int rt, Col c) {
  if (rt == 0 && c.t == 0) {
    constexpr int dxs[13] = {0, -1, 1, 0, 0, -2, 2, 0, 0, -1, 1, -1, 1};
    constexpr int dys[13] = {0, 0, 0, -1, 1, 0, 0, -2, 2, -1, -1, 1, 1};
    for (int k = 0; k < 13; ++k)
      if (dxs[k] == c.dx && dys[k] == c.dy) return k;
  } else {
    constexpr int dxs[5] = {0, -1, 1, 0, 0};
    constexpr int dys[5] = {0, 0, 0, -1, 1};
    const int base = (rt == 0) ? 13 : (c.t == 1 ? 18 : 23);
    if (rt == 1 && c.t == 0) return (c.dx == 0 && c.dy == 0) ? 23 : -1;
    for (int k = 0; k < 5; ++k)
      if (dxs[k] == c.dx && dys[k] == c.dy) return base + k;
  }
  return -1;
}
// Upper part of a u-pivot row (its columns 8..17 = diagonal first) and of a v-pivot
// row (its columns 3..5), as offsets relative to the pivot cell.
__host__ __device__ constexpr Col uupper(int e) { return ucol(8 + e); }
__host__ __device__ constexpr Col vupper(int e) { return vcol(3 + e); }

// Every pattern entry has a Jacobian slot and the upper parts match the row lists.
__host__ __device__ constexpr bool tables_consistent() {
  for (int k = 0; k < 18; ++k)
    if (jslot(0, ucol(k)) < 0 || jslot(0, ucol(k)) >= kNSlot2D) return false;
  for (int k = 0; k < 6; ++k)
    if (jslot(1, vcol(k)) < 0 || jslot(1, vcol(k)) >= kNSlot2D) return false;
  // lower columns come first and precede the diagonal in unknown order
  if (!(ucol(8).t == 0 && ucol(8).dx == 0 && ucol(8).dy == 0)) return false;
  if (!(vcol(3).t == 1 && vcol(3).dx == 0 && vcol(3).dy == 0)) return false;
  return true;
}
static_assert(tables_consistent(), "ILU pattern tables");

// Pivot-row storage in the LDS ring: 10 values of the u-row's upper part, then 3 of
// the v-row's.
constexpr int kRing = 13;

template <int P, int E>
ACCH_DEV void elim_u_entry(double (&a)[18], double l, const double *prow) {
  constexpr Col pc = ucol(P);
  constexpr Col e = (pc.t == 0) ? uupper(E) : vupper(E);
  constexpr int tgt = find_ucol(e.t, pc.dx + e.dx, pc.dy + e.dy);
  if constexpr (tgt > P) a[tgt] -= l * prow[E];
}
template <int P, int... Es>
ACCH_DEV void elim_u_row(double (&a)[18], double l, const double *prow, std::integer_sequence<int, Es...>) {
  (elim_u_entry<P, Es + 1>(a, l, prow), ...);
}
template <int P, int E>
ACCH_DEV void elim_v_entry(double (&b)[6], double l, const double *prow) {
  constexpr Col pc = vcol(P);
  constexpr Col e = (pc.t == 0) ? uupper(E) : vupper(E);
  constexpr int tgt = find_vcol(e.t, pc.dx + e.dx, pc.dy + e.dy);
  if constexpr (tgt > P) b[tgt] -= l * prow[E];
}
template <int P, int... Es>
ACCH_DEV void elim_v_row(double (&b)[6], double l, const double *prow, std::integer_sequence<int, Es...>) {
  (elim_v_entry<P, Es + 1>(b, l, prow), ...);
}

ACCH_DEV int level_lo(int w, int bw) {
  const int d = w - bw + 2;
  return d > 0 ? (d >> 1) : 0;
}

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

// ---------------------------------------------------------------------------
// Extraction of A_k = R_k J R_k^T and its ILU(0) factorisation, one box per block.
// ---------------------------------------------------------------------------
template <typename FT, int NW>
__global__ __launch_bounds__(64 * NW) void k_ilu_factor2d(BoxGeom G, const SubInfo *__restrict__ subs,
                                                          const int *__restrict__ lvl, int nx, int ny,
                                                          int periodic, const double *__restrict__ J,
                                                          double shift, FT *__restrict__ fac) {
  constexpr int T = 64 * NW;
  extern __shared__ double ring[];  // [5][bh][kRing]
  const int t = threadIdx.x;
  const SubInfo si = subs[blockIdx.x];
  const long n = (long)nx * ny;
  FT *Fk = fac + (long)blockIdx.x * kNSlot2D * G.ncb;
  for (int w = 0; w < G.nlev; ++w) {
    const int j = row_on_level<T>(w, t, G.bw, G.bh);
    if (j >= 0) {
      const int i = w - 2 * j;
      const long g = box_to_global(si, i, j, nx, ny, periodic);
      double a[18], b[6];
      if (g >= 0) {
#pragma unroll
        for (int k = 0; k < 18; ++k) {
          const Col c = ucol(k);
          const int ii = i + c.dx, jj = j + c.dy;
          const bool in = ii >= 0 && ii < G.bw && jj >= 0 && jj < G.bh &&
                          box_to_global(si, ii, jj, nx, ny, periodic) >= 0;
          a[k] = in ? J[(long)jslot(0, c) * n + g] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          const Col c = vcol(k);
          const int ii = i + c.dx, jj = j + c.dy;
          const bool in = ii >= 0 && ii < G.bw && jj >= 0 && jj < G.bh &&
                          box_to_global(si, ii, jj, nx, ny, periodic) >= 0;
          b[k] = in ? J[(long)jslot(1, c) * n + g] : 0.0;
        }
        a[8] *= 1.0 + shift;  // ILU(0) of A_k + shift diag(A_k)
        b[3] *= 1.0 + shift;
      } else {  // padding / outside the domain: a decoupled identity row pair
#pragma unroll
        for (int k = 0; k < 18; ++k) a[k] = (k == 8) ? 1.0 : 0.0;
#pragma unroll
        for (int k = 0; k < 6; ++k) b[k] = (k == 3) ? 1.0 : 0.0;
      }
      // u-row: eliminate the 8 lower columns in order
      double prow[10];
#define ACCH_UPIVOT(P)                                                                   \
  {                                                                                      \
    constexpr Col pc = ucol(P);                                                          \
    const int ii = i + pc.dx, jj = j + pc.dy;                                            \
    if (ii >= 0 && ii < G.bw && jj >= 0 && jj < G.bh) {                                   \
      const double *src = ring + ((long)((w + pc.dx + 2 * pc.dy + 5) % 5) * G.bh + jj) * kRing + \
                          (pc.t == 0 ? 0 : 10);                                          \
      constexpr int ne = (pc.t == 0) ? 10 : 3;                                           \
      _Pragma("unroll") for (int e = 0; e < ne; ++e) prow[e] = src[e];                   \
      const double l = a[P] / prow[0];                                                   \
      a[P] = l;                                                                          \
      elim_u_row<P>(a, l, prow, std::make_integer_sequence<int, ne - 1>{});              \
    } else {                                                                             \
      a[P] = 0.0;                                                                        \
    }                                                                                    \
  }
      ACCH_UPIVOT(0) ACCH_UPIVOT(1) ACCH_UPIVOT(2) ACCH_UPIVOT(3)
      ACCH_UPIVOT(4) ACCH_UPIVOT(5) ACCH_UPIVOT(6) ACCH_UPIVOT(7)
#undef ACCH_UPIVOT
      // v-row: pivots v(0,-1), v(-1,0) from the ring, then u(0,0) of this cell
#define ACCH_VPIVOT(P)                                                                   \
  {                                                                                      \
    constexpr Col pc = vcol(P);                                                          \
    const int ii = i + pc.dx, jj = j + pc.dy;                                            \
    if (ii >= 0 && ii < G.bw && jj >= 0 && jj < G.bh) {                                   \
      const double *src = ring + ((long)((w + pc.dx + 2 * pc.dy + 5) % 5) * G.bh + jj) * kRing + 10; \
      _Pragma("unroll") for (int e = 0; e < 3; ++e) prow[e] = src[e];                    \
      const double l = b[P] / prow[0];                                                   \
      b[P] = l;                                                                          \
      elim_v_row<P>(b, l, prow, std::make_integer_sequence<int, 2>{});                   \
    } else {                                                                             \
      b[P] = 0.0;                                                                        \
    }                                                                                    \
  }
      ACCH_VPIVOT(0) ACCH_VPIVOT(1)
#undef ACCH_VPIVOT
      {
        const double l = b[2] / a[8];
        b[2] = l;
        elim_v_row<2>(b, l, &a[8], std::make_integer_sequence<int, 9>{});
      }
      // publish this cell's pivot rows for the later wavefronts
      double *dst = ring + ((long)(w % 5) * G.bh + j) * kRing;
#pragma unroll
      for (int e = 0; e < 10; ++e) dst[e] = a[8 + e];
#pragma unroll
      for (int e = 0; e < 3; ++e) dst[10 + e] = b[3 + e];
      // store the factors in the solve's slot order
      const long idx = lvl[w] + (j - level_lo(w, G.bw));
      const double s[kNSlot2D] = {a[6],  a[5],       a[4],  a[2],  a[1],  a[0],  a[7],  a[3],
                                  b[1],  b[0],       b[2],  1.0 / a[8], a[10], a[12], a[13], a[14],
                                  a[16], a[17],      a[9],  a[11], a[15], 1.0 / b[3], b[4], b[5]};
#pragma unroll
      for (int k = 0; k < kNSlot2D; ++k) Fk[(long)k * G.ncb + idx] = (FT)s[k];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// z = M^{-1} r, left-restricted Schwarz (restricted extension) with ILU(0) solves.
// ---------------------------------------------------------------------------
// Values of thread t-1 (L sweep) or t+1 (U sweep) handed over between waves.
template <typename FT, int NW>
ACCH_DEV void neighbour_fetch(int dir, int w, int lane, int wave, FT o1u, FT o1v, FT a3u, FT a3v, FT &Au,
                              FT &Av, FT &Mu, FT &Mv, FT (*xch)[NW][4]) {
  const int src = (lane + (dir < 0 ? 63 : 1)) & 63;
  Au = __shfl(o1u, src, 64);
  Av = __shfl(o1v, src, 64);
  Mu = __shfl(a3u, src, 64);
  Mv = __shfl(a3v, src, 64);
  if constexpr (NW > 1) {
    const int buf = w & 1;
    const int pub = dir < 0 ? 63 : 0;    // the lane whose values cross to the next wave
    if (lane == pub) {
      xch[buf][wave][0] = o1u;
      xch[buf][wave][1] = o1v;
      xch[buf][wave][2] = a3u;
      xch[buf][wave][3] = a3v;
    }
    __syncthreads();
    const int take = dir < 0 ? 0 : 63;
    if (lane == take) {
      const int pw = dir < 0 ? (wave + NW - 1) % NW : (wave + 1) % NW;
      Au = xch[buf][pw][0];
      Av = xch[buf][pw][1];
      Mu = xch[buf][pw][2];
      Mv = xch[buf][pw][3];
    }
  }
}

template <typename FT, int NW>
__global__ __launch_bounds__(64 * NW) void k_ras_apply2d(BoxGeom G, const SubInfo *__restrict__ subs,
                                                         const int *__restrict__ lvl, int nx, int ny,
                                                         int periodic, const FT *__restrict__ fac,
                                                         FT *__restrict__ ybuf, const double *__restrict__ r,
                                                         double *__restrict__ z, const GmresState *st,
                                                         long vstride) {
  // Inside GMRES the input is the current basis vector v_j = inv_norm[j] W_j and the
  // output is z_j; the whole kernel is skipped once the cycle has finished.
  double sc = 1.0;
  if (st) {
    if (st->done) return;
    const int jj = st->j;
    r += (long)jj * vstride;
    z += (long)jj * vstride;
    sc = st->inv_norm[jj];
  }
  constexpr int T = 64 * NW;
  __shared__ FT xch[2][NW][4];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const SubInfo si = subs[blockIdx.x];
  const long n = (long)nx * ny;
  const FT *Fk = fac + (long)blockIdx.x * kNSlot2D * G.ncb;
  FT *yk = ybuf + (long)blockIdx.x * 2 * G.ncb;
  const FT zero = (FT)0;
  // ---- forward sweep: L y = R_k r -------------------------------------------
  FT o1u = zero, o1v = zero, o2u = zero, o2v = zero;
  FT a1u = zero, a1v = zero, a2u = zero, a2v = zero, a3u = zero, a3v = zero;
  for (int w = 0; w < G.nlev; ++w) {
    const int j = row_on_level<T>(w, t, G.bw, G.bh);
    FT Au, Av, Mu, Mv;
    neighbour_fetch<FT, NW>(-1, w, lane, wave, o1u, o1v, a3u, a3v, Au, Av, Mu, Mv, xch);
    FT yu = zero, yv = zero;
    if (j >= 0) {
      const int i = w - 2 * j;
      const long idx = lvl[w] + (j - level_lo(w, G.bw));
      const long g = box_to_global(si, i, j, nx, ny, periodic);
      const FT ru = g >= 0 ? (FT)(sc * r[g]) : zero;
      const FT rv = g >= 0 ? (FT)(sc * r[n + g]) : zero;
      const FT *L = Fk + idx;
      const long s = G.ncb;
      FT acc = L[0] * o1u;
      acc = fma(L[1 * s], o2u, acc);
      acc = fma(L[2 * s], Au, acc);
      acc = fma(L[3 * s], a1u, acc);
      acc = fma(L[4 * s], a2u, acc);
      acc = fma(L[5 * s], Mu, acc);
      acc = fma(L[6 * s], o1v, acc);
      acc = fma(L[7 * s], a1v, acc);
      yu = ru - acc;
      FT accv = L[8 * s] * o1v;
      accv = fma(L[9 * s], a1v, accv);
      accv = fma(L[10 * s], yu, accv);
      yv = rv - accv;
      yk[idx] = yu;
      yk[s + idx] = yv;
    }
    a3u = a2u; a3v = a2v; a2u = a1u; a2v = a1v; a1u = Au; a1v = Av;
    o2u = o1u; o2v = o1v; o1u = yu; o1v = yv;
  }
  // ---- backward sweep: U x = y, write the owned part ------------------------
  o1u = o1v = o2u = o2v = zero;
  a1u = a1v = a2u = a2v = a3u = a3v = zero;
  for (int w = G.nlev - 1; w >= 0; --w) {
    const int j = row_on_level<T>(w, t, G.bw, G.bh);
    FT Au, Av, Mu, Mv;
    neighbour_fetch<FT, NW>(1, w, lane, wave, o1u, o1v, a3u, a3v, Au, Av, Mu, Mv, xch);
    FT xu = zero, xv = zero;
    if (j >= 0) {
      const int i = w - 2 * j;
      const long idx = lvl[w] + (j - level_lo(w, G.bw));
      const long s = G.ncb;
      const FT *U = Fk + idx;
      const FT yu = yk[idx], yv = yk[s + idx];
      FT accv = U[22 * s] * o1v;
      accv = fma(U[23 * s], a1v, accv);
      xv = (yv - accv) * U[21 * s];
      FT acc = U[12 * s] * o1u;
      acc = fma(U[13 * s], o2u, acc);
      acc = fma(U[14 * s], Au, acc);
      acc = fma(U[15 * s], a1u, acc);
      acc = fma(U[16 * s], a2u, acc);
      acc = fma(U[17 * s], Mu, acc);
      acc = fma(U[18 * s], xv, acc);
      acc = fma(U[19 * s], o1v, acc);
      acc = fma(U[20 * s], a1v, acc);
      xu = (yu - acc) * U[11 * s];
      if (i >= si.own_x0 && i < si.own_x1 && j >= si.own_y0 && j < si.own_y1) {
        const long g = box_to_global(si, i, j, nx, ny, periodic);
        if (g >= 0) {
          z[g] = (double)xu;
          z[n + g] = (double)xv;
        }
      }
    }
    a3u = a2u; a3v = a2v; a2u = a1u; a2v = a1v; a1u = Au; a1v = Av;
    o2u = o1u; o2v = o1v; o1u = xu; o1v = xv;
  }
}

// Factors (wavefront order, FT) -> FP64 [sub][slot][j][i].
template <typename FT>
__global__ void k_export_factors2d(BoxGeom G, const int *__restrict__ lvl, const FT *__restrict__ fac,
                                   double *__restrict__ out) {
  const long total = (long)G.nsub * kNSlot2D * G.ncb;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < total; e += (long)gridDim.x * 256) {
    const long cell = e % G.ncb;
    const long ss = e / G.ncb;  // sub * 24 + slot
    const int j = (int)(cell / G.bw), i = (int)(cell - (long)j * G.bw);
    const int w = i + 2 * j;
    const long idx = lvl[w] + (j - level_lo(w, G.bw));
    out[e] = (double)fac[ss * G.ncb + idx];
  }
}

template <typename FT, int NW>
hipError_t factor_impl(const BoxGeom &G, const SubInfo *subs, const int *lvl, int nx, int ny, int periodic,
                       const double *J, double shift, void *fac, hipStream_t s) {
  const size_t lds = (size_t)5 * G.bh * kRing * sizeof(double);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void *)k_ilu_factor2d<FT, NW>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_ilu_factor2d<FT, NW>), dim3(G.nsub), dim3(64 * NW), lds, s, G, subs, lvl, nx, ny, periodic,
                     J, shift, (FT *)fac);
  return hipGetLastError();
}

template <typename FT, int NW>
hipError_t apply_impl(const BoxGeom &G, const SubInfo *subs, const int *lvl, int nx, int ny, int periodic,
                      const void *fac, void *ybuf, const double *r, double *z, const GmresState *st, long vstride,
                      hipStream_t s) {
  hipLaunchKernelGGL((k_ras_apply2d<FT, NW>), dim3(G.nsub), dim3(64 * NW), 0, s, G, subs, lvl, nx, ny, periodic,
                     (const FT *)fac, (FT *)ybuf, r, z, st, vstride);
  return hipGetLastError();
}

}  // namespace

int schwarz_waves(const BoxGeom &G) {
  // bw < 2T keeps one active cell per thread per wavefront (and clean histories)
  if (G.bw <= 127) return 1;
  if (G.bw <= 255) return 2;
  if (G.bw <= 511) return 4;
  return 0;
}

hipError_t launch_ilu_factor2d(const BoxGeom &G, const SubInfo *subs, const int *lvl, int nx, int ny, int periodic,
                               const double *J, double shift, void *fac, int fp32, hipStream_t s) {
  const int nw = schwarz_waves(G);
  if (fp32) {
    if (nw == 1) return factor_impl<float, 1>(G, subs, lvl, nx, ny, periodic, J, shift, fac, s);
    if (nw == 2) return factor_impl<float, 2>(G, subs, lvl, nx, ny, periodic, J, shift, fac, s);
    if (nw == 4) return factor_impl<float, 4>(G, subs, lvl, nx, ny, periodic, J, shift, fac, s);
  } else {
    if (nw == 1) return factor_impl<double, 1>(G, subs, lvl, nx, ny, periodic, J, shift, fac, s);
    if (nw == 2) return factor_impl<double, 2>(G, subs, lvl, nx, ny, periodic, J, shift, fac, s);
    if (nw == 4) return factor_impl<double, 4>(G, subs, lvl, nx, ny, periodic, J, shift, fac, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_ras_apply2d(const BoxGeom &G, const SubInfo *subs, const int *lvl, int nx, int ny, int periodic,
                              const void *fac, void *ybuf, const double *r, double *z, const GmresState *st,
                              long vstride, int fp32, hipStream_t s) {
  const int nw = schwarz_waves(G);
  if (fp32) {
    if (nw == 1) return apply_impl<float, 1>(G, subs, lvl, nx, ny, periodic, fac, ybuf, r, z, st, vstride, s);
    if (nw == 2) return apply_impl<float, 2>(G, subs, lvl, nx, ny, periodic, fac, ybuf, r, z, st, vstride, s);
    if (nw == 4) return apply_impl<float, 4>(G, subs, lvl, nx, ny, periodic, fac, ybuf, r, z, st, vstride, s);
  } else {
    if (nw == 1) return apply_impl<double, 1>(G, subs, lvl, nx, ny, periodic, fac, ybuf, r, z, st, vstride, s);
    if (nw == 2) return apply_impl<double, 2>(G, subs, lvl, nx, ny, periodic, fac, ybuf, r, z, st, vstride, s);
    if (nw == 4) return apply_impl<double, 4>(G, subs, lvl, nx, ny, periodic, fac, ybuf, r, z, st, vstride, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_export_factors2d(const BoxGeom &G, const int *lvl, const void *fac, int fp32, double *out,
                                   hipStream_t s) {
  const long total = (long)G.nsub * kNSlot2D * G.ncb;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  if (fp32)
    hipLaunchKernelGGL(k_export_factors2d<float>, dim3(blocks), dim3(256), 0, s, G, lvl, (const float *)fac, out);
  else
    hipLaunchKernelGGL(k_export_factors2d<double>, dim3(blocks), dim3(256), 0, s, G, lvl, (const double *)fac, out);
  return hipGetLastError();
}

}  // namespace acch
