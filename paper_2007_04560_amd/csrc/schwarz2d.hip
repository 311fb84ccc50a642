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
// Factors are stored per subdomain cell by cell in the padded wavefront order, the
// 24 slots of a cell contiguous (see the factor-storage note above k_ras_apply2d).
#include <utility>

#include "../../include/acch.h"
#include "boxes.h"
#include "bufio.h"
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

// ---------------------------------------------------------------------------
// Extraction of A_k = R_k J R_k^T and its ILU(0) factorisation, one box per block.
// ---------------------------------------------------------------------------
template <typename FT, int NW>
__global__ __launch_bounds__(64 * NW) void k_ilu_factor2d(Phys P0, Batch bt, BoxGeom G,
                                                          const SubInfo *__restrict__ subs,
                                                          const int *__restrict__ lvl, const double *__restrict__ J,
                                                          double shift, FT *__restrict__ fac) {
  constexpr int T = 64 * NW;
  extern __shared__ double ring[];  // [5][bh][kRing]
  const Loc Lc = locate(bt, kFamSub);
  if (!Lc.on) return;
  const Phys &Pi = bt.map[kFamSub] ? bt.inst[Lc.b].P : P0;
  const int nx = Pi.nx, ny = Pi.ny, periodic = Pi.periodic;
  if (bt.map[kFamSub]) J += bt.inst[Lc.b].joff;
  const int t = threadIdx.x;
  const SubInfo si = subs[blockIdx.x];
  const long n = (long)nx * ny;
  const long ncb = (long)G.nlev * G.bh;
  FT *Fk = fac + (long)blockIdx.x * kNSlot2D * ncb;
  // The box cells that hold a grid cell (box_to_global >= 0) form the rectangle
  // [ilo, ihi) x [jlo, jhi): the real extent, cut to the domain for Neumann boxes.
  int ilo = 0, jlo = 0, ihi = min(G.bw, si.ex), jhi = min(G.bh, si.ey);
  if (!periodic) {
    ilo = max(ilo, -si.ox);
    jlo = max(jlo, -si.oy);
    ihi = min(ihi, nx - si.ox);
    jhi = min(jhi, ny - si.oy);
  }
  const unsigned iw = (unsigned)max(ihi - ilo, 0), jw = (unsigned)max(jhi - jlo, 0);
  auto inside = [&](int ii, int jj) { return (unsigned)(ii - ilo) < iw && (unsigned)(jj - jlo) < jw; };
  for (int w = 0; w < G.nlev; ++w) {
    const int j = row_on_level<T>(w, t, G.bw, G.bh);
    if (j >= 0) {
      const int i = w - 2 * j;
      const long g = inside(i, j) ? box_to_global(si, i, j, nx, ny, periodic) : -1;
      double a[18], b[6];
      if (g >= 0) {
#pragma unroll
        for (int k = 0; k < 18; ++k) {
          const Col c = ucol(k);
          a[k] = inside(i + c.dx, j + c.dy) ? J[(long)jslot(0, c) * n + g] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          const Col c = vcol(k);
          b[k] = inside(i + c.dx, j + c.dy) ? J[(long)jslot(1, c) * n + g] : 0.0;
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
      // store the factors in the solve's slot order, wavefront-major (padded to bh rows)
      const long idx = (long)w * G.bh + j;
      const double s[kNSlot2D] = {a[6],  a[5],       a[4],  a[2],  a[1],  a[0],  a[7],  a[3],
                                  b[1],  b[0],       b[2],  1.0 / a[8], a[10], a[12], a[13], a[14],
                                  a[16], a[17],      a[9],  a[11], a[15], 1.0 / b[3], b[4], b[5]};
#pragma unroll
      for (int k = 0; k < kNSlot2D; ++k) Fk[(long)idx * kNSlot2D + k] = (FT)s[k];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Transposed records (the adjoint's M^{-T}): slot m of cell p holds the coefficient of
// column p in the row of cell q = p + (dx, dy) (zero when q is outside the box):
//   0-5  U[u_q][u_p] for q at (-1,0) (-2,0) (1,-1) (0,-1) (-1,-1) (0,-2);  6  1/U[u_p][u_p]
//   7-9  U[u_q][v_p] for q at (0,0) (-1,0) (0,-1);  10-11 U[v_q][v_p] for q at (-1,0) (0,-1)
//   12   1/U[v_p][v_p]
//   13-18 L[u_q][u_p] for q at (1,0) (2,0) (-1,1) (0,1) (1,1) (0,2);  19 L[v_p][u_p]
//   20-21 L[u_q][v_p] for q at (1,0) (0,1);  22-23 L[v_q][v_p] for q at (1,0) (0,1)
// The U^T sweep reads slots 0..12, the L^T sweep 13..23.
// ---------------------------------------------------------------------------
constexpr int kTFwd2D = 13;   // slots of the U^T sweep

struct TSrc {
  int dx, dy, slot;   // row cell q - p and the forward record slot holding the coefficient
};
__host__ __device__ constexpr TSrc tsrc2(int m) {
  constexpr TSrc tab[kNSlot2D] = {{-1, 0, 12}, {-2, 0, 13}, {1, -1, 14}, {0, -1, 15}, {-1, -1, 16}, {0, -2, 17},
                                  {0, 0, 11},  {0, 0, 18},  {-1, 0, 19}, {0, -1, 20}, {-1, 0, 22},  {0, -1, 23},
                                  {0, 0, 21},  {1, 0, 0},   {2, 0, 1},   {-1, 1, 2},  {0, 1, 3},    {1, 1, 4},
                                  {0, 2, 5},   {0, 0, 10},  {1, 0, 6},   {0, 1, 7},   {1, 0, 8},    {0, 1, 9}};
  return tab[m];
}

template <typename FT>
__global__ __launch_bounds__(256) void k_pack_t2d(BoxGeom G, const FT *__restrict__ fac, FT *__restrict__ fact) {
  const long ncb = (long)G.nlev * G.bh;   // padded wavefront-major cell slots
  const FT *Fk = fac + (long)blockIdx.x * kNSlot2D * ncb;
  FT *Tk = fact + (long)blockIdx.x * kNSlot2D * ncb;
  const int nbox = G.bw * G.bh;
  for (int e = threadIdx.x; e < nbox; e += 256) {
    const int j = e / G.bw, i = e - j * G.bw;
    FT *dst = Tk + ((long)(i + 2 * j) * G.bh + j) * kNSlot2D;
#pragma unroll
    for (int m = 0; m < kNSlot2D; ++m) {
      const TSrc q = tsrc2(m);
      const int qi = i + q.dx, qj = j + q.dy;
      const bool in = qi >= 0 && qi < G.bw && qj >= 0 && qj < G.bh;
      dst[m] = in ? Fk[((long)(qi + 2 * qj) * G.bh + qj) * kNSlot2D + q.slot] : (FT)0;
    }
  }
}

// ---------------------------------------------------------------------------
// z = M^{-1} r, left-restricted Schwarz (restricted extension) with ILU(0) solves.
// ---------------------------------------------------------------------------
// Factor storage: per subdomain, the 24 slots of a cell are contiguous (12 16-byte
// chunks in FP64, 6 in FP32) and the cells follow the padded wavefront order, so a
// sweep reads a cell's half of the slots with one address and 16-byte loads.
template <typename FT>
struct ChunkOf;
template <>
struct ChunkOf<double> {
  using T = double2;
  using Pair = double2;
  static constexpr int per = 2;
};
template <>
struct ChunkOf<float> {
  using T = float4;
  using Pair = float2;
  static constexpr int per = 4;
};

template <int K>
ACCH_DEV double comp(const double2 &c) {
  if constexpr (K == 0) return c.x;
  else return c.y;
}
template <int K>
ACCH_DEV float comp(const float4 &c) {
  if constexpr (K == 0) return c.x;
  else if constexpr (K == 1) return c.y;
  else if constexpr (K == 2) return c.z;
  else return c.w;
}

// Slot S of a cell from its loaded chunks c[0..), the first of which is chunk BASE.
template <int S, int BASE, typename FT, typename T, int N>
ACCH_DEV FT slot(const T (&c)[N]) {
  constexpr int per = ChunkOf<FT>::per;
  static_assert(S / per - BASE >= 0 && S / per - BASE < N, "slot outside the loaded chunks");
  return comp<S % per>(c[S / per - BASE]);
}

// Lane rotation inside a wave64: value of lane (t-1) mod 64 (L sweep) or (t+1) mod 64.
template <int DIR>
ACCH_DEV int rot_i(int x) {
  // wave_ror:1 / wave_rol:1; every lane has a source, so the old value is never used
  // (bound_ctrl set: the result register needs no copy of it)
  return __builtin_amdgcn_update_dpp(0, x, DIR < 0 ? 0x13C : 0x134, 0xF, 0xF, true);
}
template <int DIR>
ACCH_DEV double rot(double x) {
  const int lo = rot_i<DIR>(__double2loint(x));
  const int hi = rot_i<DIR>(__double2hiint(x));
  return __hiloint2double(hi, lo);
}
template <int DIR>
ACCH_DEV float rot(float x) {
  return __int_as_float(rot_i<DIR>(__float_as_int(x)));
}

// Values of thread t-1 (DIR < 0) or t+1 (DIR > 0): within the wave by lane rotation,
// across waves through LDS (one barrier per wavefront).
template <int DIR, typename FT, int NW>
ACCH_DEV void neighbour_fetch(int w, int lane, int wave, FT o1u, FT o1v, FT a3u, FT a3v, FT &Au, FT &Av, FT &Mu,
                              FT &Mv, FT (*xch)[NW][4]) {
  Au = rot<DIR>(o1u);
  Av = rot<DIR>(o1v);
  Mu = rot<DIR>(a3u);
  Mv = rot<DIR>(a3v);
  if constexpr (NW > 1) {
    const int buf = w & 1;
    const int pub = DIR < 0 ? 63 : 0;    // the lane whose values cross to the next wave
    if (lane == pub) {
      xch[buf][wave][0] = o1u;
      xch[buf][wave][1] = o1v;
      xch[buf][wave][2] = a3u;
      xch[buf][wave][3] = a3v;
    }
    __syncthreads();
    const int take = DIR < 0 ? 0 : 63;
    if (lane == take) {
      const int pw = DIR < 0 ? (wave + NW - 1) % NW : (wave + 1) % NW;
      Au = xch[buf][pw][0];
      Av = xch[buf][pw][1];
      Mu = xch[buf][pw][2];
      Mv = xch[buf][pw][3];
    }
  }
}

// Per-thread data of one wavefront, loaded D wavefronts ahead of its use (branch-free
// buffer accesses, see bufio.h).
template <typename FT, int NCH>
struct Stage {
  typename ChunkOf<FT>::T c[NCH];
  typename ChunkOf<FT>::Pair y;   // L sweep: R r of the cell; U sweep: y of the cell
  unsigned vf, vy;                 // per-lane byte offsets of the cell's record and value (kPastEnd: no cell)
  unsigned sf, sy;                 // the wavefront's byte offsets (uniform)
};

// Waits until at most N vector-memory operations of this wave are outstanding (vmcnt
// in bits 3:0 and 15:14; expcnt and lgkmcnt at their maxima, i.e. not waited for).
template <int N>
ACCH_DEV void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// Threads of a Schwarz block: the sweeps run on NW waves; with one sweep wave the
// block has seven more, which only share the gather / scatter passes (whose
// latency-bound loads then need few rounds).
template <int NW>
constexpr int ras_threads() {
  return NW == 1 ? 512 : 64 * NW;
}

// Global cell of box cell (i, j) for the box si (periodic wrap), -1 if padding or
// outside a Neumann domain; own: the cell is in the owned rectangle.
ACCH_DEV long box_cell(const SubInfo &si, int i, int j, int nx, int ny, int periodic, bool &own) {
  own = false;
  const long g = box_to_global(si, i, j, nx, ny, periodic);
  own = g >= 0 && i >= si.own_x0 && i < si.own_x1 && j >= si.own_y0 && j < si.own_y1;
  return g;
}

// TRP: the transposed solves (U^T y = b, then L^T x = y) with transposed records
// (k_pack_t2d); they read the same neighbour cells as the forward sweeps, since the
// rows holding column p of U (of L) are the cells p - o for the U (L) offsets o.
template <typename FT, int NW, int D, bool TRP>
__global__ __launch_bounds__(ras_threads<NW>()) void k_ras_apply2d(Phys P0, Batch bt, BoxGeom G,
                                                                   const SubInfo *__restrict__ subs,
                                                                   const int *__restrict__ lvl,
                                                                   const void *__restrict__ fac_,
                                                                   void *__restrict__ ybuf_,
                                                                   const double *__restrict__ r,
                                                                   double *__restrict__ z, double *__restrict__ dump,
                                                                   const GmresState *st, long vstride, int kind) {
  const Loc Lc = locate(bt, kFamSub);
  if (!Lc.on) return;
  const Phys &Pi = bt.map[kFamSub] ? bt.inst[Lc.b].P : P0;
  const int nx = Pi.nx, ny = Pi.ny, periodic = Pi.periodic;
  if (bt.map[kFamSub]) {
    r += bt.inst[Lc.b].xoff;
    z += bt.inst[Lc.b].xoff;
  }
  if (st) st += Lc.b;
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
  using C = ChunkOf<FT>;
  using T = typename C::T;
  using P2 = typename C::Pair;
  constexpr int per = C::per;
  constexpr int NCH = kNSlot2D / per;          // chunks per cell
  constexpr int NL = TRP ? kTFwd2D : 11;        // slots the L (U^T) sweep reads
  constexpr int NLC = (NL + per - 1) / per;    // chunks holding slots 0..NL-1
  constexpr int U0C = NL / per;                // first chunk of slots NL..23
  constexpr int NUC = NCH - U0C;
  constexpr int TT = 64 * NW;
  constexpr int TB = ras_threads<NW>();
  __shared__ FT xch[2][NW][4];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const SubInfo si = subs[blockIdx.x];
  const long n = (long)nx * ny;
  const unsigned ncb = (unsigned)G.nlev * G.bh;   // padded wavefront-major cell slots
  const T *Fk = (const T *)fac_ + (long)blockIdx.x * NCH * ncb;
  P2 *yk = (P2 *)ybuf_ + (long)blockIdx.x * (ncb + 1);   // entry ncb is this box's dump slot
  const FT zero = (FT)0;
  const int nlev = G.nlev;
  const int nbox = G.bw * G.bh;

  // ---- gather: yk[slot of (i,j)] = R_k r (scaled), zero on padding / outside cells;
  // GU cells per thread and round, all loads first
  constexpr int GU = 10;   // one round for boxes up to 5120 cells with 512 threads
  for (int e0 = t; e0 < nbox; e0 += TB * GU) {
    double ru[GU], rv[GU];
    long gq[GU];
    unsigned sq[GU];
#pragma unroll
    for (int u = 0; u < GU; ++u) {
      const int e = e0 + u * TB;
      const int ec = e < nbox ? e : 0;
      const int j = ec / G.bw, i = ec - j * G.bw;
      bool own;
      gq[u] = e < nbox ? box_cell(si, i, j, nx, ny, periodic, own) : -2;
      if (kind == ACCH_RAS_RIGHT && gq[u] >= 0 && !own) gq[u] = -1;   // restricted restriction
      sq[u] = (unsigned)(i + 2 * j) * G.bh + j;
      const long gs = gq[u] >= 0 ? gq[u] : 0;
      ru[u] = r[gs];
      rv[u] = r[n + gs];
    }
#pragma unroll
    for (int u = 0; u < GU; ++u) {
      if (gq[u] == -2) continue;
      P2 v;
      v.x = gq[u] >= 0 ? (FT)(sc * ru[u]) : zero;
      v.y = gq[u] >= 0 ? (FT)(sc * rv[u]) : zero;
      yk[sq[u]] = v;
    }
  }
  __syncthreads();

  if (t < TT) {
    const int nround = (nlev + 2 * D) / (D + 1) * (D + 1);   // >= nlev + D wavefronts
    const int niter = nround / (D + 1);
    constexpr unsigned REC = NCH * sizeof(T);   // bytes of a cell's record
    constexpr unsigned YB = sizeof(P2);
    const __amdgpu_buffer_rsrc_t rsF = buffer_rsrc(Fk, ncb * REC);
    const __amdgpu_buffer_rsrc_t rsY = buffer_rsrc(yk, ncb * YB);
    const unsigned wavF = (unsigned)G.bh * REC, wavY = (unsigned)G.bh * YB;   // bytes per wavefront
    // Lane t holds box row jA = t, and from a switch level on row jB = t + TT if the box
    // has it (bw < 2TT: row t has left the wavefronts before row t + TT enters them).
    // The switch is uniform: any level in [lo, 2TT) works, lo = 2(bh - TT - 1) + bw,
    // and the sweeps change rows between two loop iterations chosen inside it (the
    // host picks NW so that the window holds one).  A row the box lacks is parked
    // beyond every wavefront.  A lane without a cell loads zeros (zero factors and
    // right-hand side give a zero result) and its store is dropped.
    constexpr int kFar = 1 << 30;
    const bool hasB = t + TT < G.bh;
    const int j2A = t < G.bh ? 2 * t : kFar, j2B = hasB ? 2 * (t + TT) : j2A;
    const unsigned fA = t * REC, fB = hasB ? (t + TT) * REC : fA;
    const unsigned yA = t * YB, yB = hasB ? (t + TT) * YB : yA;
    const int lo = 2 * (G.bh - TT - 1) + G.bw;
    // Per-lane offsets select the cell (kPastEnd: none); the wavefront's offset is
    // uniform and goes in the scalar offset.
    auto prefetch = [&](auto &s, int w, int c0, int j2, unsigned fl, unsigned yl) {
      const bool act = (unsigned)(w - j2) < (unsigned)G.bw;
      s.vf = act ? fl : kPastEnd;
      s.vy = act ? yl : kPastEnd;
      s.sf = (unsigned)w * wavF;
      s.sy = (unsigned)w * wavY;
#pragma unroll
      for (int q = 0; q < (int)(sizeof(s.c) / sizeof(s.c[0])); ++q)
        s.c[q] = load16(rsF, s.vf + (unsigned)((c0 + q) * sizeof(T)), s.sf, (const T *)nullptr);
      s.y = load_pair(rsY, s.vy, s.sy, (const P2 *)nullptr);
    };
    // ---- forward sweep: L y = R_k r (in place in yk) -------------------------
    // D + 1 operand sets rotate by name through a loop unrolled D + 1 times: each
    // wavefront uses one set and loads wavefront w + D into the set used before it.
    // The sweep starts D empty wavefronts early (zero operands, nothing to load), so
    // every load is issued inside the loop; each wavefront waits once, for its own set
    // (the D - 1 later sets and their stores may still be in flight).
    constexpr int kWaitL = (D - 1) * (NLC + 2), kWaitU = (D - 1) * (NUC + 2);
    Stage<FT, NLC> ring[D + 1] = {};
#pragma unroll
    for (int k = 0; k <= D; ++k) ring[k].vf = ring[k].vy = kPastEnd;
    FT o1u = zero, o1v = zero, o2u = zero, o2v = zero;
    FT a1u = zero, a1v = zero, a2u = zero, a2v = zero, a3u = zero, a3v = zero;
    auto fwd_iter = [&](int w0, int j2, unsigned fl, unsigned yl) {
#pragma unroll
      for (int k = 0; k <= D; ++k) {
        const int w = w0 + k;
        wait_vm<kWaitL>();
        __builtin_amdgcn_sched_barrier(0);   // the arithmetic stays after the one wait
        FT Au, Av, Mu, Mv;
        neighbour_fetch<-1, FT, NW>(w, lane, wave, o1u, o1v, a3u, a3v, Au, Av, Mu, Mv, xch);
        const Stage<FT, NLC> &s = ring[k];
        // values of earlier wavefronts first; o1 (own, w-1) and A (neighbour, w-1) last
        FT yu, yv;
        if constexpr (!TRP) {
          FT acc = slot<1, 0, FT>(s.c) * o2u;
          acc = fma(slot<3, 0, FT>(s.c), a1u, acc);
          acc = fma(slot<4, 0, FT>(s.c), a2u, acc);
          acc = fma(slot<7, 0, FT>(s.c), a1v, acc);
          acc = fma(slot<5, 0, FT>(s.c), Mu, acc);
          acc = fma(slot<0, 0, FT>(s.c), o1u, acc);
          acc = fma(slot<6, 0, FT>(s.c), o1v, acc);
          acc = fma(slot<2, 0, FT>(s.c), Au, acc);
          yu = s.y.x - acc;
          FT accv = slot<9, 0, FT>(s.c) * a1v;
          accv = fma(slot<8, 0, FT>(s.c), o1v, accv);
          accv = fma(slot<10, 0, FT>(s.c), yu, accv);
          yv = s.y.y - accv;
        } else {   // U^T
          FT acc = slot<1, 0, FT>(s.c) * o2u;
          acc = fma(slot<3, 0, FT>(s.c), a1u, acc);
          acc = fma(slot<4, 0, FT>(s.c), a2u, acc);
          acc = fma(slot<5, 0, FT>(s.c), Mu, acc);
          acc = fma(slot<0, 0, FT>(s.c), o1u, acc);
          acc = fma(slot<2, 0, FT>(s.c), Au, acc);
          yu = (s.y.x - acc) * slot<6, 0, FT>(s.c);
          FT accv = slot<9, 0, FT>(s.c) * a1u;
          accv = fma(slot<11, 0, FT>(s.c), a1v, accv);
          accv = fma(slot<8, 0, FT>(s.c), o1u, accv);
          accv = fma(slot<10, 0, FT>(s.c), o1v, accv);
          accv = fma(slot<7, 0, FT>(s.c), yu, accv);
          yv = (s.y.y - accv) * slot<12, 0, FT>(s.c);
        }
        P2 y2;
        y2.x = yu;
        y2.y = yv;
        store_pair(rsY, s.vy, s.sy, y2);
        a3u = a2u; a3v = a2v; a2u = a1u; a2v = a1v; a1u = Au; a1v = Av;
        o2u = o1u; o2v = o1v; o1u = yu; o1v = yv;
        prefetch(ring[(k + D) % (D + 1)], w + D, 0, j2, fl, yl);
        // nothing moves across wavefronts: hoisting later wavefronts' arithmetic above
        // this point would make it wait for loads just issued
        __builtin_amdgcn_sched_barrier(0);
      }
    };
    // Row A while the loads stay below 2TT; the last row-A iteration loads up to level
    // w0 + 2D, and row B takes over from the first loaded level >= lo.
    const int mA = G.bh > TT ? min(niter, 1 + max(0, (lo - 1) / (D + 1))) : niter;
    int m = 0;
    for (; m < mA; ++m) fwd_iter(-D + m * (D + 1), j2A, fA, yA);
    for (; m < niter; ++m) fwd_iter(-D + m * (D + 1), j2B, fB, yB);
    // ---- backward sweep: U x = y (in place in yk) ----------------------------
    Stage<FT, NUC> ringu[D + 1] = {};
#pragma unroll
    for (int k = 0; k <= D; ++k) ringu[k].vf = ringu[k].vy = kPastEnd;
    o1u = o1v = o2u = o2v = zero;
    a1u = a1v = a2u = a2v = a3u = a3v = zero;
    auto bwd_iter = [&](int w0, int j2, unsigned fl, unsigned yl) {
#pragma unroll
      for (int k = 0; k <= D; ++k) {
        const int w = w0 - k;
        wait_vm<kWaitU>();
        __builtin_amdgcn_sched_barrier(0);   // the arithmetic stays after the one wait
        FT Au, Av, Mu, Mv;
        neighbour_fetch<1, FT, NW>(w, lane, wave, o1u, o1v, a3u, a3v, Au, Av, Mu, Mv, xch);
        const Stage<FT, NUC> &s = ringu[k];
        FT xu, xv;
        if constexpr (!TRP) {
          FT accv = slot<23, U0C, FT>(s.c) * a1v;
          accv = fma(slot<22, U0C, FT>(s.c), o1v, accv);
          xv = (s.y.y - accv) * slot<21, U0C, FT>(s.c);
          FT acc = slot<13, U0C, FT>(s.c) * o2u;
          acc = fma(slot<15, U0C, FT>(s.c), a1u, acc);
          acc = fma(slot<16, U0C, FT>(s.c), a2u, acc);
          acc = fma(slot<20, U0C, FT>(s.c), a1v, acc);
          acc = fma(slot<17, U0C, FT>(s.c), Mu, acc);
          acc = fma(slot<12, U0C, FT>(s.c), o1u, acc);
          acc = fma(slot<19, U0C, FT>(s.c), o1v, acc);
          acc = fma(slot<14, U0C, FT>(s.c), Au, acc);
          acc = fma(slot<18, U0C, FT>(s.c), xv, acc);
          xu = (s.y.x - acc) * slot<11, U0C, FT>(s.c);
        } else {   // L^T (unit diagonal), v before u at each cell
          FT accv = slot<21, U0C, FT>(s.c) * a1u;
          accv = fma(slot<23, U0C, FT>(s.c), a1v, accv);
          accv = fma(slot<20, U0C, FT>(s.c), o1u, accv);
          accv = fma(slot<22, U0C, FT>(s.c), o1v, accv);
          xv = s.y.y - accv;
          FT acc = slot<14, U0C, FT>(s.c) * o2u;
          acc = fma(slot<16, U0C, FT>(s.c), a1u, acc);
          acc = fma(slot<17, U0C, FT>(s.c), a2u, acc);
          acc = fma(slot<18, U0C, FT>(s.c), Mu, acc);
          acc = fma(slot<13, U0C, FT>(s.c), o1u, acc);
          acc = fma(slot<15, U0C, FT>(s.c), Au, acc);
          acc = fma(slot<19, U0C, FT>(s.c), xv, acc);
          xu = s.y.x - acc;
        }
        P2 x2;
        x2.x = xu;
        x2.y = xv;
        store_pair(rsY, s.vy, s.sy, x2);
        a3u = a2u; a3v = a2v; a2u = a1u; a2v = a1v; a1u = Au; a1v = Av;
        o2u = o1u; o2v = o1v; o1u = xu; o1v = xv;
        prefetch(ringu[(k + D) % (D + 1)], w - D, U0C, j2, fl, yl);
        __builtin_amdgcn_sched_barrier(0);
      }
    };
    // Row B while the loads stay at or above lo; the last row-B iteration loads down to
    // level w0 - 2D.
    const int m1 = G.bh > TT ? min(niter, 1 + max(0, (nlev - 1 - D - lo) / (D + 1))) : 0;
    for (m = 0; m < m1; ++m) bwd_iter(nlev - 1 + D - m * (D + 1), j2B, fB, yB);
    for (; m < niter; ++m) bwd_iter(nlev - 1 + D - m * (D + 1), j2A, fA, yA);
  }
  __syncthreads();
  // ---- scatter: z = (R_k^0)^T x on the owned cells, GU cells per round (the
  // other variants add whole boxes in k_ras_sum2d) -----------------------------
  if (kind != ACCH_RAS_LEFT) return;
  for (int e0 = t; e0 < nbox; e0 += TB * GU) {
    P2 xq[GU];
    long gq[GU];
#pragma unroll
    for (int u = 0; u < GU; ++u) {
      const int e = e0 + u * TB;
      const int ec = e < nbox ? e : 0;
      const int j = ec / G.bw, i = ec - j * G.bw;
      bool own;
      const long g = box_cell(si, i, j, nx, ny, periodic, own);
      gq[u] = (e < nbox && own) ? g : -1;
      xq[u] = yk[(unsigned)(i + 2 * j) * G.bh + j];
    }
#pragma unroll
    for (int u = 0; u < GU; ++u) {
      if (gq[u] < 0) continue;
      z[gq[u]] = (double)xq[u].x;
      z[n + gq[u]] = (double)xq[u].y;
    }
  }
  (void)dump;
}

// z = sum of the box values (in the wavefront-ordered box buffers) of every box
// holding the cell: the extension (R_k^delta)^T of the right-restricted and the
// classical variants.
template <typename FT>
__global__ __launch_bounds__(256) void k_ras_sum2d(BoxGeom G, const SubInfo *__restrict__ subs, int nx, int ny,
                                                    int periodic, int px, int py, const int *__restrict__ own_x,
                                                    const int *__restrict__ own_y, const void *__restrict__ ybuf_,
                                                    double *__restrict__ z, const GmresState *st, long vstride) {
  if (st && st->done) return;
  const int jj = st ? st->j : 0;
  const long n = (long)nx * ny;
  double *zu = z + (long)jj * vstride, *zv = zu + n;
  using P2 = typename ChunkOf<FT>::Pair;
  const long ncb = (long)G.nlev * G.bh;
  const P2 *yb = (const P2 *)ybuf_;
  for (long g = blockIdx.x * 256L + threadIdx.x; g < n; g += (long)gridDim.x * 256) {
    const int gy = (int)(g / nx), gx = (int)(g - (long)gy * nx);
    double su = 0.0, sv = 0.0;
    for_boxes_of(subs, nx, ny, periodic, px, py, own_x, own_y, gx, gy, [&](int k, int lx, int ly) {
      const P2 x2 = yb[(long)k * (ncb + 1) + (long)(lx + 2 * ly) * G.bh + ly];
      su += (double)x2.x;
      sv += (double)x2.y;
    });
    zu[g] = su;
    zv[g] = sv;
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
    const long ncbp = (long)G.nlev * G.bh;
    const long idx = (long)w * G.bh + j;
    const long sub = ss / kNSlot2D;
    const int k = (int)(ss - sub * kNSlot2D);
    out[e] = (double)fac[sub * kNSlot2D * ncbp + idx * kNSlot2D + k];
  }
}

template <typename FT, int NW>
hipError_t factor_impl(const BatchLaunch &bl, const BoxGeom &G, const SubInfo *subs, const int *lvl,
                       const double *J, double shift, void *fac, hipStream_t s) {
  const size_t lds = (size_t)5 * G.bh * kRing * sizeof(double);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void *)k_ilu_factor2d<FT, NW>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_ilu_factor2d<FT, NW>), dim3(bl.grid[kFamSub]), dim3(64 * NW), lds, s, bl.P0, bl.bt, G, subs,
                     lvl, J, shift, (FT *)fac);
  return hipGetLastError();
}

// Wavefronts loaded ahead of their use in the solves (selectable for tuning).
int g_ras_prefetch = 5;

template <typename FT, int NW, int D, bool TRP>
hipError_t apply_d(const BatchLaunch &bl, const BoxGeom &G, const SubInfo *subs, const int *lvl, const void *fac,
                   void *ybuf, const double *r, double *z, double *dump, const GmresState *st, long vstride,
                   int kind, hipStream_t s) {
  hipLaunchKernelGGL((k_ras_apply2d<FT, NW, D, TRP>), dim3(bl.grid[kFamSub]), dim3(ras_threads<NW>()), 0, s, bl.P0,
                     bl.bt, G, subs, lvl, fac, ybuf, r, z, dump, st, vstride, kind);
  return hipGetLastError();
}

template <typename FT, int NW, bool TRP = false>
hipError_t apply_impl(const BatchLaunch &bl, const BoxGeom &G, const SubInfo *subs, const int *lvl, const void *fac,
                      void *ybuf, const double *r, double *z, double *dump, const GmresState *st, long vstride,
                      int kind, hipStream_t s) {
  switch (g_ras_prefetch) {
    case 3: return apply_d<FT, NW, 3, TRP>(bl, G, subs, lvl, fac, ybuf, r, z, dump, st, vstride, kind, s);
    case 4: return apply_d<FT, NW, 4, TRP>(bl, G, subs, lvl, fac, ybuf, r, z, dump, st, vstride, kind, s);
    case 6: return apply_d<FT, NW, 6, TRP>(bl, G, subs, lvl, fac, ybuf, r, z, dump, st, vstride, kind, s);
    default: return apply_d<FT, NW, 5, TRP>(bl, G, subs, lvl, fac, ybuf, r, z, dump, st, vstride, kind, s);
  }
}

}  // namespace

void set_ras_prefetch(int d) { g_ras_prefetch = (d == 3 || d == 4 || d == 6) ? d : 5; }
int get_ras_prefetch() { return g_ras_prefetch; }

// Sweep waves of the Schwarz apply: bw < 2TT (a wavefront meets a lane's rows at most
// once), and a box taller than TT rows needs a window of at least 8 levels for the
// uniform switch of lanes from row t to row t + TT (2TT - lo >= 8, lo = 2(bh - TT - 1)
// + bw), so that an iteration boundary of the unrolled sweep falls inside it.
static int apply_waves(const BoxGeom &G) {
  for (int nw = 1; nw <= 4; nw *= 2) {
    const int tt = 64 * nw;
    if (G.bw >= 2 * tt || G.bh > 2 * tt) continue;
    if (G.bh <= tt || 2 * tt - (2 * (G.bh - tt - 1) + G.bw) >= 8) return nw;
  }
  return 0;
}

int schwarz_waves(const BoxGeom &G) {
  // bw < 2T keeps one active cell per thread per wavefront (and clean histories)
  if (apply_waves(G) == 0) return 0;
  if (G.bw <= 127) return 1;
  if (G.bw <= 255) return 2;
  if (G.bw <= 511) return 4;
  return 0;
}

hipError_t launch_ilu_factor2d(const BatchLaunch &bl, const BoxGeom &G, const SubInfo *subs, const int *lvl,
                               const double *J, double shift, void *fac, int fp32, hipStream_t s) {
  const int nw = schwarz_waves(G);
  if (fp32) {
    if (nw == 1) return factor_impl<float, 1>(bl, G, subs, lvl, J, shift, fac, s);
    if (nw == 2) return factor_impl<float, 2>(bl, G, subs, lvl, J, shift, fac, s);
    if (nw == 4) return factor_impl<float, 4>(bl, G, subs, lvl, J, shift, fac, s);
  } else {
    if (nw == 1) return factor_impl<double, 1>(bl, G, subs, lvl, J, shift, fac, s);
    if (nw == 2) return factor_impl<double, 2>(bl, G, subs, lvl, J, shift, fac, s);
    if (nw == 4) return factor_impl<double, 4>(bl, G, subs, lvl, J, shift, fac, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_ras_apply2d(const BatchLaunch &bl, const BoxGeom &G, const SubInfo *subs, const int *lvl,
                              const void *fac, void *ybuf, const double *r, double *z, double *dump,
                              const GmresState *st, long vstride, int fp32, hipStream_t s, const RasVariant &rv) {
  const int nw = apply_waves(G);
  const int kind = rv.kind;
  if (kind != ACCH_RAS_LEFT && (bl.bt.map[kFamSub] != nullptr || !rv.own_x)) return hipErrorInvalidValue;
  hipError_t e = hipErrorInvalidValue;
  if (fp32) {
    if (nw == 1) e = apply_impl<float, 1>(bl, G, subs, lvl, fac, ybuf, r, z, dump, st, vstride, kind, s);
    if (nw == 2) e = apply_impl<float, 2>(bl, G, subs, lvl, fac, ybuf, r, z, dump, st, vstride, kind, s);
    if (nw == 4) e = apply_impl<float, 4>(bl, G, subs, lvl, fac, ybuf, r, z, dump, st, vstride, kind, s);
  } else {
    if (nw == 1) e = apply_impl<double, 1>(bl, G, subs, lvl, fac, ybuf, r, z, dump, st, vstride, kind, s);
    if (nw == 2) e = apply_impl<double, 2>(bl, G, subs, lvl, fac, ybuf, r, z, dump, st, vstride, kind, s);
    if (nw == 4) e = apply_impl<double, 4>(bl, G, subs, lvl, fac, ybuf, r, z, dump, st, vstride, kind, s);
  }
  if (e != hipSuccess || kind == ACCH_RAS_LEFT) return e;
  return launch_ras_sum2d(bl, G, subs, ybuf, z, st, vstride, fp32, s, rv);
}

// M^{-T} r for the three variants: M^{-T} of the left-restricted operator has the
// shape of the right-restricted M^{-1} (owned-cell gather, whole boxes summed) and
// vice versa, so the transposed solves run with the variant swapped.
hipError_t launch_ras_t_apply2d(const BatchLaunch &bl, const BoxGeom &G, const SubInfo *subs, const int *lvl,
                                const void *fac, void *fact, bool *packed, void *ybuf, const double *r, double *z,
                                double *dump, const GmresState *st, long vstride, int fp32, hipStream_t s,
                                const RasVariant &rv) {
  const int nw = apply_waves(G);
  if (bl.bt.map[kFamSub] != nullptr || !rv.own_x) return hipErrorInvalidValue;
  if (!*packed) {
    if (fp32)
      hipLaunchKernelGGL(k_pack_t2d<float>, dim3(G.nsub), dim3(256), 0, s, G, (const float *)fac, (float *)fact);
    else
      hipLaunchKernelGGL(k_pack_t2d<double>, dim3(G.nsub), dim3(256), 0, s, G, (const double *)fac, (double *)fact);
    *packed = true;
  }
  const int kind = rv.kind == ACCH_RAS_LEFT ? ACCH_RAS_RIGHT : (rv.kind == ACCH_RAS_RIGHT ? ACCH_RAS_LEFT : rv.kind);
  hipError_t e = hipErrorInvalidValue;
  if (fp32) {
    if (nw == 1) e = apply_impl<float, 1, true>(bl, G, subs, lvl, fact, ybuf, r, z, dump, st, vstride, kind, s);
    if (nw == 2) e = apply_impl<float, 2, true>(bl, G, subs, lvl, fact, ybuf, r, z, dump, st, vstride, kind, s);
    if (nw == 4) e = apply_impl<float, 4, true>(bl, G, subs, lvl, fact, ybuf, r, z, dump, st, vstride, kind, s);
  } else {
    if (nw == 1) e = apply_impl<double, 1, true>(bl, G, subs, lvl, fact, ybuf, r, z, dump, st, vstride, kind, s);
    if (nw == 2) e = apply_impl<double, 2, true>(bl, G, subs, lvl, fact, ybuf, r, z, dump, st, vstride, kind, s);
    if (nw == 4) e = apply_impl<double, 4, true>(bl, G, subs, lvl, fact, ybuf, r, z, dump, st, vstride, kind, s);
  }
  if (e != hipSuccess || kind == ACCH_RAS_LEFT) return e;
  return launch_ras_sum2d(bl, G, subs, ybuf, z, st, vstride, fp32, s, rv);
}

hipError_t launch_ras_sum2d(const BatchLaunch &bl, const BoxGeom &G, const SubInfo *subs, const void *ybuf, double *z,
                            const GmresState *st, long vstride, int fp32, hipStream_t s, const RasVariant &rv) {
  const Phys &P = bl.P0;
  const int nb = reduce_blocks((long)P.nx * P.ny);
  if (fp32)
    hipLaunchKernelGGL(k_ras_sum2d<float>, dim3(nb), dim3(256), 0, s, G, subs, P.nx, P.ny, P.periodic, rv.px, rv.py,
                       rv.own_x, rv.own_y, ybuf, z, st, vstride);
  else
    hipLaunchKernelGGL(k_ras_sum2d<double>, dim3(nb), dim3(256), 0, s, G, subs, P.nx, P.ny, P.periodic, rv.px, rv.py,
                       rv.own_x, rv.own_y, ybuf, z, st, vstride);
  return hipGetLastError();
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
