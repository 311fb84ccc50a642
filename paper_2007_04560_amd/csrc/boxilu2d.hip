// ILU(0) on the width-2 box pattern as the subdomain solver of the 2D Schwarz
// preconditioner (Section 3.1; the ILU(0) of Tables 2-5 under the reading that its
// pattern is the structure a structured-grid matrix library allocates for this stencil).
//
// Pattern: both rows of box cell c couple to both unknowns of every box cell q with
// |q - c| <= 2 along each axis, 50 entries per row; unknowns cell by cell, x fastest,
// u before v.  A row's entries are indexed e = ((dy + 2) 5 + dx + 2) 2 + t, which is the
// unknown order: the 12 lower cells give e = 0..23, the cell itself 24 (u) and 25 (v),
// the 12 upper cells 26..49.  With wavefronts w = i + 3 j (boxilu.h) all lower cells lie
// on earlier wavefronts, so the factorisation and both triangular sweeps run the
// wavefronts in order, one box per workgroup: in the factorisation thread j owns box
// row j, in the sweeps four lanes share each cell of the current wavefront.
//
// Records (FT, kBoxIluRec = 52 slots per cell, cells in the wavefront order of boxilu.h):
//   L: for each lower cell k (unknown order) L(u_c,u_q) L(u_c,v_q) L(v_c,u_q) L(v_c,v_q)
//      at 4k .. 4k+3; L(v_c,u_c) at 48; zeros at 49..51.
//   U: for each upper cell k U(u_c,u_q) U(u_c,v_q) U(v_c,u_q) U(v_c,v_q) at 4k .. 4k+3;
//      1/U(u_c,u_c) at 48, U(u_c,v_c) at 49, 1/U(v_c,v_c) at 50, zero at 51.
// Entries towards cells outside the grid (padding, beyond a Neumann boundary) are zero,
// and such cells are decoupled identity rows, as in the other subdomain solvers.
#include <algorithm>
#include <utility>

#include "../../include/acch.h"
#include "boxes.h"
#include "boxilu.h"
#include "bufio.h"
#include "kernels.h"

namespace acch {
namespace {

struct Off {
  int dx, dy;
};
// Lower cells in unknown order: (dx, -2) and (dx, -1) for dx = -2..2, then (-2, 0), (-1, 0).
__host__ __device__ constexpr Off lower_cell(int k) { return k < 10 ? Off{k % 5 - 2, k / 5 - 2} : Off{k - 12, 0}; }
// Upper cells in unknown order: (1, 0), (2, 0), then (dx, 1) and (dx, 2) for dx = -2..2.
__host__ __device__ constexpr Off upper_cell(int k) {
  return k < 2 ? Off{k + 1, 0} : Off{(k - 2) % 5 - 2, (k - 2) / 5 + 1};
}
// Row entry of column (c + (dx, dy), type t); -1 outside the pattern.
__host__ __device__ constexpr int entry(int dx, int dy, int t) {
  return (dx < -2 || dx > 2 || dy < -2 || dy > 2) ? -1 : ((dy + 2) * 5 + dx + 2) * 2 + t;
}

// The 24 Jacobian slots of include/acch.h: row type, column type, column offset.
struct JSlot {
  int rt, ct, dx, dy;
};
__host__ __device__ constexpr JSlot jslot(int s) {
  constexpr JSlot tab[kNSlot2D] = {
      {0, 0, 0, 0},   {0, 0, -1, 0}, {0, 0, 1, 0},  {0, 0, 0, -1}, {0, 0, 0, 1},   {0, 0, -2, 0},
      {0, 0, 2, 0},   {0, 0, 0, -2}, {0, 0, 0, 2},  {0, 0, -1, -1}, {0, 0, 1, -1}, {0, 0, -1, 1},
      {0, 0, 1, 1},   {0, 1, 0, 0},  {0, 1, -1, 0}, {0, 1, 1, 0},  {0, 1, 0, -1},  {0, 1, 0, 1},
      {1, 1, 0, 0},   {1, 1, -1, 0}, {1, 1, 1, 0},  {1, 1, 0, -1}, {1, 1, 0, 1},   {1, 0, 0, 0}};
  return tab[s];
}

constexpr bool tables_consistent() {
  for (int k = 0; k < 12; ++k) {
    const Off l = lower_cell(k), u = upper_cell(k);
    if (entry(l.dx, l.dy, 0) != 2 * k || entry(u.dx, u.dy, 0) != 26 + 2 * k) return false;
  }
  for (int s = 0; s < kNSlot2D; ++s)
    if (entry(jslot(s).dx, jslot(s).dy, jslot(s).ct) < 0) return false;
  return entry(0, 0, 0) == 24;
}
static_assert(tables_consistent(), "box pattern tables");

// Cells of the padded box that hold a grid cell: the rectangle [ilo, ihi) x [jlo, jhi).
struct Rect {
  int ilo, ihi, jlo, jhi;
  ACCH_DEV bool in(int i, int j) const { return i >= ilo && i < ihi && j >= jlo && j < jhi; }
};
ACCH_DEV Rect grid_rect(const SubInfo &si, int bw, int bh, int nx, int ny, int periodic) {
  Rect r{0, min(bw, si.ex), 0, min(bh, si.ey)};
  if (!periodic) {
    r.ilo = max(r.ilo, -si.ox);
    r.jlo = max(r.jlo, -si.oy);
    r.ihi = min(r.ihi, nx - si.ox);
    r.jhi = min(r.jhi, ny - si.oy);
  }
  return r;
}

// Barrier for LDS traffic only (no global memory is exchanged between the threads).
ACCH_DEV void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Record position of cell (i, j) (on wavefront i + 3 j).
ACCH_DEV long cell_pos(const int *lvoff, int i, int j, int bw) {
  const int w = i + 3 * j;
  return lvoff[w] + j - level_jlo(w, bw);
}

// ---------------------------------------------------------------------------
// Factorisation: extraction of A_k = R_k J R_k^T (+ sigma diag(A_k)) and ILU(0) on the box
// pattern in IKJ order.  Both rows of a cell are eliminated together: the pivots are the
// rows of the 12 lower cells (u row, then v row, in unknown order), whose U records were
// stored on earlier wavefronts by the threads of their box rows, then the cell's own u
// row for its v row.  The elimination is FP64; the pivot rows are read back in FT.
// ---------------------------------------------------------------------------
template <int S>
ACCH_DEV void load_slot(double (&a)[50], double (&b)[50], const double *J, long n, long g, const Rect &rc, int i,
                        int j) {
  constexpr JSlot q = jslot(S);
  constexpr int e = entry(q.dx, q.dy, q.ct);
  if (rc.in(i + q.dx, j + q.dy)) {
    const double v = J[(long)S * n + g];
    if constexpr (q.rt == 0) a[e] = v;
    else b[e] = v;
  }
}
template <int... S>
ACCH_DEV void load_row(double (&a)[50], double (&b)[50], const double *J, long n, long g, const Rect &rc, int i,
                       int j, std::integer_sequence<int, S...>) {
  (load_slot<S>(a, b, J, n, g, rc, i, j), ...);
}

// a[target] -= la * U(pivot row, column); pivot row (lower cell K, type TP), its column
// in upper cell KU of the pivot cell (both types); dropped when outside the pattern.
template <int K, int TP, int KU>
ACCH_DEV void update(double (&a)[50], double (&b)[50], double la, double lb, const double (&u)[kBoxIluRec]) {
  constexpr Off o = lower_cell(K), e = upper_cell(KU);
  constexpr int t0 = entry(o.dx + e.dx, o.dy + e.dy, 0);
  if constexpr (t0 >= 0) {
    constexpr int s = 4 * KU + 2 * TP;
    a[t0] -= la * u[s];
    a[t0 + 1] -= la * u[s + 1];
    b[t0] -= lb * u[s];
    b[t0 + 1] -= lb * u[s + 1];
  }
}
template <int K, int TP, int... KU>
ACCH_DEV void update_all(double (&a)[50], double (&b)[50], double la, double lb, const double (&u)[kBoxIluRec],
                         std::integer_sequence<int, KU...>) {
  (update<K, TP, KU>(a, b, la, lb, u), ...);
}

template <typename FT, int K>
ACCH_DEV void eliminate_cell(double (&a)[50], double (&b)[50], const FT *Uk, const int *lvoff, const Rect &rc,
                             int i, int j, int bw) {
  constexpr Off o = lower_cell(K);
  if (!rc.in(i + o.dx, j + o.dy)) {   // no such cell: its columns are outside the pattern
    a[2 * K] = a[2 * K + 1] = b[2 * K] = b[2 * K + 1] = 0.0;
    return;
  }
  const FT *rec = Uk + cell_pos(lvoff, i + o.dx, j + o.dy, bw) * kBoxIluRec;
  double u[kBoxIluRec];
#pragma unroll
  for (int s = 0; s < kBoxIluRec - 1; ++s) u[s] = (double)rec[s];
  u[kBoxIluRec - 1] = 0.0;
  {  // pivot row u_q
    const double la = a[2 * K] * u[48], lb = b[2 * K] * u[48];
    a[2 * K] = la;
    b[2 * K] = lb;
    a[2 * K + 1] -= la * u[49];
    b[2 * K + 1] -= lb * u[49];
    update_all<K, 0>(a, b, la, lb, u, std::make_integer_sequence<int, 12>{});
  }
  {  // pivot row v_q
    const double la = a[2 * K + 1] * u[50], lb = b[2 * K + 1] * u[50];
    a[2 * K + 1] = la;
    b[2 * K + 1] = lb;
    update_all<K, 1>(a, b, la, lb, u, std::make_integer_sequence<int, 12>{});
  }
}
template <typename FT, int... K>
ACCH_DEV void eliminate(double (&a)[50], double (&b)[50], const FT *Uk, const int *lvoff, const Rect &rc, int i,
                        int j, int bw, std::integer_sequence<int, K...>) {
  (eliminate_cell<FT, K>(a, b, Uk, lvoff, rc, i, j, bw), ...);
}

template <typename FT, int TH>
__global__ __launch_bounds__(TH) void k_boxilu_factor2d(Phys P0, Batch bt, BoxIluGeom X,
                                                          const SubInfo *__restrict__ subs,
                                                                  const int *__restrict__ lvoff,
                                                                  const double *__restrict__ J, double shift,
                                                                  FT *__restrict__ Lrec, FT *__restrict__ Urec) {
  // batched: the block's instance (its grid, its rows of J); the whole block leaves
  // together when the instance is inactive
  const Loc Lc = locate(bt, kFamSub);
  if (!Lc.on) return;
  const Phys &P = bt.map[kFamSub] ? bt.inst[Lc.b].P : P0;
  if (bt.map[kFamSub]) J += bt.inst[Lc.b].joff;
  const int j = threadIdx.x;   // box row
  const SubInfo si = subs[blockIdx.x];
  const Rect rc = grid_rect(si, X.bw, X.bh, P.nx, P.ny, P.periodic);
  const long n = (long)P.nx * P.ny;
  FT *Lk = Lrec + (long)blockIdx.x * X.ncell * kBoxIluRec;
  FT *Uk = Urec + (long)blockIdx.x * X.ncell * kBoxIluRec;
  for (int w = 0; w < X.nlev; ++w) {
    const int i = w - 3 * j;
    if (j < X.bh && i >= 0 && i < X.bw) {
      double a[50], b[50];
#pragma unroll
      for (int e = 0; e < 50; ++e) a[e] = b[e] = 0.0;
      if (rc.in(i, j)) {
        const long g = box_to_global(si, i, j, P.nx, P.ny, P.periodic);
        load_row(a, b, J, n, g, rc, i, j, std::make_integer_sequence<int, kNSlot2D>{});
        a[24] *= 1.0 + shift;
        b[25] *= 1.0 + shift;
        eliminate<FT>(a, b, Uk, lvoff, rc, i, j, X.bw, std::make_integer_sequence<int, 12>{});
        const double lb = b[24] / a[24];   // v row: the cell's own u row
        b[24] = lb;
#pragma unroll
        for (int e = 25; e < 50; ++e) b[e] -= lb * a[e];
      } else {
        a[24] = 1.0;
        b[25] = 1.0;
      }
      const long p = (long)lvoff[w] + j - level_jlo(w, X.bw);
      FT *L = Lk + p * kBoxIluRec;
      FT *U = Uk + p * kBoxIluRec;
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        const Off lo = lower_cell(k), up = upper_cell(k);
        const bool lin = rc.in(i + lo.dx, j + lo.dy), uin = rc.in(i + up.dx, j + up.dy);
        L[4 * k + 0] = (FT)(lin ? a[2 * k] : 0.0);
        L[4 * k + 1] = (FT)(lin ? a[2 * k + 1] : 0.0);
        L[4 * k + 2] = (FT)(lin ? b[2 * k] : 0.0);
        L[4 * k + 3] = (FT)(lin ? b[2 * k + 1] : 0.0);
        U[4 * k + 0] = (FT)(uin ? a[26 + 2 * k] : 0.0);
        U[4 * k + 1] = (FT)(uin ? a[27 + 2 * k] : 0.0);
        U[4 * k + 2] = (FT)(uin ? b[26 + 2 * k] : 0.0);
        U[4 * k + 3] = (FT)(uin ? b[27 + 2 * k] : 0.0);
      }
      L[48] = (FT)b[24];
      L[49] = L[50] = L[51] = (FT)0;
      U[48] = (FT)(1.0 / a[24]);
      U[49] = (FT)a[25];
      U[50] = (FT)(1.0 / b[25]);
      U[51] = (FT)0;
    }
    __syncthreads();   // this wavefront's U records are read by the next ones
  }
}

// ---------------------------------------------------------------------------
// z = M^{-1} r: forward sweep L y = R_k r, backward sweep U x = y, one box per block,
// in the precision of the records (FP64, or FP32 for the mixed-precision form).
// The records of one wavefront are contiguous; all 256 threads load them with 16-byte
// loads into registers D - 1 wavefronts ahead and copy them to LDS one wavefront ahead
// (double-buffered).  Four threads share a cell of the wavefront (its p-th, threads
// 4p .. 4p + 3), each taking 3 of the 12 neighbour cells, and add their partial sums
// across the quad.  Each box row keeps its last 16 finished (u, v) pairs in an LDS ring,
// every pair stored at column c mod 16 and again 16 further, so the 5 columns around a
// cell are consecutive: the neighbours of cell (i, j) on rows j - 2 .. j + 2 are at most
// 8 wavefronts old, and within one wavefront no row writes a slot that another row
// reads.  The ring starts at zero and holds finite values only; neighbours outside the
// grid carry zero coefficients.
// ---------------------------------------------------------------------------
constexpr int kRingW = 16;

// (u, v) pair in FT
template <typename FT>
struct ChunkOf2;
template <>
struct ChunkOf2<double> {
  using T = double2;
};
template <>
struct ChunkOf2<float> {
  using T = float2;
};

// the 4 slots 4k .. 4k+3 of a record in LDS
ACCH_DEV void slots4(const double *rec, int k, double &c0, double &c1, double &c2, double &c3) {
  const double2 p = *(const double2 *)(rec + 4 * k), q = *(const double2 *)(rec + 4 * k + 2);
  c0 = p.x;
  c1 = p.y;
  c2 = q.x;
  c3 = q.y;
}
ACCH_DEV void slots4(const float *rec, int k, float &c0, float &c1, float &c2, float &c3) {
  const float4 p = *(const float4 *)(rec + 4 * k);
  c0 = p.x;
  c1 = p.y;
  c2 = p.z;
  c3 = p.w;
}

// Sum over the 4 lanes of a quad (DPP quad permutations [1,0,3,2] and [2,3,0,1]); every
// lane of the quad takes part.
template <int CTRL>
ACCH_DEV int dpp_i(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
ACCH_DEV double dpp(double x) {
  return __hiloint2double(dpp_i<CTRL>(__double2hiint(x)), dpp_i<CTRL>(__double2loint(x)));
}
template <int CTRL>
ACCH_DEV float dpp(float x) {
  return __int_as_float(dpp_i<CTRL>(__float_as_int(x)));
}
template <typename T>
ACCH_DEV T quad_sum(T x) {
  x += dpp<0xB1>(x);
  return x + dpp<0x4E>(x);
}

// Cells on wavefront w of a bw x bh box (0 outside [0, nlev)).
ACCH_DEV int level_count(int w, int bw, int bh, int nlev) {
  if (w < 0 || w >= nlev) return 0;
  return max(0, min(bh - 1, w / 3) - level_jlo(w, bw) + 1);
}

// Records of the wavefront whose first record is `first` and which has `cnt` cells:
// 16-byte chunks t + TH m of a block of TH threads.
template <typename FT, int NCH, int TH>
ACCH_DEV void stage_load(__amdgpu_buffer_rsrc_t rs, int first, int cnt, word4 (&R)[NCH]) {
  const unsigned base = (unsigned)first * kBoxIluRec * (unsigned)sizeof(FT);
  const unsigned bytes = (unsigned)cnt * kBoxIluRec * (unsigned)sizeof(FT);
#pragma unroll
  for (int m = 0; m < NCH; ++m) {
    const unsigned e = (unsigned)(threadIdx.x + TH * m) * 16u;
    R[m] = __builtin_amdgcn_raw_buffer_load_b128(rs, e < bytes ? base + e : kPastEnd, 0, 0);
  }
}
template <int NCH, int TH>
ACCH_DEV void stage_store(word4 *buf, const word4 (&R)[NCH]) {
#pragma unroll
  for (int m = 0; m < NCH; ++m) buf[threadIdx.x + TH * m] = R[m];
}

// Waits until at most N vector-memory operations (loads and stores) of this wave are
// outstanding (vmcnt in bits 3:0 and 15:14; expcnt and lgkmcnt not waited for).
template <int N>
ACCH_DEV void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// Gather of R_k r into the box vector (in the cell order of the records) and scatter of x
// from it to z (left RAS) or to the box buffer of the overlap sum, by the threads of the
// box's block before and after the sweeps; kGS cells per thread are handled together, so
// their loads are in flight at once.
constexpr int kGS = 4;

template <typename FT, int TH>
ACCH_DEV void gather_box(const Phys &P, const BoxIluGeom &X, const SubInfo &si, const Rect &rc,
                         const int *__restrict__ cellof, const double *__restrict__ r, double sc,
                         typename ChunkOf2<FT>::T *yk, int kind) {
  using V2 = typename ChunkOf2<FT>::T;
  const long n = (long)P.nx * P.ny;
  for (int p0 = 0; p0 < X.ncell; p0 += kGS * TH) {
    long g[kGS];
    int pos[kGS];
#pragma unroll
    for (int u = 0; u < kGS; ++u) {
      pos[u] = p0 + u * TH + (int)threadIdx.x;
      const int ij = pos[u] < X.ncell ? cellof[pos[u]] : 0, i = ij & 0xffff, j = ij >> 16;
      g[u] = -1;
      if (pos[u] < X.ncell && rc.in(i, j)) {
        const bool own = i >= si.own_x0 && i < si.own_x1 && j >= si.own_y0 && j < si.own_y1;
        if (kind != ACCH_RAS_RIGHT || own) g[u] = box_to_global(si, i, j, P.nx, P.ny, P.periodic);
      }
    }
    V2 v[kGS];
#pragma unroll
    for (int u = 0; u < kGS; ++u)
      v[u] = g[u] >= 0 ? V2{(FT)(sc * r[g[u]]), (FT)(sc * r[g[u] + n])} : V2{(FT)0, (FT)0};
#pragma unroll
    for (int u = 0; u < kGS; ++u)
      if (pos[u] < X.ncell) yk[pos[u]] = v[u];
  }
}

template <typename FT, int TH>
ACCH_DEV void scatter_box(const Phys &P, const BoxIluGeom &X, const BoxGeom &G, const SubInfo &si, const Rect &rc,
                          const int *__restrict__ cellof, const typename ChunkOf2<FT>::T *yk, FT *boxbuf,
                          double *__restrict__ z, int kind) {
  using V2 = typename ChunkOf2<FT>::T;
  const long n = (long)P.nx * P.ny;
  const long ncb = (long)G.nlev * G.bh;
  for (int p0 = 0; p0 < X.ncell; p0 += kGS * TH) {
    int ij[kGS];
    V2 x[kGS];
#pragma unroll
    for (int u = 0; u < kGS; ++u) {
      const int pos = p0 + u * TH + (int)threadIdx.x;
      ij[u] = pos < X.ncell ? cellof[pos] : -1;
      x[u] = pos < X.ncell ? yk[pos] : V2{(FT)0, (FT)0};
    }
#pragma unroll
    for (int u = 0; u < kGS; ++u) {
      if (ij[u] < 0) continue;
      const int i = ij[u] & 0xffff, j = ij[u] >> 16;
      if (!rc.in(i, j)) continue;
      if (kind == ACCH_RAS_LEFT) {
        if (i >= si.own_x0 && i < si.own_x1 && j >= si.own_y0 && j < si.own_y1) {
          const long g = box_to_global(si, i, j, P.nx, P.ny, P.periodic);
          z[g] = (double)x[u].x;
          z[g + n] = (double)x[u].y;
        }
      } else {
        ((V2 *)boxbuf)[(long)blockIdx.x * (ncb + 1) + (long)(i + 2 * j) * G.bh + j] = x[u];
      }
    }
  }
}

// Every global access of the sweeps is a buffer access issued by every thread on every
// step; a thread without a cell there passes an offset past the end (bufio.h).  A sweep
// runs D steps before its first wavefront (nothing to compute, only loads) and is padded
// to a multiple of D steps, so every access is issued inside a loop unrolled D times and
// each step issues the same accesses: step s handles wavefront s - D of the sweep's order,
// copies the records and box values of the next wavefront (loaded D - 1 steps earlier) to
// LDS and loads those of wavefront s.  The two waits of a step are exact counts of the
// accesses issued after the ones it needs.
template <typename FT, int NCH, int D, int TH, bool FWD, bool TRANS = false>
ACCH_DEV void sweep(const BoxIluGeom &X, __amdgpu_buffer_rsrc_t rsRec, __amdgpu_buffer_rsrc_t rsV,
                    word4 (*stage)[NCH * TH], typename ChunkOf2<FT>::T (*stv)[64],
                    typename ChunkOf2<FT>::T (*ring)[2 * kRingW], const int (&off)[3]) {
  using V2 = typename ChunkOf2<FT>::T;
  const int t = threadIdx.x, p = t >> 2, part = t & 3;
  const int nlev = X.nlev;
  const int nstep = (nlev + D + D - 1) / D * D;   // D lead-in steps, padded to a multiple of D
  constexpr int kOps = NCH + 2;                    // a step: 1 store, NCH + 1 loads
  auto count = [&](int w) { return level_count(w, X.bw, X.bh, nlev); };
  word4 R[D][NCH];
  V2 RV[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    RV[d] = V2{(FT)0, (FT)0};
#pragma unroll
    for (int m = 0; m < NCH; ++m) R[d][m] = word4{0u, 0u, 0u, 0u};
  }
  const int top = nlev - 1;
  // first record of wavefronts w and the one D further in the sweep's order
  int first_c = FWD ? 0 : X.ncell, first_l = FWD ? 0 : X.ncell - count(top);
  for (int s0 = 0; s0 < nstep; s0 += D) {
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const int w = FWD ? s0 + k - D : top - (s0 + k - D);
      const int wl = FWD ? w + D : w - D;          // wavefront loaded on this step
      const int wn = FWD ? w + 1 : w - 1;          // next wavefront
      const int cw = count(w), cl = count(wl);
      if constexpr (TH > 64) lds_barrier();   // one wave: its LDS accesses are performed in order
      const bool act = p < cw;
      const int j = level_jlo(w, X.bw) + p, i = w - 3 * j;
      V2 v = stv[w & 1][p & 63];
      if (act) {   // whole quads
        const FT *rec = (const FT *)&stage[w & 1][0] + p * kBoxIluRec;
        const V2 *rb = &ring[j + 2][(i - 2) & (kRingW - 1)];
        FT au = (FT)0, av = (FT)0;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          const V2 x = rb[off[m]];
          FT c0, c1, c2, c3;
          slots4(rec + 12 * part, m, c0, c1, c2, c3);
          au += c0 * x.x + c1 * x.y;
          av += c2 * x.x + c3 * x.y;
        }
        v.x -= quad_sum(au);
        v.y -= quad_sum(av);
        if constexpr (FWD && TRANS) {   // U^T: 1/U(u,u) at 49, U(u,v) at 48, 1/U(v,v) at 50
          v.x *= rec[49];
          v.y = (v.y - rec[48] * v.x) * rec[50];
        } else if constexpr (FWD) {
          v.y -= rec[48] * v.x;
        } else {
          v.y *= rec[50];
          v.x = (v.x - rec[49] * v.y) * rec[48];
        }
        if (part == 0) {
          ring[j + 2][i & (kRingW - 1)] = v;
          ring[j + 2][(i & (kRingW - 1)) + kRingW] = v;
        }
      }
      store_pair(rsV, act && part == 0 ? (unsigned)((first_c + p) * sizeof(V2)) : kPastEnd, 0, v);
      // the records and values of the next wavefront (loaded D - 1 steps ago) to LDS
      wait_vm<(D - 2) * kOps + 1>();
      __builtin_amdgcn_sched_barrier(0);
      stage_store<NCH, TH>(&stage[wn & 1][0], R[(k + 1) % D]);
      if (t < 64) stv[wn & 1][t] = RV[(k + 1) % D];
      stage_load<FT, NCH, TH>(rsRec, first_l, cl, R[k]);
      RV[k] = load_pair(rsV, t < cl ? (unsigned)((first_l + t) * sizeof(V2)) : kPastEnd, 0, (const V2 *)nullptr);
      if (FWD) {
        first_c += cw;
        first_l += cl;
      } else {
        first_c -= count(w - 1);
        first_l -= count(wl - 1);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

template <typename FT, int NCH, int D, int TH, bool TRANS>
__global__ __launch_bounds__(TH) void k_boxilu_apply2d(Phys P0, Batch bt, BoxIluGeom X, BoxGeom G,
                                                      const SubInfo *__restrict__ subs,
                                                      const int *__restrict__ cellof, const FT *__restrict__ Lrec,
                                                      const FT *__restrict__ Urec, void *__restrict__ ybox_,
                                                      void *__restrict__ boxbuf, const double *__restrict__ r,
                                                      double *__restrict__ z, const GmresState *st, long vstride,
                                                      int kind) {
  using V2 = typename ChunkOf2<FT>::T;
  // batched: the block's instance (its grid, its slice of r and z, its GMRES state)
  const Loc Lc = locate(bt, kFamSub);
  if (!Lc.on) return;
  const Phys &P = bt.map[kFamSub] ? bt.inst[Lc.b].P : P0;
  if (bt.map[kFamSub]) {
    r += bt.inst[Lc.b].xoff;
    z += bt.inst[Lc.b].xoff;
  }
  if (st) st += Lc.b;
  double sc = 1.0;
  if (st) {
    if (st->done) return;
    r += (long)st->j * vstride;
    z += (long)st->j * vstride;
    sc = st->inv_norm[st->j];
  }
  __shared__ word4 stage[2][NCH * TH];
  __shared__ V2 stv[2][64];
  // ring: box row j at ring row j + 2, bh + 4 rows (dynamic LDS, so that blocks of small
  // boxes share a CU)
  extern __shared__ char dyn_lds[];
  V2(*ring)[2 * kRingW] = reinterpret_cast<V2(*)[2 * kRingW]>(dyn_lds);
  const int t = threadIdx.x;
  const int part = t & 3;   // the lane's 3 of the cell's 12 neighbour cells: 3 part .. 3 part + 2
  for (int e = t; e < (X.bh + 4) * 2 * kRingW; e += TH) (&ring[0][0])[e] = V2{(FT)0, (FT)0};
  const long cbase = (long)blockIdx.x * X.ncell;
  const unsigned rbytes = (unsigned)(X.ncell * kBoxIluRec * sizeof(FT));
  const __amdgpu_buffer_rsrc_t rsL = buffer_rsrc(Lrec + cbase * kBoxIluRec, rbytes);
  const __amdgpu_buffer_rsrc_t rsU = buffer_rsrc(Urec + cbase * kBoxIluRec, rbytes);
  const __amdgpu_buffer_rsrc_t rsV = buffer_rsrc((V2 *)ybox_ + cbase, (unsigned)(X.ncell * sizeof(V2)));
  // ring offsets (from column (i - 2) mod 16 of the cell's row) of this lane's neighbours
  int offL[3], offU[3];
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    const Off lo = lower_cell(3 * part + m), up = upper_cell(3 * part + m);
    offL[m] = lo.dy * 2 * kRingW + lo.dx + 2;
    offU[m] = up.dy * 2 * kRingW + up.dx + 2;
  }
  const SubInfo si = subs[blockIdx.x];
  const Rect rc = grid_rect(si, X.bw, X.bh, P.nx, P.ny, P.periodic);
  V2 *yk = (V2 *)ybox_ + cbase;
  gather_box<FT, TH>(P, X, si, rc, cellof, r, sc, yk, kind);
  __syncthreads();   // the box vector, written by other threads, before the L sweep loads it
  sweep<FT, NCH, D, TH, true, TRANS>(X, rsL, rsV, stage, stv, ring, offL);
  wait_vm<0>();
  __syncthreads();   // y of every cell in ybox, written by other threads, before the U sweep
  sweep<FT, NCH, D, TH, false>(X, rsU, rsV, stage, stv, ring, offU);
  wait_vm<0>();
  __syncthreads();   // x of every cell, before the scatter reads it
  scatter_box<FT, TH>(P, X, G, si, rc, cellof, yk, (FT *)boxbuf, z, kind);
}

// Records of the transposed solves (L U)^{-T}: U^T is swept forward, L^T backward, with the
// same sweeps.  The U^T record of cell p holds, for its lower cell k (q = p + lower(k), so
// p = q + upper(11 - k)), the entries of q's U row towards p: U(u_q,u_p) U(v_q,u_p)
// U(u_q,v_p) U(v_q,v_p) at 4k .. 4k+3, then U(u_p,v_p), 1/U(u_p,u_p), 1/U(v_p,v_p) at 48..50.
// The L^T record holds, for its upper cell k (q = p + upper(k), p = q + lower(11 - k)),
// L(u_q,u_p) L(v_q,u_p) L(u_q,v_p) L(v_q,v_p), then 1, L(v_p,u_p), 1 at 48..50 (the
// backward sweep's diagonal form with a unit diagonal).
template <typename FT>
__global__ __launch_bounds__(256) void k_boxilu_pack_t(BoxIluGeom X, const int *__restrict__ lvoff,
                                                       const int *__restrict__ cellof, const FT *__restrict__ Lrec,
                                                       const FT *__restrict__ Urec, FT *__restrict__ Tf,
                                                       FT *__restrict__ Tb) {
  const int pos = blockIdx.x * 256 + threadIdx.x;
  if (pos >= X.ncell) return;
  const long base = (long)blockIdx.y * X.ncell;
  const int ij = cellof[pos], i = ij & 0xffff, j = ij >> 16;
  const FT *Lp = Lrec + (base + pos) * kBoxIluRec, *Up = Urec + (base + pos) * kBoxIluRec;
  FT *F = Tf + (base + pos) * kBoxIluRec, *B = Tb + (base + pos) * kBoxIluRec;
  auto in_box = [&](int a, int b) { return a >= 0 && a < X.bw && b >= 0 && b < X.bh; };
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const Off lo = lower_cell(k), up = upper_cell(k);
    const int s = 4 * (11 - k);
    if (in_box(i + lo.dx, j + lo.dy)) {
      const FT *Uq = Urec + (base + cell_pos(lvoff, i + lo.dx, j + lo.dy, X.bw)) * kBoxIluRec;
      F[4 * k] = Uq[s];
      F[4 * k + 1] = Uq[s + 2];
      F[4 * k + 2] = Uq[s + 1];
      F[4 * k + 3] = Uq[s + 3];
    } else {
      F[4 * k] = F[4 * k + 1] = F[4 * k + 2] = F[4 * k + 3] = (FT)0;
    }
    if (in_box(i + up.dx, j + up.dy)) {
      const FT *Lq = Lrec + (base + cell_pos(lvoff, i + up.dx, j + up.dy, X.bw)) * kBoxIluRec;
      B[4 * k] = Lq[s];
      B[4 * k + 1] = Lq[s + 2];
      B[4 * k + 2] = Lq[s + 1];
      B[4 * k + 3] = Lq[s + 3];
    } else {
      B[4 * k] = B[4 * k + 1] = B[4 * k + 2] = B[4 * k + 3] = (FT)0;
    }
  }
  F[48] = Up[49];
  F[49] = Up[48];
  F[50] = Up[50];
  F[51] = (FT)0;
  B[48] = (FT)1;
  B[49] = Lp[48];
  B[50] = (FT)1;
  B[51] = (FT)0;
}

// Factors (FT records) -> FP64 [sub][cell j bw + i][L record, U record].
template <typename FT>
__global__ void k_boxilu_export(BoxIluGeom X, int nsub, const int *__restrict__ lvoff, const FT *__restrict__ Lrec,
                                const FT *__restrict__ Urec, double *__restrict__ out) {
  const long total = (long)nsub * X.ncell * 2 * kBoxIluRec;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < total; e += (long)gridDim.x * 256) {
    const int s = (int)(e % (2 * kBoxIluRec));
    const long cell = (e / (2 * kBoxIluRec)) % X.ncell;
    const long b = e / (2 * kBoxIluRec * (long)X.ncell);
    const int j = (int)(cell / X.bw), i = (int)(cell - (long)j * X.bw);
    const long p = (b * X.ncell + cell_pos(lvoff, i, j, X.bw)) * kBoxIluRec;
    out[e] = (double)(s < kBoxIluRec ? Lrec[p + s] : Urec[p + s - kBoxIluRec]);
  }
}

template <typename FT, int NCH, int TH>
void apply_launch(const BatchLaunch &bl, const BoxIluGeom &X, const BoxGeom &G, const SubInfo *subs, const int *cellof,
                  const void *L, const void *U, double *ybox, void *boxbuf, const double *r, double *z,
                  const GmresState *st, long vstride, int kind, bool trans, hipStream_t s) {
  constexpr int D = TH == 64 ? (NCH <= 7 ? 4 : 3) : (NCH <= 3 ? 6 : 4);   // register stages
  const size_t ring_bytes = (size_t)(X.bh + 4) * 2 * kRingW * 2 * sizeof(FT);
  if (trans)
    hipLaunchKernelGGL((k_boxilu_apply2d<FT, NCH, D, TH, true>), dim3(G.nsub), dim3(TH), ring_bytes, s, bl.P0, bl.bt, X,
                       G, subs,
                       cellof, (const FT *)L, (const FT *)U, (void *)ybox, boxbuf, r, z, st, vstride, kind);
  else
    hipLaunchKernelGGL((k_boxilu_apply2d<FT, NCH, D, TH, false>), dim3(G.nsub), dim3(TH), ring_bytes, s, bl.P0, bl.bt, X,
                       G, subs,
                       cellof, (const FT *)L, (const FT *)U, (void *)ybox, boxbuf, r, z, st, vstride, kind);
}

template <typename FT>
hipError_t apply_t(const BatchLaunch &bl, const BoxIluGeom &X, const BoxGeom &G, const SubInfo *subs, const int *cellof,
                   const void *L, const void *U, double *ybox, void *boxbuf, const double *r, double *z,
                   const GmresState *st, long vstride, int kind, bool trans, hipStream_t s) {
  const int bytes = X.maxcount * kBoxIluRec * (int)sizeof(FT);   // one wavefront's records
  // One wave per box when the quads of a wavefront fit it (no barriers) and there are
  // enough boxes for several blocks per CU; otherwise 256 threads, whose four waves share
  // the loads.
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
  }
  if (X.maxcount <= 16 && G.nsub >= 2 * cus) {
    const int nch = (bytes + 1023) / 1024;
    if (nch <= 3) apply_launch<FT, 3, 64>(bl, X, G, subs, cellof, L, U, ybox, boxbuf, r, z, st, vstride, kind, trans, s);
    else if (nch <= 5) apply_launch<FT, 5, 64>(bl, X, G, subs, cellof, L, U, ybox, boxbuf, r, z, st, vstride, kind, trans, s);
    else if (nch <= 7) apply_launch<FT, 7, 64>(bl, X, G, subs, cellof, L, U, ybox, boxbuf, r, z, st, vstride, kind, trans, s);
    else if (nch <= 10) apply_launch<FT, 10, 64>(bl, X, G, subs, cellof, L, U, ybox, boxbuf, r, z, st, vstride, kind, trans, s);
    else apply_launch<FT, 13, 64>(bl, X, G, subs, cellof, L, U, ybox, boxbuf, r, z, st, vstride, kind, trans, s);
  } else {
    switch ((bytes + 16 * kBoxIluThreads - 1) / (16 * kBoxIluThreads)) {
      case 1: apply_launch<FT, 1, kBoxIluThreads>(bl, X, G, subs, cellof, L, U, ybox, boxbuf, r, z, st, vstride, kind, trans, s); break;
      case 2: apply_launch<FT, 2, kBoxIluThreads>(bl, X, G, subs, cellof, L, U, ybox, boxbuf, r, z, st, vstride, kind, trans, s); break;
      case 3: apply_launch<FT, 3, kBoxIluThreads>(bl, X, G, subs, cellof, L, U, ybox, boxbuf, r, z, st, vstride, kind, trans, s); break;
      case 4: apply_launch<FT, 4, kBoxIluThreads>(bl, X, G, subs, cellof, L, U, ybox, boxbuf, r, z, st, vstride, kind, trans, s); break;
      case 5: apply_launch<FT, 5, kBoxIluThreads>(bl, X, G, subs, cellof, L, U, ybox, boxbuf, r, z, st, vstride, kind, trans, s); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

}  // namespace

bool boxilu_fits(const BoxIluGeom &X) {
  return X.bw >= 1 && X.bh >= 1 && X.bw <= kBoxIluMaxW && X.bh <= kBoxIluMaxH && X.bh <= kBoxIluThreads &&
         X.maxcount * kBoxIluRec * 8 <= 5 * 16 * kBoxIluThreads;
}

namespace {
template <typename FT, int TH>
void factor_launch(const BatchLaunch &bl, const BoxIluGeom &X, int nsub, const SubInfo *subs, const int *lvoff,
                   const double *J, double shift, void *L, void *U, hipStream_t s) {
  hipLaunchKernelGGL((k_boxilu_factor2d<FT, TH>), dim3(nsub), dim3(TH), 0, s, bl.P0, bl.bt, X, subs, lvoff, J, shift,
                     (FT *)L, (FT *)U);
}
template <typename FT>
void factor_t(const BatchLaunch &bl, const BoxIluGeom &X, int nsub, const SubInfo *subs, const int *lvoff,
              const double *J, double shift, void *L, void *U, hipStream_t s) {
  // one thread per box row; short boxes take smaller blocks, so that several share a CU
  if (X.bh <= 64) factor_launch<FT, 64>(bl, X, nsub, subs, lvoff, J, shift, L, U, s);
  else if (X.bh <= 128) factor_launch<FT, 128>(bl, X, nsub, subs, lvoff, J, shift, L, U, s);
  else factor_launch<FT, kBoxIluThreads>(bl, X, nsub, subs, lvoff, J, shift, L, U, s);
}
}  // namespace

hipError_t launch_boxilu_factor2d(const BatchLaunch &bl, const BoxIluGeom &X, int nsub, const SubInfo *subs,
                                  const int *lvoff, const double *J, double shift, void *L, void *U, int fp32,
                                  hipStream_t s) {
  if (!boxilu_fits(X)) return hipErrorInvalidValue;
  if (fp32)
    factor_t<float>(bl, X, nsub, subs, lvoff, J, shift, L, U, s);
  else
    factor_t<double>(bl, X, nsub, subs, lvoff, J, shift, L, U, s);
  return hipGetLastError();
}

hipError_t launch_boxilu_apply2d(const BatchLaunch &bl, const BoxIluGeom &X, const BoxGeom &G, const SubInfo *subs,
                                 const int *cellof, const void *L, const void *U, double *ybox, void *boxbuf,
                                 const double *r, double *z, const GmresState *st, long vstride, int fp32,
                                 hipStream_t s, const RasVariant &rv, bool trans) {
  if (!boxilu_fits(X)) return hipErrorInvalidValue;
  // batches: the left-restricted forward operator only
  if (bl.bt.map[kFamSub] != nullptr && (rv.kind != ACCH_RAS_LEFT || trans)) return hipErrorInvalidValue;
  if (rv.kind != ACCH_RAS_LEFT && !rv.own_x) return hipErrorInvalidValue;
  hipError_t e = fp32 ? apply_t<float>(bl, X, G, subs, cellof, L, U, ybox, boxbuf, r, z, st, vstride, rv.kind, trans, s)
                      : apply_t<double>(bl, X, G, subs, cellof, L, U, ybox, boxbuf, r, z, st, vstride, rv.kind, trans,
                                        s);
  if (e != hipSuccess || rv.kind == ACCH_RAS_LEFT) return e;
  return launch_ras_sum2d(bl, G, subs, boxbuf, z, st, vstride, fp32, s, rv);
}

hipError_t launch_boxilu_export(const BoxIluGeom &X, int nsub, const int *lvoff, const void *L, const void *U,
                                int fp32, double *out, hipStream_t s) {
  const long total = (long)nsub * X.ncell * 2 * kBoxIluRec;
  const int blocks = (int)std::min<long>((total + 255) / 256, 4096);
  if (fp32)
    hipLaunchKernelGGL(k_boxilu_export<float>, dim3(blocks), dim3(256), 0, s, X, nsub, lvoff, (const float *)L,
                       (const float *)U, out);
  else
    hipLaunchKernelGGL(k_boxilu_export<double>, dim3(blocks), dim3(256), 0, s, X, nsub, lvoff, (const double *)L,
                       (const double *)U, out);
  return hipGetLastError();
}

hipError_t launch_boxilu_pack_t(const BoxIluGeom &X, int nsub, const int *lvoff, const int *cellof, const void *L,
                                const void *U, void *Tf, void *Tb, int fp32, hipStream_t s) {
  const dim3 grid((X.ncell + 255) / 256, nsub);
  if (fp32)
    hipLaunchKernelGGL(k_boxilu_pack_t<float>, grid, dim3(256), 0, s, X, lvoff, cellof, (const float *)L,
                       (const float *)U, (float *)Tf, (float *)Tb);
  else
    hipLaunchKernelGGL(k_boxilu_pack_t<double>, grid, dim3(256), 0, s, X, lvoff, cellof, (const double *)L,
                       (const double *)U, (double *)Tf, (double *)Tb);
  return hipGetLastError();
}

}  // namespace acch
