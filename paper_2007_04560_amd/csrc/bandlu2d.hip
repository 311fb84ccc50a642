// Exact-LU and ILU(k) subdomain solvers of the 2D Schwarz preconditioner (Section 3.1,
// the subdomain solvers compared in Table 2), in the band storage of band.h.
//
// Extraction: every box matrix A_k = R_k J R_k^T (plus sigma diag(A_k) for ILU(k)) is
// written into a zeroed band; cells of the padded box outside the grid are decoupled
// identity rows, as in the ILU(0) path.
//
// Factorisation (one workgroup of 256 threads per box): Gaussian elimination without
// pivoting in the natural order, through a register window of the active part of the
// band (details at k_band_factor2d).  With an ILU(k) pattern (a bit per band entry, from
// the host's symbolic level-of-fill elimination) the entries outside the pattern are
// zero wherever they are used, which is ILU(k) in IKJ form.  The elimination runs in the
// precision of the stored factors: FP64 factors in FP64, FP32 factors (the
// mixed-precision form) in FP32.
//
// Solve (eight waves per box): forward substitution with L, then backward with U, 64 rows
// at a time (details at k_band_solve2d), in FP64 arithmetic on FP64 or FP32 factors.
#include <algorithm>

#include "../../include/acch.h"
#include "band.h"
#include "boxes.h"
#include "bufio.h"
#include "kernels.h"

namespace acch {
namespace {

// The 24 Jacobian slots of include/acch.h: row type, column type, column offset.
struct BSlot {
  int rt, ct, dx, dy;
};
__host__ __device__ constexpr BSlot bslot(int s) {
  constexpr BSlot tab[kNSlot2D] = {
      {0, 0, 0, 0},   {0, 0, -1, 0}, {0, 0, 1, 0},  {0, 0, 0, -1}, {0, 0, 0, 1},  {0, 0, -2, 0},
      {0, 0, 2, 0},   {0, 0, 0, -2}, {0, 0, 0, 2},  {0, 0, -1, -1}, {0, 0, 1, -1}, {0, 0, -1, 1},
      {0, 0, 1, 1},   {0, 1, 0, 0},  {0, 1, -1, 0}, {0, 1, 1, 0},  {0, 1, 0, -1}, {0, 1, 0, 1},
      {1, 1, 0, 0},   {1, 1, -1, 0}, {1, 1, 1, 0},  {1, 1, 0, -1}, {1, 1, 0, 1},  {1, 0, 0, 0}};
  return tab[s];
}

// Cells of the padded box that hold a grid cell: the rectangle [ilo, ihi) x [jlo, jhi).
struct Rect {
  int ilo, ihi, jlo, jhi;
};
ACCH_DEV Rect inside_rect(const SubInfo &si, const BandGeom &B, int nx, int ny, int periodic) {
  Rect r{0, min(B.bw, si.ex), 0, min(B.bh, si.ey)};
  if (!periodic) {
    r.ilo = max(r.ilo, -si.ox);
    r.jlo = max(r.jlo, -si.oy);
    r.ihi = min(r.ihi, nx - si.ox);
    r.jhi = min(r.jhi, ny - si.oy);
  }
  return r;
}
ACCH_DEV bool in_rect(const Rect &r, int i, int j) { return i >= r.ilo && i < r.ihi && j >= r.jlo && j < r.jhi; }

ACCH_DEV long band_at(const BandGeom &B, int R, int d) { return ((long)(R >> 6) * B.nd + d) * 64 + (R & 63); }

template <typename FT>
__global__ __launch_bounds__(256) void k_band_zero(FT *__restrict__ band, long total) {
  for (long e = blockIdx.x * 256L + threadIdx.x; e < total; e += (long)gridDim.x * 256) band[e] = (FT)0;
}

// A_k (+ shift diag(A_k)) into the zeroed band of each box: one block per box.
template <typename FT>
__global__ __launch_bounds__(256) void k_band_extract2d(Phys P, BandGeom B, const SubInfo *__restrict__ subs,
                                                         const double *__restrict__ J, double shift,
                                                         FT *__restrict__ band) {
  const SubInfo si = subs[blockIdx.x];
  const Rect rc = inside_rect(si, B, P.nx, P.ny, P.periodic);
  FT *Bk = band + (long)blockIdx.x * B.box_elems;
  const long n = (long)P.nx * P.ny;
  for (int c = threadIdx.x; c < B.bw * B.bh; c += 256) {
    const int j = c / B.bw, i = c - j * B.bw;
    const int R0 = 2 * c;
    if (!in_rect(rc, i, j)) {
      Bk[band_at(B, R0, B.kl)] = (FT)1;
      Bk[band_at(B, R0 + 1, B.kl)] = (FT)1;
      continue;
    }
    const long g = box_to_global(si, i, j, P.nx, P.ny, P.periodic);
#pragma unroll
    for (int s = 0; s < kNSlot2D; ++s) {
      const BSlot q = bslot(s);
      const int ii = i + q.dx, jj = j + q.dy;
      if (!in_rect(rc, ii, jj)) continue;
      const int R = R0 + q.rt, C = 2 * (jj * B.bw + ii) + q.ct;
      double v = J[(long)s * n + g];
      if (R == C) v *= 1.0 + shift;
      Bk[band_at(B, R, C - R + B.kl)] = (FT)v;
    }
  }
}

// Barrier for values exchanged through LDS only: device-memory loads and stores issued
// before it stay in flight (__syncthreads would wait for them).
ACCH_DEV void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Band LU (or ILU(k) on the pattern `mask`, MASKED) of one box matrix per block, in
// place.  Right-looking elimination through a W x W register window (W = 16 NR >= kl + 1)
// that holds the active part of the Schur complement; all fill of the band LU stays
// within kl of the diagonal, so nothing outside the window is touched.  Steps go in
// groups of 16: before the steps 16 g .. 16 g + 15, register tile (p, q) of thread
// (ty, tx) holds entry (16 g + 16 p + ty, 16 g + 16 q + tx).  Step k = 16 g + tr pivots
// on tile row and column 0 of the threads with ty == tr and tx == tr, publishes the pivot
// row and column through LDS, updates the window, stores row k of U and column k of L,
// and puts row and column k + W of the original matrix in the pivot's place.  After the
// group the tiles rotate by one (tile 0, now holding rows and columns 16 g + W + ..., is
// the last), so the pivot tile is always tile 0 and every register is named at compile
// time.
//
// The rows and columns that enter during group g are loaded at the start of group
// g - 1: thread (ty, tx) loads the row entering at step 16 g + ty and the column entering
// at step 16 g + tx into registers and moves them to LDS at the start of group g.  The
// only wait for device memory is therefore the one at a group's start, for loads issued
// 16 steps earlier.
template <typename FT, int NR, bool MASKED>
__global__ __launch_bounds__(256) void k_band_factor2d(BandGeom B, FT *__restrict__ band,
                                                        const unsigned *__restrict__ mask) {
  constexpr int W = 16 * NR;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  FT *Bk = band + (long)blockIdx.x * B.box_elems;
  const unsigned *Mk = MASKED ? mask + (long)blockIdx.x * B.n * B.mwords : nullptr;
  const int n = B.n, kl = B.kl, nd = B.nd;
  __shared__ FT urow[2][W], acol[2][W];
  __shared__ FT srow[NR][256], scol[NR][256];
  __shared__ unsigned srw[MASKED ? NR : 1][256], scw[MASKED ? NR : 1][256];

  auto in_band = [&](int R, int C) {
    const int d = C - R + kl;
    return R < n && C < n && (unsigned)d < (unsigned)nd;
  };
  // Range-checked buffer accesses: an entry outside the matrix or the band has an offset
  // past the end, so it loads as zero (pattern word zero) and a store to it is dropped.
  const __amdgpu_buffer_rsrc_t rsB = buffer_rsrc(Bk, (unsigned)(B.box_elems * sizeof(FT)));
  const __amdgpu_buffer_rsrc_t rsM = buffer_rsrc(Mk, MASKED ? (unsigned)(B.n * B.mwords * 4) : 0u);
  auto boff = [&](int R, int C) -> unsigned {
    return in_band(R, C) ? (unsigned)band_at(B, R, C - R + kl) * (unsigned)sizeof(FT) : kPastEnd;
  };
  auto raw = [&](int R, int C) -> FT { return load_one(rsB, boff(R, C), 0, (const FT *)nullptr); };
  // the ILU(k) pattern word holding (R, C)
  auto raw_mask = [&](int R, int C) -> unsigned {
    const unsigned o = in_band(R, C) ? (unsigned)(R * B.mwords + ((C - R + kl) >> 5)) * 4u : kPastEnd;
    return load_one(rsM, o, 0, (const unsigned *)nullptr);
  };
  // bit of (R, C) in its pattern word (a word loaded for an entry outside the band is 0)
  auto mask_bit = [&](int R, int C, unsigned word) -> unsigned { return (word >> ((C - R + kl) & 31)) & 1u; };
  // column of tile q of this thread after step kg + t of the group starting at kg (row of
  // tile p: the same with ty)
  auto col_after = [&](int kg, int t, int q) { return kg + 16 * q + tx + (q == 0 && tx <= t ? W : 0); };
  auto row_after = [&](int kg, int t, int p) { return kg + 16 * p + ty + (p == 0 && ty <= t ? W : 0); };

  FT a[NR][NR];
  unsigned m[NR];   // bit q: entry (row of tile p, column of tile q) is in the pattern
#pragma unroll
  for (int p = 0; p < NR; ++p) {
    m[p] = 0;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const int R = ty + 16 * p, C = tx + 16 * q;
      a[p][q] = raw(R, C);
      if (MASKED) m[p] |= mask_bit(R, C, raw_mask(R, C)) << q;
    }
  }

  // rows (at this thread's columns) and columns (at its rows) entering during the next
  // group, in registers; those of the current group in LDS (read by the same thread)
  FT nrow[NR], ncol[NR];
  unsigned nrw[NR], ncw[NR];
  auto load_group = [&](int kg) {
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const int C = col_after(kg, ty, q);
      nrow[q] = raw(kg + ty + W, C);
      if (MASKED) nrw[q] = raw_mask(kg + ty + W, C);
    }
#pragma unroll
    for (int p = 0; p < NR; ++p) {
      const int R = row_after(kg, tx, p);
      ncol[p] = raw(R, kg + tx + W);
      if (MASKED) ncw[p] = raw_mask(R, kg + tx + W);
    }
  };
  load_group(0);
  __syncthreads();

  for (int kg = 0; kg < n; kg += 16) {
    // this group's entering rows and columns (loaded a group ago) move to LDS; the
    // next group's loads start
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      srow[q][tid] = nrow[q];
      scol[q][tid] = ncol[q];
      if (MASKED) {
        srw[q][tid] = nrw[q];
        scw[q][tid] = ncw[q];
      }
    }
    if (kg + 16 < n) load_group(kg + 16);
    const int tend = min(16, n - kg);
    for (int tr = 0; tr < tend; ++tr) {
      const int k = kg + tr, buf = k & 1;
      const bool prow_t = ty == tr, pcol_t = tx == tr;   // owns the pivot row / column
      // ILU(k): entries off the pattern are updated like the others but never read --
      // they are dropped here, the only place an entry's value is used (as part of the
      // pivot row or column), which is the same as dropping every update to them
      if (prow_t) {
#pragma unroll
        for (int q = 0; q < NR; ++q)
          urow[buf][tx + 16 * q] = (!MASKED || ((m[0] >> q) & 1u)) ? a[0][q] : (FT)0;
      }
      if (pcol_t) {
#pragma unroll
        for (int p = 0; p < NR; ++p) acol[buf][ty + 16 * p] = (!MASKED || (m[p] & 1u)) ? a[p][0] : (FT)0;
      }
      // LDS only: the band stores of earlier steps and the loads of the next group
      // touch other entries and stay in flight
      lds_barrier();
      const FT inv = (FT)1 / urow[buf][tr];
      FT l[NR], u[NR];
#pragma unroll
      for (int p = 0; p < NR; ++p) l[p] = acol[buf][ty + 16 * p] * inv;
#pragma unroll
      for (int q = 0; q < NR; ++q) u[q] = urow[buf][tx + 16 * q];
      if (prow_t) l[0] = (FT)0;   // the pivot row and column are not updated
      if (pcol_t) u[0] = (FT)0;
#pragma unroll
      for (int p = 0; p < NR; ++p)
#pragma unroll
        for (int q = 0; q < NR; ++q) a[p][q] -= l[p] * u[q];

      // row k of U (1/u_kk on the diagonal) and column k of L over the band: entry (k, k + off)
      // lies kl + off diagonals into row k's chunk (a uniform base plus 64 off), entry
      // (k + off, k) at diagonal kl - off of row k + off
      if (prow_t) {
        const unsigned u0 = (unsigned)(((k >> 6) * nd + kl) * 64 + (k & 63));
#pragma unroll
        for (int q = 0; q < NR; ++q) {
          const int off = 16 * q + tx - tr + (q == 0 && tx < tr ? W : 0);   // column k + off
          const bool ok = off <= kl && k + off < n;
          store_one(rsB, ok ? (u0 + 64u * (unsigned)off) * (unsigned)sizeof(FT) : kPastEnd, 0, off == 0 ? inv : u[q]);
        }
      }
      if (pcol_t) {
#pragma unroll
        for (int p = 0; p < NR; ++p) {
          const int off = 16 * p + ty - tr + (p == 0 && ty < tr ? W : 0);   // row k + off
          const int R = k + off;
          const bool ok = off >= 1 && off <= kl && R < n;
          const unsigned o = (unsigned)(((R >> 6) * nd + kl - off) * 64 + (R & 63));
          store_one(rsB, ok ? o * (unsigned)sizeof(FT) : kPastEnd, 0, l[p]);
        }
      }
      // row and column k + W take the pivot's place
      if (prow_t) {
        unsigned mr = 0;
#pragma unroll
        for (int q = 0; q < NR; ++q) {
          const int C = col_after(kg, tr, q);
          a[0][q] = srow[q][tid];
          if (MASKED) mr |= mask_bit(k + W, C, srw[q][tid]) << q;
        }
        if (MASKED) m[0] = mr;
      }
      if (pcol_t) {
#pragma unroll
        for (int p = 0; p < NR; ++p) {
          const int R = row_after(kg, tr, p);
          a[p][0] = scol[p][tid];
          if (MASKED) m[p] = (m[p] & ~1u) | mask_bit(R, k + W, scw[p][tid]);
        }
      }
    }
    // tiles move down by one: tile (p, q) takes tile (p + 1, q + 1), cyclically
    {
      FT t[NR];
#pragma unroll
      for (int q = 0; q < NR; ++q) t[q] = a[0][q];
#pragma unroll
      for (int p = 0; p + 1 < NR; ++p)
#pragma unroll
        for (int q = 0; q < NR; ++q) a[p][q] = a[p + 1][(q + 1) % NR];
#pragma unroll
      for (int q = 0; q < NR; ++q) a[NR - 1][q] = t[(q + 1) % NR];
      if (MASKED) {
        const unsigned full = (1u << NR) - 1u;
        const unsigned m0 = m[0];
#pragma unroll
        for (int p = 0; p + 1 < NR; ++p) m[p] = ((m[p + 1] >> 1) | (m[p + 1] << (NR - 1))) & full;
        m[NR - 1] = ((m0 >> 1) | (m0 << (NR - 1))) & full;
      }
    }
  }
}

// Broadcast of lane s (wave-uniform s) of a double.
ACCH_DEV double bcast(double v, int s) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), s);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), s);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

constexpr int kRing = 512;   // finished values kept for the band (kl + 64 <= kRing)
constexpr int kSolveWaves = 8;   // waves per box: all share the finished-chunk terms

// Forward and backward substitution with the band factors of one box per block, for
// z = sum_k R_k^T (LU)_k^{-1} R_k r (left RAS: owned cells only; right and classical:
// into the box buffer for the overlap sum).  The 64 rows of a chunk are solved together.
// Phase 1 adds the terms of all columns within kl of the rows (diagonals 1..kl split
// between the waves, partial sums through LDS); the ring slots of the chunk's own rows
// hold zeros at that point, so the terms of its own columns vanish there, and their
// coefficients go to tri (column s of the chunk, row lane) for phase 2, in which one wave
// takes the 64 rows in order, row s broadcast from its lane.  The lower (forward) and
// upper (backward) tri are separate and start as zeros, so phase 2 needs no masks; the
// backward sweep broadcasts acc / u_ss and scales every row by 1 / u_ss at the end.
// Each wave's coefficients of the chunk after next (and the right-hand side values of
// its rows) are loaded while the current chunk is solved, into the third of three
// register sets; the loads use clamped addresses and no condition, so the only wait is for
// data issued a chunk earlier.
template <typename FT, int PER>
__global__ __launch_bounds__(64 * kSolveWaves) void k_band_solve2d(Phys P, BandGeom B, BoxGeom G, const SubInfo *__restrict__ subs,
                                                      const FT *__restrict__ band, double *__restrict__ ybox,
                                                      void *__restrict__ boxbuf_, const double *__restrict__ r,
                                                      double *__restrict__ z, const GmresState *st, long vstride,
                                                      int kind) {
  double sc = 1.0;
  if (st) {
    if (st->done) return;
    const int jj = st->j;
    r += (long)jj * vstride;
    z += (long)jj * vstride;
    sc = st->inv_norm[jj];
  }
  // finished values: row x at x mod kRing and again kRing further, so the kl rows before
  // (after) a chunk's rows lie at increasing addresses without wrapping
  __shared__ double ring[2 * kRing];
  // the chunk's own coefficients; rows 64..127 take stores of other columns, never read
  __shared__ double trl[128][64], tru[128][64];
  __shared__ double psum[kSolveWaves][64];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: scalar
  const SubInfo si = subs[blockIdx.x];
  const Rect rc = inside_rect(si, B, P.nx, P.ny, P.periodic);
  const FT *Bk = band + (long)blockIdx.x * B.box_elems;
  // the coefficients through a buffer: 32-bit offsets, the diagonal's in a scalar register
  const __amdgpu_buffer_rsrc_t rsB = buffer_rsrc(Bk, (unsigned)(B.box_elems * sizeof(FT)));
  double *yk = ybox + (long)blockIdx.x * B.nchunk * 64;
  const long n = (long)P.nx * P.ny;
  const int kl = B.kl, nd = B.nd, nch = B.nchunk;
  for (int e = threadIdx.x; e < 2 * kRing; e += 64 * kSolveWaves) ring[e] = 0.0;
  for (int e = threadIdx.x; e < 128 * 64; e += 64 * kSolveWaves) {
    (&trl[0][0])[e] = 0.0;
    (&tru[0][0])[e] = 0.0;
  }
  // value of row x (both copies) and the ring rows of a chunk's rows
  auto ring_put = [&](int x, double v) {
    ring[x & (kRing - 1)] = v;
    ring[(x & (kRing - 1)) + kRing] = v;
  };
  __syncthreads();
  // this wave's diagonals: dlo .. dlo + PER - 1 (8 PER >= kl); those beyond kl belong to no
  // other wave and load as zero (offset past the end of the buffer)
  const int dlo = 1 + wave * PER;
  // offset (relative to the chunk's row) of diagonal d = kl - dp (L) or kl + dp (U)
  auto coef_off = [&](int dp, int sign) -> unsigned {
    return dp <= kl ? (unsigned)((kl + sign * dp) * 64) * (unsigned)sizeof(FT) : kPastEnd;
  };

  // grid cell of box row R (-1: none), whether its cell is owned
  auto cell_of = [&](int R, bool &own) -> long {
    own = false;
    if (R >= B.n) return -1;
    const int c = R >> 1, j = c / B.bw, i = c - j * B.bw;
    if (!in_rect(rc, i, j)) return -1;
    own = i >= si.own_x0 && i < si.own_x1 && j >= si.own_y0 && j < si.own_y1;
    return box_to_global(si, i, j, P.nx, P.ny, P.periodic);
  };

  // ---- forward: L y = R_k r
  {
    FT ca[PER], cb[PER], cc3[PER];
    double ra = 0.0, rb = 0.0, rc3 = 0.0, fa = 0.0, fb = 0.0, fc = 0.0;   // wave 0: r of the rows, its scale
    auto load = [&](int c, FT (&cf)[PER], double &rv, double &rf) {
      const int cc = min(c, nch - 1);
      const unsigned vo = (unsigned)(cc * nd * 64 + lane) * (unsigned)sizeof(FT);
#pragma unroll
      for (int i = 0; i < PER; ++i) cf[i] = load_one(rsB, vo, coef_off(dlo + i, -1), (const FT *)nullptr);
      if (wave == 0) {
        bool own;
        const int R = 64 * cc + lane;
        const long g = cell_of(R, own);
        rv = r[max(g, 0L) + (R & 1) * n];
        rf = g >= 0 && (kind != ACCH_RAS_RIGHT || own) ? sc : 0.0;   // R_k: rows of the box
      }
    };
    auto chunk = [&](int c, const FT (&cf)[PER], double rv, double rf) {
      const int R = 64 * c + lane;
      double part[4] = {wave == 0 ? rf * rv : 0.0, 0.0, 0.0, 0.0};
      // rd[PER - 1 - i]: row R - (dlo + i); the coefficient goes to trl row 63 - s for the
      // chunk's own column s = lane - dp, to a row >= 64 (not read) for the others
      const double *rd = &ring[(R & (kRing - 1)) + kRing - dlo - (PER - 1)];
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const double coef = (double)cf[i];
        part[i & 3] -= coef * rd[PER - 1 - i];
        trl[min(63 - lane + dlo + i, 127)][lane] = coef;
      }
      psum[wave][lane] = (part[0] + part[1]) + (part[2] + part[3]);
      lds_barrier();
      if (wave == 0) {
        double acc = psum[0][lane];
#pragma unroll
        for (int q = 1; q < kSolveWaves; ++q) acc += psum[q][lane];
#pragma unroll
        for (int s = 0; s < 63; ++s) acc -= trl[63 - s][lane] * bcast(acc, s);
        ring_put(R, acc);
        ring_put(R + 64, 0.0);   // the next chunk's rows
        yk[R] = acc;
      }
      lds_barrier();
    };
    // three register sets rotate by name: chunk c + 2 loads while chunk c is solved
    load(0, ca, ra, fa);
    load(1, cb, rb, fb);
    for (int c = 0; c < nch; c += 3) {
      load(c + 2, cc3, rc3, fc);
      chunk(c, ca, ra, fa);
      if (c + 1 >= nch) break;
      load(c + 3, ca, ra, fa);
      chunk(c + 1, cb, rb, fb);
      if (c + 2 >= nch) break;
      load(c + 4, cb, rb, fb);
      chunk(c + 2, cc3, rc3, fc);
    }
  }
  // ---- backward: U x = y
  if (wave == 0) ring_put(64 * (nch - 1) + lane, 0.0);   // the last chunk's rows
  __syncthreads();
  FT *boxbuf = (FT *)boxbuf_;
  const long ncb = (long)G.nlev * G.bh;
  {
    FT ca[PER], cb[PER], cc3[PER];
    double ya = 0.0, yb = 0.0, yc = 0.0, ia = 0.0, ib = 0.0, ic = 0.0;
    auto load = [&](int c, FT (&cf)[PER], double &yv, double &iv) {
      const int cc = max(c, 0);
      const unsigned vo = (unsigned)(cc * nd * 64 + lane) * (unsigned)sizeof(FT);
#pragma unroll
      for (int i = 0; i < PER; ++i) cf[i] = load_one(rsB, vo, coef_off(dlo + i, 1), (const FT *)nullptr);
      if (wave == 0) {
        yv = yk[64 * cc + lane];
        iv = (double)load_one(rsB, vo, (unsigned)(kl * 64) * (unsigned)sizeof(FT), (const FT *)nullptr);
      }
    };
    auto chunk = [&](int c, const FT (&cf)[PER], double yv, double inv) {
      const int R = 64 * c + lane;
      double part[4] = {wave == 0 ? yv : 0.0, 0.0, 0.0, 0.0};
      // rd[i]: row R + dlo + i; the coefficient goes to tru row s = lane + dp for the
      // chunk's own column s <= 63, to a row >= 64 (not read) for the others
      const double *rd = &ring[(R & (kRing - 1)) + dlo];
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const double coef = (double)cf[i];
        part[i & 3] -= coef * rd[i];
        tru[min(lane + dlo + i, 127)][lane] = coef;
      }
      psum[wave][lane] = (part[0] + part[1]) + (part[2] + part[3]);
      lds_barrier();
      if (wave == 0) {
        double acc = psum[0][lane];
#pragma unroll
        for (int q = 1; q < kSolveWaves; ++q) acc += psum[q][lane];
#pragma unroll
        for (int s = 63; s >= 1; --s) acc -= tru[s][lane] * bcast(acc * inv, s);
        acc *= inv;
        ring_put(R, acc);
        ring_put(R - 64, 0.0);   // the next chunk's rows
        bool own;
        const long g = cell_of(R, own);
        if (g >= 0) {
          if (kind == ACCH_RAS_LEFT) {
            if (own) z[g + (R & 1) * n] = acc;
          } else {
            const int cc = R >> 1, j = cc / B.bw, i = cc - j * B.bw;
            boxbuf[2 * ((long)blockIdx.x * (ncb + 1) + (long)(i + 2 * j) * G.bh + j) + (R & 1)] = (FT)acc;
          }
        }
      }
      lds_barrier();
    };
    // the y values of the chunk were stored by the same threads (wave 0) in the forward
    // sweep
    load(nch - 1, ca, ya, ia);
    load(nch - 2, cb, yb, ib);
    for (int c = nch - 1; c >= 0; c -= 3) {
      load(c - 2, cc3, yc, ic);
      chunk(c, ca, ya, ia);
      if (c - 1 < 0) break;
      load(c - 3, ca, ya, ia);
      chunk(c - 1, cb, yb, ib);
      if (c - 2 < 0) break;
      load(c - 4, cb, yb, ib);
      chunk(c - 2, cc3, yc, ic);
    }
  }
}

// Band (FT) -> FP64 [sub][R][d].
template <typename FT>
__global__ void k_band_export(BandGeom B, int nsub, const FT *__restrict__ band, double *__restrict__ out) {
  const long total = (long)nsub * B.n * B.nd;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < total; e += (long)gridDim.x * 256) {
    const int d = (int)(e % B.nd);
    const long rs = e / B.nd;
    const long sub = rs / B.n;
    const int R = (int)(rs - sub * B.n);
    out[e] = (double)band[sub * B.box_elems + band_at(B, R, d)];
  }
}

template <typename FT>
hipError_t factor_t(const Phys &P, const BandGeom &B, int nsub, const SubInfo *subs, const double *J, double shift,
                    const unsigned *mask, void *band, hipStream_t s) {
  FT *bd = (FT *)band;
  const long total = (long)nsub * B.box_elems;
  int blocks = (int)std::min<long>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(k_band_zero<FT>, dim3(blocks), dim3(256), 0, s, bd, total);
  hipLaunchKernelGGL(k_band_extract2d<FT>, dim3(nsub), dim3(256), 0, s, P, B, subs, J, shift, bd);
  if (mask) {
    switch (B.nr) {
#define ACCH_FACTOR(NR) \
  case NR: hipLaunchKernelGGL((k_band_factor2d<FT, NR, true>), dim3(nsub), dim3(256), 0, s, B, bd, mask); break;
      ACCH_FACTOR(4) ACCH_FACTOR(5) ACCH_FACTOR(6) ACCH_FACTOR(7) ACCH_FACTOR(8) ACCH_FACTOR(9) ACCH_FACTOR(10)
      ACCH_FACTOR(11) ACCH_FACTOR(12) ACCH_FACTOR(13) ACCH_FACTOR(14)
#undef ACCH_FACTOR
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (B.nr) {
#define ACCH_FACTOR(NR) \
  case NR: hipLaunchKernelGGL((k_band_factor2d<FT, NR, false>), dim3(nsub), dim3(256), 0, s, B, bd, nullptr); break;
      ACCH_FACTOR(4) ACCH_FACTOR(5) ACCH_FACTOR(6) ACCH_FACTOR(7) ACCH_FACTOR(8) ACCH_FACTOR(9) ACCH_FACTOR(10)
      ACCH_FACTOR(11) ACCH_FACTOR(12) ACCH_FACTOR(13) ACCH_FACTOR(14)
#undef ACCH_FACTOR
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

template <typename FT>
hipError_t solve_t(int per, const Phys &P, const BandGeom &B, const BoxGeom &G, const SubInfo *subs, const void *band,
                   double *ybox, void *boxbuf, const double *r, double *z, const GmresState *st, long vstride,
                   int kind, hipStream_t s) {
  const FT *bd = (const FT *)band;
  const dim3 grid(G.nsub), block(64 * kSolveWaves);
  if (per <= 4)
    hipLaunchKernelGGL((k_band_solve2d<FT, 4>), grid, block, 0, s, P, B, G, subs, bd, ybox, boxbuf, r, z, st, vstride, kind);
  else if (per <= 8)
    hipLaunchKernelGGL((k_band_solve2d<FT, 8>), grid, block, 0, s, P, B, G, subs, bd, ybox, boxbuf, r, z, st, vstride, kind);
  else if (per <= 12)
    hipLaunchKernelGGL((k_band_solve2d<FT, 12>), grid, block, 0, s, P, B, G, subs, bd, ybox, boxbuf, r, z, st, vstride, kind);
  else if (per <= 16)
    hipLaunchKernelGGL((k_band_solve2d<FT, 16>), grid, block, 0, s, P, B, G, subs, bd, ybox, boxbuf, r, z, st, vstride, kind);
  else if (per <= 20)
    hipLaunchKernelGGL((k_band_solve2d<FT, 20>), grid, block, 0, s, P, B, G, subs, bd, ybox, boxbuf, r, z, st, vstride, kind);
  else if (per <= 24)
    hipLaunchKernelGGL((k_band_solve2d<FT, 24>), grid, block, 0, s, P, B, G, subs, bd, ybox, boxbuf, r, z, st, vstride, kind);
  else if (per <= 28)
    hipLaunchKernelGGL((k_band_solve2d<FT, 28>), grid, block, 0, s, P, B, G, subs, bd, ybox, boxbuf, r, z, st, vstride, kind);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace

hipError_t launch_band_factor2d(const BatchLaunch &bl, const BandGeom &B, int nsub, const SubInfo *subs,
                                const double *J, double shift, const unsigned *mask, void *band, int fp32,
                                hipStream_t s) {
  if (bl.bt.map[kFamSub] != nullptr || B.nr == 0 || B.kl + 64 > kRing) return hipErrorInvalidValue;
  return fp32 ? factor_t<float>(bl.P0, B, nsub, subs, J, shift, mask, band, s)
              : factor_t<double>(bl.P0, B, nsub, subs, J, shift, mask, band, s);
}

hipError_t launch_band_apply2d(const BatchLaunch &bl, const BandGeom &B, const BoxGeom &G, const SubInfo *subs,
                               const void *band, double *ybox, void *boxbuf, const double *r, double *z,
                               const GmresState *st, long vstride, int fp32, hipStream_t s, const RasVariant &rv) {
  if (bl.bt.map[kFamSub] != nullptr) return hipErrorInvalidValue;
  if (rv.kind != ACCH_RAS_LEFT && !rv.own_x) return hipErrorInvalidValue;
  const int per = (B.kl + kSolveWaves - 1) / kSolveWaves;
  hipError_t e = fp32 ? solve_t<float>(per, bl.P0, B, G, subs, band, ybox, boxbuf, r, z, st, vstride, rv.kind, s)
                      : solve_t<double>(per, bl.P0, B, G, subs, band, ybox, boxbuf, r, z, st, vstride, rv.kind, s);
  if (e != hipSuccess) return e;
  e = hipGetLastError();
  if (e != hipSuccess || rv.kind == ACCH_RAS_LEFT) return e;
  return launch_ras_sum2d(bl, G, subs, boxbuf, z, st, vstride, fp32, s, rv);
}

hipError_t launch_band_export(const BandGeom &B, int nsub, const void *band, int fp32, double *out, hipStream_t s) {
  const long total = (long)nsub * B.n * B.nd;
  int blocks = (int)std::min<long>((total + 255) / 256, 4096);
  if (fp32)
    hipLaunchKernelGGL(k_band_export<float>, dim3(blocks), dim3(256), 0, s, B, nsub, (const float *)band, out);
  else
    hipLaunchKernelGGL(k_band_export<double>, dim3(blocks), dim3(256), 0, s, B, nsub, (const double *)band, out);
  return hipGetLastError();
}

}  // namespace acch
