// Exact-LU and ILU(k) subdomain solvers of the 2D Schwarz preconditioner (Section 3.1,
// the subdomain solvers compared in Table 2), in the band storage of band.h.
//
// Extraction: every box matrix A_k = R_k J R_k^T (plus sigma diag(A_k) for ILU(k)) is
// written into a zeroed band; cells of the padded box outside the grid are decoupled
// identity rows, as in the ILU(0) path.
//
// Factorisation (one workgroup of 256 threads per box): Gaussian elimination without
// pivoting in the natural order.  The active part of the band -- rows k..k+W-1 and
// columns k..k+W-1 at step k, W = 16 nr >= kl + 1 -- lives in registers: thread
// (ty, tx) of the 16 x 16 grid owns the window rows R = ty (mod 16) and columns
// C = tx (mod 16), at the circular slots R mod W and C mod W.  A step publishes the
// pivot row and column through LDS (double buffered, one barrier per step), applies
// the rank-1 update to every owned entry, stores row k of U and column k of L over the
// band, and loads row k+W and column k+W into the freed slots.  With an ILU(k) pattern
// (a bit per band entry, from the host's symbolic level-of-fill elimination) updates
// of entries outside the pattern are dropped, which is ILU(k) in IKJ form.
//
// Solve (four waves per box): forward substitution with L, then backward with U, 64 rows
// at a time.  For a chunk, the four waves split the up to kl earlier (later) rows that lie
// in finished chunks and subtract their contributions -- coalesced loads along each
// diagonal, the finished values from an LDS ring -- keeping the coefficients of the
// chunk's own columns in LDS; one wave then sums the four partial sums and finishes the
// 64 rows one after another, each broadcast from its lane.  Arithmetic is FP64; the
// factors are FP64 or FP32.
#include <algorithm>

#include "../../include/acch.h"
#include "band.h"
#include "boxes.h"
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

// Selects register row p == sel of a[NR][NR] (sel uniform over the block).
template <int NR>
ACCH_DEV void row_out(const double (&a)[NR][NR], int sel, double (&out)[NR]) {
#pragma unroll
  for (int p = 0; p < NR; ++p)
    if (p == sel) {
#pragma unroll
      for (int q = 0; q < NR; ++q) out[q] = a[p][q];
    }
}

template <typename FT, int NR>
__global__ __launch_bounds__(256) void k_band_factor2d(BandGeom B, FT *__restrict__ band,
                                                        const unsigned *__restrict__ mask) {
  constexpr int W = 16 * NR;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  FT *Bk = band + (long)blockIdx.x * B.box_elems;
  const unsigned *Mk = mask ? mask + (long)blockIdx.x * B.n * B.mwords : nullptr;
  const int n = B.n, kl = B.kl, nd = B.nd;
  __shared__ double urow[2][W], acol[2][W];

  // original entry (R, C) of A_k, zero outside the matrix or the band
  auto orig = [&](int R, int C) -> double {
    const int d = C - R + kl;
    if (R >= n || C >= n || (unsigned)d >= (unsigned)nd) return 0.0;
    return (double)Bk[band_at(B, R, d)];
  };
  // (R, C) in the ILU(k) pattern (always, for the exact LU)
  auto inpat = [&](int R, int C) -> bool {
    if (!Mk) return true;
    const int d = C - R + kl;
    if (R >= n || C >= n || (unsigned)d >= (unsigned)nd) return false;
    return (Mk[(long)R * B.mwords + (d >> 5)] >> (d & 31)) & 1u;
  };

  double a[NR][NR];
  unsigned m[NR];   // bit q: entry (row of slot p, column of slot q) may be updated
#pragma unroll
  for (int p = 0; p < NR; ++p) {
    m[p] = 0;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const int R = ty + 16 * p, C = tx + 16 * q;
      a[p][q] = orig(R, C);
      m[p] |= inpat(R, C) ? (1u << q) : 0u;
    }
  }
  // Rows and columns enter the window kPf steps after their loads are issued: the
  // thread row (column) of the slot freed at step kk is kk mod 16, so a thread has at
  // most one pending row and one pending column (kPf < 16).
  constexpr int kPf = 8;
  double prow[NR], pcol[NR];
  unsigned pmrow = 0, pmcol = 0;
  // row or column held by slot s after step kk
  auto held_after = [&](int kk, int s) {
    const int kw = kk % W;
    return s == kw ? kk + W : kk + (s > kw ? s - kw : s - kw + W);
  };
  auto issue_row = [&](int kk) {   // row kk + W at the columns this thread owns after step kk
    pmrow = 0;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const int C = held_after(kk, tx + 16 * q);
      prow[q] = orig(kk + W, C);
      pmrow |= inpat(kk + W, C) ? (1u << q) : 0u;
    }
  };
  auto issue_col = [&](int kk) {   // column kk + W at the rows this thread owns after step kk
    pmcol = 0;
#pragma unroll
    for (int p = 0; p < NR; ++p) {
      const int R = held_after(kk, ty + 16 * p);
      pcol[p] = orig(R, kk + W);
      pmcol |= inpat(R, kk + W) ? (1u << p) : 0u;
    }
  };
  if (ty < kPf) issue_row(ty);
  if (tx < kPf) issue_col(tx);
  __syncthreads();

  int ks = 0;   // window slot of the pivot row and column: k mod W
  for (int k = 0; k < n; ++k) {
    const int buf = k & 1;
    const int pr = ks >> 4, tr = ks & 15;
    if (ty == tr) {
      double row[NR];
      row_out<NR>(a, pr, row);
#pragma unroll
      for (int q = 0; q < NR; ++q) urow[buf][tx + 16 * q] = row[q];
    }
    if (tx == tr) {
#pragma unroll
      for (int p = 0; p < NR; ++p) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < NR; ++q)
          if (q == pr) v = a[p][q];
        acol[buf][ty + 16 * p] = v;
      }
    }
    // LDS only: the band stores of earlier steps and the loads of entering rows and
    // columns (kPf steps ahead) touch disjoint entries and stay in flight
    lds_barrier();
    const double inv = 1.0 / urow[buf][ks];
    double l[NR], u[NR];
#pragma unroll
    for (int p = 0; p < NR; ++p) {
      const int s = ty + 16 * p;
      l[p] = s == ks ? 0.0 : acol[buf][s] * inv;
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const int s = tx + 16 * q;
      u[q] = s == ks ? 0.0 : urow[buf][s];
    }
#pragma unroll
    for (int p = 0; p < NR; ++p)
#pragma unroll
      for (int q = 0; q < NR; ++q)
        if ((m[p] >> q) & 1u) a[p][q] -= l[p] * u[q];

    // row k of U (1/u_kk on the diagonal) and column k of L over the band
    if (ty == tr) {
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        const int s = tx + 16 * q;
        const int off = s >= ks ? s - ks : s - ks + W;   // column k + off
        if (off <= kl && k + off < n) Bk[band_at(B, k, kl + off)] = (FT)(off == 0 ? inv : urow[buf][s]);
      }
    }
    if (tx == tr) {
#pragma unroll
      for (int p = 0; p < NR; ++p) {
        const int s = ty + 16 * p;
        const int off = s >= ks ? s - ks : s - ks + W;   // row k + off
        if (off >= 1 && off <= kl && k + off < n) Bk[band_at(B, k + off, kl - off)] = (FT)l[p];
      }
    }
    // slot ks takes row k + W and column k + W (loaded kPf steps ahead); the other
    // slots keep theirs
    if (ty == tr) {
#pragma unroll
      for (int p = 0; p < NR; ++p)
        if (p == pr) {
#pragma unroll
          for (int q = 0; q < NR; ++q) a[p][q] = prow[q];
          m[p] = pmrow;
        }
    }
    if (tx == tr) {
#pragma unroll
      for (int p = 0; p < NR; ++p)
#pragma unroll
        for (int q = 0; q < NR; ++q)
          if (q == pr) {
            a[p][q] = pcol[p];
            m[p] = (m[p] & ~(1u << q)) | (((pmcol >> p) & 1u) << q);
          }
    }
    {
      const int kk = k + kPf;
      if (ty == (kk & 15)) issue_row(kk);
      if (tx == (kk & 15)) issue_col(kk);
    }
    ks = ks + 1 == W ? 0 : ks + 1;
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
constexpr int kBatch = 16;   // band coefficients loaded together by a solve sweep

// use(dp, load(dp)) for dp = lo..hi in order, the loads issued kBatch at a time with
// the next batch in flight while the current one is used (loads past hi read dp = hi)
template <typename Load, typename Use>
ACCH_DEV void sweep_batches(int lo, int hi, Load &&load, Use &&use) {
  if (lo > hi) return;
  double cur[kBatch], nxt[kBatch];
#pragma unroll
  for (int u = 0; u < kBatch; ++u) cur[u] = (double)load(min(lo + u, hi));
  for (int d0 = lo; d0 <= hi; d0 += 2 * kBatch) {
#pragma unroll
    for (int u = 0; u < kBatch; ++u) nxt[u] = (double)load(min(d0 + kBatch + u, hi));
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
      if (d0 + u <= hi) use(d0 + u, cur[u]);
#pragma unroll
    for (int u = 0; u < kBatch; ++u) cur[u] = (double)load(min(d0 + 2 * kBatch + u, hi));
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
      if (d0 + kBatch + u <= hi) use(d0 + kBatch + u, nxt[u]);
  }
}

constexpr int kSolveWaves = 4;   // waves per box: all share the finished-chunk terms

template <typename FT>
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
  __shared__ double ring[kRing];
  __shared__ double tri[64][64];
  __shared__ double psum[kSolveWaves][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const SubInfo si = subs[blockIdx.x];
  const Rect rc = inside_rect(si, B, P.nx, P.ny, P.periodic);
  const FT *Bk = band + (long)blockIdx.x * B.box_elems;
  double *yk = ybox + (long)blockIdx.x * B.nchunk * 64;
  const long n = (long)P.nx * P.ny;
  const int kl = B.kl, nd = B.nd;
  for (int e = threadIdx.x; e < kRing; e += 64 * kSolveWaves) ring[e] = 0.0;
  __syncthreads();
  // this wave's share of the diagonals 1..kl
  const int per = (kl + kSolveWaves - 1) / kSolveWaves;
  const int dlo = 1 + wave * per, dhi = min(kl, (wave + 1) * per);

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
  // Phase 1: the terms of columns in finished chunks, branch-free over four partial
  // sums; the coefficients of this chunk's own columns go to tri[s][lane] (column s of
  // the chunk, row lane).  Phase 2: the 64 rows in order, row s broadcast from its lane.
  for (int c = 0; c < B.nchunk; ++c) {
    const int R = 64 * c + lane;
    bool own;
    const long g = cell_of(R, own);
    double part[4] = {0.0, 0.0, 0.0, 0.0};
    if (wave == 0 && g >= 0 && (kind != ACCH_RAS_RIGHT || own)) part[0] = sc * r[g + (R & 1) * n];
    const FT *Lc = Bk + (long)c * nd * 64 + lane;
    sweep_batches(dlo, dhi, [&](int dp) { return Lc[(long)(kl - dp) * 64]; }, [&](int dp, double coef) {
      const bool fin = dp > lane;
      const double y = ring[(R - dp) & (kRing - 1)];
      part[dp & 3] -= (fin ? coef : 0.0) * y;
      if (!fin) tri[lane - dp][lane] = coef;
    });
    psum[wave][lane] = (part[0] + part[1]) + (part[2] + part[3]);
    lds_barrier();
    if (wave == 0) {
      double acc = psum[0][lane];
#pragma unroll
      for (int q = 1; q < kSolveWaves; ++q) acc += psum[q][lane];
#pragma unroll
      for (int s = 0; s < 63; ++s) {
        const double cs = lane > s ? tri[s][lane] : 0.0;
        acc -= cs * bcast(acc, s);
      }
      ring[R & (kRing - 1)] = acc;
      yk[R] = acc;
    }
    lds_barrier();
  }
  // ---- backward: U x = y
  FT *boxbuf = (FT *)boxbuf_;
  const long ncb = (long)G.nlev * G.bh;
  for (int c = B.nchunk - 1; c >= 0; --c) {
    const int R = 64 * c + lane;
    double part[4] = {wave == 0 ? yk[R] : 0.0, 0.0, 0.0, 0.0};
    const FT *Uc = Bk + (long)c * nd * 64 + lane;
    sweep_batches(dlo, dhi, [&](int dp) { return Uc[(long)(kl + dp) * 64]; }, [&](int dp, double coef) {
      const bool fin = dp > 63 - lane;
      const double x = ring[(R + dp) & (kRing - 1)];
      part[dp & 3] -= (fin ? coef : 0.0) * x;
      if (!fin) tri[lane + dp][lane] = coef;
    });
    psum[wave][lane] = (part[0] + part[1]) + (part[2] + part[3]);
    lds_barrier();
    if (wave == 0) {
      double acc = psum[0][lane];
#pragma unroll
      for (int q = 1; q < kSolveWaves; ++q) acc += psum[q][lane];
      const double inv = (double)Uc[(long)kl * 64];
#pragma unroll
      for (int s = 63; s >= 0; --s) {
        if (lane == s) acc *= inv;
        const double cs = lane < s ? tri[s][lane] : 0.0;
        acc -= cs * bcast(acc, s);
      }
      ring[R & (kRing - 1)] = acc;
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
  switch (B.nr) {
    case 4: hipLaunchKernelGGL((k_band_factor2d<FT, 4>), dim3(nsub), dim3(256), 0, s, B, bd, mask); break;
    case 6: hipLaunchKernelGGL((k_band_factor2d<FT, 6>), dim3(nsub), dim3(256), 0, s, B, bd, mask); break;
    case 8: hipLaunchKernelGGL((k_band_factor2d<FT, 8>), dim3(nsub), dim3(256), 0, s, B, bd, mask); break;
    case 10: hipLaunchKernelGGL((k_band_factor2d<FT, 10>), dim3(nsub), dim3(256), 0, s, B, bd, mask); break;
    case 12: hipLaunchKernelGGL((k_band_factor2d<FT, 12>), dim3(nsub), dim3(256), 0, s, B, bd, mask); break;
    case 14: hipLaunchKernelGGL((k_band_factor2d<FT, 14>), dim3(nsub), dim3(256), 0, s, B, bd, mask); break;
    default: return hipErrorInvalidValue;
  }
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
  if (fp32)
    hipLaunchKernelGGL(k_band_solve2d<float>, dim3(G.nsub), dim3(64 * kSolveWaves), 0, s, bl.P0, B, G, subs, (const float *)band,
                       ybox, boxbuf, r, z, st, vstride, rv.kind);
  else
    hipLaunchKernelGGL(k_band_solve2d<double>, dim3(G.nsub), dim3(64 * kSolveWaves), 0, s, bl.P0, B, G, subs,
                       (const double *)band, ybox, boxbuf, r, z, st, vstride, rv.kind);
  hipError_t e = hipGetLastError();
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
