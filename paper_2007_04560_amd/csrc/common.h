// Shared definitions of the acch HIP library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace acch {

constexpr int kMaxRestart = 30;     // GMRES(m) with m <= 30 (device Hessenberg storage)
constexpr int kMaxS = 64;           // series order limit of Lemma 2.2's truncation
constexpr int kRedBlocks = 512;     // grid size of the vector reduction kernels
constexpr int kNSlot2D = 24;        // Jacobian / factor slots per cell in 2D

// Physical and mesh parameters seen by the stencil kernels.
struct Phys {
  int nx, ny;
  int periodic;
  double wx, wy;          // 1/hx^2, 1/hy^2
  double alpha, beta, theta, gamma, rho;
  int S;
  int mob;                // 0 midpoint, 1 average, 2 explicit
  int nz;                 // 1 in 2D
  double wz;              // 1/hz^2 (3D)
};

// Scratch of the two-kernel reductions: per-block partial sums and final values.
struct RedBuf {
  double *partials;       // [nv][gridblocks]
  unsigned *counter;      // unused (kept zero)
  double *out;            // [nv] final sums
};

// Geometry of the padded subdomain boxes Omega_k^delta (all boxes share bw x bh).
// Per-box factor and scratch storage is wavefront-major: cell (i, j) lives at slot
// (i + 2j) * bh + j of nlev * bh slots, so a wavefront's cells are contiguous.
struct BoxGeom {
  int bw, bh;             // padded box width/height (cells)
  int bd;                 // padded box depth (1 in 2D)
  int nlev;               // levels of the i + 2j wavefront: bw + 2(bh-1)
  int ncb;                // bw * bh (cells of a box; storage is padded to nlev * bh slots)
  int nsub;
  int wmax;               // 3D: most cells on one level
};

// One subdomain: unwrapped box origin, its real extent inside the padded box and
// the owned rectangle Omega_k in box coordinates.
struct SubInfo {
  int ox, oy;             // global coordinates of box cell (0,0), may be negative
  int ex, ey;             // real box extent (<= bw, bh); cells beyond are padding
  int own_x0, own_x1, own_y0, own_y1;
  int oz, ez, own_z0, own_z1;   // third direction (0, 1, 0, 1 in 2D)
};

// Device-resident state of one restarted GMRES cycle (flexible, right preconditioned).
struct GmresState {
  double H[(kMaxRestart + 1) * kMaxRestart];   // column-major Hessenberg, after rotations
  double cs[kMaxRestart], sn[kMaxRestart];
  double g[kMaxRestart + 1];
  double y[kMaxRestart];
  double hcol[kMaxRestart + 1];                // dots of the current Arnoldi step
  double inv_norm[kMaxRestart + 1];            // V_i is stored unnormalised: v_i = inv_norm[i] * W_i
  double beta;            // ||r_0|| of the cycle
  double tol;             // absolute stopping tolerance
  double resid;           // current residual estimate |g[j]|
  double shift;           // mean of the u part of the final direction (mass projection)
  int j;                  // Arnoldi steps done in this cycle
  int m;                  // restart length
  int done;               // cycle finished (converged, breakdown or j == m)
  int converged;
  int total_its;
  int first;              // the next cycle is the first of a solve (fixes tol)
  int applied;            // this cycle's update has been added to S
  int pad;
};

// ---- batches of independent instances ---------------------------------------
// Kernels are launched over "families" of blocks; in a batch every block belongs to
// one instance, found through a per-family map (global block -> instance, local
// block).  A null map means a single instance whose blocks are the whole grid.
enum { kFamTile = 0, kFamCell = 1, kFamElem = 2, kFamSub = 3, kFamilies = 4 };

struct Inst {
  Phys P;
  long xoff;              // first element of the instance in a batched state vector (2 n)
  long joff;              // first element of its Jacobian block (24 n)
  int blk0[kFamilies];    // first global block of each family
  int nblk[kFamilies];    // blocks of each family
};

struct Batch {
  const Inst *inst;
  const int2 *map[kFamilies];
  const int *active;      // per-instance mask (null: all active)
};

// Small pinned-host mirror of the values the host control flow reads.
struct HostMirror {
  double vals[8];
  int ivals[8];
};

#define ACCH_DEV __device__ __forceinline__

constexpr int pow2_at_least(int v) { return v <= 1 ? 1 : 2 * pow2_at_least((v + 1) / 2); }

// Periodic wrap, or clamping (the Neumann ghost copies the boundary cell, which
// makes every boundary difference vanish, as in Section 2).  Offsets are within
// +-2 of the domain and periodic grids have at least 5 cells.
ACCH_DEV int wrap_index(int g, int n, int periodic) {
  if (periodic) return g < 0 ? g + n : (g >= n ? g - n : g);
  return g < 0 ? 0 : (g >= n ? n - 1 : g);
}

ACCH_DEV bool face_exists(int g, int dir, int n, int periodic) {
  return periodic || (dir < 0 ? g > 0 : g < n - 1);
}

// ---------------------------------------------------------------------------
// Reductions: wave64 shuffles, then LDS across waves, then a last-block pass.
// ---------------------------------------------------------------------------

ACCH_DEV double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sums NV values over the block; the result is valid in thread 0.  nthreads must
// be a multiple of 64 and at most 1024.
template <int NV>
ACCH_DEV void block_sum(double (&v)[NV], int tid, int nthreads) {
  __shared__ double s_red[NV][16];
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  const int lane = tid & 63, wid = tid >> 6;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) s_red[k][wid] = v[k];
  }
  __syncthreads();
  if (tid == 0) {
    const int nw = nthreads >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double a = 0.0;
      for (int w = 0; w < nw; ++w) a += s_red[k][w];
      v[k] = a;
    }
  }
}

// Many sums at once (NV a power of two): each butterfly step halves the number of
// values a lane carries and trades the other half with its partner, so NV values
// need about NV shuffles instead of 6 NV.  On return lane l holds the wave total of
// value l / (64 / NV).
template <int C, int O, int NV>
ACCH_DEV void multi_step(double (&v)[NV], int lane) {
  if constexpr (C >= 1) {
    const bool up = (lane & O) != 0;
#pragma unroll
    for (int k = 0; k < C; ++k) {
      const double send = up ? v[k] : v[k + C];
      const double keep = up ? v[k + C] : v[k];
      v[k] = keep + __shfl_xor(send, O, 64);
    }
    multi_step<C / 2, O / 2, NV>(v, lane);
  }
}

template <int NV>
ACCH_DEV double wave_multi_sum(double (&v)[NV], int lane) {
  static_assert(NV >= 1 && NV <= 64 && (NV & (NV - 1)) == 0, "NV must be a power of two <= 64");
  multi_step<NV / 2, 32, NV>(v, lane);
  double r = v[0];
#pragma unroll
  for (int o = 32 / NV; o > 0; o >>= 1) r += __shfl_xor(r, o, 64);
  return r;
}

// Block totals of the first nv_used of NV values, written by threads 0..nv_used-1.
template <int NV>
ACCH_DEV void block_multi_sum(double (&v)[NV], int tid, int nthreads, int nv_used, double *s_out) {
  __shared__ double s_red[16][NV];
  constexpr int R = 64 / NV;
  const int lane = tid & 63, wid = tid >> 6;
  const double r = wave_multi_sum<NV>(v, lane);
  if (lane % R == 0) s_red[wid][lane / R] = r;
  __syncthreads();
  if (tid < nv_used) {
    double a = 0.0;
    for (int w = 0; w < (nthreads >> 6); ++w) a += s_red[w][tid];
    *s_out = a;
  }
}

// Two-kernel grid reductions.  A reduction kernel stores one partial sum per block
// (block_partial); a one-block finalize kernel adds the partials in block order
// (final_sum), which makes the result independent of scheduling.  The kernel
// boundary orders the two: no device-scope fence (on this GPU a full L2 write-back
// per block) is needed.
template <int NV>
ACCH_DEV void block_partial(double (&v)[NV], double *partials, int tid, int nthreads, int bid, int nblocks,
                            int nv_used = NV) {
  block_sum<NV>(v, tid, nthreads);
  if (tid == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k)
      if (k < nv_used) partials[k * nblocks + bid] = v[k];
  }
}

// block_partial for many values (NV a power of two, see wave_multi_sum).
template <int NV>
ACCH_DEV void block_partial_multi(double (&v)[NV], double *partials, int tid, int nthreads, int bid, int nblocks,
                                  int nv_used) {
  double a;
  block_multi_sum<NV>(v, tid, nthreads, nv_used, &a);
  if (tid < nv_used) partials[tid * nblocks + bid] = a;
}

// Sum of the partials of blocks [b0, b0 + nb) of the first nv_used values, the
// partials of value k being stored at k * stride + block; valid in thread 0.
template <int NV>
ACCH_DEV void final_sum(const double *partials, int stride, int b0, int nb, int tid, int nthreads,
                        double (&acc)[NV], int nv_used = NV) {
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double a = 0.0;
    if (k < nv_used)
      for (int b = tid; b < nb; b += nthreads) a += partials[(long)k * stride + b0 + b];
    acc[k] = a;
  }
  block_sum<NV>(acc, tid, nthreads);
}

// Where a block of a (possibly batched) launch works.
struct Loc {
  int b;      // instance
  int lb;     // block index within the instance
  int nb;     // blocks of the instance
  bool on;    // instance active
};

ACCH_DEV Loc locate(const Batch &bt, int fam) {
  Loc L;
  if (bt.map[fam] == nullptr) {
    L.b = 0;
    L.lb = blockIdx.x;
    L.nb = gridDim.x;
    L.on = true;
    return L;
  }
  const int2 m = bt.map[fam][blockIdx.x];
  L.b = m.x;
  L.lb = m.y;
  L.nb = bt.inst[m.x].nblk[fam];
  L.on = bt.active == nullptr || bt.active[m.x] != 0;
  return L;
}

}  // namespace acch
