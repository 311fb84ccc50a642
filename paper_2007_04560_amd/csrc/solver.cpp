// Host driver of the acch library: parameter validation, subdomain maps, workspace
// layout, and the control flow of one time step (Sections 3.1 and 3.2): inexact
// Newton with a backtracking line search, restarted flexible GMRES preconditioned
// by restricted additive Schwarz with subdomain ILU(0) (factored once per step
// attempt), and the adaptive time step with sqrt(2) retries and eta doubling.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cstring>
#include <functional>
#include <new>
#include <string>
#include <vector>

#include "../../include/acch.h"
#include "driver.h"
#include "kernels.h"
#include "stencil3d.h"

using namespace acch;

namespace acch {
thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}
}  // namespace acch

namespace {

struct Layout {
  size_t off_Xn, off_Xprev, off_X, off_Xt, off_F, off_Ft, off_S, off_W;
  size_t off_J, off_V, off_Z, off_fac, off_wfac, off_wfact, off_q3, off_y, off_dump, off_subs, off_lvl, off_state, off_part, off_cnt, off_out;
  size_t off_tbox, off_own;
  size_t off_band, off_bandy, off_mask;   // exact-LU / ILU(k) subdomain solvers (2D)
  size_t off_bxL, off_bxU, off_bxy, off_lvoff, off_cellof;   // box-pattern ILU(0) (2D)
  size_t off_bxTf, off_bxTb;                                  // its transposed records (adjoint)
  size_t total;
};

// Optional per-kernel-class timing with HIP events recorded on the context's stream
// around each launch; harvested whenever the host synchronises anyway.
struct KernelTimer {
  static constexpr int kPool = 2048;
  static constexpr int kSample = 16;   // sampled mode: one Schwarz launch in kSample
  bool on = false;
  bool sampled = false;
  long seen = 0;
  std::vector<hipEvent_t> ev;  // pairs (start, stop)
  std::vector<int> kind;
  int used = 0;
  double total_ms[ACCH_KERNEL_KINDS] = {};
  long count[ACCH_KERNEL_KINDS] = {};
};

}  // namespace

struct acch_ctx {
  acch_params p{};
  Phys P{};
  Geometry geo;
  Layout lay{};
  hipStream_t stream = nullptr;
  char *ws = nullptr;
  double *Xn, *Xprev, *X, *Xt, *F, *Ft, *S, *W, *J, *V, *Z;
  void *fac, *wfac, *ybuf;   // wfac: level-major factor copy of the 3D windowed apply (or null)
  double *q3;                // 3D: cell quantities of the residual / Jacobian passes
  void *wfact = nullptr;     // transposed records for M^{-T} (3D: level-major, windowed form)
  bool tpacked = false;      // wfact holds the current factorisation
  double *dump, *tbox;
  SubInfo *d_subs;
  int *d_lvl, *d_own;
  GmresState *st;
  RedBuf red{};
  HostMirror *host = nullptr;  // pinned
  char *host_state = nullptr;  // pinned, holds the tail of GmresState
  double hvol = 1.0;           // cell volume
  double t = 0.0, dt_prev = 0.0, eta = 0.0;
  bool have_history = false;
  bool factored = false;
  int its_guess = 4;
  long launches = 0, syncs = 0;
  KernelTimer timer;
  BatchLaunch bl{};   // single-instance launch shapes
  RasVariant ras{};   // Schwarz variant and owner maps
  bool d3 = false;    // 3D grid
  bool band = false;  // exact-LU / ILU(k) subdomain solver (band storage)
  BandGeom bg{};
  void *bandf = nullptr;        // band factors
  double *bandy = nullptr;      // forward-sweep values of the band solve
  unsigned *bandmask = nullptr; // ILU(k) pattern bits (null: exact LU)
  bool boxilu = false;          // ILU(0) on the box pattern (its own kernels)
  BoxIluGeom bx{};
  std::vector<int> lvoff_h;     // wavefront offsets of the box records
  std::vector<int> cellof_h;    // box cell of each record position
  void *bxL = nullptr, *bxU = nullptr;
  void *bxTf = nullptr, *bxTb = nullptr;   // transposed records, packed on the first transposed apply
  double *bxy = nullptr;        // forward-sweep values, (u, v) per box cell
  int *d_lvoff = nullptr;
  int *d_cellof = nullptr;
};

// ---------------------------------------------------------------------------
// parameters, geometry, workspace
// ---------------------------------------------------------------------------
extern "C" void acch_params_default(acch_params *p) {
  if (!p) return;
  if (p->dim == 0) p->dim = 2;
  for (int d = 0; d < 3; ++d)
    if (p->L[d] == 0.0) p->L[d] = 1.0;
  if (p->S == 0) p->S = 10;
  if (p->newton_rtol == 0.0) p->newton_rtol = 1e-8;
  if (p->newton_atol == 0.0) p->newton_atol = 1e-13;
  if (p->newton_max_it == 0) p->newton_max_it = 50;
  if (p->gmres_rtol == 0.0) p->gmres_rtol = 1e-8;
  if (p->gmres_atol == 0.0) p->gmres_atol = 1e-14;
  if (p->gmres_restart == 0) p->gmres_restart = 30;
  if (p->gmres_max_restarts == 0) p->gmres_max_restarts = 10;
  for (int d = 0; d < 3; ++d)
    if (p->sub[d] == 0) p->sub[d] = 1;
  // switches: 0 (a zero-filled struct) means the documented default, on
  if (p->ilu_reuse == 0) p->ilu_reuse = ACCH_ON;
  if (p->mass_projection == 0) p->mass_projection = ACCH_ON;
  if (p->log_energy == 0) p->log_energy = ACCH_ON;
}

// ILU(0) on the box pattern: its own kernels (boxilu2d.hip); levels >= 1 use the band.
static bool box_ilu0(const acch_params &p) { return p.subsolver == ACCH_SUB_ILUK_BOX && p.fill_level == 0; }
// Subdomain solvers in band storage, and those whose band factorisation keeps a pattern.
static bool band_sub(const acch_params &p) { return p.subsolver != ACCH_SUB_ILU0 && !box_ilu0(p); }
static bool masked_sub(const acch_params &p) {
  return band_sub(p) && (p.subsolver == ACCH_SUB_ILUK || p.subsolver == ACCH_SUB_ILUK_BOX);
}

int acch::validate_params(const acch_params &p) {
  if (p.dim != 2 && p.dim != 3) return fail(ACCH_EUNSUPPORTED, "dim must be 2 or 3");
  const int nd = p.dim;
  for (int d = 0; d < nd; ++d)
    if (p.n[d] < 2) return fail(ACCH_EINVAL, "need at least 2 cells per direction");
  if (p.bc != ACCH_BC_PERIODIC && p.bc != ACCH_BC_NEUMANN) return fail(ACCH_EINVAL, "bc");
  for (int d = 0; d < nd; ++d)
    if (p.bc == ACCH_BC_PERIODIC && p.n[d] < 5)
      return fail(ACCH_EINVAL, "periodic grids need at least 5 cells per direction");
  if (!(p.alpha > 0 && p.beta > 0 && p.theta > 0 && p.gamma > 0 && p.rho > 0))
    return fail(ACCH_EINVAL, "alpha, beta, theta, gamma, rho must be positive");
  if (p.S < 1 || p.S > kMaxS) return fail(ACCH_EINVAL, "S out of range");
  if (p.gmres_restart < 1 || p.gmres_restart > kMaxRestart) return fail(ACCH_EINVAL, "gmres_restart must be 1..30");
  if (p.ras_type != ACCH_RAS_LEFT && p.ras_type != ACCH_RAS_RIGHT && p.ras_type != ACCH_AS_CLASSICAL)
    return fail(ACCH_EINVAL, "ras_type");
  if (p.precision != ACCH_PREC_FP64 && p.precision != ACCH_PREC_MIXED) return fail(ACCH_EINVAL, "precision");
  if (p.mobility_mode < 0 || p.mobility_mode > 2) return fail(ACCH_EINVAL, "mobility_mode");
  if (p.overlap < 0) return fail(ACCH_EINVAL, "overlap");
  if (!(p.ilu_shift >= 0.0 && p.ilu_shift < 10.0)) return fail(ACCH_EINVAL, "ilu_shift must be in [0, 10)");
  if (p.subsolver != ACCH_SUB_ILU0 && p.subsolver != ACCH_SUB_ILUK && p.subsolver != ACCH_SUB_LU &&
      p.subsolver != ACCH_SUB_ILUK_BOX)
    return fail(ACCH_EINVAL, "subsolver");
  if (p.subsolver == ACCH_SUB_ILUK && (p.fill_level < 1 || p.fill_level > 8))
    return fail(ACCH_EINVAL, "fill_level must be 1..8 for ILU(k)");
  if (p.subsolver == ACCH_SUB_ILUK_BOX && (p.fill_level < 0 || p.fill_level > 8))
    return fail(ACCH_EINVAL, "fill_level must be 0..8 for box ILU(k)");
  if (box_ilu0(p)) {
    if (nd != 2) return fail(ACCH_EUNSUPPORTED, "the box-pattern subdomain ILU(0) is 2D");
    const int bw = (p.n[0] + p.sub[0] - 1) / p.sub[0] + 2 * p.overlap;
    const int bh = (p.n[1] + p.sub[1] - 1) / p.sub[1] + 2 * p.overlap;
    if (!boxilu_fits(make_boxilu_geom(bw, bh, nullptr)))
      return fail(ACCH_EUNSUPPORTED, "box-pattern ILU(0) subdomain boxes must be at most " +
                                         std::to_string(kBoxIluMaxW) + " x " + std::to_string(kBoxIluMaxH) +
                                         " cells (owned size + 2 overlap)");
  } else if (p.subsolver != ACCH_SUB_ILU0) {
    if (nd != 2) return fail(ACCH_EUNSUPPORTED, "ILU(k) and exact-LU subdomain solvers are 2D");
    const bool box = p.subsolver == ACCH_SUB_ILUK_BOX;
    const int maxw = box ? kBandMaxWidthBox : kBandMaxWidth;
    const int bw = (p.n[0] + p.sub[0] - 1) / p.sub[0] + 2 * p.overlap;
    if (bw > maxw)
      return fail(ACCH_EUNSUPPORTED, "ILU(k) / exact-LU subdomain boxes must be at most " + std::to_string(maxw) +
                                         " cells wide (owned width + 2 overlap)");
    // one box's band is addressed with 31-bit byte offsets
    const int bh = (p.n[1] + p.sub[1] - 1) / p.sub[1] + 2 * p.overlap;
    const BandGeom bg = make_band_geom(bw, bh, box);
    if ((double)bg.box_elems * (p.precision == ACCH_PREC_MIXED ? 4.0 : 8.0) >= 2147483648.0)
      return fail(ACCH_EUNSUPPORTED, "ILU(k) / exact-LU subdomain box too large (its band must stay below 2 GiB)");
  }
  if (p.adaptive) {
    if (!(p.dt_min > 0 && p.dt_max >= p.dt_min && p.eta0 > 0)) return fail(ACCH_EINVAL, "dt_min, dt_max, eta0");
  } else if (!(p.dt_fixed > 0)) {
    return fail(ACCH_EINVAL, "dt_fixed");
  }
  for (int d = 0; d < nd; ++d) {
    if (p.sub[d] < 1 || p.sub[d] > p.n[d]) return fail(ACCH_EINVAL, "sub");
    if (p.bc == ACCH_BC_PERIODIC) {
      if (p.sub[d] < 2) return fail(ACCH_EINVAL, "periodic directions need at least 2 subdomains");
      const int longest = (p.n[d] + p.sub[d] - 1) / p.sub[d] + 2 * p.overlap;
      if (longest > p.n[d] - 2) return fail(ACCH_EINVAL, "overlapping box would touch itself across the periodic wrap");
    }
  }
  return ACCH_OK;
}

// 3D: boxes in x, y, z; levels w = i + 2j + 3k listed cell by cell.
static int build_geometry3(const acch_params &p, Geometry &geo) {
  const int nx = p.n[0], ny = p.n[1], nz = p.n[2], d = p.overlap;
  geo.ncell = (long)nx * ny * nz;
  std::vector<int> s3[3], l3[3];
  for (int a = 0; a < 3; ++a) split(p.n[a], p.sub[a], s3[a], l3[a]);
  int b3[3] = {0, 0, 0};
  for (int a = 0; a < 3; ++a)
    for (int v : l3[a]) b3[a] = std::max(b3[a], v + 2 * d);
  if (std::max(b3[0], std::max(b3[1], b3[2])) > 1023) return fail(ACCH_EINVAL, "subdomain box longer than 1023 cells");
  BoxGeom &G = geo.G;
  G.bw = b3[0];
  G.bh = b3[1];
  G.bd = b3[2];
  G.nlev = (G.bw - 1) + 2 * (G.bh - 1) + 3 * (G.bd - 1) + 1;
  G.ncb = G.bw * G.bh * G.bd;
  G.nsub = p.sub[0] * p.sub[1] * p.sub[2];
  geo.subs.clear();
  for (int bz = 0; bz < p.sub[2]; ++bz)
    for (int by = 0; by < p.sub[1]; ++by)
      for (int bx = 0; bx < p.sub[0]; ++bx) {
        SubInfo s{};
        s.ox = s3[0][bx] - d;
        s.oy = s3[1][by] - d;
        s.oz = s3[2][bz] - d;
        s.ex = l3[0][bx] + 2 * d;
        s.ey = l3[1][by] + 2 * d;
        s.ez = l3[2][bz] + 2 * d;
        s.own_x0 = s.own_y0 = s.own_z0 = d;
        s.own_x1 = d + l3[0][bx];
        s.own_y1 = d + l3[1][by];
        s.own_z1 = d + l3[2][bz];
        geo.subs.push_back(s);
      }
  geo.own.assign(nx + ny + nz, 0);
  int base = 0;
  geo.min_part = 1 << 30;
  for (int a = 0; a < 3; ++a) {
    for (int k = 0; k < p.sub[a]; ++k) {
      for (int x = s3[a][k]; x < s3[a][k] + l3[a][k]; ++x) geo.own[base + x] = k;
      geo.min_part = std::min(geo.min_part, l3[a][k]);
    }
    base += p.n[a];
  }
  // cells of the padded box grouped by level w = i + 2j + 3k, as i | j << 10 | k << 20
  geo.lvl.assign(G.nlev + 1, 0);
  geo.cells.assign(G.ncb, 0);
  std::vector<int> count(G.nlev, 0);
  for (int k = 0; k < G.bd; ++k)
    for (int j = 0; j < G.bh; ++j)
      for (int i = 0; i < G.bw; ++i) count[i + 2 * j + 3 * k]++;
  for (int w = 0; w < G.nlev; ++w) geo.lvl[w + 1] = geo.lvl[w] + count[w];
  std::vector<int> fill(geo.lvl.begin(), geo.lvl.end() - 1);
  for (int k = 0; k < G.bd; ++k)
    for (int j = 0; j < G.bh; ++j)
      for (int i = 0; i < G.bw; ++i) geo.cells[fill[i + 2 * j + 3 * k]++] = i | j << 10 | k << 20;
  // Columns (j, k) of the box for the windowed apply: column (j, k) holds the cell of
  // level w at i = w - (2j + 3k), so it is busy on bw consecutive levels.  Columns in
  // order of their first level go to the thread that became free first (equal
  // lengths: a queue), which needs as many threads as the largest level.
  {
    std::vector<std::pair<int, int>> col;   // (first level, packed j | k << 10)
    for (int k = 0; k < G.bd; ++k)
      for (int j = 0; j < G.bh; ++j) col.push_back({2 * j + 3 * k, j | k << 10});
    std::stable_sort(col.begin(), col.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
    std::vector<std::vector<int>> per;   // columns of each thread
    std::vector<int> free_at;            // level from which a thread is free
    size_t head = 0;                     // queue of threads in order of free_at
    std::vector<int> queue;
    for (const auto &c : col) {
      int t;
      if (head < queue.size() && free_at[queue[head]] <= c.first) {
        t = queue[head++];
      } else {
        t = (int)per.size();
        per.emplace_back();
        free_at.push_back(0);
      }
      per[t].push_back(c.second);
      free_at[t] = c.first + G.bw;
      queue.push_back(t);
    }
    bool fits = (int)per.size() <= kWin3DThreads;
    for (const auto &v : per) fits = fits && (int)v.size() <= kWin3DCols;
    if (fits) {
      G.wmax = (int)per.size();
      const size_t base = geo.cells.size();
      // each thread's columns in order (forward sweep), then in reverse (backward)
      geo.cells.resize(base + (size_t)2 * kWin3DCols * kWin3DThreads, -1);
      for (size_t t = 0; t < per.size(); ++t)
        for (size_t m = 0; m < per[t].size(); ++m) {
          geo.cells[base + m * kWin3DThreads + t] = per[t][m];
          geo.cells[base + (kWin3DCols + m) * kWin3DThreads + t] = per[t][per[t].size() - 1 - m];
        }
      // then the thread owning each column (j, k), at j + bh k
      std::vector<int> owner((size_t)G.bh * G.bd, -1);
      for (size_t t = 0; t < per.size(); ++t)
        for (int c : per[t]) owner[(size_t)(c & 1023) + (size_t)G.bh * (c >> 10)] = (int)t;
      geo.cells.insert(geo.cells.end(), owner.begin(), owner.end());
    } else {
      G.wmax = 0;
    }
  }
  geo.tile_blocks = 0;
  return ACCH_OK;
}

Phys acch::phys_of(const acch_params &p) {
  Phys P{};
  P.nx = p.n[0];
  P.ny = p.n[1];
  P.nz = p.dim == 3 ? p.n[2] : 1;
  P.periodic = p.bc == ACCH_BC_PERIODIC;
  const double hx = p.L[0] / p.n[0], hy = p.L[1] / p.n[1];
  const double hz = p.dim == 3 ? p.L[2] / p.n[2] : 1.0;
  P.wx = 1.0 / (hx * hx);
  P.wy = 1.0 / (hy * hy);
  P.wz = p.dim == 3 ? 1.0 / (hz * hz) : 0.0;
  P.alpha = p.alpha;
  P.beta = p.beta;
  P.theta = p.theta;
  P.gamma = p.gamma;
  P.rho = p.rho;
  P.S = p.S;
  P.mob = p.mobility_mode;
  return P;
}

int acch::build_geometry(const acch_params &p, Geometry &geo) {
  if (p.dim == 3) return build_geometry3(p, geo);
  const int nx = p.n[0], ny = p.n[1], d = p.overlap;
  geo.ncell = (long)nx * ny;
  std::vector<int> sx, lx, sy, ly;
  split(nx, p.sub[0], sx, lx);
  split(ny, p.sub[1], sy, ly);
  int bw = 0, bh = 0;
  for (int v : lx) bw = std::max(bw, v + 2 * d);
  for (int v : ly) bh = std::max(bh, v + 2 * d);
  geo.G.bw = bw;
  geo.G.bh = bh;
  geo.G.bd = 1;
  geo.G.nlev = bw + 2 * (bh - 1);
  geo.G.ncb = bw * bh;
  geo.G.nsub = p.sub[0] * p.sub[1];
  if (schwarz_waves(geo.G) == 0) return fail(ACCH_EINVAL, "subdomain box too large (at most 511 cells wide, 512 tall)");
  geo.subs.clear();
  for (int by = 0; by < p.sub[1]; ++by)
    for (int bx = 0; bx < p.sub[0]; ++bx) {
      SubInfo s{};
      s.ox = sx[bx] - d;
      s.oy = sy[by] - d;
      s.ex = lx[bx] + 2 * d;
      s.ey = ly[by] + 2 * d;
      s.own_x0 = d;
      s.own_x1 = d + lx[bx];
      s.own_y0 = d;
      s.own_y1 = d + ly[by];
      s.oz = 0;
      s.ez = 1;
      s.own_z0 = 0;
      s.own_z1 = 1;
      geo.subs.push_back(s);
    }
  geo.own.assign(nx + ny, 0);
  for (int k = 0; k < p.sub[0]; ++k)
    for (int x = sx[k]; x < sx[k] + lx[k]; ++x) geo.own[x] = k;
  for (int k = 0; k < p.sub[1]; ++k)
    for (int y = sy[k]; y < sy[k] + ly[k]; ++y) geo.own[nx + y] = k;
  geo.min_part = std::min(*std::min_element(lx.begin(), lx.end()), *std::min_element(ly.begin(), ly.end()));
  // wavefront w = i + 2j holds rows j in [lo(w), hi(w)]
  geo.lvl.assign(geo.G.nlev + 1, 0);
  for (int w = 0; w < geo.G.nlev; ++w) {
    const int lo = std::max(0, (w - bw + 2) >> 1);
    const int hi = std::min(bh - 1, w >> 1);
    geo.lvl[w + 1] = geo.lvl[w] + std::max(0, hi - lo + 1);
  }
  if (geo.lvl[geo.G.nlev] != geo.G.ncb) return fail(ACCH_EINVAL, "internal: wavefront table");
  geo.tile_blocks = ((nx + 31) / 32) * ((ny + 7) / 8);
  return ACCH_OK;
}

static void make_layout(const acch_params &p, const Geometry &geo, Layout &L) {
  const size_t n2 = 2 * (size_t)geo.ncell * sizeof(double);
  const int m = p.gmres_restart;
  const size_t fsz = p.precision == ACCH_PREC_MIXED ? sizeof(float) : sizeof(double);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L.off_Xn = take(n2);
  L.off_Xprev = take(n2);
  L.off_X = take(n2);
  L.off_Xt = take(n2);
  L.off_F = take(n2);
  L.off_Ft = take(n2);
  L.off_S = take(n2);
  L.off_W = take(n2);
  const bool d3 = p.dim == 3;
  const bool band = p.subsolver != ACCH_SUB_ILU0;   // neither path keeps 24-slot factors
  const int nslot = d3 ? kNSlot3D : kNSlot2D;
  L.off_J = take((size_t)nslot * geo.ncell * sizeof(double));
  L.off_V = take((size_t)(m + 1) * n2);
  L.off_Z = take((size_t)m * n2);
  // 2D: padded wavefront-major cells per box; 3D: box cells
  const size_t slots = d3 ? (size_t)geo.G.ncb : (size_t)geo.G.nlev * geo.G.bh;
  L.off_fac = take(band ? 0 : (size_t)geo.G.nsub * nslot * slots * fsz);
  // 2D: FT pairs + one dump slot per box; 3D: FP64 pairs
  // (3D: one more pair, where the windowed apply's idle threads write)
  L.off_y = d3 ? take((box3_ypairs(geo.G) + 1) * 2 * sizeof(double))
               : take((size_t)geo.G.nsub * 2 * (slots + 1) * fsz);
  L.off_wfac = take(d3 ? win3d_fac_elems(geo.G) * fsz : 0);
  // transposed records (adjoint): 3D level-major copy, 2D same layout as the factors
  L.off_wfact = take(d3 ? win3d_fac_elems(geo.G) * fsz : (band ? 0 : (size_t)geo.G.nsub * nslot * slots * fsz));
  L.off_q3 = take(d3 ? (size_t)8 * geo.ncell * sizeof(double) : 0);   // 3D cell quantities
  L.off_dump = take(64 * sizeof(double));
  L.off_subs = take(geo.subs.size() * sizeof(SubInfo));
  L.off_lvl = take((geo.lvl.size() + geo.cells.size()) * sizeof(int));
  L.off_state = take(sizeof(GmresState));
  const size_t nparts = std::max<size_t>((size_t)(kMaxRestart + 1) * kRedBlocks, 2 * (size_t)geo.tile_blocks);
  L.off_part = take(nparts * sizeof(double));
  L.off_cnt = take(64);
  L.off_out = take(64 * sizeof(double));
  L.off_tbox = take(d3 ? (size_t)geo.G.nsub * 2 * geo.G.ncb * sizeof(double) : 0);   // 3D transposed boxes
  L.off_own = take(geo.own.size() * sizeof(int));
  const BandGeom B = make_band_geom(geo.G.bw, geo.G.bh, p.subsolver == ACCH_SUB_ILUK_BOX);
  L.off_band = take(band_sub(p) ? (size_t)geo.G.nsub * B.box_elems * fsz : 0);
  L.off_bandy = take(band_sub(p) ? (size_t)geo.G.nsub * B.nchunk * 64 * sizeof(double) : 0);
  L.off_mask = take(masked_sub(p) ? (size_t)geo.G.nsub * B.n * B.mwords * sizeof(unsigned) : 0);
  const bool bx = box_ilu0(p);
  const BoxIluGeom X = bx ? make_boxilu_geom(geo.G.bw, geo.G.bh, nullptr) : BoxIluGeom{};
  L.off_bxL = take(bx ? (size_t)geo.G.nsub * X.ncell * kBoxIluRec * fsz : 0);
  L.off_bxU = take(bx ? (size_t)geo.G.nsub * X.ncell * kBoxIluRec * fsz : 0);
  L.off_bxy = take(bx ? (size_t)geo.G.nsub * X.ncell * 2 * sizeof(double) : 0);
  L.off_lvoff = take(bx ? (size_t)(X.nlev + 1) * sizeof(int) : 0);
  L.off_cellof = take(bx ? (size_t)X.ncell * sizeof(int) : 0);
  L.off_bxTf = take(bx ? (size_t)geo.G.nsub * X.ncell * kBoxIluRec * fsz : 0);
  L.off_bxTb = take(bx ? (size_t)geo.G.nsub * X.ncell * kBoxIluRec * fsz : 0);
  L.total = o;
}

extern "C" int acch_workspace_bytes(const acch_params *pin, size_t *bytes) {
  if (!pin || !bytes) return fail(ACCH_EINVAL, "null argument");
  acch_params p = *pin;
  acch_params_default(&p);
  int rc = validate_params(p);
  if (rc) return rc;
  Geometry geo;
  rc = build_geometry(p, geo);
  if (rc) return rc;
  Layout L;
  make_layout(p, geo, L);
  *bytes = L.total;
  return ACCH_OK;
}

static bool admissible_host(const double *u, const double *v, long n) {
  for (long k = 0; k < n; ++k) {
    const double pp = u[k] + v[k], q = u[k] - v[k];
    if (!(pp > 0.0 && pp < 1.0 && q > 0.0 && q < 1.0)) return false;
  }
  return true;
}

// ---------------------------------------------------------------------------
// ILU(k) pattern of a box matrix (band.h numbering): symbolic elimination with
// levels of fill.  Entries of A_k (with box: every coupling of two cells at most 2
// apart along each axis, both types) have level 0; eliminating pivot p from row R gives
// entry (R, C), C > p, the level lev(R, p) + lev(p, C) + 1 (the smallest over the
// pivots); entries of level above k are dropped.  Rows are processed in order and the
// pivots of a row in increasing column order, fill of the same row included.  Cells
// of the padded box outside the rectangle [ilo, ihi) x [jlo, jhi) are identity rows.
// Bit d of word d / 32 of row R is set for entry (R, R + d - kl).
// ---------------------------------------------------------------------------
static void iluk_pattern(const BandGeom &B, int ilo, int ihi, int jlo, int jhi, int k, bool box, unsigned *bits) {
  static const int kSl[24][4] = {{0, 0, 0, 0},  {0, 0, -1, 0}, {0, 0, 1, 0},  {0, 0, 0, -1}, {0, 0, 0, 1},
                                 {0, 0, -2, 0}, {0, 0, 2, 0},  {0, 0, 0, -2}, {0, 0, 0, 2},  {0, 0, -1, -1},
                                 {0, 0, 1, -1}, {0, 0, -1, 1}, {0, 0, 1, 1},  {0, 1, 0, 0},  {0, 1, -1, 0},
                                 {0, 1, 1, 0},  {0, 1, 0, -1}, {0, 1, 0, 1},  {1, 1, 0, 0},  {1, 1, -1, 0},
                                 {1, 1, 1, 0},  {1, 1, 0, -1}, {1, 1, 0, 1},  {1, 0, 0, 0}};
  const int n = B.n, bw = B.bw;
  auto inside = [&](int i, int j) { return i >= ilo && i < ihi && j >= jlo && j < jhi; };
  std::vector<std::vector<std::pair<int, int>>> upper(n);   // (column, level) right of the diagonal
  std::vector<int> lev(n, -1), cols;
  std::vector<char> queued(n, 0);
  std::memset(bits, 0, sizeof(unsigned) * (size_t)n * B.mwords);
  for (int R = 0; R < n; ++R) {
    cols.clear();
    const int c = R >> 1, t = R & 1, j = c / bw, i = c - j * bw;
    auto add = [&](int C, int l) {
      lev[C] = l;
      cols.push_back(C);
    };
    if (inside(i, j) && box) {   // level 0: both types of every cell up to 2 away per axis
      for (int dy = -2; dy <= 2; ++dy)
        for (int dx = -2; dx <= 2; ++dx)
          if (inside(i + dx, j + dy))
            for (int tc = 0; tc < 2; ++tc) add(2 * ((j + dy) * bw + i + dx) + tc, 0);
    } else if (inside(i, j)) {
      for (const auto &q : kSl) {
        if (q[0] != t || !inside(i + q[2], j + q[3])) continue;
        add(2 * ((j + q[3]) * bw + i + q[2]) + q[1], 0);
      }
    } else {
      add(R, 0);
    }
    // pivots of the row in increasing order (a min-heap; a column enters it once)
    std::vector<int> heap;
    for (int C : cols)
      if (C < R) {
        heap.push_back(C);
        queued[C] = 1;
      }
    std::make_heap(heap.begin(), heap.end(), std::greater<int>());
    while (!heap.empty()) {
      std::pop_heap(heap.begin(), heap.end(), std::greater<int>());
      const int p = heap.back();
      heap.pop_back();
      for (const auto &e : upper[p]) {
        const int nl = lev[p] + e.second + 1;
        if (nl > k) continue;
        const int C = e.first;
        if (lev[C] < 0) {
          add(C, nl);
          if (C < R && !queued[C]) {
            heap.push_back(C);
            std::push_heap(heap.begin(), heap.end(), std::greater<int>());
            queued[C] = 1;
          }
        } else if (nl < lev[C]) {
          lev[C] = nl;
        }
      }
    }
    for (int C : cols) {
      const int d = C - R + B.kl;
      bits[(size_t)R * B.mwords + (d >> 5)] |= 1u << (d & 31);
      if (C > R) upper[R].push_back({C, lev[C]});
      lev[C] = -1;
      queued[C] = 0;
    }
    std::sort(upper[R].begin(), upper[R].end());
  }
}

// ---------------------------------------------------------------------------
// small helpers on a context
// ---------------------------------------------------------------------------
namespace {

// Fold the completed event pairs into the per-kind totals (the stream is idle).
int harvest_timer(acch_ctx *c) {
  KernelTimer &T = c->timer;
  for (int i = 0; i < T.used; ++i) {
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, T.ev[2 * i], T.ev[2 * i + 1]));
    T.total_ms[T.kind[i]] += ms;
    T.count[T.kind[i]] += 1;
  }
  T.used = 0;
  return ACCH_OK;
}

int sync_read(acch_ctx *c, const void *dev, void *host, size_t bytes) {
  HIP_TRY(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->syncs++;
  if (c->timer.on && c->timer.used) return harvest_timer(c);
  return ACCH_OK;
}

int timer_begin(acch_ctx *c, int kind) {
  KernelTimer &T = c->timer;
  if (!T.on) return -1;
  if (T.sampled && (kind != ACCH_KERNEL_RAS || T.seen++ % KernelTimer::kSample != 0)) return -1;
  if (T.used == KernelTimer::kPool) {
    HIP_TRY(hipStreamSynchronize(c->stream));
    int rc = harvest_timer(c);
    if (rc) return -1;
  }
  const int slot = T.used++;
  T.kind[slot] = kind;
  if (hipEventRecord(T.ev[2 * slot], c->stream) != hipSuccess) return -1;
  return slot;
}

void timer_end(acch_ctx *c, int slot) {
  if (slot >= 0) (void)hipEventRecord(c->timer.ev[2 * slot + 1], c->stream);
}

// Launch helper: counts the launch, optionally times it, maps errors.
#define LAUNCHK(c, kind, expr)                                                                     \
  do {                                                                                             \
    const int slot_ = timer_begin((c), (kind));                                                    \
    hipError_t e_ = (expr);                                                                        \
    timer_end((c), slot_);                                                                         \
    (c)->launches++;                                                                               \
    if (e_ != hipSuccess) return fail(ACCH_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)
#define LAUNCH(c, expr) LAUNCHK(c, ACCH_KERNEL_OTHER, expr)

// Kernel launches by dimension.
const int *level_cells(acch_ctx *c) { return c->d_lvl + c->geo.lvl.size(); }
int fp32_of(acch_ctx *c) { return c->p.precision == ACCH_PREC_MIXED; }

hipError_t run_residual(acch_ctx *c, const double *X, const double *Sdir, double lam, const GmresState *shift,
                        const double *Xn, double dt, double *Xt, double *F) {
  return c->d3 ? launch_residual3d(c->bl, X, Sdir, lam, shift, Xn, dt, Xt, F, c->q3, c->red, c->stream)
               : launch_residual2d(c->bl, X, Sdir, lam, nullptr, shift, Xn, dt, Xt, F, c->red, c->stream);
}
hipError_t run_jacobian(acch_ctx *c, const double *X, const double *Xn, double dt) {
  return c->d3 ? launch_jacobian3d(c->bl, X, Xn, dt, c->J, c->q3, c->stream)
               : launch_jacobian2d(c->bl, X, Xn, dt, c->J, c->stream);
}
hipError_t run_spmv(acch_ctx *c, const double *x, double *y, int transpose) {
  return c->d3 ? launch_spmv3d(c->bl, c->J, x, y, transpose, c->stream)
               : launch_spmv2d(c->bl, c->J, x, y, transpose, c->stream);
}
hipError_t run_spmv_dots(acch_ctx *c, long vs, int j, int transpose) {
  return c->d3 ? launch_spmv_dots3d(c->bl, c->J, c->Z, c->V, vs, j, transpose, c->st, c->red, c->stream)
               : launch_spmv_dots2d(c->bl, c->J, c->Z, c->V, vs, j, transpose, c->st, c->red, c->stream);
}
hipError_t run_energy(acch_ctx *c, const double *X) {
  return c->d3 ? launch_energy3d(c->bl, X, c->red, c->stream) : launch_energy2d(c->bl, X, c->red, c->stream);
}
hipError_t run_factor(acch_ctx *c) {
  c->tpacked = false;
  if (c->boxilu)
    return launch_boxilu_factor2d(c->bl, c->bx, c->geo.G.nsub, c->d_subs, c->d_lvoff, c->J, c->p.ilu_shift, c->bxL,
                                  c->bxU, fp32_of(c), c->stream);
  if (c->band)
    return launch_band_factor2d(c->bl, c->bg, c->geo.G.nsub, c->d_subs, c->J,
                                c->p.subsolver == ACCH_SUB_LU ? 0.0 : c->p.ilu_shift, c->bandmask, c->bandf,
                                fp32_of(c), c->stream);
  if (c->d3)
    return launch_ilu_factor3d(c->P, c->geo.G, c->d_subs, c->d_lvl, level_cells(c), c->J, c->p.ilu_shift, c->fac,
                               c->wfac, fp32_of(c), c->stream);
  return launch_ilu_factor2d(c->bl, c->geo.G, c->d_subs, c->d_lvl, c->J, c->p.ilu_shift, c->fac, fp32_of(c),
                             c->stream);
}
hipError_t run_ras(acch_ctx *c, const double *r, double *z, const GmresState *st, long vs) {
  if (c->boxilu)
    return launch_boxilu_apply2d(c->bl, c->bx, c->geo.G, c->d_subs, c->d_cellof, c->bxL, c->bxU, c->bxy, c->ybuf, r, z,
                                 st, vs, fp32_of(c), c->stream, c->ras);
  if (c->band)
    return launch_band_apply2d(c->bl, c->bg, c->geo.G, c->d_subs, c->bandf, c->bandy, c->ybuf, r, z, st, vs,
                               fp32_of(c), c->stream, c->ras);
  if (c->d3)
    return launch_ras_apply3d(c->P, c->geo.G, c->d_subs, c->d_lvl, level_cells(c), c->fac, c->wfac, c->ybuf, r, z,
                              st, vs, fp32_of(c), c->stream, c->ras);
  return launch_ras_apply2d(c->bl, c->geo.G, c->d_subs, c->d_lvl, c->fac, c->ybuf, r, z, c->dump, st, vs, fp32_of(c),
                            c->stream, c->ras);
}
hipError_t run_ras_t(acch_ctx *c, const double *r, double *z, const GmresState *st, long vs) {
  if (c->boxilu) {
    // M^{-T}: the transposed solves with the restriction and extension of the variant
    // exchanged (left <-> right; classical is its own transpose)
    if (!c->tpacked) {
      hipError_t e = launch_boxilu_pack_t(c->bx, c->geo.G.nsub, c->d_lvoff, c->d_cellof, c->bxL, c->bxU, c->bxTf,
                                          c->bxTb, fp32_of(c), c->stream);
      if (e != hipSuccess) return e;
      c->tpacked = true;
    }
    RasVariant rv = c->ras;
    rv.kind = rv.kind == ACCH_RAS_LEFT ? ACCH_RAS_RIGHT : (rv.kind == ACCH_RAS_RIGHT ? ACCH_RAS_LEFT : rv.kind);
    return launch_boxilu_apply2d(c->bl, c->bx, c->geo.G, c->d_subs, c->d_cellof, c->bxTf, c->bxTb, c->bxy, c->ybuf, r,
                                 z, st, vs, fp32_of(c), c->stream, rv, true);
  }
  if (c->d3)
    return launch_ras_t_apply3d(c->P, c->geo.G, c->d_subs, c->d_lvl, level_cells(c), c->p.sub[0], c->p.sub[1],
                                c->p.sub[2], c->d_own, c->fac, c->wfact, &c->tpacked, c->ybuf, c->tbox, r, z, st, vs,
                                fp32_of(c), c->stream);
  return launch_ras_t_apply2d(c->bl, c->geo.G, c->d_subs, c->d_lvl, c->fac, c->wfact, &c->tpacked, c->ybuf, r, z,
                              c->dump, st, vs, fp32_of(c), c->stream, c->ras);
}

int residual_eval(acch_ctx *c, const double *X, const double *Sdir, double lam, const GmresState *shift,
                  const double *Xn, double dt, double *Xt, double *F, double &f2, double &bad) {
  LAUNCHK(c, ACCH_KERNEL_RESIDUAL, run_residual(c, X, Sdir, lam, shift, Xn, dt, Xt, F));
  int rc = sync_read(c, c->red.out, c->host->vals, 2 * sizeof(double));
  if (rc) return rc;
  f2 = c->host->vals[0];
  bad = c->host->vals[1];
  return ACCH_OK;
}

int factor(acch_ctx *c) {
  LAUNCHK(c, ACCH_KERNEL_FACTOR, run_factor(c));
  c->factored = true;
  return ACCH_OK;
}

int precondition_t(acch_ctx *c, const double *r, double *z, const GmresState *st, long vs) {
  LAUNCHK(c, ACCH_KERNEL_RAS, run_ras_t(c, r, z, st, vs));
  return ACCH_OK;
}

// Solve J S = -F (J^T S = -F when transpose) with S from 0.  Returns ACCH_OK when
// converged, ACCH_EDIVERGED if not.  The transposed solve is preconditioned by the
// transposed Schwarz operator and never projects the mass.
int gmres(acch_ctx *c, const double *F, double *S, int &its, double &resid, int transpose = 0) {
  const long n2 = 2 * c->geo.ncell;
  const long vs = n2;
  const int m = c->p.gmres_restart;
  const int project = transpose ? 0 : (c->p.mass_projection > 0);
  LAUNCH(c, launch_reset_state(c->bl, c->st, c->stream));
  its = 0;
  resid = 0.0;
  const size_t tail = offsetof(GmresState, beta);
  GmresState hs{};
  for (int cycle = 0; cycle < c->p.gmres_max_restarts; ++cycle) {
    if (cycle > 0) LAUNCHK(c, ACCH_KERNEL_SPMV, run_spmv(c, S, c->W, transpose));
    LAUNCHK(c, ACCH_KERNEL_GMRES_START, launch_gmres_start(c->bl, F, cycle > 0 ? c->W : nullptr, c->V, c->st, m, c->p.gmres_rtol,
                                 c->p.gmres_atol, c->red, c->stream));
    int launched = 0;
    // Steps enqueued before the first convergence check of the cycle: what the
    // previous solve needed in this cycle, plus one (extra steps are no-ops once the
    // cycle is done), or half a cycle beyond that solve's count; then two at a time.
    const int rem = c->its_guess - cycle * m + 1;
    int chunk = rem >= 1 ? std::min(m, rem) : std::max(1, m / 2);
    while (true) {
      for (int k = 0; k < chunk && launched < m; ++k, ++launched) {
        if (transpose) {
          int rc = precondition_t(c, c->V, c->Z, c->st, vs);
          if (rc) return rc;
        } else {
          LAUNCHK(c, ACCH_KERNEL_RAS, run_ras(c, c->V, c->Z, c->st, vs));
        }
        LAUNCHK(c, ACCH_KERNEL_SPMV_DOTS, run_spmv_dots(c, vs, launched, transpose));
        LAUNCHK(c, ACCH_KERNEL_ORTH, launch_gmres_orth(c->bl, c->V, vs, launched, c->st, c->red, c->stream));
      }
      LAUNCHK(c, ACCH_KERNEL_GMRES_UPDATE, launch_gmres_update(c->bl, S, c->Z, vs, c->st, cycle > 0, project, c->red, c->stream));
      int rc = sync_read(c, (const char *)c->st + tail, c->host_state, sizeof(GmresState) - tail);
      if (rc) return rc;
      memcpy((char *)&hs + tail, c->host_state, sizeof(GmresState) - tail);
      if (hs.done || launched >= m) break;
      chunk = 2;
    }
    its = hs.total_its;
    resid = hs.resid;
    if (!hs.done) return fail(ACCH_EDIVERGED, "GMRES cycle did not finish");
    if (hs.converged) {
      c->its_guess = std::max(1, its);   // over all cycles
      return ACCH_OK;
    }
    if (!(resid == resid)) return fail(ACCH_EDIVERGED, "GMRES residual is not finite");
    if (hs.total_its == 0) return fail(ACCH_EDIVERGED, "GMRES made no progress");
  }
  return fail(ACCH_EDIVERGED, "GMRES did not converge within the restart limit");
}

// Backtracking line search along S (with the mass shift) from X (LineSearch in
// driver.h).  On success Xt/Ft hold the accepted point.
int line_search(acch_ctx *c, double dt, double fnorm, double &f2_new, double &lam_out) {
  LineSearch ls;
  ls.start(fnorm);
  const GmresState *shift = c->p.mass_projection > 0 ? c->st : nullptr;
  while (ls.state == LineSearch::kSearching) {
    double f2, bad;
    int rc = residual_eval(c, c->X, c->S, ls.lam, shift, c->Xn, dt, c->Xt, c->Ft, f2, bad);
    if (rc) return rc;
    ls.trial(f2, bad);
  }
  if (ls.state != LineSearch::kAccepted) return fail(ACCH_EDIVERGED, "line search failed");
  f2_new = ls.f2;
  lam_out = ls.lam;
  return ACCH_OK;
}

struct SolveStats {
  int newton = 0, gmres = 0;
  double fnorm = 0.0;
};

// Newton solve of scheme (2.20) at dt from Xn; on success X holds the root.
int nks_solve(acch_ctx *c, double dt, SolveStats &stats) {
  const long n2 = 2 * c->geo.ncell;
  HIP_TRY(hipMemcpyAsync(c->X, c->Xn, n2 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  double f2, bad;
  int rc = residual_eval(c, c->X, nullptr, 0.0, nullptr, c->Xn, dt, nullptr, c->F, f2, bad);
  if (rc) return rc;
  double fnorm = sqrt(f2);
  stats.fnorm = fnorm;
  if (!isfinite(fnorm)) return fail(ACCH_EDIVERGED, "initial residual is not finite");
  const double tol = std::max(c->p.newton_rtol * fnorm, c->p.newton_atol);
  if (fnorm <= tol) return ACCH_OK;
  for (int it = 1; it <= c->p.newton_max_it; ++it) {
    // counted before any early return, so a failed attempt's last iteration counts too
    stats.newton = it;
    LAUNCHK(c, ACCH_KERNEL_JACOBIAN, run_jacobian(c, c->X, c->Xn, dt));
    if (it == 1 || c->p.ilu_reuse < 0) {
      rc = factor(c);
      if (rc) return rc;
    }
    int its = 0;
    double lres = 0.0;
    rc = gmres(c, c->F, c->S, its, lres);
    stats.gmres += its;
    if (rc) return rc;
    double f2n, lam;
    rc = line_search(c, dt, fnorm, f2n, lam);
    if (rc) return rc;
    std::swap(c->X, c->Xt);
    std::swap(c->F, c->Ft);
    fnorm = sqrt(f2n);
    stats.fnorm = fnorm;
    if (!isfinite(fnorm)) return fail(ACCH_EDIVERGED, "residual is not finite");
    if (fnorm <= tol) return ACCH_OK;
  }
  return fail(ACCH_EDIVERGED, "Newton iteration limit reached");
}

int energy_mass(acch_ctx *c, const double *X, double &E, double &M) {
  LAUNCHK(c, ACCH_KERNEL_ENERGY, run_energy(c, X));
  int rc = sync_read(c, c->red.out, c->host->vals, 2 * sizeof(double));
  if (rc) return rc;
  E = c->host->vals[0] * c->hvol;
  M = c->host->vals[1] * c->hvol;
  return ACCH_OK;
}

// Accept the iterate X as the new state.
void accept(acch_ctx *c, double dt) {
  std::swap(c->Xprev, c->Xn);  // Xprev <- old state
  std::swap(c->Xn, c->X);      // Xn <- root; X gets the free buffer
  c->t += dt;
  c->dt_prev = dt;
  c->have_history = true;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" int acch_create(const acch_params *pin, const double *u0, const double *v0, acch_ctx **out) {
  if (!pin || !u0 || !v0 || !out) return fail(ACCH_EINVAL, "null argument");
  *out = nullptr;
  acch_params p = *pin;
  acch_params_default(&p);
  int rc = validate_params(p);
  if (rc) return rc;
  acch_ctx *c = new (std::nothrow) acch_ctx();
  if (!c) return fail(ACCH_EINVAL, "host allocation failed");
  c->p = p;
  rc = build_geometry(p, c->geo);
  if (rc) {
    delete c;
    return rc;
  }
  if (p.ras_type != ACCH_RAS_LEFT && p.overlap > c->geo.min_part) {
    delete c;
    return fail(ACCH_EUNSUPPORTED, "right-restricted / classical Schwarz needs overlap <= the smallest subdomain width");
  }
  make_layout(p, c->geo, c->lay);
  if (!p.workspace || p.workspace_bytes < c->lay.total) {
    delete c;
    return fail(ACCH_EINVAL, "workspace missing or smaller than acch_workspace_bytes()");
  }
  if (((uintptr_t)p.workspace) % kAlign) {
    delete c;
    return fail(ACCH_EINVAL, "workspace must be 256-byte aligned");
  }
  const long n = c->geo.ncell;
  if (!admissible_host(u0, v0, n)) {
    delete c;
    return fail(ACCH_EDOMAIN, "initial state outside the admissible set");
  }
  c->stream = (hipStream_t)p.stream;
  c->ws = (char *)p.workspace;
  const Layout &L = c->lay;
  c->Xn = (double *)(c->ws + L.off_Xn);
  c->Xprev = (double *)(c->ws + L.off_Xprev);
  c->X = (double *)(c->ws + L.off_X);
  c->Xt = (double *)(c->ws + L.off_Xt);
  c->F = (double *)(c->ws + L.off_F);
  c->Ft = (double *)(c->ws + L.off_Ft);
  c->S = (double *)(c->ws + L.off_S);
  c->W = (double *)(c->ws + L.off_W);
  c->J = (double *)(c->ws + L.off_J);
  c->V = (double *)(c->ws + L.off_V);
  c->Z = (double *)(c->ws + L.off_Z);
  c->fac = c->ws + L.off_fac;
  c->wfac = c->geo.G.wmax > 0 ? (void *)(c->ws + L.off_wfac) : nullptr;
  c->wfact = (p.dim == 2 || c->geo.G.wmax > 0) ? (void *)(c->ws + L.off_wfact) : nullptr;
  c->q3 = (double *)(c->ws + L.off_q3);
  c->ybuf = c->ws + L.off_y;
  c->dump = (double *)(c->ws + L.off_dump);
  c->tbox = (double *)(c->ws + L.off_tbox);
  c->d_subs = (SubInfo *)(c->ws + L.off_subs);
  c->d_lvl = (int *)(c->ws + L.off_lvl);
  c->d_own = (int *)(c->ws + L.off_own);
  c->ras.own_x = c->d_own;
  c->ras.own_y = c->d_own + p.n[0];
  c->st = (GmresState *)(c->ws + L.off_state);
  c->red.partials = (double *)(c->ws + L.off_part);
  c->red.counter = (unsigned *)(c->ws + L.off_cnt);
  c->red.out = (double *)(c->ws + L.off_out);
  c->P = phys_of(p);
  c->hvol = (p.L[0] / p.n[0]) * (p.L[1] / p.n[1]) * (p.dim == 3 ? p.L[2] / p.n[2] : 1.0);
  c->d3 = p.dim == 3;
  c->eta = p.eta0;
  c->bl = single_launch(c->P, c->geo.G.nsub);
  c->ras.kind = p.ras_type;
  c->ras.px = p.sub[0];
  c->ras.py = p.sub[1];
  c->ras.pz = p.dim == 3 ? p.sub[2] : 1;
  c->band = band_sub(p);
  c->boxilu = box_ilu0(p);
  if (c->boxilu) {
    c->bx = make_boxilu_geom(c->geo.G.bw, c->geo.G.bh, &c->lvoff_h, &c->cellof_h);
    c->bxL = c->ws + L.off_bxL;
    c->bxU = c->ws + L.off_bxU;
    c->bxy = (double *)(c->ws + L.off_bxy);
    c->d_lvoff = (int *)(c->ws + L.off_lvoff);
    c->d_cellof = (int *)(c->ws + L.off_cellof);
    c->bxTf = c->ws + L.off_bxTf;
    c->bxTb = c->ws + L.off_bxTb;
  }
  std::vector<unsigned> maskh;
  if (c->band) {
    c->bg = make_band_geom(c->geo.G.bw, c->geo.G.bh, p.subsolver == ACCH_SUB_ILUK_BOX);
    c->bandf = c->ws + L.off_band;
    c->bandy = (double *)(c->ws + L.off_bandy);
    if (masked_sub(p)) {
      c->bandmask = (unsigned *)(c->ws + L.off_mask);
      // one pattern per distinct rectangle of grid cells inside the padded box
      const size_t per = (size_t)c->bg.n * c->bg.mwords;
      maskh.resize(per * c->geo.G.nsub);
      std::vector<std::vector<int>> keys;
      std::vector<size_t> first;
      for (int b = 0; b < c->geo.G.nsub; ++b) {
        const SubInfo &si = c->geo.subs[b];
        int ilo = 0, jlo = 0, ihi = std::min(c->bg.bw, si.ex), jhi = std::min(c->bg.bh, si.ey);
        if (p.bc != ACCH_BC_PERIODIC) {
          ilo = std::max(ilo, -si.ox);
          jlo = std::max(jlo, -si.oy);
          ihi = std::min(ihi, p.n[0] - si.ox);
          jhi = std::min(jhi, p.n[1] - si.oy);
        }
        const std::vector<int> key = {ilo, ihi, jlo, jhi};
        size_t at = keys.size();
        for (size_t q = 0; q < keys.size(); ++q)
          if (keys[q] == key) at = q;
        if (at == keys.size()) {
          keys.push_back(key);
          first.push_back((size_t)b);
          iluk_pattern(c->bg, ilo, ihi, jlo, jhi, p.fill_level, p.subsolver == ACCH_SUB_ILUK_BOX,
                       maskh.data() + per * b);
        } else {
          std::memcpy(maskh.data() + per * b, maskh.data() + per * first[at], per * sizeof(unsigned));
        }
      }
    }
  }
  if (hipHostMalloc((void **)&c->host, sizeof(GmresState) + sizeof(HostMirror), hipHostMallocDefault) != hipSuccess) {
    delete c;
    return fail(ACCH_EDEVICE, "hipHostMalloc failed");
  }
  c->host_state = (char *)c->host + sizeof(HostMirror);
  auto cleanup = [&](int code) {
    (void)hipHostFree(c->host);
    delete c;
    return code;
  };
  if (hipMemcpyAsync(c->Xn, u0, n * sizeof(double), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      hipMemcpyAsync(c->Xn + n, v0, n * sizeof(double), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      hipMemcpyAsync(c->d_subs, c->geo.subs.data(), c->geo.subs.size() * sizeof(SubInfo), hipMemcpyHostToDevice,
                     c->stream) != hipSuccess ||
      hipMemcpyAsync(c->d_lvl, c->geo.lvl.data(), c->geo.lvl.size() * sizeof(int), hipMemcpyHostToDevice,
                     c->stream) != hipSuccess ||
      (!c->geo.cells.empty() &&
       hipMemcpyAsync(c->d_lvl + c->geo.lvl.size(), c->geo.cells.data(), c->geo.cells.size() * sizeof(int),
                      hipMemcpyHostToDevice, c->stream) != hipSuccess) ||
      hipMemcpyAsync(c->d_own, c->geo.own.data(), c->geo.own.size() * sizeof(int), hipMemcpyHostToDevice,
                     c->stream) != hipSuccess ||
      hipMemsetAsync(c->red.counter, 0, 64, c->stream) != hipSuccess ||
      hipMemsetAsync(c->st, 0, sizeof(GmresState), c->stream) != hipSuccess ||
      (!maskh.empty() && hipMemcpyAsync(c->bandmask, maskh.data(), maskh.size() * sizeof(unsigned),
                                        hipMemcpyHostToDevice, c->stream) != hipSuccess) ||
      (c->boxilu && hipMemcpyAsync(c->d_lvoff, c->lvoff_h.data(), c->lvoff_h.size() * sizeof(int),
                                   hipMemcpyHostToDevice, c->stream) != hipSuccess) ||
      (c->boxilu && hipMemcpyAsync(c->d_cellof, c->cellof_h.data(), c->cellof_h.size() * sizeof(int),
                                   hipMemcpyHostToDevice, c->stream) != hipSuccess) ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return cleanup(fail(ACCH_EDEVICE, "initial upload failed"));
  *out = c;
  return ACCH_OK;
}

extern "C" int acch_timing(acch_ctx *c, int enable) {
  if (!c) return fail(ACCH_EINVAL, "null context");
  KernelTimer &T = c->timer;
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (T.on && T.used) {
    int rc = harvest_timer(c);
    if (rc) return rc;
  }
  if (enable && T.ev.empty()) {
    T.ev.resize(2 * KernelTimer::kPool);
    T.kind.resize(KernelTimer::kPool);
    for (auto &e : T.ev) HIP_TRY(hipEventCreate(&e));
  }
  T.on = enable != 0;
  T.sampled = enable == 2;
  T.seen = 0;
  for (int k = 0; k < ACCH_KERNEL_KINDS; ++k) {
    T.total_ms[k] = 0.0;
    T.count[k] = 0;
  }
  c->launches = 0;
  c->syncs = 0;
  return ACCH_OK;
}

extern "C" int acch_kernel_stats(acch_ctx *c, int kind, double *total_ms, long *count) {
  if (!c || kind < 0 || kind >= ACCH_KERNEL_KINDS) return fail(ACCH_EINVAL, "bad arguments");
  if (c->timer.on && c->timer.used) {
    HIP_TRY(hipStreamSynchronize(c->stream));
    int rc = harvest_timer(c);
    if (rc) return rc;
  }
  if (total_ms) *total_ms = c->timer.total_ms[kind];
  if (count) *count = c->timer.count[kind];
  return ACCH_OK;
}

extern "C" int acch_set_option(acch_ctx *c, int option, long value) {
  (void)c;
  if (option == ACCH_OPT_RAS_PREFETCH) {
    set_ras_prefetch((int)value);
    return ACCH_OK;
  }
  if (option == ACCH_OPT_RAS3D_WINDOW) {
    set_ras3d_window(value != 0);
    return ACCH_OK;
  }
  return fail(ACCH_EINVAL, "unknown option");
}

extern "C" int acch_counters(acch_ctx *c, long *launches, long *syncs) {
  if (!c) return fail(ACCH_EINVAL, "null context");
  if (launches) *launches = c->launches;
  if (syncs) *syncs = c->syncs;
  return ACCH_OK;
}

extern "C" int acch_destroy(acch_ctx *c) {
  if (!c) return ACCH_OK;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (auto &e : c->timer.ev) (void)hipEventDestroy(e);
  if (c->host) (void)hipHostFree(c->host);
  delete c;
  return ACCH_OK;
}

extern "C" int acch_step(acch_ctx *c, int nsteps, acch_step_info *info, int *accepted) {
  if (!c || nsteps < 0) return fail(ACCH_EINVAL, "bad arguments");
  if (accepted) *accepted = 0;
  const acch_params &p = c->p;
  for (int s = 0; s < nsteps; ++s) {
    double dt;
    if (!p.adaptive) {
      dt = p.dt_fixed;
    } else if (!c->have_history) {
      dt = p.dt_min;
    } else {
      LAUNCH(c, launch_norm2_diff(c->bl, c->Xn, c->Xprev, c->red, c->stream));
      int rc = sync_read(c, c->red.out, c->host->vals, sizeof(double));
      if (rc) return rc;
      double dn = sqrt(c->host->vals[0]);
      if (p.xd_norm == 1) dn *= sqrt(c->hvol);
      const double xd = dn / c->dt_prev;
      dt = std::max(p.dt_min, p.dt_max / sqrt(1.0 + c->eta * xd * xd));
    }
    SolveStats tot;
    int retries = 0;
    while (true) {
      SolveStats st;
      int rc = nks_solve(c, dt, st);
      tot.newton += st.newton;
      tot.gmres += st.gmres;
      tot.fnorm = st.fnorm;
      if (rc == ACCH_OK) break;
      if (rc != ACCH_EDIVERGED) return rc;
      if (!p.adaptive) return fail(ACCH_EDIVERGED, "NKS diverged at the fixed dt: " + g_last_error);
      c->eta *= 2.0;
      if (dt <= p.dt_min) return fail(ACCH_EDIVERGED, "NKS diverged at dt_min: " + g_last_error);
      dt = std::max(dt / sqrt(2.0), p.dt_min);
      ++retries;
    }
    accept(c, dt);
    acch_step_info rec{};
    rec.t = c->t;
    rec.dt = dt;
    rec.eta = c->eta;
    rec.fnorm = tot.fnorm;
    rec.newton_its = tot.newton;
    rec.gmres_its = tot.gmres;
    rec.retries = retries;
    rec.status = ACCH_OK;
    rec.energy = rec.mass = NAN;
    if (p.log_energy > 0) {
      int rc = energy_mass(c, c->Xn, rec.energy, rec.mass);
      if (rc) return rc;
    }
    if (info) info[s] = rec;
    if (accepted) *accepted = s + 1;
  }
  return ACCH_OK;
}

extern "C" int acch_solve_step(acch_ctx *c, double dt, acch_step_info *info) {
  if (!c || !(dt > 0)) return fail(ACCH_EINVAL, "bad arguments");
  SolveStats st;
  int rc = nks_solve(c, dt, st);
  if (rc) return rc;
  accept(c, dt);
  if (info) {
    acch_step_info rec{};
    rec.t = c->t;
    rec.dt = dt;
    rec.eta = c->eta;
    rec.fnorm = st.fnorm;
    rec.newton_its = st.newton;
    rec.gmres_its = st.gmres;
    rec.energy = rec.mass = NAN;
    if (c->p.log_energy > 0) {
      rc = energy_mass(c, c->Xn, rec.energy, rec.mass);
      if (rc) return rc;
    }
    *info = rec;
  }
  return ACCH_OK;
}

extern "C" int acch_energy(acch_ctx *c, double *energy, double *mass) {
  if (!c) return fail(ACCH_EINVAL, "null context");
  double E, M;
  int rc = energy_mass(c, c->Xn, E, M);
  if (rc) return rc;
  if (energy) *energy = E;
  if (mass) *mass = M;
  return ACCH_OK;
}

extern "C" int acch_get_fields(acch_ctx *c, double *u, double *v) {
  if (!c || !u || !v) return fail(ACCH_EINVAL, "null argument");
  const long n = c->geo.ncell;
  HIP_TRY(hipMemcpyAsync(u, c->Xn, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipMemcpyAsync(v, c->Xn + n, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return ACCH_OK;
}

extern "C" int acch_set_fields(acch_ctx *c, const double *u, const double *v) {
  if (!c || !u || !v) return fail(ACCH_EINVAL, "null argument");
  const long n = c->geo.ncell;
  if (!admissible_host(u, v, n)) return fail(ACCH_EDOMAIN, "state outside the admissible set");
  HIP_TRY(hipMemcpyAsync(c->Xn, u, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(c->Xn + n, v, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->have_history = false;
  return ACCH_OK;
}

extern "C" int acch_get_time(acch_ctx *c, double *t, double *dt_prev, double *eta) {
  if (!c) return fail(ACCH_EINVAL, "null context");
  if (t) *t = c->t;
  if (dt_prev) *dt_prev = c->dt_prev;
  if (eta) *eta = c->eta;
  return ACCH_OK;
}

extern "C" int acch_residual(acch_ctx *c, const double *X, const double *Xn, double dt, double *F, double *fnorm2,
                             int *inadmissible) {
  if (!c || !X || !Xn || !F || !(dt > 0)) return fail(ACCH_EINVAL, "bad arguments");
  double f2, bad;
  int rc = residual_eval(c, X, nullptr, 0.0, nullptr, Xn, dt, nullptr, F, f2, bad);
  if (rc) return rc;
  if (fnorm2) *fnorm2 = f2;
  if (inadmissible) *inadmissible = (int)bad;
  return ACCH_OK;
}

extern "C" int acch_jacobian(acch_ctx *c, const double *X, const double *Xn, double dt) {
  if (!c || !X || !Xn || !(dt > 0)) return fail(ACCH_EINVAL, "bad arguments");
  LAUNCHK(c, ACCH_KERNEL_JACOBIAN, run_jacobian(c, X, Xn, dt));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return ACCH_OK;
}

extern "C" int acch_apply_jacobian(acch_ctx *c, const double *x, double *y) {
  if (!c || !x || !y) return fail(ACCH_EINVAL, "bad arguments");
  LAUNCH(c, run_spmv(c, x, y, 0));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return ACCH_OK;
}

extern "C" int acch_apply_jacobian_transpose(acch_ctx *c, const double *x, double *y) {
  if (!c || !x || !y) return fail(ACCH_EINVAL, "bad arguments");
  LAUNCHK(c, ACCH_KERNEL_SPMV, run_spmv(c, x, y, 1));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return ACCH_OK;
}

static int adjoint_ready(acch_ctx *c) {
  if (c->d3 && c->p.ras_type != ACCH_RAS_LEFT)
    return fail(ACCH_EUNSUPPORTED, "the 3D transposed Schwarz operator is built for the left-restricted variant");
  if (c->band)
    return fail(ACCH_EUNSUPPORTED, "the transposed Schwarz operator uses an ILU(0) subdomain solver");
  if (c->p.overlap > c->geo.min_part)
    return fail(ACCH_EUNSUPPORTED, "transposed Schwarz operator needs overlap <= the smallest subdomain width");
  return ACCH_OK;
}

extern "C" int acch_precondition_transpose(acch_ctx *c, const double *r, double *z) {
  if (!c || !r || !z) return fail(ACCH_EINVAL, "bad arguments");
  if (!c->factored) return fail(ACCH_EINVAL, "no factorisation: call acch_factor first");
  int rc = adjoint_ready(c);
  if (rc) return rc;
  rc = precondition_t(c, r, z, nullptr, 0);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(c->stream));
  return ACCH_OK;
}

extern "C" int acch_energy_gradient(acch_ctx *c, const double *X, double *g, double *dparams) {
  if (!c || !g || !dparams) return fail(ACCH_EINVAL, "bad arguments");
  LAUNCHK(c, ACCH_KERNEL_ENERGY,
          c->d3 ? launch_energy_grad3d(c->P, X ? X : c->Xn, c->hvol, g, c->red, c->stream)
                : launch_energy_grad2d(c->P, X ? X : c->Xn, c->hvol, g, c->red, c->stream));
  int rc = sync_read(c, c->red.out, c->host->vals, 4 * sizeof(double));
  if (rc) return rc;
  for (int k = 0; k < 4; ++k) dparams[k] = c->host->vals[k];
  return ACCH_OK;
}

extern "C" int acch_adjoint_step(acch_ctx *c, const double *X1, const double *X0, double dt, const double *g,
                                 double *g_prev, double *dparams, int *gmres_its, double *resid) {
  if (!c || !X1 || !X0 || !g || !g_prev || !dparams) return fail(ACCH_EINVAL, "bad arguments");
  if (!(dt > 0.0)) return fail(ACCH_EINVAL, "dt must be positive");
  int rc = adjoint_ready(c);
  if (rc) return rc;
  LAUNCHK(c, ACCH_KERNEL_JACOBIAN, run_jacobian(c, X1, X0, dt));
  rc = factor(c);
  if (rc) return rc;
  int its = 0;
  double res = 0.0;
  rc = gmres(c, g, c->S, its, res, 1);   // J^T S = -g: S = -lambda
  if (gmres_its) *gmres_its = its;
  if (resid) *resid = res;
  if (rc) return rc;
  // g_prev = (dF/dX0)^T S and red.out = S . dF/dp, i.e. -lambda . dF/dp
  LAUNCH(c, c->d3 ? launch_adjoint_prev3d(c->P, X1, X0, dt, c->S, 1.0, c->W, g_prev, c->red, c->stream)
                  : launch_adjoint_prev2d(c->P, X1, X0, dt, c->S, 1.0, c->W, g_prev, c->red, c->stream));
  rc = sync_read(c, c->red.out, c->host->vals, 4 * sizeof(double));
  if (rc) return rc;
  for (int k = 0; k < 4; ++k) dparams[k] += c->host->vals[k];
  return ACCH_OK;
}

extern "C" int acch_factor(acch_ctx *c) {
  if (!c) return fail(ACCH_EINVAL, "null context");
  int rc = factor(c);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(c->stream));
  return ACCH_OK;
}

extern "C" int acch_precondition(acch_ctx *c, const double *r, double *z) {
  if (!c || !r || !z) return fail(ACCH_EINVAL, "bad arguments");
  if (!c->factored) return fail(ACCH_EINVAL, "no factorisation: call acch_factor first");
  LAUNCHK(c, ACCH_KERNEL_RAS, run_ras(c, r, z, nullptr, 0));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return ACCH_OK;
}

extern "C" int acch_gmres(acch_ctx *c, const double *F, double *S, int *iterations, double *resid) {
  if (!c || !F || !S) return fail(ACCH_EINVAL, "bad arguments");
  if (!c->factored) return fail(ACCH_EINVAL, "no factorisation: call acch_factor first");
  int its = 0;
  double r = 0.0;
  int rc = gmres(c, F, S, its, r);
  if (iterations) *iterations = its;
  if (resid) *resid = r;
  return rc;
}

extern "C" int acch_export(acch_ctx *c, int which, void *out, size_t *bytes) {
  if (!c || !bytes) return fail(ACCH_EINVAL, "bad arguments");
  const BoxGeom &G = c->geo.G;
  size_t need = 0;
  const int nslot = c->d3 ? kNSlot3D : kNSlot2D;
  if (which == ACCH_EXPORT_JACOBIAN) need = (size_t)nslot * c->geo.ncell * sizeof(double);
  else if (which == ACCH_EXPORT_FACTORS && c->boxilu) need = (size_t)G.nsub * c->bx.ncell * 2 * kBoxIluRec * sizeof(double);
  else if (which == ACCH_EXPORT_FACTORS) need = (size_t)G.nsub * nslot * G.ncb * sizeof(double);
  else if (which == ACCH_EXPORT_BOXES) need = (size_t)G.nsub * 4 * sizeof(int);
  else if (which == ACCH_EXPORT_BAND && c->band) need = (size_t)G.nsub * c->bg.n * c->bg.nd * sizeof(double);
  else return fail(ACCH_EINVAL, "unknown export");
  if (!out) {
    *bytes = need;
    return ACCH_OK;
  }
  if (*bytes < need) return fail(ACCH_EINVAL, "output buffer too small");
  if (which == ACCH_EXPORT_JACOBIAN) {
    HIP_TRY(hipMemcpyAsync(out, c->J, need, hipMemcpyDeviceToDevice, c->stream));
  } else if (which == ACCH_EXPORT_BAND) {
    if (!c->factored) return fail(ACCH_EINVAL, "no factorisation");
    LAUNCH(c, launch_band_export(c->bg, G.nsub, c->bandf, c->p.precision == ACCH_PREC_MIXED, (double *)out, c->stream));
  } else if (which == ACCH_EXPORT_FACTORS) {
    if (!c->factored) return fail(ACCH_EINVAL, "no factorisation");
    if (c->band) return fail(ACCH_EINVAL, "the factors of ILU(k) / exact LU are exported by ACCH_EXPORT_BAND");
    if (c->boxilu)
      LAUNCH(c, launch_boxilu_export(c->bx, G.nsub, c->d_lvoff, c->bxL, c->bxU, fp32_of(c), (double *)out, c->stream));
    else if (c->d3)
      LAUNCH(c, launch_export_factors3d(G, c->fac, c->p.precision == ACCH_PREC_MIXED, (double *)out, c->stream));
    else
      LAUNCH(c, launch_export_factors2d(G, c->d_lvl, c->fac, c->p.precision == ACCH_PREC_MIXED, (double *)out,
                                        c->stream));
  } else {
    std::vector<int> b;
    for (const SubInfo &s : c->geo.subs) {
      b.push_back(s.ox);
      b.push_back(s.oy);
      b.push_back(G.bw);
      b.push_back(G.bh);
    }
    HIP_TRY(hipMemcpyAsync(out, b.data(), need, hipMemcpyHostToDevice, c->stream));
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  *bytes = need;
  return ACCH_OK;
}

extern "C" int acch_info(acch_ctx *c, long *ncell, int *nsub, int *box_w, int *box_h) {
  if (!c) return fail(ACCH_EINVAL, "null context");
  if (ncell) *ncell = c->geo.ncell;
  if (nsub) *nsub = c->geo.G.nsub;
  if (box_w) *box_w = c->geo.G.bw;
  if (box_h) *box_h = c->geo.G.bh;
  return ACCH_OK;
}

extern "C" const char *acch_strerror(int code) {
  switch (code) {
    case ACCH_OK: return "ok";
    case ACCH_EINVAL: return "invalid argument";
    case ACCH_EDOMAIN: return "state outside the admissible set";
    case ACCH_EDIVERGED: return "Newton-Krylov-Schwarz diverged";
    case ACCH_EDEVICE: return "HIP runtime error";
    case ACCH_EUNSUPPORTED: return "unsupported configuration";
    default: return "unknown error";
  }
}

extern "C" const char *acch_last_error(void) { return g_last_error.c_str(); }
