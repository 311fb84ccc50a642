// Batched driver: many independent instances of scheme (2.20) (own grid, parameters
// and subdomains each) advanced together at a common fixed dt.  Every kernel of the
// Newton–Krylov–Schwarz step runs once per stage for all instances (all subdomain
// factorisations and triangular solves of all instances in one launch); instances
// that have converged are masked off.  Newton iterations, line searches and GMRES
// cycles run in lockstep with a per-instance state, so each instance follows exactly
// the operation sequence of its single-instance run.  The Arnoldi steps of a GMRES
// cycle are recorded once into HIP graphs (chunks of steps) and replayed.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "driver.h"
#include "kernels.h"

using namespace acch;

namespace {

constexpr int kChunk = 8;   // Arnoldi steps per recorded graph

struct BLayout {
  size_t off_Xn, off_X, off_Xt, off_F, off_Ft, off_S, off_W, off_J, off_V, off_Z, off_fac, off_y, off_dump;
  size_t off_subs, off_lvl, off_state, off_part, off_out, off_inst, off_map[kFamilies], off_mask[3], off_lam;
  size_t off_bxL, off_bxU, off_bxy, off_bxlv, off_bxcell;   // box-pattern ILU(0) records and tables
  size_t total;
};

struct Plan {
  int count = 0;
  long ncell = 0;                 // all instances
  BoxGeom G{};                    // common padded box geometry
  std::vector<Inst> inst;
  std::vector<SubInfo> subs;      // all subdomains, instance by instance
  std::vector<int> lvl;
  std::vector<int2> map[kFamilies];
  int grid[kFamilies] = {};
  bool box = false;               // ILU(0) on the box pattern (its own kernels)
  BoxIluGeom bx{};                // its record geometry for the common padded box
  std::vector<int> bxlvoff, bxcellof;
};

int make_plan(const acch_params *ps, int count, Plan &pl) {
  if (count < 1) return fail(ACCH_EINVAL, "a batch needs at least one instance");
  const acch_params &p0 = ps[0];
  pl.count = count;
  pl.inst.assign(count, Inst{});
  std::vector<Geometry> geos(count);
  int bw = 0, bh = 0;
  for (int b = 0; b < count; ++b) {
    acch_params p = ps[b];
    acch_params_default(&p);
    int rc = validate_params(p);
    if (rc) return fail(rc, "instance " + std::to_string(b) + ": " + acch_last_error());
    if (p.dim != 2) return fail(ACCH_EUNSUPPORTED, "batches are 2D");
    if (p.adaptive) return fail(ACCH_EUNSUPPORTED, "batches step at a common fixed dt (adaptive = 0)");
    if (p.ras_type != ACCH_RAS_LEFT) return fail(ACCH_EUNSUPPORTED, "batches use the left-restricted Schwarz variant");
    const bool box = p.subsolver == ACCH_SUB_ILUK_BOX && p.fill_level == 0;
    if (p.subsolver != ACCH_SUB_ILU0 && !box)
      return fail(ACCH_EUNSUPPORTED, "batches use ILU(0) on the stencil or on the box pattern");
    if (p.overlap != p0.overlap || p.precision != p0.precision || p.dt_fixed != p0.dt_fixed ||
        p.subsolver != p0.subsolver || p.fill_level != p0.fill_level)
      return fail(ACCH_EINVAL, "instances must share overlap, precision, dt_fixed and the subdomain solver");
    pl.box = box;
    rc = build_geometry(p, geos[b]);
    if (rc) return rc;
    bw = std::max(bw, geos[b].G.bw);
    bh = std::max(bh, geos[b].G.bh);
  }
  pl.G.bw = bw;
  pl.G.bh = bh;
  pl.G.nlev = bw + 2 * (bh - 1);
  pl.G.ncb = bw * bh;
  if (schwarz_waves(pl.G) == 0) return fail(ACCH_EINVAL, "subdomain box too large (at most 511 cells wide, 512 tall)");
  if (pl.box) {
    pl.bx = make_boxilu_geom(bw, bh, &pl.bxlvoff, &pl.bxcellof);
    if (!boxilu_fits(pl.bx))
      return fail(ACCH_EINVAL, "box-pattern ILU(0): subdomain box too large (at most 144 cells wide, 160 tall)");
  }
  long xoff = 0, joff = 0;
  int blk[kFamilies] = {};
  for (int b = 0; b < count; ++b) {
    acch_params p = ps[b];
    acch_params_default(&p);
    Inst &I = pl.inst[b];
    Phys &P = I.P;
    P.nx = p.n[0];
    P.ny = p.n[1];
    P.periodic = p.bc == ACCH_BC_PERIODIC;
    const double hx = p.L[0] / p.n[0], hy = p.L[1] / p.n[1];
    P.wx = 1.0 / (hx * hx);
    P.wy = 1.0 / (hy * hy);
    P.alpha = p.alpha;
    P.beta = p.beta;
    P.theta = p.theta;
    P.gamma = p.gamma;
    P.rho = p.rho;
    P.S = p.S;
    P.mob = p.mobility_mode;
    P.nz = 1;
    P.wz = 0.0;
    const long n = (long)P.nx * P.ny;
    I.xoff = xoff;
    I.joff = joff;
    xoff += 2 * n;
    joff += (long)kNSlot2D * n;
    pl.ncell += n;
    int nb[kFamilies];
    family_blocks(P, (int)geos[b].subs.size(), nb);
    for (int f = 0; f < kFamilies; ++f) {
      I.blk0[f] = blk[f];
      I.nblk[f] = nb[f];
      for (int k = 0; k < nb[f]; ++k) pl.map[f].push_back(make_int2(b, k));
      blk[f] += nb[f];
    }
    pl.subs.insert(pl.subs.end(), geos[b].subs.begin(), geos[b].subs.end());
  }
  for (int f = 0; f < kFamilies; ++f) pl.grid[f] = blk[f];
  pl.G.nsub = (int)pl.subs.size();
  pl.lvl.assign(pl.G.nlev + 1, 0);
  for (int w = 0; w < pl.G.nlev; ++w) {
    const int lo = std::max(0, (w - bw + 2) >> 1);
    const int hi = std::min(bh - 1, w >> 1);
    pl.lvl[w + 1] = pl.lvl[w] + std::max(0, hi - lo + 1);
  }
  return ACCH_OK;
}

void make_layout(const acch_params &p0, const Plan &pl, BLayout &L) {
  const size_t n2 = 2 * (size_t)pl.ncell * sizeof(double);
  const int m = p0.gmres_restart;
  const size_t fsz = p0.precision == ACCH_PREC_MIXED ? sizeof(float) : sizeof(double);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L.off_Xn = take(n2);
  L.off_X = take(n2);
  L.off_Xt = take(n2);
  L.off_F = take(n2);
  L.off_Ft = take(n2);
  L.off_S = take(n2);
  L.off_W = take(n2);
  L.off_J = take((size_t)kNSlot2D * pl.ncell * sizeof(double));
  L.off_V = take((size_t)(m + 1) * n2);
  L.off_Z = take((size_t)m * n2);
  const size_t slots = (size_t)pl.G.nlev * pl.G.bh;
  L.off_fac = take(pl.box ? 0 : (size_t)pl.G.nsub * kNSlot2D * slots * fsz);
  const size_t brec = pl.box ? (size_t)pl.G.nsub * pl.bx.ncell * kBoxIluRec * fsz : 0;
  L.off_bxL = take(brec);
  L.off_bxU = take(brec);
  L.off_bxy = take(pl.box ? (size_t)pl.G.nsub * pl.bx.ncell * 2 * sizeof(double) : 0);
  L.off_bxlv = take(pl.bxlvoff.size() * sizeof(int));
  L.off_bxcell = take(pl.bxcellof.size() * sizeof(int));
  L.off_y = take((size_t)pl.G.nsub * 2 * (slots + 1) * fsz);
  L.off_dump = take(64 * sizeof(double));
  L.off_subs = take(pl.subs.size() * sizeof(SubInfo));
  L.off_lvl = take(pl.lvl.size() * sizeof(int));
  L.off_state = take((size_t)pl.count * sizeof(GmresState));
  // dot rows of the Arnoldi SpMV, then the Gram–Schmidt kernel's norm rows after them
  const size_t nparts = std::max<size_t>((size_t)kMaxRestart * pl.grid[kFamCell] + pl.grid[kFamElem],
                                         std::max<size_t>((size_t)(kMaxRestart + 1) * pl.grid[kFamCell],
                                                          std::max<size_t>(2 * (size_t)pl.grid[kFamTile],
                                                                           4 * (size_t)pl.grid[kFamElem])));
  L.off_part = take(nparts * sizeof(double));
  L.off_out = take((size_t)4 * pl.count * sizeof(double));
  L.off_inst = take((size_t)pl.count * sizeof(Inst));
  for (int f = 0; f < kFamilies; ++f) L.off_map[f] = take((size_t)pl.grid[f] * sizeof(int2));
  for (int k = 0; k < 3; ++k) L.off_mask[k] = take((size_t)pl.count * sizeof(int));
  L.off_lam = take((size_t)pl.count * sizeof(double));
  L.total = o;
}

}  // namespace

struct acch_batch {
  acch_params p{};          // batch-wide settings (instance 0)
  Plan pl;
  BLayout lay{};
  hipStream_t stream = nullptr;
  char *ws = nullptr;
  double *Xn, *X, *Xt, *F, *Ft, *S, *W, *J, *V, *Z, *dump, *out, *lam;
  void *fac, *ybuf;
  void *bxL = nullptr, *bxU = nullptr;   // box-pattern ILU(0) records
  double *bxy = nullptr;
  int *d_bxlv = nullptr, *d_bxcell = nullptr;
  SubInfo *d_subs;
  int *d_lvl;
  GmresState *st;
  int *mask[3];             // 0: Newton-active, 1: line-search trials, 2: GMRES cycle
  RedBuf red{};
  BatchLaunch all{}, newton{}, trial{}, cyc{};
  // pinned host mirrors
  char *pinned = nullptr;
  double *h_out, *h_lam;
  int *h_mask[3];
  GmresState *h_state;
  double t = 0.0;
  int use_graph = 1;
  bool graphs_ready = false;
  bool factored = false;
  std::vector<hipGraphExec_t> graphs;   // chunk c holds Arnoldi steps [c kChunk, (c+1) kChunk)
  long launches = 0, syncs = 0, graph_launches = 0;
};

namespace {

#define BLAUNCH(b, expr)                                                                                 \
  do {                                                                                                   \
    hipError_t e_ = (expr);                                                                              \
    (b)->launches++;                                                                                     \
    if (e_ != hipSuccess) return fail(ACCH_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

int bsync(acch_batch *b) {
  HIP_TRY(hipStreamSynchronize(b->stream));
  b->syncs++;
  return ACCH_OK;
}

int upload_mask(acch_batch *b, int k) {
  HIP_TRY(hipMemcpyAsync(b->mask[k], b->h_mask[k], b->pl.count * sizeof(int), hipMemcpyHostToDevice, b->stream));
  return ACCH_OK;
}

// out[4 i + k] of every instance to the host (synchronises).
int read_out(acch_batch *b) {
  HIP_TRY(hipMemcpyAsync(b->h_out, b->out, 4 * b->pl.count * sizeof(double), hipMemcpyDeviceToHost, b->stream));
  return bsync(b);
}

int read_states(acch_batch *b) {
  HIP_TRY(hipMemcpyAsync(b->h_state, b->st, b->pl.count * sizeof(GmresState), hipMemcpyDeviceToHost, b->stream));
  return bsync(b);
}

// z = M^{-1} r over every subdomain of the instances bl selects (left-restricted Schwarz).
hipError_t apply_m(acch_batch *b, const BatchLaunch &bl, const double *r, double *z, const GmresState *st, long vs,
                   int fp32) {
  if (b->pl.box)
    return launch_boxilu_apply2d(bl, b->pl.bx, b->pl.G, b->d_subs, b->d_bxcell, b->bxL, b->bxU, b->bxy, b->ybuf, r, z,
                                 st, vs, fp32, b->stream, RasVariant{});
  return launch_ras_apply2d(bl, b->pl.G, b->d_subs, b->d_lvl, b->fac, b->ybuf, r, z, b->dump, st, vs, fp32, b->stream);
}

int enqueue_steps(acch_batch *b, int j0, int j1, int fp32, long vs) {
  for (int j = j0; j < j1; ++j) {
    BLAUNCH(b, apply_m(b, b->cyc, b->V, b->Z, b->st, vs, fp32));
    BLAUNCH(b, launch_spmv_dots2d(b->cyc, b->J, b->Z, b->V, vs, j, 0, b->st, b->red, b->stream));
    BLAUNCH(b, launch_gmres_orth(b->cyc, b->V, vs, j, b->st, b->red, b->stream));
  }
  BLAUNCH(b, launch_gmres_update(b->cyc, b->S, b->Z, vs, b->st, 1, b->p.mass_projection > 0, b->red, b->stream));
  return ACCH_OK;
}

// Records the chunks of a cycle: chunk 0 also computes J S and starts the cycle.
int record_graphs(acch_batch *b) {
  const int m = b->p.gmres_restart;
  const long vs = 2 * b->pl.ncell;
  const int fp32 = b->p.precision == ACCH_PREC_MIXED;
  const int nchunk = (m + kChunk - 1) / kChunk;
  for (int c = 0; c < nchunk; ++c) {
    HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    int rc = ACCH_OK;
    if (c == 0) {
      hipError_t e = launch_spmv2d(b->cyc, b->J, b->S, b->W, 0, b->stream);
      if (e == hipSuccess)
        e = launch_gmres_start(b->cyc, b->F, b->W, b->V, b->st, m, b->p.gmres_rtol, b->p.gmres_atol, b->red,
                               b->stream);
      if (e != hipSuccess) rc = fail(ACCH_EDEVICE, std::string("graph start: ") + hipGetErrorString(e));
    }
    if (!rc) rc = enqueue_steps(b, c * kChunk, std::min(m, (c + 1) * kChunk), fp32, vs);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return fail(ACCH_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(ACCH_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    b->graphs.push_back(x);
  }
  b->graphs_ready = true;
  return ACCH_OK;
}

// Lockstep GMRES for the Newton-active instances: J S = -F per instance, S from 0.
int gmres_batch(acch_batch *b, std::vector<int> &its) {
  const int count = b->pl.count;
  const int m = b->p.gmres_restart;
  const long vs = 2 * b->pl.ncell;
  const int fp32 = b->p.precision == ACCH_PREC_MIXED;
  BLAUNCH(b, launch_reset_state(b->all, b->st, b->stream));
  BLAUNCH(b, launch_copy2(b->newton, b->S, nullptr, nullptr, nullptr, b->stream));
  for (int i = 0; i < count; ++i) b->h_mask[2][i] = b->h_mask[0][i];
  std::vector<int> total(count, 0);
  auto add_its = [&]() {
    for (int i = 0; i < count; ++i) its[i] += total[i];
  };
  if (b->use_graph && !b->graphs_ready) {
    int rc = record_graphs(b);
    if (rc) return rc;
  }
  for (int cycle = 0; cycle < b->p.gmres_max_restarts; ++cycle) {
    int rc = upload_mask(b, 2);
    if (rc) return rc;
    const int nchunk = (m + kChunk - 1) / kChunk;
    for (int c = 0; c < nchunk; ++c) {
      if (b->use_graph) {
        HIP_TRY(hipGraphLaunch(b->graphs[c], b->stream));
        b->graph_launches++;
      } else {
        if (c == 0) {
          BLAUNCH(b, launch_spmv2d(b->cyc, b->J, b->S, b->W, 0, b->stream));
          BLAUNCH(b, launch_gmres_start(b->cyc, b->F, b->W, b->V, b->st, m, b->p.gmres_rtol, b->p.gmres_atol,
                                        b->red, b->stream));
        }
        rc = enqueue_steps(b, c * kChunk, std::min(m, (c + 1) * kChunk), fp32, vs);
        if (rc) return rc;
      }
      rc = read_states(b);
      if (rc) return rc;
      bool all_done = true;
      for (int i = 0; i < count; ++i)
        if (b->h_mask[2][i] && !b->h_state[i].done) all_done = false;
      if (all_done) break;
    }
    bool all_conv = true;
    for (int i = 0; i < count; ++i) {
      if (!b->h_mask[2][i]) continue;
      const GmresState &g = b->h_state[i];
      if (!g.done) return fail(ACCH_EDIVERGED, "instance " + std::to_string(i) + ": GMRES cycle did not finish");
      total[i] = g.total_its;
      if (g.converged) {
        b->h_mask[2][i] = 0;
      } else {
        all_conv = false;
        if (!(g.resid == g.resid)) return fail(ACCH_EDIVERGED, "instance " + std::to_string(i) + ": GMRES residual is not finite");
      }
    }
    if (all_conv) {
      add_its();
      return ACCH_OK;
    }
  }
  add_its();
  return fail(ACCH_EDIVERGED, "GMRES did not converge within the restart limit");
}

// Residual of every instance selected by bl (trial state X + lam_i (S - shift_i e_u)
// when Sdir is given); f2/bad per instance in h_out[4 i], h_out[4 i + 1].
int residual_batch(acch_batch *b, const BatchLaunch &bl, const double *Sdir, double *Xt, double *F) {
  const GmresState *shift = (Sdir && b->p.mass_projection > 0) ? b->st : nullptr;
  BLAUNCH(b, launch_residual2d(bl, b->X, Sdir, 0.0, Sdir ? b->lam : nullptr, shift, b->Xn, b->p.dt_fixed, Xt, F,
                               b->red, b->stream));
  return read_out(b);
}

struct BStats {
  std::vector<int> newton, gmres;
};

int nks_batch(acch_batch *b, BStats &stats) {
  const int count = b->pl.count;
  const acch_params &p = b->p;
  HIP_TRY(hipMemcpyAsync(b->X, b->Xn, 2 * b->pl.ncell * sizeof(double), hipMemcpyDeviceToDevice, b->stream));
  int rc = residual_batch(b, b->all, nullptr, nullptr, b->F);
  if (rc) return rc;
  std::vector<double> fnorm(count), tol(count);
  for (int i = 0; i < count; ++i) {
    fnorm[i] = sqrt(b->h_out[4 * i]);
    if (!std::isfinite(fnorm[i])) return fail(ACCH_EDIVERGED, "instance " + std::to_string(i) + ": residual is not finite");
    tol[i] = std::max(p.newton_rtol * fnorm[i], p.newton_atol);
  }
  std::vector<LineSearch> ls(count);
  for (int it = 1;; ++it) {
    int nact = 0;
    for (int i = 0; i < count; ++i) {
      b->h_mask[0][i] = fnorm[i] > tol[i] ? 1 : 0;
      nact += b->h_mask[0][i];
    }
    if (nact == 0) return ACCH_OK;
    if (it > p.newton_max_it) return fail(ACCH_EDIVERGED, "Newton iteration limit reached");
    // counted before any early return, so a failed attempt's last iteration counts too
    for (int i = 0; i < count; ++i)
      if (b->h_mask[0][i]) stats.newton[i] = it;
    rc = upload_mask(b, 0);
    if (rc) return rc;
    BLAUNCH(b, launch_jacobian2d(b->newton, b->X, b->Xn, p.dt_fixed, b->J, b->stream));
    if (it == 1 || p.ilu_reuse < 0) {
      if (b->pl.box)
        BLAUNCH(b, launch_boxilu_factor2d(b->newton, b->pl.bx, b->pl.G.nsub, b->d_subs, b->d_bxlv, b->J, p.ilu_shift,
                                          b->bxL, b->bxU, p.precision == ACCH_PREC_MIXED, b->stream));
      else
        BLAUNCH(b, launch_ilu_factor2d(b->newton, b->pl.G, b->d_subs, b->d_lvl, b->J, p.ilu_shift, b->fac,
                                       p.precision == ACCH_PREC_MIXED, b->stream));
      b->factored = true;
    }
    rc = gmres_batch(b, stats.gmres);
    if (rc) return rc;
    // line searches of the active instances, in lockstep rounds
    for (int i = 0; i < count; ++i) {
      if (b->h_mask[0][i]) ls[i].start(fnorm[i]);
      else ls[i].state = LineSearch::kAccepted;
    }
    while (true) {
      int ntrial = 0;
      for (int i = 0; i < count; ++i) {
        const bool on = b->h_mask[0][i] && ls[i].state == LineSearch::kSearching;
        b->h_mask[1][i] = on ? 1 : 0;
        b->h_lam[i] = ls[i].lam;
        ntrial += on;
      }
      if (ntrial == 0) break;
      rc = upload_mask(b, 1);
      if (rc) return rc;
      HIP_TRY(hipMemcpyAsync(b->lam, b->h_lam, count * sizeof(double), hipMemcpyHostToDevice, b->stream));
      rc = residual_batch(b, b->trial, b->S, b->Xt, b->Ft);
      if (rc) return rc;
      for (int i = 0; i < count; ++i)
        if (b->h_mask[1][i]) ls[i].trial(b->h_out[4 * i], b->h_out[4 * i + 1]);
    }
    for (int i = 0; i < count; ++i)
      if (b->h_mask[0][i] && ls[i].state != LineSearch::kAccepted)
        return fail(ACCH_EDIVERGED, "instance " + std::to_string(i) + ": line search failed");
    BLAUNCH(b, launch_copy2(b->newton, b->X, b->Xt, b->F, b->Ft, b->stream));
    for (int i = 0; i < count; ++i) {
      if (!b->h_mask[0][i]) continue;
      fnorm[i] = sqrt(ls[i].f2);
      if (!std::isfinite(fnorm[i])) return fail(ACCH_EDIVERGED, "instance " + std::to_string(i) + ": residual is not finite");
    }
  }
}

}  // namespace

extern "C" int acch_batch_workspace_bytes(const acch_params *inst, int count, size_t *bytes) {
  if (!inst || !bytes) return fail(ACCH_EINVAL, "null argument");
  Plan pl;
  int rc = make_plan(inst, count, pl);
  if (rc) return rc;
  acch_params p0 = inst[0];
  acch_params_default(&p0);
  BLayout L;
  make_layout(p0, pl, L);
  *bytes = L.total;
  return ACCH_OK;
}

extern "C" int acch_batch_create(const acch_params *inst, int count, const double *const *u0,
                                 const double *const *v0, acch_batch **out) {
  if (!inst || !u0 || !v0 || !out) return fail(ACCH_EINVAL, "null argument");
  *out = nullptr;
  acch_batch *b = new (std::nothrow) acch_batch();
  if (!b) return fail(ACCH_EINVAL, "host allocation failed");
  int rc = make_plan(inst, count, b->pl);
  if (rc) {
    delete b;
    return rc;
  }
  b->p = inst[0];
  acch_params_default(&b->p);
  make_layout(b->p, b->pl, b->lay);
  const BLayout &L = b->lay;
  if (!b->p.workspace || b->p.workspace_bytes < L.total || ((uintptr_t)b->p.workspace) % kAlign) {
    delete b;
    return fail(ACCH_EINVAL, "workspace missing, misaligned or smaller than acch_batch_workspace_bytes()");
  }
  for (int i = 0; i < count; ++i) {
    const long n = (long)b->pl.inst[i].P.nx * b->pl.inst[i].P.ny;
    if (!u0[i] || !v0[i]) {
      delete b;
      return fail(ACCH_EINVAL, "null initial field");
    }
    for (long k = 0; k < n; ++k) {
      const double pp = u0[i][k] + v0[i][k], q = u0[i][k] - v0[i][k];
      if (!(pp > 0.0 && pp < 1.0 && q > 0.0 && q < 1.0)) {
        delete b;
        return fail(ACCH_EDOMAIN, "instance " + std::to_string(i) + ": initial state outside the admissible set");
      }
    }
  }
  b->stream = (hipStream_t)b->p.stream;
  b->ws = (char *)b->p.workspace;
  char *w = b->ws;
  b->Xn = (double *)(w + L.off_Xn);
  b->X = (double *)(w + L.off_X);
  b->Xt = (double *)(w + L.off_Xt);
  b->F = (double *)(w + L.off_F);
  b->Ft = (double *)(w + L.off_Ft);
  b->S = (double *)(w + L.off_S);
  b->W = (double *)(w + L.off_W);
  b->J = (double *)(w + L.off_J);
  b->V = (double *)(w + L.off_V);
  b->Z = (double *)(w + L.off_Z);
  b->fac = w + L.off_fac;
  b->ybuf = w + L.off_y;
  if (b->pl.box) {
    b->bxL = w + L.off_bxL;
    b->bxU = w + L.off_bxU;
    b->bxy = (double *)(w + L.off_bxy);
    b->d_bxlv = (int *)(w + L.off_bxlv);
    b->d_bxcell = (int *)(w + L.off_bxcell);
  }
  b->dump = (double *)(w + L.off_dump);
  b->d_subs = (SubInfo *)(w + L.off_subs);
  b->d_lvl = (int *)(w + L.off_lvl);
  b->st = (GmresState *)(w + L.off_state);
  b->red.partials = (double *)(w + L.off_part);
  b->red.counter = nullptr;
  b->red.out = b->out = (double *)(w + L.off_out);
  b->lam = (double *)(w + L.off_lam);
  Inst *d_inst = (Inst *)(w + L.off_inst);
  for (int k = 0; k < 3; ++k) b->mask[k] = (int *)(w + L.off_mask[k]);
  BatchLaunch base{};
  base.count = count;
  base.ncell = b->pl.ncell;
  base.bt.inst = d_inst;
  for (int f = 0; f < kFamilies; ++f) {
    base.grid[f] = b->pl.grid[f];
    base.bt.map[f] = (const int2 *)(w + L.off_map[f]);
  }
  b->all = b->newton = b->trial = b->cyc = base;
  b->newton.bt.active = b->mask[0];
  b->trial.bt.active = b->mask[1];
  b->cyc.bt.active = b->mask[2];
  const size_t pin = 4 * count * sizeof(double) + count * sizeof(double) + 3 * count * sizeof(int) +
                     count * sizeof(GmresState) + 256;
  if (hipHostMalloc((void **)&b->pinned, pin, hipHostMallocDefault) != hipSuccess) {
    delete b;
    return fail(ACCH_EDEVICE, "hipHostMalloc failed");
  }
  char *h = b->pinned;
  b->h_state = (GmresState *)h;
  h += count * sizeof(GmresState);
  b->h_out = (double *)h;
  h += 4 * count * sizeof(double);
  b->h_lam = (double *)h;
  h += count * sizeof(double);
  for (int k = 0; k < 3; ++k) {
    b->h_mask[k] = (int *)h;
    h += count * sizeof(int);
  }
  auto cleanup = [&](int code) {
    (void)hipHostFree(b->pinned);
    delete b;
    return code;
  };
  bool ok = hipMemcpyAsync(d_inst, b->pl.inst.data(), count * sizeof(Inst), hipMemcpyHostToDevice, b->stream) ==
                hipSuccess &&
            hipMemcpyAsync(b->d_subs, b->pl.subs.data(), b->pl.subs.size() * sizeof(SubInfo), hipMemcpyHostToDevice,
                           b->stream) == hipSuccess &&
            hipMemcpyAsync(b->d_lvl, b->pl.lvl.data(), b->pl.lvl.size() * sizeof(int), hipMemcpyHostToDevice,
                           b->stream) == hipSuccess &&
            hipMemsetAsync(b->st, 0, count * sizeof(GmresState), b->stream) == hipSuccess &&
            (!b->pl.box || (hipMemcpyAsync(b->d_bxlv, b->pl.bxlvoff.data(), b->pl.bxlvoff.size() * sizeof(int),
                                           hipMemcpyHostToDevice, b->stream) == hipSuccess &&
                            hipMemcpyAsync(b->d_bxcell, b->pl.bxcellof.data(), b->pl.bxcellof.size() * sizeof(int),
                                           hipMemcpyHostToDevice, b->stream) == hipSuccess));
  for (int f = 0; ok && f < kFamilies; ++f)
    ok = hipMemcpyAsync((void *)base.bt.map[f], b->pl.map[f].data(), b->pl.map[f].size() * sizeof(int2),
                        hipMemcpyHostToDevice, b->stream) == hipSuccess;
  for (int i = 0; ok && i < count; ++i) {
    const Inst &I = b->pl.inst[i];
    const long n = (long)I.P.nx * I.P.ny;
    ok = hipMemcpyAsync(b->Xn + I.xoff, u0[i], n * sizeof(double), hipMemcpyHostToDevice, b->stream) == hipSuccess &&
         hipMemcpyAsync(b->Xn + I.xoff + n, v0[i], n * sizeof(double), hipMemcpyHostToDevice, b->stream) ==
             hipSuccess;
  }
  if (!ok || hipStreamSynchronize(b->stream) != hipSuccess) return cleanup(fail(ACCH_EDEVICE, "initial upload failed"));
  *out = b;
  return ACCH_OK;
}

extern "C" int acch_batch_step(acch_batch *b, int nsteps, int *newton_its, int *gmres_its) {
  if (!b || nsteps < 0) return fail(ACCH_EINVAL, "bad arguments");
  const int count = b->pl.count;
  for (int s = 0; s < nsteps; ++s) {
    BStats st;
    st.newton.assign(count, 0);
    st.gmres.assign(count, 0);
    int rc = nks_batch(b, st);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(b->Xn, b->X, 2 * b->pl.ncell * sizeof(double), hipMemcpyDeviceToDevice, b->stream));
    b->t += b->p.dt_fixed;
    for (int i = 0; i < count; ++i) {
      if (newton_its) newton_its[i] += st.newton[i];
      if (gmres_its) gmres_its[i] += st.gmres[i];
    }
  }
  return bsync(b);
}

extern "C" int acch_batch_energy(acch_batch *b, double *energy, double *mass) {
  if (!b) return fail(ACCH_EINVAL, "null batch");
  BLAUNCH(b, launch_energy2d(b->all, b->Xn, b->red, b->stream));
  int rc = read_out(b);
  if (rc) return rc;
  for (int i = 0; i < b->pl.count; ++i) {
    const Phys &P = b->pl.inst[i].P;
    const double vol = 1.0 / sqrt(P.wx * P.wy);
    if (energy) energy[i] = b->h_out[4 * i] * vol;
    if (mass) mass[i] = b->h_out[4 * i + 1] * vol;
  }
  return ACCH_OK;
}

extern "C" int acch_batch_get_fields(acch_batch *b, int i, double *u, double *v) {
  if (!b || !u || !v || i < 0 || i >= b->pl.count) return fail(ACCH_EINVAL, "bad arguments");
  const Inst &I = b->pl.inst[i];
  const long n = (long)I.P.nx * I.P.ny;
  HIP_TRY(hipMemcpyAsync(u, b->Xn + I.xoff, n * sizeof(double), hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipMemcpyAsync(v, b->Xn + I.xoff + n, n * sizeof(double), hipMemcpyDeviceToHost, b->stream));
  return bsync(b);
}

extern "C" int acch_batch_precondition(acch_batch *b, const double *r, double *z) {
  if (!b || !r || !z) return fail(ACCH_EINVAL, "bad arguments");
  if (!b->factored) return fail(ACCH_EINVAL, "no factorisation yet: take a step first");
  BLAUNCH(b, apply_m(b, b->all, r, z, nullptr, 0, b->p.precision == ACCH_PREC_MIXED));
  return ACCH_OK;
}

extern "C" int acch_batch_info(acch_batch *b, long *ncell, int *nsub, int *box_w, int *box_h, long *xoff) {
  if (!b) return fail(ACCH_EINVAL, "null batch");
  if (ncell) *ncell = b->pl.ncell;
  if (nsub) *nsub = b->pl.G.nsub;
  if (box_w) *box_w = b->pl.G.bw;
  if (box_h) *box_h = b->pl.G.bh;
  if (xoff)
    for (int i = 0; i < b->pl.count; ++i) xoff[i] = b->pl.inst[i].xoff;
  return ACCH_OK;
}

extern "C" int acch_batch_set_option(acch_batch *b, int option, long value) {
  if (!b) return fail(ACCH_EINVAL, "null batch");
  if (option == ACCH_BATCH_OPT_GRAPH) {
    b->use_graph = value != 0;
    if (b->use_graph && !b->graphs_ready) return record_graphs(b);
    return ACCH_OK;
  }
  return fail(ACCH_EINVAL, "unknown batch option");
}

extern "C" int acch_batch_counters(acch_batch *b, long *launches, long *graph_launches, long *syncs) {
  if (!b) return fail(ACCH_EINVAL, "null batch");
  if (launches) *launches = b->launches;
  if (graph_launches) *graph_launches = b->graph_launches;
  if (syncs) *syncs = b->syncs;
  return ACCH_OK;
}

extern "C" int acch_batch_destroy(acch_batch *b) {
  if (!b) return ACCH_OK;
  (void)hipStreamSynchronize(b->stream);
  for (hipGraphExec_t g : b->graphs) (void)hipGraphExecDestroy(g);
  (void)hipHostFree(b->pinned);
  delete b;
  return ACCH_OK;
}
