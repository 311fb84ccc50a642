// Host-side launchers of the acch HIP kernels (one stream-ordered launch each).
#pragma once

#include "band.h"
#include "boxilu.h"
#include "common.h"

namespace acch {

int reduce_blocks(long n);

// A launch over one instance (null maps in bt) or over a whole batch.
struct BatchLaunch {
  Phys P0;               // the instance of a single-instance launch
  Batch bt;              // device description (maps null for one instance)
  int grid[kFamilies];   // blocks of each family over the launch
  int count;             // instances
  long ncell;            // cells of a single instance
};
BatchLaunch single_launch(const Phys &P, int nsub);
// Blocks of each family for one instance (tiles, cells, elements, subdomains).
void family_blocks(const Phys &P, int nsub, int (&nb)[kFamilies]);

// Second stage of the two-kernel reductions (krylov.hip): one block per instance,
// out[4 b + k] for kFinPlain.
enum { kFinPlain = 0, kFinStart = 1, kFinOrth = 3, kFinUpdate = 4 };
struct FinalizeArgs {
  int m, project;
  double rtol, atol;
  long ncell;
};
hipError_t launch_finalize(int mode, int nv, const RedBuf &red, const BatchLaunch &bl, int fam, GmresState *st,
                           const FinalizeArgs &fa, hipStream_t s);
int schwarz_waves(const BoxGeom &G);
void set_ras_prefetch(int d);
int get_ras_prefetch();
void set_ras3d_window(bool on);
// 3D windowed Schwarz apply: threads per box and box columns (j, k) per thread.  The
// host lists each thread's columns after the level-ordered cells, in order and then
// in reverse ([2][kWin3DCols][kWin3DThreads], -1 unused; wmax = 0: no list), then
// the thread owning each column (bh * bd ints, index j + bh k).
constexpr int kWin3DThreads = 512;
constexpr int kWin3DCols = 8;
constexpr int kWin3DSlots = 40;   // factor values per cell (3D)
// Threads of the windowed apply = row width of its level-major arrays (0: no window).
__host__ __device__ inline int win3d_row(const BoxGeom &G) { return G.wmax > 0 ? (G.wmax + 63) / 64 * 64 : 0; }
// Level-major factor copy of the windowed apply: [sub][level][slot][row] (elements).
inline size_t win3d_fac_elems(const BoxGeom &G) {
  return (size_t)G.nsub * G.nlev * kWin3DSlots * win3d_row(G);
}
// 3D box-buffer pairs: cell-ordered boxes of the general apply, or the level-major
// rows of the windowed one, whichever is larger; one spare pair follows.
inline size_t box3_ypairs(const BoxGeom &G) {
  const size_t a = (size_t)G.nsub * G.ncb, b = (size_t)G.nsub * G.nlev * win3d_row(G);
  return a > b ? a : b;
}

// stencil2d.hip.  lam_b (per instance, may be null: lam0) and shift_st (the mass
// shift of each instance's GMRES state, may be null) describe the trial state.
hipError_t launch_residual2d(const BatchLaunch &bl, const double *X, const double *Sdir, double lam0,
                             const double *lam_b, const GmresState *shift_st, const double *Xn, double dt, double *Xt,
                             double *F, const RedBuf &red, hipStream_t s);
hipError_t launch_energy2d(const BatchLaunch &bl, const double *X, const RedBuf &red, hipStream_t s);
hipError_t launch_jacobian2d(const BatchLaunch &bl, const double *X, const double *Xn, double dt, double *J,
                             hipStream_t s);
// y = J x, or J^T x when transpose
hipError_t launch_spmv2d(const BatchLaunch &bl, const double *J, const double *x, double *y, int transpose,
                         hipStream_t s);
// Arnoldi step j of the cycle (the device state's j must equal it unless the cycle is done);
// the block partials of the dots are summed by the Gram–Schmidt kernel of the step
hipError_t launch_spmv_dots2d(const BatchLaunch &bl, const double *J, const double *Z, double *V, long vstride, int j,
                              int transpose, GmresState *st, const RedBuf &red, hipStream_t s);

// schwarz2d.hip (subs: every subdomain of the launch, in block order)
hipError_t launch_ilu_factor2d(const BatchLaunch &bl, const BoxGeom &G, const SubInfo *subs, const int *lvl,
                               const double *J, double shift, void *fac, int fp32, hipStream_t s);
// Schwarz variant (ACCH_RAS_LEFT / ACCH_RAS_RIGHT / ACCH_AS_CLASSICAL); the last two
// add whole boxes and need the owner maps (single-instance launches only).
struct RasVariant {
  int kind = 0;
  const int *own_x = nullptr, *own_y = nullptr;   // 3D: own_x is the whole x | y | z owner map
  int px = 0, py = 0, pz = 1;
};
hipError_t launch_ras_apply2d(const BatchLaunch &bl, const BoxGeom &G, const SubInfo *subs, const int *lvl,
                              const void *fac, void *ybuf, const double *r, double *z, double *dump,
                              const GmresState *st, long vstride, int fp32, hipStream_t s,
                              const RasVariant &rv = RasVariant{});
hipError_t launch_export_factors2d(const BoxGeom &G, const int *lvl, const void *fac, int fp32, double *out,
                                   hipStream_t s);
// z = sum over the boxes holding each cell of their values in the box buffer (the
// extension of the right-restricted and classical variants; single instance)
hipError_t launch_ras_sum2d(const BatchLaunch &bl, const BoxGeom &G, const SubInfo *subs, const void *ybuf, double *z,
                            const GmresState *st, long vstride, int fp32, hipStream_t s, const RasVariant &rv);

// bandlu2d.hip: the exact-LU / ILU(k) subdomain solvers in band storage (band.h),
// single instance.  mask: the ILU(k) pattern, n * mwords words per box (null: exact LU).
hipError_t launch_band_factor2d(const BatchLaunch &bl, const BandGeom &B, int nsub, const SubInfo *subs,
                                const double *J, double shift, const unsigned *mask, void *band, int fp32,
                                hipStream_t s);
// z = M^{-1} r with the band factors; ybox: nchunk * 64 doubles per box; boxbuf: the
// box buffer of the right-restricted / classical variants (layout of launch_ras_apply2d)
hipError_t launch_band_apply2d(const BatchLaunch &bl, const BandGeom &B, const BoxGeom &G, const SubInfo *subs,
                               const void *band, double *ybox, void *boxbuf, const double *r, double *z,
                               const GmresState *st, long vstride, int fp32, hipStream_t s, const RasVariant &rv);
hipError_t launch_band_export(const BandGeom &B, int nsub, const void *band, int fp32, double *out, hipStream_t s);

// boxilu2d.hip: ILU(0) on the width-2 box pattern (boxilu.h); L, U: nsub * ncell * 52
// FT records each; ybox: nsub * ncell (u, v) pairs; boxbuf as for the band solve; lvoff:
// the wavefront offsets; cellof: box cell (j << 16 | i) of each record position.
bool boxilu_fits(const BoxIluGeom &X);
hipError_t launch_boxilu_factor2d(const BatchLaunch &bl, const BoxIluGeom &X, int nsub, const SubInfo *subs,
                                  const int *lvoff, const double *J, double shift, void *L, void *U, int fp32,
                                  hipStream_t s);
hipError_t launch_boxilu_apply2d(const BatchLaunch &bl, const BoxIluGeom &X, const BoxGeom &G, const SubInfo *subs,
                                 const int *cellof, const void *L, const void *U, double *ybox, void *boxbuf,
                                 const double *r, double *z, const GmresState *st, long vstride, int fp32,
                                 hipStream_t s, const RasVariant &rv, bool trans = false);
// Transposed records (Tf for the U^T sweep, Tb for the L^T sweep), same layout and size as L, U.
hipError_t launch_boxilu_pack_t(const BoxIluGeom &X, int nsub, const int *lvoff, const int *cellof, const void *L,
                                const void *U, void *Tf, void *Tb, int fp32, hipStream_t s);
hipError_t launch_boxilu_export(const BoxIluGeom &X, int nsub, const int *lvoff, const void *L, const void *U,
                                int fp32, double *out, hipStream_t s);

// krylov.hip
hipError_t launch_gmres_start(const BatchLaunch &bl, const double *F, const double *JS, double *V0, GmresState *st,
                              int m, double rtol, double atol, const RedBuf &red, hipStream_t s);
hipError_t launch_gmres_orth(const BatchLaunch &bl, double *V, long vstride, int j, GmresState *st,
                             const RedBuf &red, hipStream_t s);
hipError_t launch_gmres_update(const BatchLaunch &bl, double *S, const double *Z, long vstride, GmresState *st,
                               int accumulate, int project, const RedBuf &red, hipStream_t s);
hipError_t launch_norm2_diff(const BatchLaunch &bl, const double *a, const double *b, const RedBuf &red,
                             hipStream_t s);
hipError_t launch_reset_state(const BatchLaunch &bl, GmresState *st, hipStream_t s);
// d1 = s1 (d1 = 0 when s1 is null) and d2 = s2 (if d2) on the active instances; a
// kernel, so it may be part of a captured graph.
hipError_t launch_copy2(const BatchLaunch &bl, double *d1, const double *s1, double *d2, const double *s2,
                        hipStream_t s);

// z = M^{-T} r (the transpose of the variant rv.kind with the current factors, one
// instance): fact holds the transposed records, filled from fac unless *packed (set
// once filled); ybuf / dump as for launch_ras_apply2d.
hipError_t launch_ras_t_apply2d(const BatchLaunch &bl, const BoxGeom &G, const SubInfo *subs, const int *lvl,
                                const void *fac, void *fact, bool *packed, void *ybuf, const double *r, double *z,
                                double *dump, const GmresState *st, long vstride, int fp32, hipStream_t s,
                                const RasVariant &rv);
// adjoint2d.hip
// out = (dF/dU^n)^T (lam_scale lam) at (X1; X0, dt); bar is a 2n scratch; red.out[0..3]
// receives (lam_scale lam) . dF/dp for p = alpha, beta, theta, gamma.
hipError_t launch_adjoint_prev2d(const Phys &P, const double *X1, const double *X0, double dt, const double *lam,
                                 double lam_scale, double *bar, double *out, const RedBuf &red, hipStream_t s);
// g = dE~/dX at X; red.out[0..3] = dE~/d(alpha, beta, theta, gamma).
hipError_t launch_energy_grad2d(const Phys &P, const double *X, double vol, double *g, const RedBuf &red,
                                hipStream_t s);

// stencil3d.hip / schwarz3d.hip (single instance; cells listed per level in `cells`)
// Q: scratch of 3 (residual) / 8 (Jacobian) FP64 values per cell
hipError_t launch_residual3d(const BatchLaunch &bl, const double *X, const double *Sdir, double lam,
                             const GmresState *shift_st, const double *Xn, double dt, double *Xt, double *F,
                             double *Q, const RedBuf &red, hipStream_t s);
hipError_t launch_energy3d(const BatchLaunch &bl, const double *X, const RedBuf &red, hipStream_t s);
hipError_t launch_jacobian3d(const BatchLaunch &bl, const double *X, const double *Xn, double dt, double *J,
                             double *Q, hipStream_t s);
hipError_t launch_spmv3d(const BatchLaunch &bl, const double *J, const double *x, double *y, int transpose,
                         hipStream_t s);
hipError_t launch_spmv_dots3d(const BatchLaunch &bl, const double *J, const double *Z, double *V, long vstride, int j,
                              int transpose, GmresState *st, const RedBuf &red, hipStream_t s);
hipError_t launch_adjoint_prev3d(const Phys &P, const double *X1, const double *X0, double dt, const double *lam,
                                 double lam_scale, double *bar, double *out, const RedBuf &red, hipStream_t s);
hipError_t launch_energy_grad3d(const Phys &P, const double *X, double vol, double *g, const RedBuf &red,
                                hipStream_t s);
// wfac (may be null): also fill the level-major copy of the windowed apply
hipError_t launch_ilu_factor3d(const Phys &P, const BoxGeom &G, const SubInfo *subs, const int *lvl, const int *cells,
                               const double *J, double shift, void *fac, void *wfac, int fp32, hipStream_t s);
// rv: the Schwarz variant; right-restricted and classical run the box-buffer sweeps and
// sum the boxes of each cell (owner maps in rv.own_x: x, then y, then z)
hipError_t launch_ras_apply3d(const Phys &P, const BoxGeom &G, const SubInfo *subs, const int *lvl, const int *cells,
                              const void *fac, const void *wfac, void *ybuf, const double *r, double *z,
                              const GmresState *st, long vstride, int fp32, hipStream_t s, const RasVariant &rv);
// wfact (may be null): transposed-record copy of the windowed form, filled from fac
// unless *packed (set once filled); tbox: 2 ncb doubles per box
hipError_t launch_ras_t_apply3d(const Phys &P, const BoxGeom &G, const SubInfo *subs, const int *lvl,
                                const int *cells, int px, int py, int pz, const int *own, const void *fac,
                                void *wfact, bool *packed, void *ybuf, double *tbox, const double *r, double *z,
                                const GmresState *st, long vstride, int fp32, hipStream_t s);
hipError_t launch_export_factors3d(const BoxGeom &G, const void *fac, int fp32, double *out, hipStream_t s);

}  // namespace acch
