// Host-side launchers of the acch HIP kernels (one stream-ordered launch each).
#pragma once

#include "common.h"

namespace acch {

int reduce_blocks(long n);

// Second stage of the two-kernel reductions (krylov.hip).
enum { kFinPlain = 0, kFinStart = 1, kFinDots = 2, kFinOrth = 3, kFinUpdate = 4 };
struct FinalizeArgs {
  int first, m, project;
  double rtol, atol;
  long ncell;
};
hipError_t launch_finalize(int mode, int nv, const RedBuf &red, int nblocks, GmresState *st, const FinalizeArgs &fa,
                           hipStream_t s);
// second stage of the Arnoldi dots of step j (0 <= j < kMaxRestart)
hipError_t launch_finalize_dots(int j, const RedBuf &red, int nblocks, GmresState *st, hipStream_t s);
int schwarz_waves(const BoxGeom &G);
void set_ras_prefetch(int d);
int get_ras_prefetch();

// stencil2d.hip
hipError_t launch_residual2d(const Phys &P, const double *X, const double *Sdir, double lam, const double *shift,
                             const double *Xn, double dt, double *Xt, double *F, const RedBuf &red, hipStream_t s);
hipError_t launch_energy2d(const Phys &P, const double *X, const RedBuf &red, hipStream_t s);
hipError_t launch_jacobian2d(const Phys &P, const double *X, const double *Xn, double dt, double *J, hipStream_t s);
// y = J x, or J^T x when transpose
hipError_t launch_spmv2d(const Phys &P, const double *J, const double *x, double *y, int transpose, hipStream_t s);
// Arnoldi step j of the cycle (the device state's j must equal it unless the cycle is done)
hipError_t launch_spmv_dots2d(const Phys &P, const double *J, const double *Z, double *V, long vstride, int j,
                              int transpose, GmresState *st, const RedBuf &red, hipStream_t s);

// schwarz2d.hip
hipError_t launch_ilu_factor2d(const BoxGeom &G, const SubInfo *subs, const int *lvl, int nx, int ny, int periodic,
                               const double *J, double shift, void *fac, int fp32, hipStream_t s);
hipError_t launch_ras_apply2d(const BoxGeom &G, const SubInfo *subs, const int *lvl, int nx, int ny, int periodic,
                              const void *fac, void *ybuf, const double *r, double *z, double *dump,
                              const GmresState *st, long vstride, int fp32, hipStream_t s);
hipError_t launch_export_factors2d(const BoxGeom &G, const int *lvl, const void *fac, int fp32, double *out,
                                   hipStream_t s);

// krylov.hip
hipError_t launch_gmres_start(long n2, const double *F, const double *JS, double *V0, GmresState *st, int m,
                              double rtol, double atol, const RedBuf &red, hipStream_t s);
hipError_t launch_gmres_orth(long n2, double *V, long vstride, int j, GmresState *st, const RedBuf &red,
                             hipStream_t s);
hipError_t launch_gmres_update(long ncell, double *S, const double *Z, long vstride, GmresState *st, int accumulate,
                               int project, const RedBuf &red, hipStream_t s);
hipError_t launch_norm2_diff(long n2, const double *a, const double *b, const RedBuf &red, hipStream_t s);
hipError_t launch_reset_state(GmresState *st, hipStream_t s);

// adjoint2d.hip
// z = M^{-T} r (the transposed left-restricted Schwarz operator with the current
// factors); box is a scratch of nsub * 2 * bw * bh doubles; own_x / own_y give the
// owner subdomain index of each grid column / row.
hipError_t launch_ras_t_apply2d(const BoxGeom &G, const SubInfo *subs, int nx, int ny, int periodic, int px, int py,
                                const int *own_x, const int *own_y, const void *fac, double *box, const double *r,
                                double *z, const GmresState *st, long vstride, int fp32, hipStream_t s);
// out = (dF/dU^n)^T (lam_scale lam) at (X1; X0, dt); bar is a 2n scratch; red.out[0..3]
// receives (lam_scale lam) . dF/dp for p = alpha, beta, theta, gamma.
hipError_t launch_adjoint_prev2d(const Phys &P, const double *X1, const double *X0, double dt, const double *lam,
                                 double lam_scale, double *bar, double *out, const RedBuf &red, hipStream_t s);
// g = dE~/dX at X; red.out[0..3] = dE~/d(alpha, beta, theta, gamma).
hipError_t launch_energy_grad2d(const Phys &P, const double *X, double vol, double *g, const RedBuf &red,
                                hipStream_t s);

}  // namespace acch
