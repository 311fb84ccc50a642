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
int schwarz_waves(const BoxGeom &G);
void set_ras_prefetch(int d);
int get_ras_prefetch();

// stencil2d.hip
hipError_t launch_residual2d(const Phys &P, const double *X, const double *Sdir, double lam, const double *shift,
                             const double *Xn, double dt, double *Xt, double *F, const RedBuf &red, hipStream_t s);
hipError_t launch_energy2d(const Phys &P, const double *X, const RedBuf &red, hipStream_t s);
hipError_t launch_jacobian2d(const Phys &P, const double *X, const double *Xn, double dt, double *J, hipStream_t s);
hipError_t launch_spmv2d(const Phys &P, const double *J, const double *x, double *y, hipStream_t s);
hipError_t launch_spmv_dots2d(const Phys &P, const double *J, const double *Z, double *V, long vstride,
                              GmresState *st, const RedBuf &red, hipStream_t s);

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
hipError_t launch_gmres_orth(long n2, double *V, long vstride, GmresState *st, const RedBuf &red, hipStream_t s);
hipError_t launch_gmres_update(long ncell, double *S, const double *Z, long vstride, GmresState *st, int accumulate,
                               int project, const RedBuf &red, hipStream_t s);
hipError_t launch_norm2_diff(long n2, const double *a, const double *b, const RedBuf &red, hipStream_t s);
hipError_t launch_reset_state(GmresState *st, hipStream_t s);

}  // namespace acch
