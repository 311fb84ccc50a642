// Restarted flexible GMRES kernels (Section 3.1: right-preconditioned GMRES for
// J H^{-1} (H S) = -F).  The basis vectors are stored unnormalised (W_i) with
// v_i = inv_norm[i] W_i, so no separate normalisation pass is needed; the
// preconditioned vectors z_j = M^{-1} v_j are kept (flexible variant), which makes
// x = Z y valid also for the single-precision preconditioner.  Every kernel of an
// Arnoldi step returns at once when the cycle is finished, so the host may enqueue
// several steps ahead of its convergence check.
#include <math.h>

#include "kernels.h"

namespace acch {
namespace {

// V_0 = -(F + J S) (J S computed by the caller into JS, or absent on the first
// cycle) and beta = ||V_0||; the last block starts the cycle.
// On the first cycle the absolute tolerance becomes max(rtol * beta, atol); later
// cycles keep it.
__global__ __launch_bounds__(256) void k_gmres_start(long n2, const double *__restrict__ F,
                                                      const double *__restrict__ JS, double *__restrict__ V0,
                                                      GmresState *st, int m, double rtol, double atol, RedBuf red) {
  double acc[1] = {0.0};
  for (long e = blockIdx.x * 256L + threadIdx.x; e < n2; e += (long)gridDim.x * 256) {
    const double r = JS ? -(F[e] + JS[e]) : -F[e];
    V0[e] = r;
    acc[0] = fma(r, r, acc[0]);
  }
  block_partial<1>(acc, red.partials, threadIdx.x, 256, blockIdx.x, gridDim.x);
}

ACCH_DEV void start_tail(GmresState *st, double sum, int first, int m, double rtol, double atol) {
  const double beta = sqrt(sum);
  st->beta = beta;
  if (first) st->tol = fmax(rtol * beta, atol);
  const double tol = st->tol;
  st->m = m;
  st->j = 0;
  st->g[0] = beta;
  st->resid = beta;
  st->inv_norm[0] = beta > 0.0 ? 1.0 / beta : 0.0;
  st->converged = (beta <= tol) ? 1 : 0;
  st->done = st->converged;
}

// W_{j+1} -= sum_{i<=j} h_ij v_i (classical Gram–Schmidt, one pass), then the norm,
// the Givens update of the Hessenberg column and the convergence test.
__global__ __launch_bounds__(256) void k_gmres_orth(long n2, double *__restrict__ V, long vstride, GmresState *st,
                                                     RedBuf red) {
  if (st->done) return;
  const int j = st->j;
  __shared__ double coef[kMaxRestart + 1];
  if (threadIdx.x <= j) coef[threadIdx.x] = st->hcol[threadIdx.x] * st->inv_norm[threadIdx.x];
  __syncthreads();
  double *w = V + (long)(j + 1) * vstride;
  double acc[1] = {0.0};
  for (long e = blockIdx.x * 256L + threadIdx.x; e < n2; e += (long)gridDim.x * 256) {
    double x = w[e];
    for (int i = 0; i <= j; ++i) x = fma(-coef[i], V[(long)i * vstride + e], x);
    w[e] = x;
    acc[0] = fma(x, x, acc[0]);
  }
  block_partial<1>(acc, red.partials, threadIdx.x, 256, blockIdx.x, gridDim.x);
}

// The serial part of an Arnoldi step (one thread): Hessenberg column, Givens
// rotations, residual estimate, stopping test and, at the end of a cycle, y.
ACCH_DEV void orth_tail(GmresState *st, double sum) {
  const int j = st->j;
  const double hn = sqrt(sum);
  const int M1 = kMaxRestart + 1;
  // new Hessenberg column: the dots, then ||w||; apply the previous rotations
  double *h = st->H + j * M1;
  for (int i = 0; i <= j; ++i) h[i] = st->hcol[i];
  double hj1 = hn;
  for (int i = 0; i < j; ++i) {
    const double a = h[i], b = h[i + 1];
    h[i] = st->cs[i] * a + st->sn[i] * b;
    h[i + 1] = -st->sn[i] * a + st->cs[i] * b;
  }
  const double rr = hypot(h[j], hj1);
  double c = 1.0, s = 0.0;
  if (rr > 0.0) {
    c = h[j] / rr;
    s = hj1 / rr;
  }
  st->cs[j] = c;
  st->sn[j] = s;
  h[j] = rr;
  const double gj = st->g[j];
  st->g[j] = c * gj;
  st->g[j + 1] = -s * gj;
  const double resid = fabs(st->g[j + 1]);
  st->resid = resid;
  const int jn = j + 1;
  st->j = jn;
  st->total_its += 1;
  const bool breakdown = !(hn > 1e-300 * st->beta);
  st->inv_norm[jn] = breakdown ? 0.0 : 1.0 / hn;
  if (resid <= st->tol || breakdown) {
    st->converged = 1;
    st->done = 1;
  } else if (jn >= st->m || !(resid == resid)) {
    st->done = 1;
  }
  if (st->done) {
    // back substitution H(0:jn,0:jn) y = g
    for (int i = jn - 1; i >= 0; --i) {
      double a = st->g[i];
      for (int k = i + 1; k < jn; ++k) a -= st->H[k * M1 + i] * st->y[k];
      const double d = st->H[i * M1 + i];
      st->y[i] = d != 0.0 ? a / d : 0.0;
    }
  }
}

// S (+)= sum_{i<k} y_i Z_i, with the sum of the u part for the mass projection.
__global__ __launch_bounds__(256) void k_gmres_update(long ncell, double *__restrict__ S, const double *__restrict__ Z,
                                                       long vstride, GmresState *st, int accumulate, int project,
                                                       RedBuf red) {
  if (!st->done) return;   // enqueued speculatively after each chunk of Arnoldi steps
  const int k = st->j;
  __shared__ double y[kMaxRestart];
  if (threadIdx.x < k) y[threadIdx.x] = st->y[threadIdx.x];
  __syncthreads();
  const long n2 = 2 * ncell;
  double acc[1] = {0.0};
  for (long e = blockIdx.x * 256L + threadIdx.x; e < n2; e += (long)gridDim.x * 256) {
    double x = accumulate ? S[e] : 0.0;
    for (int i = 0; i < k; ++i) x = fma(y[i], Z[(long)i * vstride + e], x);
    S[e] = x;
    if (e < ncell) acc[0] += x;
  }
  block_partial<1>(acc, red.partials, threadIdx.x, 256, blockIdx.x, gridDim.x);
}

// ||a - b||^2 (b may be null), for the dt controller and diagnostics.
__global__ __launch_bounds__(256) void k_norm2_diff(long n2, const double *__restrict__ a, const double *__restrict__ b,
                                                     RedBuf red) {
  double acc[1] = {0.0};
  for (long e = blockIdx.x * 256L + threadIdx.x; e < n2; e += (long)gridDim.x * 256) {
    const double d = b ? a[e] - b[e] : a[e];
    acc[0] = fma(d, d, acc[0]);
  }
  block_partial<1>(acc, red.partials, threadIdx.x, 256, blockIdx.x, gridDim.x);
}

// One-block second stage of every reduction (see block_partial / final_sum).
template <int NV>
__global__ __launch_bounds__(256) void k_finalize(const double *__restrict__ partials, int nblocks, int nv,
                                                   double *__restrict__ out, GmresState *st, int mode,
                                                   FinalizeArgs fa) {
  if (mode == kFinDots || mode == kFinOrth) {
    if (st->done) return;   // the partial kernel skipped as well
  } else if (mode == kFinUpdate) {
    if (!st->done) return;
  }
  if (mode == kFinDots) nv = st->j + 1;
  double acc[NV];
  final_sum<NV>(partials, nblocks, threadIdx.x, 256, acc, nv);
  if (threadIdx.x != 0) return;
  switch (mode) {
    case kFinPlain:
      for (int k = 0; k < NV; ++k)
        if (k < nv) out[k] = acc[k];
      break;
    case kFinStart:
      start_tail(st, acc[0], fa.first, fa.m, fa.rtol, fa.atol);
      break;
    case kFinDots:
      for (int k = 0; k < NV; ++k)
        if (k < nv) st->hcol[k] = acc[k] * st->inv_norm[k];
      break;
    case kFinOrth:
      orth_tail(st, acc[0]);
      break;
    case kFinUpdate:
      st->shift = fa.project ? acc[0] / (double)fa.ncell : 0.0;
      break;
  }
}

__global__ __launch_bounds__(256) void k_reset_state(GmresState *st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->total_its = 0;
    st->done = 0;
    st->converged = 0;
    st->j = 0;
    st->shift = 0.0;
  }
}

}  // namespace

hipError_t launch_finalize(int mode, int nv, const RedBuf &red, int nblocks, GmresState *st, const FinalizeArgs &fa,
                           hipStream_t s) {
  if (nv > 2)
    hipLaunchKernelGGL(k_finalize<kMaxRestart + 1>, dim3(1), dim3(256), 0, s, red.partials, nblocks, nv, red.out, st,
                       mode, fa);
  else
    hipLaunchKernelGGL(k_finalize<2>, dim3(1), dim3(256), 0, s, red.partials, nblocks, nv, red.out, st, mode, fa);
  return hipGetLastError();
}

hipError_t launch_gmres_start(long n2, const double *F, const double *JS, double *V0, GmresState *st, int m,
                              double rtol, double atol, const RedBuf &red, hipStream_t s) {
  const int nb = reduce_blocks(n2);
  hipLaunchKernelGGL(k_gmres_start, dim3(nb), dim3(256), 0, s, n2, F, JS, V0, st, m, rtol, atol, red);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  FinalizeArgs fa{};
  fa.first = JS ? 0 : 1;
  fa.m = m;
  fa.rtol = rtol;
  fa.atol = atol;
  return launch_finalize(kFinStart, 1, red, nb, st, fa, s);
}

hipError_t launch_gmres_orth(long n2, double *V, long vstride, GmresState *st, const RedBuf &red, hipStream_t s) {
  const int nb = reduce_blocks(n2);
  hipLaunchKernelGGL(k_gmres_orth, dim3(nb), dim3(256), 0, s, n2, V, vstride, st, red);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(kFinOrth, 1, red, nb, st, FinalizeArgs{}, s);
}

hipError_t launch_gmres_update(long ncell, double *S, const double *Z, long vstride, GmresState *st, int accumulate,
                               int project, const RedBuf &red, hipStream_t s) {
  const int nb = reduce_blocks(2 * ncell);
  hipLaunchKernelGGL(k_gmres_update, dim3(nb), dim3(256), 0, s, ncell, S, Z, vstride, st, accumulate, project, red);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  FinalizeArgs fa{};
  fa.project = project;
  fa.ncell = ncell;
  return launch_finalize(kFinUpdate, 1, red, nb, st, fa, s);
}

hipError_t launch_norm2_diff(long n2, const double *a, const double *b, const RedBuf &red, hipStream_t s) {
  const int nb = reduce_blocks(n2);
  hipLaunchKernelGGL(k_norm2_diff, dim3(nb), dim3(256), 0, s, n2, a, b, red);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(kFinPlain, 1, red, nb, nullptr, FinalizeArgs{}, s);
}

hipError_t launch_reset_state(GmresState *st, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_state, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

}  // namespace acch
