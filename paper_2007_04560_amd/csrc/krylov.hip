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
// the Givens update of the Hessenberg column and the convergence test.  One
// instantiation per step j, like k_spmv_dots2d.
template <int J>
__global__ __launch_bounds__(256) void k_gmres_orth(long n2, double *__restrict__ V, long vstride, GmresState *st,
                                                     RedBuf red) {
  if (st->done) return;
  __shared__ double coef[J + 1];
  if (threadIdx.x <= J) coef[threadIdx.x] = st->hcol[threadIdx.x] * st->inv_norm[threadIdx.x];
  __syncthreads();
  double c[J + 1];
#pragma unroll
  for (int i = 0; i <= J; ++i) c[i] = coef[i];
  double *w = V + (long)(J + 1) * vstride;
  double acc[1] = {0.0};
  for (long e = blockIdx.x * 256L + threadIdx.x; e < n2; e += (long)gridDim.x * 256) {
    double b[J + 1];
#pragma unroll
    for (int i = 0; i <= J; ++i) b[i] = V[(long)i * vstride + e];
    double x = w[e];
#pragma unroll
    for (int i = 0; i <= J; ++i) x = fma(-c[i], b[i], x);
    w[e] = x;
    acc[0] = fma(x, x, acc[0]);
  }
  block_partial<1>(acc, red.partials, threadIdx.x, 256, blockIdx.x, gridDim.x);
}

// The serial part of an Arnoldi step: Hessenberg column, Givens rotations, residual
// estimate, stopping test and, at the end of a cycle, y.  The block first stages the
// small GMRES arrays in LDS (one round trip), thread 0 works on LDS only, then the
// block writes the results back.
ACCH_DEV void orth_tail(GmresState *st, double sum) {
  constexpr int M1 = kMaxRestart + 1;
  __shared__ double sH[M1 * kMaxRestart];
  __shared__ double sc_[kMaxRestart], ss_[kMaxRestart], sg[M1], sy[kMaxRestart];
  __shared__ int s_done;
  const int tid = threadIdx.x;
  const int j = st->j;
  for (int e = tid; e < (j + 1) * M1; e += blockDim.x) {
    const int col = e / M1, row = e - col * M1;
    sH[e] = (col < j) ? st->H[e] : (row <= j ? st->hcol[row] : 0.0);
  }
  if (tid < j) {
    sc_[tid] = st->cs[tid];
    ss_[tid] = st->sn[tid];
  }
  if (tid <= j) sg[tid] = st->g[tid];
  __syncthreads();
  const double hn = sqrt(sum);
  if (tid == 0) {
    double *h = sH + j * M1;
    for (int i = 0; i < j; ++i) {
      const double a = h[i], b = h[i + 1];
      h[i] = sc_[i] * a + ss_[i] * b;
      h[i + 1] = -ss_[i] * a + sc_[i] * b;
    }
    const double rr = hypot(h[j], hn);
    double c = 1.0, s = 0.0;
    if (rr > 0.0) {
      c = h[j] / rr;
      s = hn / rr;
    }
    sc_[j] = c;
    ss_[j] = s;
    h[j] = rr;
    const double gj = sg[j];
    sg[j] = c * gj;
    sg[j + 1] = -s * gj;
    const double resid = fabs(sg[j + 1]);
    const int jn = j + 1;
    const bool breakdown = !(hn > 1e-300 * st->beta);
    int done = 0;
    if (resid <= st->tol || breakdown) {
      st->converged = 1;
      done = 1;
    } else if (jn >= st->m || !(resid == resid)) {
      done = 1;
    }
    if (done) {  // back substitution H(0:jn,0:jn) y = g
      for (int i = jn - 1; i >= 0; --i) {
        double a = sg[i];
        for (int q = i + 1; q < jn; ++q) a -= sH[q * M1 + i] * sy[q];
        const double d = sH[i * M1 + i];
        sy[i] = d != 0.0 ? a / d : 0.0;
      }
    }
    st->resid = resid;
    st->inv_norm[jn] = breakdown ? 0.0 : 1.0 / hn;
    st->total_its += 1;
    s_done = done;
  }
  __syncthreads();
  const int jn = j + 1;
  if (tid <= j) st->H[j * M1 + tid] = sH[j * M1 + tid];
  if (tid == 0) {
    st->cs[j] = sc_[j];
    st->sn[j] = ss_[j];
    st->g[j] = sg[j];
    st->g[j + 1] = sg[j + 1];
  }
  if (s_done && tid < jn) st->y[tid] = sy[tid];
  __syncthreads();
  if (tid == 0) {
    st->j = jn;
    st->done = s_done;
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

// One-block second stages of the reductions (see block_partial / final_sum), one
// kernel per kind so that profiles tell them apart.
// h_ij = inv_norm_i * (sum of the block partials of dot i), i <= J.
template <int J>
__global__ __launch_bounds__(256) void k_finalize_dots(const double *__restrict__ partials, int nblocks,
                                                        GmresState *st) {
  if (st->done) return;
  constexpr int NV = pow2_at_least(J + 1);
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += 256) {
    double p[J + 1];
#pragma unroll
    for (int k = 0; k <= J; ++k) p[k] = partials[k * nblocks + b];
#pragma unroll
    for (int k = 0; k <= J; ++k) acc[k] += p[k];
  }
  double tot;
  block_multi_sum<NV>(acc, threadIdx.x, 256, J + 1, &tot);
  if ((int)threadIdx.x <= J) st->hcol[threadIdx.x] = tot * st->inv_norm[threadIdx.x];
}

template <int MODE>
__global__ __launch_bounds__(256) void k_finalize(const double *__restrict__ partials, int nblocks, int nv,
                                                   double *__restrict__ out, GmresState *st, FinalizeArgs fa) {
  if constexpr (MODE == kFinDots || MODE == kFinOrth) {
    if (st->done) return;   // the partial kernel skipped as well
  } else if constexpr (MODE == kFinUpdate) {
    if (!st->done) return;
  }
  if constexpr (MODE == kFinOrth) {
    double acc[1];
    final_sum<1>(partials, nblocks, threadIdx.x, 256, acc);
    __shared__ double s_sum;
    if (threadIdx.x == 0) s_sum = acc[0];
    __syncthreads();
    orth_tail(st, s_sum);
  } else if constexpr (MODE == kFinPlain) {
    double acc[4];
    final_sum<4>(partials, nblocks, threadIdx.x, 256, acc, nv);
    if (threadIdx.x == 0)
      for (int k = 0; k < 4; ++k)
        if (k < nv) out[k] = acc[k];
  } else {
    double acc[1];
    final_sum<1>(partials, nblocks, threadIdx.x, 256, acc);
    if (threadIdx.x != 0) return;
    if constexpr (MODE == kFinStart)
      start_tail(st, acc[0], fa.first, fa.m, fa.rtol, fa.atol);
    else
      st->shift = fa.project ? acc[0] / (double)fa.ncell : 0.0;
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
  switch (mode) {
    case kFinPlain:
      if (nv > 4) return hipErrorInvalidValue;
      hipLaunchKernelGGL(k_finalize<kFinPlain>, dim3(1), dim3(256), 0, s, red.partials, nblocks, nv, red.out, st, fa);
      break;
    case kFinStart:
      hipLaunchKernelGGL(k_finalize<kFinStart>, dim3(1), dim3(256), 0, s, red.partials, nblocks, nv, red.out, st, fa);
      break;
    case kFinOrth:
      hipLaunchKernelGGL(k_finalize<kFinOrth>, dim3(1), dim3(256), 0, s, red.partials, nblocks, nv, red.out, st, fa);
      break;
    case kFinUpdate:
      hipLaunchKernelGGL(k_finalize<kFinUpdate>, dim3(1), dim3(256), 0, s, red.partials, nblocks, nv, red.out, st, fa);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int J>
static hipError_t finalize_dots_at(int j, const RedBuf &red, int nblocks, GmresState *st, hipStream_t s) {
  if (j == J) {
    hipLaunchKernelGGL(k_finalize_dots<J>, dim3(1), dim3(256), 0, s, red.partials, nblocks, st);
    return hipGetLastError();
  }
  if constexpr (J + 1 < kMaxRestart) return finalize_dots_at<J + 1>(j, red, nblocks, st, s);
  return hipErrorInvalidValue;
}

hipError_t launch_finalize_dots(int j, const RedBuf &red, int nblocks, GmresState *st, hipStream_t s) {
  if (j < 0 || j >= kMaxRestart) return hipErrorInvalidValue;
  return finalize_dots_at<0>(j, red, nblocks, st, s);
}

template <int J>
static hipError_t orth_at(int j, long n2, double *V, long vstride, GmresState *st, const RedBuf &red, int nb,
                          hipStream_t s) {
  if (j == J) {
    hipLaunchKernelGGL(k_gmres_orth<J>, dim3(nb), dim3(256), 0, s, n2, V, vstride, st, red);
    return hipGetLastError();
  }
  if constexpr (J + 1 < kMaxRestart) return orth_at<J + 1>(j, n2, V, vstride, st, red, nb, s);
  return hipErrorInvalidValue;
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

hipError_t launch_gmres_orth(long n2, double *V, long vstride, int j, GmresState *st, const RedBuf &red,
                             hipStream_t s) {
  if (j < 0 || j >= kMaxRestart) return hipErrorInvalidValue;
  const int nb = reduce_blocks(n2);
  hipError_t e = orth_at<0>(j, n2, V, vstride, st, red, nb, s);
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
