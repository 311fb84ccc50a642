// Restarted flexible GMRES kernels (Section 3.1: right-preconditioned GMRES for
// J H^{-1} (H S) = -F).  The basis vectors are stored unnormalised (W_i) with
// v_i = inv_norm[i] W_i, so no separate normalisation pass is needed; the
// preconditioned vectors z_j = M^{-1} v_j are kept (flexible variant), which makes
// x = Z y valid also for the single-precision preconditioner.  Every kernel of an
// Arnoldi step returns at once when the cycle is finished, so the host may enqueue
// several steps ahead of its convergence check.  Every kernel also runs batched: a
// block finds its instance through the launch family's map (common.h), and the
// one-block second stages run one block per instance.
#include <math.h>

#include "kernels.h"

namespace acch {
namespace {

// Instance of this block in a (possibly batched) vector launch over 2n elements.
struct ElemLoc {
  Loc L;
  long n2;
  long xo;
};
ACCH_DEV ElemLoc elem_loc(const Batch &bt, long n2_single) {
  ElemLoc E;
  E.L = locate(bt, kFamElem);
  if (bt.map[kFamElem]) {
    const Inst &I = bt.inst[E.L.b];
    E.n2 = 2L * I.P.nx * I.P.ny;
    E.xo = I.xoff;
  } else {
    E.n2 = n2_single;
    E.xo = 0;
  }
  return E;
}

// V_0 = -(F + J S) (J S computed by the caller into JS, or absent) and beta = ||V_0||.
__global__ __launch_bounds__(256) void k_gmres_start(Batch bt, long n2s, const double *__restrict__ F,
                                                      const double *__restrict__ JS, double *__restrict__ V0,
                                                      RedBuf red) {
  const ElemLoc E = elem_loc(bt, n2s);
  if (!E.L.on) return;
  F += E.xo;
  V0 += E.xo;
  if (JS) JS += E.xo;
  double acc[1] = {0.0};
  for (long e = E.L.lb * 256L + threadIdx.x; e < E.n2; e += (long)E.L.nb * 256) {
    const double r = JS ? -(F[e] + JS[e]) : -F[e];
    V0[e] = r;
    acc[0] = fma(r, r, acc[0]);
  }
  block_partial<1>(acc, red.partials, threadIdx.x, 256, blockIdx.x, gridDim.x);
}

// Starts a cycle.  The first cycle after a reset fixes the absolute tolerance
// max(rtol * beta, atol); later cycles keep it.
ACCH_DEV void start_tail(GmresState *st, double sum, int m, double rtol, double atol) {
  const double beta = sqrt(sum);
  st->beta = beta;
  if (st->first) st->tol = fmax(rtol * beta, atol);
  st->first = 0;
  const double tol = st->tol;
  st->m = m;
  st->j = 0;
  st->applied = 0;
  st->g[0] = beta;
  st->resid = beta;
  st->inv_norm[0] = beta > 0.0 ? 1.0 / beta : 0.0;
  st->converged = (beta <= tol) ? 1 : 0;
  st->done = st->converged;
}

// W_{j+1} -= sum_{i<=j} h_ij v_i (classical Gram–Schmidt, one pass), then the block
// partials of ||W_{j+1}||^2 (red: their own rows of the partial buffer).  The dots of
// the SpMV kernel are summed here, by every block for itself in block order (so all
// blocks hold the same h_ij, and the same values as a separate one-block sum would
// give); the instance's first block records the Hessenberg column for the serial tail.
// One instantiation per step j, like k_spmv_dots2d.
template <int J>
__global__ __launch_bounds__(256) void k_gmres_orth(Batch bt, long n2s, double *__restrict__ V, long vstride,
                                                     GmresState *st, RedBuf red, const double *__restrict__ dots,
                                                     int dstride) {
  const ElemLoc E = elem_loc(bt, n2s);
  if (!E.L.on) return;
  GmresState *sb = st + E.L.b;
  if (sb->done) return;
  V += E.xo;
  const int db0 = bt.map[kFamElem] ? bt.inst[E.L.b].blk0[kFamCell] : 0;
  const int dnb = bt.map[kFamElem] ? bt.inst[E.L.b].nblk[kFamCell] : dstride;
  constexpr int NV = pow2_at_least(J + 1);
  __shared__ double coef[J + 1];
  {
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
    for (int b = threadIdx.x; b < dnb; b += 256) {
      double p[J + 1];
#pragma unroll
      for (int k = 0; k <= J; ++k) p[k] = dots[(long)k * dstride + db0 + b];
#pragma unroll
      for (int k = 0; k <= J; ++k) acc[k] += p[k];
    }
    double tot;
    block_multi_sum<NV>(acc, threadIdx.x, 256, J + 1, &tot);
    if ((int)threadIdx.x <= J) {
      const double h = tot * sb->inv_norm[threadIdx.x];   // h_ij
      coef[threadIdx.x] = h * sb->inv_norm[threadIdx.x];
      if (E.L.lb == 0) sb->hcol[threadIdx.x] = h;
    }
  }
  __syncthreads();
  double c[J + 1];
#pragma unroll
  for (int i = 0; i <= J; ++i) c[i] = coef[i];
  double *w = V + (long)(J + 1) * vstride;
  double acc[1] = {0.0};
  for (long e = E.L.lb * 256L + threadIdx.x; e < E.n2; e += (long)E.L.nb * 256) {
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
// estimate, stopping test and, at the end of a cycle, y.  The block stages the new
// column, the rotations and g in LDS (one round trip), thread 0 works on LDS only,
// then the block writes the results back; the earlier columns of H are read only for
// the back substitution at the end of a cycle.
// The state it reads (new column, rotations, g) is loaded by the caller's threads
// together with the partial sums of ||W_{j+1}||^2, so the two loads overlap.
struct OrthIn {
  double hc, g, c, s;   // this thread's entries (thread t: row / rotation t)
};
ACCH_DEV OrthIn orth_load(const GmresState *st) {
  const int tid = threadIdx.x;
  const int j = st->j;
  OrthIn in{0.0, 0.0, 0.0, 0.0};
  if (tid <= j) {
    in.hc = st->hcol[tid];
    in.g = st->g[tid];
  }
  if (tid < j) {
    in.c = st->cs[tid];
    in.s = st->sn[tid];
  }
  return in;
}
ACCH_DEV void orth_tail(GmresState *st, double sum, const OrthIn &in) {
  constexpr int M1 = kMaxRestart + 1;
  __shared__ double sH[M1 * kMaxRestart];   // columns 0..j, for the back substitution
  __shared__ double shc[M1];                // the new column j
  __shared__ double sc_[kMaxRestart], ss_[kMaxRestart], sg[M1], sy[kMaxRestart];
  __shared__ int s_done;
  const int tid = threadIdx.x;
  const int j = st->j;
  if (tid <= j) {
    shc[tid] = in.hc;
    sg[tid] = in.g;
  }
  if (tid < j) {
    sc_[tid] = in.c;
    ss_[tid] = in.s;
  }
  __syncthreads();
  const double hn = sqrt(sum);
  if (tid == 0) {
    double *h = shc;
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
    st->resid = resid;
    st->inv_norm[jn] = breakdown ? 0.0 : 1.0 / hn;
    st->total_its += 1;
    s_done = done;
  }
  __syncthreads();
  const int jn = j + 1;
  if (s_done) {   // back substitution H(0:jn,0:jn) y = g
    for (int e = tid; e < jn * M1; e += blockDim.x) {
      const int col = e / M1, row = e - col * M1;
      sH[e] = (col < j) ? st->H[e] : (row <= j ? shc[row] : 0.0);
    }
    __syncthreads();
    if (tid == 0) {
      for (int i = jn - 1; i >= 0; --i) {
        double a = sg[i];
        for (int q = i + 1; q < jn; ++q) a -= sH[q * M1 + i] * sy[q];
        const double d = sH[i * M1 + i];
        sy[i] = d != 0.0 ? a / d : 0.0;
      }
    }
    __syncthreads();
  }
  if (tid <= j) st->H[j * M1 + tid] = shc[tid];
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
__global__ __launch_bounds__(256) void k_gmres_update(Batch bt, long n2s, double *__restrict__ S,
                                                       const double *__restrict__ Z, long vstride, GmresState *st,
                                                       int accumulate, RedBuf red) {
  const ElemLoc E = elem_loc(bt, n2s);
  if (!E.L.on) return;
  GmresState *sb = st + E.L.b;
  if (!sb->done || sb->applied) return;   // enqueued speculatively after each chunk of Arnoldi steps
  S += E.xo;
  Z += E.xo;
  const int k = sb->j;
  __shared__ double y[kMaxRestart];
  if (threadIdx.x < k) y[threadIdx.x] = sb->y[threadIdx.x];
  __syncthreads();
  const long ncell = E.n2 / 2;
  double acc[1] = {0.0};
  for (long e = E.L.lb * 256L + threadIdx.x; e < E.n2; e += (long)E.L.nb * 256) {
    double x = accumulate ? S[e] : 0.0;
    for (int i = 0; i < k; ++i) x = fma(y[i], Z[(long)i * vstride + e], x);
    S[e] = x;
    if (e < ncell) acc[0] += x;
  }
  block_partial<1>(acc, red.partials, threadIdx.x, 256, blockIdx.x, gridDim.x);
}

// ||a - b||^2 (b may be null), for the dt controller and diagnostics.
__global__ __launch_bounds__(256) void k_norm2_diff(Batch bt, long n2s, const double *__restrict__ a,
                                                     const double *__restrict__ b, RedBuf red) {
  const ElemLoc E = elem_loc(bt, n2s);
  if (!E.L.on) return;
  a += E.xo;
  if (b) b += E.xo;
  double acc[1] = {0.0};
  for (long e = E.L.lb * 256L + threadIdx.x; e < E.n2; e += (long)E.L.nb * 256) {
    const double d = b ? a[e] - b[e] : a[e];
    acc[0] = fma(d, d, acc[0]);
  }
  block_partial<1>(acc, red.partials, threadIdx.x, 256, blockIdx.x, gridDim.x);
}

// d1 = s1 and d2 = s2 (d2 may be null) on the active instances; with s1 null, d1 = 0.
__global__ __launch_bounds__(256) void k_copy2(Batch bt, long n2s, double *__restrict__ d1,
                                                const double *__restrict__ s1, double *__restrict__ d2,
                                                const double *__restrict__ s2) {
  const ElemLoc E = elem_loc(bt, n2s);
  if (!E.L.on) return;
  for (long e = E.L.lb * 256L + threadIdx.x; e < E.n2; e += (long)E.L.nb * 256) {
    d1[E.xo + e] = s1 ? s1[E.xo + e] : 0.0;
    if (d2) d2[E.xo + e] = s2[E.xo + e];
  }
}

// Second stages of the reductions (see block_partial / final_sum): one block per
// instance, summing that instance's blocks of the partial kernel; one kernel per
// kind so that profiles tell them apart.
struct FinRange {
  int b, b0, nb;
  bool on;
};
ACCH_DEV FinRange fin_range(const Inst *inst, const int *active, int fam, int nblocks) {
  FinRange R;
  R.b = blockIdx.x;
  if (inst) {
    R.b0 = inst[R.b].blk0[fam];
    R.nb = inst[R.b].nblk[fam];
  } else {
    R.b0 = 0;
    R.nb = nblocks;
  }
  R.on = active == nullptr || active[R.b] != 0;
  return R;
}

template <int MODE>
__global__ __launch_bounds__(256) void k_finalize(const double *__restrict__ partials, int stride, int fam,
                                                   const Inst *inst, const int *active, int nv,
                                                   double *__restrict__ out, GmresState *st, FinalizeArgs fa) {
  const FinRange R = fin_range(inst, active, fam, stride);
  GmresState *sb = st ? st + R.b : nullptr;
  if constexpr (MODE == kFinStart) {
    if (!R.on) {   // an inactive instance does not take part in this solve
      if (threadIdx.x == 0) {
        sb->done = 1;
        sb->converged = 1;
        sb->applied = 1;
        sb->j = 0;
      }
      return;
    }
  } else {
    if (!R.on) return;
  }
  if constexpr (MODE == kFinOrth) {
    if (sb->done) return;   // the partial kernel skipped as well
  } else if constexpr (MODE == kFinUpdate) {
    if (!sb->done || sb->applied) return;
  }
  if constexpr (MODE == kFinOrth) {
    const OrthIn in = orth_load(sb);
    double acc[1];
    final_sum<1>(partials, stride, R.b0, R.nb, threadIdx.x, 256, acc);
    __shared__ double s_sum;
    if (threadIdx.x == 0) s_sum = acc[0];
    __syncthreads();
    orth_tail(sb, s_sum, in);
  } else if constexpr (MODE == kFinPlain) {
    double acc[4];
    final_sum<4>(partials, stride, R.b0, R.nb, threadIdx.x, 256, acc, nv);
    if (threadIdx.x == 0)
      for (int k = 0; k < 4; ++k)
        if (k < nv) out[4 * R.b + k] = acc[k];
  } else {
    double acc[1];
    final_sum<1>(partials, stride, R.b0, R.nb, threadIdx.x, 256, acc);
    if (threadIdx.x != 0) return;
    if constexpr (MODE == kFinStart) {
      start_tail(sb, acc[0], fa.m, fa.rtol, fa.atol);
    } else {
      const long ncell = inst ? (long)inst[R.b].P.nx * inst[R.b].P.ny : fa.ncell;
      sb->shift = fa.project ? acc[0] / (double)ncell : 0.0;
      sb->applied = 1;
    }
  }
}

__global__ __launch_bounds__(64) void k_reset_state(GmresState *st, int count) {
  const int b = blockIdx.x * 64 + threadIdx.x;
  if (b < count) {
    st[b].total_its = 0;
    st[b].done = 0;
    st[b].converged = 0;
    st[b].j = 0;
    st[b].first = 1;
    st[b].applied = 0;
    st[b].shift = 0.0;
  }
}

}  // namespace

static const Inst *fin_inst(const BatchLaunch &bl, int fam) { return bl.bt.map[fam] ? bl.bt.inst : nullptr; }

hipError_t launch_finalize(int mode, int nv, const RedBuf &red, const BatchLaunch &bl, int fam, GmresState *st,
                           const FinalizeArgs &fa, hipStream_t s) {
  const dim3 g(bl.count);
  const int stride = bl.grid[fam];
  const Inst *in = fin_inst(bl, fam);
  const int *act = bl.bt.active;
  switch (mode) {
    case kFinPlain:
      if (nv > 4) return hipErrorInvalidValue;
      hipLaunchKernelGGL(k_finalize<kFinPlain>, g, dim3(256), 0, s, red.partials, stride, fam, in, act, nv, red.out,
                         st, fa);
      break;
    case kFinStart:
      hipLaunchKernelGGL(k_finalize<kFinStart>, g, dim3(256), 0, s, red.partials, stride, fam, in, act, nv, red.out,
                         st, fa);
      break;
    case kFinOrth:
      hipLaunchKernelGGL(k_finalize<kFinOrth>, g, dim3(256), 0, s, red.partials, stride, fam, in, act, nv, red.out,
                         st, fa);
      break;
    case kFinUpdate:
      hipLaunchKernelGGL(k_finalize<kFinUpdate>, g, dim3(256), 0, s, red.partials, stride, fam, in, act, nv, red.out,
                         st, fa);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int J>
static hipError_t orth_at(int j, const BatchLaunch &bl, double *V, long vstride, GmresState *st, const RedBuf &nred,
                          const double *dots, hipStream_t s) {
  if (j == J) {
    hipLaunchKernelGGL(k_gmres_orth<J>, dim3(bl.grid[kFamElem]), dim3(256), 0, s, bl.bt, 2 * bl.ncell, V, vstride, st,
                       nred, dots, bl.grid[kFamCell]);
    return hipGetLastError();
  }
  if constexpr (J + 1 < kMaxRestart) return orth_at<J + 1>(j, bl, V, vstride, st, nred, dots, s);
  return hipErrorInvalidValue;
}

hipError_t launch_gmres_start(const BatchLaunch &bl, const double *F, const double *JS, double *V0, GmresState *st,
                              int m, double rtol, double atol, const RedBuf &red, hipStream_t s) {
  hipLaunchKernelGGL(k_gmres_start, dim3(bl.grid[kFamElem]), dim3(256), 0, s, bl.bt, 2 * bl.ncell, F, JS, V0, red);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  FinalizeArgs fa{};
  fa.m = m;
  fa.rtol = rtol;
  fa.atol = atol;
  return launch_finalize(kFinStart, 1, red, bl, kFamElem, st, fa, s);
}

hipError_t launch_gmres_orth(const BatchLaunch &bl, double *V, long vstride, int j, GmresState *st,
                             const RedBuf &red, hipStream_t s) {
  if (j < 0 || j >= kMaxRestart) return hipErrorInvalidValue;
  // the norm partials go after the dot rows, which the kernel is still reading
  RedBuf nred = red;
  nred.partials = red.partials + (long)kMaxRestart * bl.grid[kFamCell];
  hipError_t e = orth_at<0>(j, bl, V, vstride, st, nred, red.partials, s);
  if (e != hipSuccess) return e;
  return launch_finalize(kFinOrth, 1, nred, bl, kFamElem, st, FinalizeArgs{}, s);
}

hipError_t launch_gmres_update(const BatchLaunch &bl, double *S, const double *Z, long vstride, GmresState *st,
                               int accumulate, int project, const RedBuf &red, hipStream_t s) {
  hipLaunchKernelGGL(k_gmres_update, dim3(bl.grid[kFamElem]), dim3(256), 0, s, bl.bt, 2 * bl.ncell, S, Z, vstride,
                     st, accumulate, red);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  FinalizeArgs fa{};
  fa.project = project;
  fa.ncell = bl.ncell;
  return launch_finalize(kFinUpdate, 1, red, bl, kFamElem, st, fa, s);
}

hipError_t launch_norm2_diff(const BatchLaunch &bl, const double *a, const double *b, const RedBuf &red,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_norm2_diff, dim3(bl.grid[kFamElem]), dim3(256), 0, s, bl.bt, 2 * bl.ncell, a, b, red);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(kFinPlain, 1, red, bl, kFamElem, nullptr, FinalizeArgs{}, s);
}

hipError_t launch_copy2(const BatchLaunch &bl, double *d1, const double *s1, double *d2, const double *s2,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_copy2, dim3(bl.grid[kFamElem]), dim3(256), 0, s, bl.bt, 2 * bl.ncell, d1, s1, d2, s2);
  return hipGetLastError();
}

hipError_t launch_reset_state(const BatchLaunch &bl, GmresState *st, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_state, dim3((bl.count + 63) / 64), dim3(64), 0, s, st, bl.count);
  return hipGetLastError();
}

}  // namespace acch
