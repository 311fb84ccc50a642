// Discrete adjoint of the time-step map of scheme (2.20) with the step sizes held
// fixed, 2D.  A step solves F(U^{n+1}; U^n) = 0, so for a loss L(U^N)
//   A^T lambda = dL/dU^{n+1},  dL/dU^n = -B^T lambda,  dL/dp -= lambda . dF/dp,
// with A = dF/dU^{n+1} (the Newton Jacobian J) and B = dF/dU^n.  This file holds
//   - the transposed Schwarz preconditioner M^{-T} = sum_k (R_k^delta)^T (L_k U_k)^{-T} R_k^0
//     (the exact transpose of the left-restricted operator, with the same factors),
//   - B^T lambda and the parameter terms by reverse differentiation of the residual
//     stencil (no B is assembled),
//   - the gradient of the discrete energy (eq. freeenergy).
// J^T x itself is the slot-transposed product in the stencil file.
#include "../../include/acch.h"
#include "boxes.h"
#include "kernels.h"
#include "physics.h"

namespace acch {
namespace {

// ---------------------------------------------------------------------------
// M^{-T} r: per box, restrict r to the owned cells, solve U^T y = r (forward over
// the wavefronts), then L^T x = y (backward); the whole box is then added into z.
// The factor layout is the one written by the factorisation kernel: the 24 slots of
// box cell (i, j) are contiguous at padded wavefront index (i + 2j) bh + j.
// Slots: 0-7 u-row L at u(-1,0) u(-2,0) u(1,-1) u(0,-1) u(-1,-1) u(0,-2) v(-1,0)
// v(0,-1); 8-10 v-row L at v(-1,0) v(0,-1) u(0,0); 11 1/U_uu; 12-17 u-row U at
// u(1,0) u(2,0) u(-1,1) u(0,1) u(1,1) u(0,2); 18-20 u-row U at v(0,0) v(1,0) v(0,1);
// 21 1/U_vv; 22-23 v-row U at v(1,0) v(0,1).
// ---------------------------------------------------------------------------
template <typename FT>
struct TCoef {
  const FT *F;
  long ncb;
  int bh;
  template <int S>
  ACCH_DEV double at(int i, int j) const {
    const long idx = (long)(i + 2 * j) * bh + j;
    return (double)F[idx * kNSlot2D + S];
  }
};

template <typename FT, int NW, bool INLDS>
__global__ __launch_bounds__(64 * NW) void k_ras_t_sweep2d(BoxGeom G, const SubInfo *__restrict__ subs, int nx,
                                                           int ny, int periodic, int kind,
                                                           const FT *__restrict__ fac, const double *__restrict__ r,
                                                           double *__restrict__ box, double *__restrict__ z,
                                                           const GmresState *st, long vstride) {
  constexpr int T = 64 * NW;
  extern __shared__ double lds_vals[];
  if (st && st->done) return;
  const int jj = st ? st->j : 0;
  const double sc = st ? st->inv_norm[jj] : 1.0;
  const long n = (long)nx * ny;
  const double *ru = r + (long)jj * vstride, *rv = ru + n;
  const int t = threadIdx.x;
  const SubInfo si = subs[blockIdx.x];
  const int bw = G.bw, bh = G.bh, nb = bw * bh;
  const TCoef<FT> C{fac + (long)blockIdx.x * kNSlot2D * (long)G.nlev * bh, (long)G.nlev * bh, bh};
  double *gvals = box + (long)blockIdx.x * 2 * nb;
  double *vu = INLDS ? lds_vals : gvals;
  double *vv = vu + nb;
  // U^T y = R^0 r
  for (int w = 0; w < G.nlev; ++w) {
    const int j = row_on_level<T>(w, t, bw, bh);
    if (j >= 0) {
      const int i = w - 2 * j;
      const long g = box_to_global(si, i, j, nx, ny, periodic);
      const bool own = g >= 0 && i >= si.own_x0 && i < si.own_x1 && j >= si.own_y0 && j < si.own_y1;
      const bool in = kind == ACCH_RAS_LEFT ? own : g >= 0;   // the transpose of the extension
      double a = in ? sc * ru[g] : 0.0;
      double b = in ? sc * rv[g] : 0.0;
      const int e = j * bw + i;
      if (i >= 1) a -= C.template at<12>(i - 1, j) * vu[e - 1];
      if (i >= 2) a -= C.template at<13>(i - 2, j) * vu[e - 2];
      if (j >= 1 && i + 1 < bw) a -= C.template at<14>(i + 1, j - 1) * vu[e - bw + 1];
      if (j >= 1) a -= C.template at<15>(i, j - 1) * vu[e - bw];
      if (j >= 1 && i >= 1) a -= C.template at<16>(i - 1, j - 1) * vu[e - bw - 1];
      if (j >= 2) a -= C.template at<17>(i, j - 2) * vu[e - 2 * bw];
      const double yu = a * C.template at<11>(i, j);
      b -= C.template at<18>(i, j) * yu;
      if (i >= 1) b -= C.template at<19>(i - 1, j) * vu[e - 1] + C.template at<22>(i - 1, j) * vv[e - 1];
      if (j >= 1) b -= C.template at<20>(i, j - 1) * vu[e - bw] + C.template at<23>(i, j - 1) * vv[e - bw];
      vu[e] = yu;
      vv[e] = b * C.template at<21>(i, j);
    }
    __syncthreads();
  }
  // L^T x = y (unit diagonal), v before u at each cell
  for (int w = G.nlev - 1; w >= 0; --w) {
    const int j = row_on_level<T>(w, t, bw, bh);
    if (j >= 0) {
      const int i = w - 2 * j;
      const int e = j * bw + i;
      double b = vv[e];
      if (i + 1 < bw) b -= C.template at<6>(i + 1, j) * vu[e + 1] + C.template at<8>(i + 1, j) * vv[e + 1];
      if (j + 1 < bh) b -= C.template at<7>(i, j + 1) * vu[e + bw] + C.template at<9>(i, j + 1) * vv[e + bw];
      double a = vu[e] - C.template at<10>(i, j) * b;
      if (i + 1 < bw) a -= C.template at<0>(i + 1, j) * vu[e + 1];
      if (i + 2 < bw) a -= C.template at<1>(i + 2, j) * vu[e + 2];
      if (j + 1 < bh && i >= 1) a -= C.template at<2>(i - 1, j + 1) * vu[e + bw - 1];
      if (j + 1 < bh) a -= C.template at<3>(i, j + 1) * vu[e + bw];
      if (j + 1 < bh && i + 1 < bw) a -= C.template at<4>(i + 1, j + 1) * vu[e + bw + 1];
      if (j + 2 < bh) a -= C.template at<5>(i, j + 2) * vu[e + 2 * bw];
      vu[e] = a;
      vv[e] = b;
    }
    __syncthreads();
  }
  if (kind == ACCH_RAS_RIGHT) {
    // the transpose of the owned-cell restriction: each owned cell written once
    double *zu = z + (long)jj * vstride, *zv = zu + n;
    for (int e = t; e < nb; e += T) {
      const int j = e / bw, i = e - j * bw;
      const long g = box_to_global(si, i, j, nx, ny, periodic);
      if (g >= 0 && i >= si.own_x0 && i < si.own_x1 && j >= si.own_y0 && j < si.own_y1) {
        zu[g] = vu[e];
        zv[g] = vv[e];
      }
    }
  } else if constexpr (INLDS) {
    for (int e = t; e < nb; e += T) {
      gvals[e] = vu[e];
      gvals[nb + e] = vv[e];
    }
  }
}

// z = sum over the boxes that contain a cell of their values there, in a fixed
// order (for_boxes_of).
__global__ __launch_bounds__(256) void k_ras_t_gather2d(BoxGeom G, const SubInfo *__restrict__ subs, int nx, int ny,
                                                         int periodic, int px, int py, const int *__restrict__ own_x,
                                                         const int *__restrict__ own_y,
                                                         const double *__restrict__ box, double *__restrict__ z,
                                                         const GmresState *st, long vstride) {
  if (st && st->done) return;
  const int jj = st ? st->j : 0;
  const long n = (long)nx * ny;
  double *zu = z + (long)jj * vstride, *zv = zu + n;
  const int nb = G.bw * G.bh;
  for (long g = blockIdx.x * 256L + threadIdx.x; g < n; g += (long)gridDim.x * 256) {
    const int gy = (int)(g / nx), gx = (int)(g - (long)gy * nx);
    double su = 0.0, sv = 0.0;
    for_boxes_of(subs, nx, ny, periodic, px, py, own_x, own_y, gx, gy, [&](int k, int lx, int ly) {
      const double *bk = box + (long)k * 2 * nb;
      su += bk[ly * G.bw + lx];
      sv += bk[nb + ly * G.bw + lx];
    });
    zu[g] = su;
    zv[g] = sv;
  }
}

// ---------------------------------------------------------------------------
// B^T lambda = (dF/dU^n)^T lambda and lambda . dF/dp by reverse differentiation
// of the residual stencil.  With mu, nu the discrete variational derivative and c the
// mobility, lambda . F = sum_c [lambda_u F_u + lambda_v F_v] has the adjoints
//   mubar = -div(ct grad lambda_u)          (the flux operator is symmetric)
//   nubar = lambda_v c / rho
//   cbar  = sum_faces w (mu_nb - mu)(lambda_u,nb - lambda_u)/2 + lambda_v nu / rho,
// and U^n enters through -U^n/dt, the pointwise parts of mu, nu and c, and the
// -gamma/2 Lap U^n terms of mu and nu (the Laplacian is symmetric as well).
// Pass 1 computes everything but the Laplacian terms and the parameter sums.
// ---------------------------------------------------------------------------
struct CellQ {
  double mu, nu, c;
};

ACCH_DEV double ld(const double *f, const Phys &P, int x, int y) {
  return f[(long)wrap_index(y, P.ny, P.periodic) * P.nx + wrap_index(x, P.nx, P.periodic)];
}

ACCH_DEV double lap_at(const double *f, const Phys &P, int x, int y) {
  const double c = ld(f, P, x, y);
  return (ld(f, P, x - 1, y) - c + (ld(f, P, x + 1, y) - c)) * P.wx +
         (ld(f, P, x, y - 1) - c + (ld(f, P, x, y + 1) - c)) * P.wy;
}

ACCH_DEV CellQ cell_q(const Phys &P, const double *X1, const double *X0, long n, int x, int y) {
  const double u1 = ld(X1, P, x, y), v1 = ld(X1 + n, P, x, y), u0 = ld(X0, P, x, y), v0 = ld(X0 + n, P, x, y);
  const double hg = 0.5 * P.gamma;
  const double phi = g2s(u1 + v1, u0 + v0, P.S), psi = g2s(u1 - v1, u0 - v0, P.S);
  CellQ q;
  q.mu = -0.5 * P.alpha * (u1 + u0 - 1.0) + P.theta * (phi + psi) -
         hg * (lap_at(X1, P, x, y) + lap_at(X0, P, x, y));
  q.nu = -0.5 * P.beta * (v1 + v0) + P.theta * (phi - psi) -
         hg * (lap_at(X1 + n, P, x, y) + lap_at(X0 + n, P, x, y));
  q.c = mobility_of(P.mob, u1, v1, u0, v0);
  return q;
}

__global__ __launch_bounds__(256) void k_adjoint_prev_a2d(Phys P, const double *__restrict__ X1,
                                                           const double *__restrict__ X0, double inv_dt,
                                                           const double *__restrict__ lam, double lam_scale,
                                                           double *__restrict__ bar, double *__restrict__ out,
                                                           RedBuf red) {
  const long n = (long)P.nx * P.ny;
  const double hg = 0.5 * P.gamma;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (long g = blockIdx.x * 256L + threadIdx.x; g < n; g += (long)gridDim.x * 256) {
    const int y = (int)(g / P.nx), x = (int)(g - (long)y * P.nx);
    const double u1 = X1[g], v1 = X1[n + g], u0 = X0[g], v0 = X0[n + g];
    const double lu = lam_scale * lam[g], lv = lam_scale * lam[n + g];
    double phi, dphi1, dphi0, psi, dpsi1, dpsi0, c, cu0, cv0;
    g2s_d01(u1 + v1, u0 + v0, P.S, phi, dphi1, dphi0);
    g2s_d01(u1 - v1, u0 - v0, P.S, psi, dpsi1, dpsi0);
    mobility_d0(P.mob, u1, v1, u0, v0, c, cu0, cv0);
    const double lapu = lap_at(X1, P, x, y) + lap_at(X0, P, x, y);
    const double lapv = lap_at(X1 + n, P, x, y) + lap_at(X0 + n, P, x, y);
    const double mu = -0.5 * P.alpha * (u1 + u0 - 1.0) + P.theta * (phi + psi) - hg * lapu;
    const double nu = -0.5 * P.beta * (v1 + v0) + P.theta * (phi - psi) - hg * lapv;
    double mubar = 0.0, cbar = lv * nu / P.rho;
    const int fdx[4] = {-1, 1, 0, 0}, fdy[4] = {0, 0, -1, 1};
    const bool fe[4] = {face_exists(x, -1, P.nx, P.periodic), face_exists(x, 1, P.nx, P.periodic),
                        face_exists(y, -1, P.ny, P.periodic), face_exists(y, 1, P.ny, P.periodic)};
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      if (!fe[f]) continue;
      const double wf = f < 2 ? P.wx : P.wy;
      const CellQ qn = cell_q(P, X1, X0, n, x + fdx[f], y + fdy[f]);
      const double lun = lam_scale * ld(lam, P, x + fdx[f], y + fdy[f]);
      mubar += wf * 0.5 * (c + qn.c) * (lu - lun);
      cbar += 0.5 * wf * (qn.mu - mu) * (lun - lu);
    }
    const double nubar = lv * c / P.rho;
    const double mu_u0 = -0.5 * P.alpha + P.theta * (dphi0 + dpsi0), mu_v0 = P.theta * (dphi0 - dpsi0);
    const double nu_u0 = P.theta * (dphi0 - dpsi0), nu_v0 = -0.5 * P.beta + P.theta * (dphi0 + dpsi0);
    out[g] = -lu * inv_dt + mubar * mu_u0 + nubar * nu_u0 + cbar * cu0;
    out[n + g] = -lv * inv_dt + mubar * mu_v0 + nubar * nu_v0 + cbar * cv0;
    bar[g] = mubar;
    bar[n + g] = nubar;
    // lambda . dF/dp for p = alpha, beta, theta, gamma
    acc[0] = fma(mubar, -0.5 * (u1 + u0 - 1.0), acc[0]);
    acc[1] = fma(nubar, -0.5 * (v1 + v0), acc[1]);
    acc[2] += mubar * (phi + psi) + nubar * (phi - psi);
    acc[3] += -0.5 * (mubar * lapu + nubar * lapv);
  }
  block_partial<4>(acc, red.partials, threadIdx.x, 256, blockIdx.x, gridDim.x);
}

// Pass 2: out -= gamma/2 Lap(mubar, nubar).
__global__ __launch_bounds__(256) void k_adjoint_prev_b2d(Phys P, const double *__restrict__ bar,
                                                           double *__restrict__ out) {
  const long n = (long)P.nx * P.ny;
  const double hg = 0.5 * P.gamma;
  for (long g = blockIdx.x * 256L + threadIdx.x; g < n; g += (long)gridDim.x * 256) {
    const int y = (int)(g / P.nx), x = (int)(g - (long)y * P.nx);
    out[g] -= hg * lap_at(bar, P, x, y);
    out[n + g] -= hg * lap_at(bar + n, P, x, y);
  }
}

// dE~/dU at X (cell volume vol) and the sums giving dE~/d(alpha, beta, theta, gamma).
__global__ __launch_bounds__(256) void k_energy_grad2d(Phys P, const double *__restrict__ X, double vol,
                                                        double *__restrict__ gout, RedBuf red) {
  const long n = (long)P.nx * P.ny;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (long g = blockIdx.x * 256L + threadIdx.x; g < n; g += (long)gridDim.x * 256) {
    const int y = (int)(g / P.nx), x = (int)(g - (long)y * P.nx);
    const double u = X[g], v = X[n + g];
    const double p = u + v, q = u - v;
    const double dp = dPhi(p), dq = dPhi(q);
    gout[g] = vol * (0.5 * P.alpha * (1.0 - 2.0 * u) + P.theta * (dp + dq) - P.gamma * lap_at(X, P, x, y));
    gout[n + g] = vol * (-P.beta * v + P.theta * (dp - dq) - P.gamma * lap_at(X + n, P, x, y));
    // |grad|^2 density: half of the squared differences over the cell's faces
    double gd = 0.0;
    const double ex = ld(X, P, x + 1, y) - u, wx_ = ld(X, P, x - 1, y) - u;
    const double ny_ = ld(X, P, x, y + 1) - u, sy_ = ld(X, P, x, y - 1) - u;
    const double fx = ld(X + n, P, x + 1, y) - v, gx_ = ld(X + n, P, x - 1, y) - v;
    const double fy = ld(X + n, P, x, y + 1) - v, gy_ = ld(X + n, P, x, y - 1) - v;
    gd += 0.5 * P.wx * (ex * ex + wx_ * wx_ + fx * fx + gx_ * gx_);
    gd += 0.5 * P.wy * (ny_ * ny_ + sy_ * sy_ + fy * fy + gy_ * gy_);
    acc[0] = fma(0.5 * u, 1.0 - u, acc[0]);
    acc[1] = fma(-0.5 * v, v, acc[1]);
    acc[2] += Phi(p) + Phi(q);
    acc[3] = fma(0.5, gd, acc[3]);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) acc[k] *= vol;
  block_partial<4>(acc, red.partials, threadIdx.x, 256, blockIdx.x, gridDim.x);
}

// Box values stay in LDS when both fields of a box fit (gfx950 has 160 KB per CU;
// above 64 KB the kernel has to be allowed the larger allocation first).
constexpr size_t kLdsDefault = 64 * 1024;
constexpr size_t kLdsMax = 160 * 1024;

template <typename FT, int NW>
hipError_t ras_t_impl(const BoxGeom &G, const SubInfo *subs, int nx, int ny, int periodic, int kind, const void *fac,
                      double *box, const double *r, double *z, const GmresState *st, long vstride, hipStream_t s) {
  const size_t lds = (size_t)2 * G.bw * G.bh * sizeof(double);
  static size_t lds_allowed = kLdsDefault;   // per instantiation
  bool inlds = lds <= lds_allowed;
  if (!inlds && lds <= kLdsMax &&
      hipFuncSetAttribute((const void *)k_ras_t_sweep2d<FT, NW, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)kLdsMax) == hipSuccess) {
    lds_allowed = kLdsMax;
    inlds = true;
  }
  (void)hipGetLastError();   // a refused attribute leaves the global-memory variant
  if (inlds)
    hipLaunchKernelGGL((k_ras_t_sweep2d<FT, NW, true>), dim3(G.nsub), dim3(64 * NW), lds, s, G, subs, nx, ny,
                       periodic, kind, (const FT *)fac, r, box, z, st, vstride);
  else
    hipLaunchKernelGGL((k_ras_t_sweep2d<FT, NW, false>), dim3(G.nsub), dim3(64 * NW), 0, s, G, subs, nx, ny,
                       periodic, kind, (const FT *)fac, r, box, z, st, vstride);
  return hipGetLastError();
}

template <typename FT>
hipError_t ras_t_waves(int nw, const BoxGeom &G, const SubInfo *subs, int nx, int ny, int periodic, int kind,
                       const void *fac, double *box, const double *r, double *z, const GmresState *st, long vstride,
                       hipStream_t s) {
  if (nw == 1) return ras_t_impl<FT, 1>(G, subs, nx, ny, periodic, kind, fac, box, r, z, st, vstride, s);
  if (nw == 2) return ras_t_impl<FT, 2>(G, subs, nx, ny, periodic, kind, fac, box, r, z, st, vstride, s);
  if (nw == 4) return ras_t_impl<FT, 4>(G, subs, nx, ny, periodic, kind, fac, box, r, z, st, vstride, s);
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_ras_t_apply2d(const BoxGeom &G, const SubInfo *subs, int nx, int ny, int periodic, int px, int py,
                                const int *own_x, const int *own_y, int kind, const void *fac, double *box,
                                const double *r, double *z, const GmresState *st, long vstride, int fp32,
                                hipStream_t s) {
  const int nw = schwarz_waves(G);
  hipError_t e = fp32 ? ras_t_waves<float>(nw, G, subs, nx, ny, periodic, kind, fac, box, r, z, st, vstride, s)
                      : ras_t_waves<double>(nw, G, subs, nx, ny, periodic, kind, fac, box, r, z, st, vstride, s);
  if (e != hipSuccess) return e;
  if (kind == ACCH_RAS_RIGHT) return hipSuccess;
  const int nb = reduce_blocks((long)nx * ny);
  hipLaunchKernelGGL(k_ras_t_gather2d, dim3(nb), dim3(256), 0, s, G, subs, nx, ny, periodic, px, py, own_x, own_y,
                     box, z, st, vstride);
  return hipGetLastError();
}

hipError_t launch_adjoint_prev2d(const Phys &P, const double *X1, const double *X0, double dt, const double *lam,
                                 double lam_scale, double *bar, double *out, const RedBuf &red, hipStream_t s) {
  const int nb = reduce_blocks((long)P.nx * P.ny);
  hipLaunchKernelGGL(k_adjoint_prev_a2d, dim3(nb), dim3(256), 0, s, P, X1, X0, 1.0 / dt, lam, lam_scale, bar, out,
                     red);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_finalize(kFinPlain, 4, red, single_launch(P, 0), kFamCell, nullptr, FinalizeArgs{}, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_adjoint_prev_b2d, dim3(nb), dim3(256), 0, s, P, bar, out);
  return hipGetLastError();
}

hipError_t launch_energy_grad2d(const Phys &P, const double *X, double vol, double *g, const RedBuf &red,
                                hipStream_t s) {
  const int nb = reduce_blocks((long)P.nx * P.ny);
  hipLaunchKernelGGL(k_energy_grad2d, dim3(nb), dim3(256), 0, s, P, X, vol, g, red);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(kFinPlain, 4, red, single_launch(P, 0), kFamCell, nullptr, FinalizeArgs{}, s);
}

}  // namespace acch
