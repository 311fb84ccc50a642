// Discrete adjoint of the time-step map of scheme (2.20) with the step sizes held
// fixed, 2D.  A step solves F(U^{n+1}; U^n) = 0, so for a loss L(U^N)
//   A^T lambda = dL/dU^{n+1},  dL/dU^n = -B^T lambda,  dL/dp -= lambda . dF/dp,
// with A = dF/dU^{n+1} (the Newton Jacobian J) and B = dF/dU^n.  This file holds
//   - B^T lambda and the parameter terms by reverse differentiation of the residual
//     stencil (no B is assembled),
//   - the gradient of the discrete energy (eq. freeenergy).
// J^T x itself is the slot-transposed product in the stencil file, and the transposed
// Schwarz preconditioner runs in the Schwarz file (transposed records, same sweeps).
#include "../../include/acch.h"
#include "kernels.h"
#include "physics.h"

namespace acch {
namespace {

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

}  // namespace

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
