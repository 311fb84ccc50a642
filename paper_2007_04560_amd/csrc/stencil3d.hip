// 3D stencil kernels of scheme (2.20): residual, discrete energy and mass, the
// analytic Jacobian in 40 slots per cell and its products, and the adjoint pieces
// (B^T lambda, parameter terms, energy gradient).  The residual and the Jacobian first
// store the cell quantities (mu, nu, c and their derivatives) of every cell, then a
// second pass reads them at the face neighbours; the same formulas as the 2D tile
// kernels with a third face pair.
//
// Slots (include/acch.h): u-row/u-col 0..24 on uu3, u-row/v-col 25..31 on star3,
// v-row/v-col 32..38 on star3, v-row/u-col 39 at the cell.
#include "kernels.h"
#include "physics.h"
#include "stencil3d.h"

namespace acch {
namespace {

struct C3 {
  int x, y, z;
};

ACCH_DEV long gidx(const Phys &P, int x, int y, int z) {
  return ((long)wrap_index(z, P.nz, P.periodic) * P.ny + wrap_index(y, P.ny, P.periodic)) * P.nx +
         wrap_index(x, P.nx, P.periodic);
}

ACCH_DEV double ld3(const double *f, const Phys &P, int x, int y, int z) { return f[gidx(P, x, y, z)]; }

ACCH_DEV double lap3(const double *f, const Phys &P, int x, int y, int z) {
  const double c = ld3(f, P, x, y, z);
  return (ld3(f, P, x - 1, y, z) - c + (ld3(f, P, x + 1, y, z) - c)) * P.wx +
         (ld3(f, P, x, y - 1, z) - c + (ld3(f, P, x, y + 1, z) - c)) * P.wy +
         (ld3(f, P, x, y, z - 1) - c + (ld3(f, P, x, y, z + 1) - c)) * P.wz;
}

ACCH_DEV double face_w(const Phys &P, int f) { return f < 2 ? P.wx : (f < 4 ? P.wy : P.wz); }

ACCH_DEV bool face3(const Phys &P, int x, int y, int z, int f) {
  switch (f) {
    case 0: return face_exists(x, -1, P.nx, P.periodic);
    case 1: return face_exists(x, 1, P.nx, P.periodic);
    case 2: return face_exists(y, -1, P.ny, P.periodic);
    case 3: return face_exists(y, 1, P.ny, P.periodic);
    case 4: return face_exists(z, -1, P.nz, P.periodic);
    default: return face_exists(z, 1, P.nz, P.periodic);
  }
}

ACCH_DEV C3 step(C3 c, int f) {
  const Off3 o = star3(1 + f);
  return C3{c.x + o.dx, c.y + o.dy, c.z + o.dz};
}

// Cell quantities of the trial state (X1 possibly X + lam (S - shift e_u)) and X0.
struct Q3 {
  double u1, v1, u0, v0, mu, nu, c, phi, psi;
};

struct Trial {
  const double *X, *S, *X0;
  double lam, shift;
  long n;
  ACCH_DEV double u1(long g) const { return S ? fma(lam, S[g] - shift, X[g]) : X[g]; }
  ACCH_DEV double v1(long g) const { return S ? fma(lam, S[n + g], X[n + g]) : X[n + g]; }
};

ACCH_DEV double lap_trial(const Trial &T, const Phys &P, C3 c, int field) {
  auto val = [&](int x, int y, int z) {
    const long g = gidx(P, x, y, z);
    return field == 0 ? T.u1(g) : T.v1(g);
  };
  const double m = val(c.x, c.y, c.z);
  return (val(c.x - 1, c.y, c.z) - m + (val(c.x + 1, c.y, c.z) - m)) * P.wx +
         (val(c.x, c.y - 1, c.z) - m + (val(c.x, c.y + 1, c.z) - m)) * P.wy +
         (val(c.x, c.y, c.z - 1) - m + (val(c.x, c.y, c.z + 1) - m)) * P.wz;
}

ACCH_DEV Q3 cell_q3(const Trial &T, const Phys &P, C3 c) {
  Q3 q;
  const long g = gidx(P, c.x, c.y, c.z);
  q.u1 = T.u1(g);
  q.v1 = T.v1(g);
  q.u0 = T.X0[g];
  q.v0 = T.X0[T.n + g];
  const double hg = 0.5 * P.gamma;
  q.phi = g2s(q.u1 + q.v1, q.u0 + q.v0, P.S);
  q.psi = g2s(q.u1 - q.v1, q.u0 - q.v0, P.S);
  const double lapu = lap_trial(T, P, c, 0) + lap3(T.X0, P, c.x, c.y, c.z);
  const double lapv = lap_trial(T, P, c, 1) + lap3(T.X0 + T.n, P, c.x, c.y, c.z);
  q.mu = -0.5 * P.alpha * (q.u1 + q.u0 - 1.0) + P.theta * (q.phi + q.psi) - hg * lapu;
  q.nu = -0.5 * P.beta * (q.v1 + q.v0) + P.theta * (q.phi - q.psi) - hg * lapv;
  q.c = mobility_of(P.mob, q.u1, q.v1, q.u0, q.v0);
  return q;
}

ACCH_DEV C3 cell_of_index(const Phys &P, long g) {
  const long plane = (long)P.nx * P.ny;
  C3 c;
  c.z = (int)(g / plane);
  const long r = g - (long)c.z * plane;
  c.y = (int)(r / P.nx);
  c.x = (int)(r - (long)c.y * P.nx);
  return c;
}

// mu, nu and c of every cell at the trial state, stored [mu | nu | c][cell], so that
// the residual reads them at the neighbours instead of recomputing them there.
__global__ __launch_bounds__(256) void k_cellq3d(Phys P, const double *__restrict__ X, const double *__restrict__ Sdir,
                                                  double lam, const GmresState *shift_st,
                                                  const double *__restrict__ Xn, double *__restrict__ Q) {
  const long n = (long)P.nx * P.ny * P.nz;
  const Trial T{X, Sdir, Xn, lam, shift_st ? shift_st->shift : 0.0, n};
  for (long g = blockIdx.x * 256L + threadIdx.x; g < n; g += (long)gridDim.x * 256) {
    const Q3 q = cell_q3(T, P, cell_of_index(P, g));
    Q[g] = q.mu;
    Q[n + g] = q.nu;
    Q[2 * n + g] = q.c;
  }
}

// F (optionally at the trial state, which is also written to Xt), ||F||^2 and the
// number of inadmissible cells, from the cell quantities of k_cellq3d.
__global__ __launch_bounds__(256) void k_residual3d(Phys P, const double *__restrict__ X,
                                                     const double *__restrict__ Sdir, double lam,
                                                     const GmresState *shift_st, const double *__restrict__ Xn,
                                                     double inv_dt, const double *__restrict__ Q,
                                                     double *__restrict__ Xt, double *__restrict__ F, RedBuf red) {
  const long n = (long)P.nx * P.ny * P.nz;
  const Trial T{X, Sdir, Xn, lam, shift_st ? shift_st->shift : 0.0, n};
  const double *Qmu = Q, *Qnu = Q + n, *Qc = Q + 2 * n;
  double acc[2] = {0.0, 0.0};
  for (long g = blockIdx.x * 256L + threadIdx.x; g < n; g += (long)gridDim.x * 256) {
    const C3 c = cell_of_index(P, g);
    Q3 q;
    q.u1 = T.u1(g);
    q.v1 = T.v1(g);
    q.u0 = Xn[g];
    q.v0 = Xn[n + g];
    q.mu = Qmu[g];
    q.nu = Qnu[g];
    q.c = Qc[g];
    double div = 0.0;
    for (int f = 0; f < 6; ++f) {
      if (!face3(P, c.x, c.y, c.z, f)) continue;
      const C3 cn = step(c, f);
      const long h = gidx(P, cn.x, cn.y, cn.z);
      div += 0.5 * (q.c + Qc[h]) * (Qmu[h] - q.mu) * face_w(P, f);
    }
    const double Fu = (q.u1 - q.u0) * inv_dt - div;
    const double Fv = (q.v1 - q.v0) * inv_dt + q.c * q.nu / P.rho;
    F[g] = Fu;
    F[n + g] = Fv;
    if (Xt) {
      Xt[g] = q.u1;
      Xt[n + g] = q.v1;
    }
    acc[0] += Fu * Fu + Fv * Fv;
    const double p = q.u1 + q.v1, qq = q.u1 - q.v1;
    acc[1] += (p > 0.0 && p < 1.0 && qq > 0.0 && qq < 1.0) ? 0.0 : 1.0;
  }
  block_partial<2>(acc, red.partials, threadIdx.x, 256, blockIdx.x, gridDim.x);
}

// Discrete energy density (without the cell volume) and u, summed.
__global__ __launch_bounds__(256) void k_energy3d(Phys P, const double *__restrict__ X, RedBuf red) {
  const long n = (long)P.nx * P.ny * P.nz;
  double acc[2] = {0.0, 0.0};
  for (long g = blockIdx.x * 256L + threadIdx.x; g < n; g += (long)gridDim.x * 256) {
    const C3 c = cell_of_index(P, g);
    const double u = X[g], v = X[n + g];
    double e = 0.5 * P.alpha * u * (1.0 - u) - 0.5 * P.beta * v * v + P.theta * (Phi(u + v) + Phi(u - v));
    double grad = 0.0;
    for (int fld = 0; fld < 2; ++fld) {
      const double *fp = X + fld * n;
      const double m = fp[g];
      for (int f = 0; f < 6; ++f) {
        const C3 nb = step(c, f);
        const double d = ld3(fp, P, nb.x, nb.y, nb.z) - m;
        grad += 0.5 * d * d * face_w(P, f);
      }
    }
    acc[0] += e + 0.5 * P.gamma * grad;
    acc[1] += u;
  }
  block_partial<2>(acc, red.partials, threadIdx.x, 256, blockIdx.x, gridDim.x);
}

// Cell quantities with the derivatives the Jacobian needs.
struct D3 {
  double mu, c, cu, cv, Am, av, nu, Bnu;
};

ACCH_DEV D3 cell_d3(const double *X, const double *Xn, const Phys &P, long n, C3 c) {
  const long g = gidx(P, c.x, c.y, c.z);
  const double u1 = X[g], v1 = X[n + g], u0 = Xn[g], v0 = Xn[n + g];
  const double hg = 0.5 * P.gamma;
  double phi, dphi, psi, dpsi;
  g2s_d(u1 + v1, u0 + v0, P.S, phi, dphi);
  g2s_d(u1 - v1, u0 - v0, P.S, psi, dpsi);
  D3 d;
  mobility_d(P.mob, u1, v1, u0, v0, d.c, d.cu, d.cv);
  double wsum = 0.0;
  for (int f = 0; f < 6; ++f)
    if (face3(P, c.x, c.y, c.z, f)) wsum += face_w(P, f);
  const double lapu = lap3(X, P, c.x, c.y, c.z) + lap3(Xn, P, c.x, c.y, c.z);
  const double lapv = lap3(X + n, P, c.x, c.y, c.z) + lap3(Xn + n, P, c.x, c.y, c.z);
  d.mu = -0.5 * P.alpha * (u1 + u0 - 1.0) + P.theta * (phi + psi) - hg * lapu;
  d.nu = -0.5 * P.beta * (v1 + v0) + P.theta * (phi - psi) - hg * lapv;
  d.Am = -0.5 * P.alpha + P.theta * (dphi + dpsi) + hg * wsum;
  d.av = P.theta * (dphi - dpsi);
  d.Bnu = -0.5 * P.beta + P.theta * (dphi + dpsi) + hg * wsum;
  return d;
}

constexpr int kD3 = 8;   // values of D3 per cell

// D3 of every cell, stored [field][cell] in the order of the struct.
__global__ __launch_bounds__(256) void k_celld3d(Phys P, const double *__restrict__ X, const double *__restrict__ Xn,
                                                  double *__restrict__ Q) {
  const long n = (long)P.nx * P.ny * P.nz;
  for (long g = blockIdx.x * 256L + threadIdx.x; g < n; g += (long)gridDim.x * 256) {
    const D3 d = cell_d3(X, Xn, P, n, cell_of_index(P, g));
    const double v[kD3] = {d.mu, d.c, d.cu, d.cv, d.Am, d.av, d.nu, d.Bnu};
#pragma unroll
    for (int k = 0; k < kD3; ++k) Q[k * n + g] = v[k];
  }
}

ACCH_DEV D3 load_d3(const double *__restrict__ Q, long n, long g) {
  return D3{Q[g], Q[n + g], Q[2 * n + g], Q[3 * n + g], Q[4 * n + g], Q[5 * n + g], Q[6 * n + g], Q[7 * n + g]};
}

// The 40 slots of every cell from the cell quantities of k_celld3d.
__global__ __launch_bounds__(256) void k_jacobian3d(Phys P, const double *__restrict__ Q, double inv_dt,
                                                     double *__restrict__ J) {
  const long n = (long)P.nx * P.ny * P.nz;
  const double hg = 0.5 * P.gamma;
  for (long g = blockIdx.x * 256L + threadIdx.x; g < n; g += (long)gridDim.x * 256) {
    const C3 c = cell_of_index(P, g);
    const D3 k = load_d3(Q, n, g);
    D3 nb[6];
    bool fe[6];
    double D[6], ct[6];
    double Wc = 0.0, sWD = 0.0, sW2c = 0.0;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      fe[f] = face3(P, c.x, c.y, c.z, f);
      const C3 cn = step(c, f);
      nb[f] = load_d3(Q, n, gidx(P, cn.x, cn.y, cn.z));
      D[f] = nb[f].mu - k.mu;
      ct[f] = 0.5 * (k.c + nb[f].c);
      if (fe[f]) {
        const double w = face_w(P, f);
        Wc += w * ct[f];
        sWD += w * D[f];
        sW2c += w * w * ct[f];
      }
    }
    double s[kNSlot3D];
    s[0] = inv_dt - 0.5 * k.cu * sWD + k.Am * Wc + hg * sW2c;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      const double w = face_w(P, f);
      s[1 + f] = fe[f] ? -w * (0.5 * nb[f].cu * D[f] + ct[f] * nb[f].Am + hg * Wc) : 0.0;
      // second neighbour along the face normal: both faces must exist
      const C3 c1 = step(c, f);
      s[7 + f] = (fe[f] && face3(P, c1.x, c1.y, c1.z, f)) ? hg * w * w * ct[f] : 0.0;
      s[26 + f] = fe[f] ? -w * (0.5 * nb[f].cv * D[f] + ct[f] * nb[f].av) : 0.0;
      s[33 + f] = fe[f] ? -k.c * hg * w / P.rho : 0.0;
    }
    // edge neighbours: two paths, one through each face
#pragma unroll
    for (int e = 13; e < 25; ++e) {
      const Off3 o = uu3(e);
      int fa = -1, fb = -1;
      if (o.dx) fa = o.dx < 0 ? 0 : 1;
      if (o.dy) (fa < 0 ? fa : fb) = o.dy < 0 ? 2 : 3;
      if (o.dz) fb = o.dz < 0 ? 4 : 5;
      s[e] = (fe[fa] && fe[fb]) ? hg * face_w(P, fa) * face_w(P, fb) * (ct[fa] + ct[fb]) : 0.0;
    }
    s[25] = -0.5 * k.cv * sWD + k.av * Wc;
    s[32] = inv_dt + (k.cv * k.nu + k.c * k.Bnu) / P.rho;
    s[39] = (k.cu * k.nu + k.c * k.av) / P.rho;
#pragma unroll
    for (int q = 0; q < kNSlot3D; ++q) J[(long)q * n + g] = s[q];
  }
}

}  // namespace

// y = J x (40 slots); neighbours outside a Neumann domain carry zero coefficients.
ACCH_DEV void spmv3d_cell(const Phys &P, const double *__restrict__ J, const double *__restrict__ x, long n, long g,
                          double &yu, double &yv) {
  const C3 c = cell_of_index(P, g);
  const double *xu = x, *xv = x + n;
  double a = 0.0, b = 0.0;
#pragma unroll
  for (int k = 0; k < 25; ++k) {
    const Off3 o = uu3(k);
    a = fma(J[(long)k * n + g], xu[gidx(P, c.x + o.dx, c.y + o.dy, c.z + o.dz)], a);
  }
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    const Off3 o = star3(k);
    const long h = gidx(P, c.x + o.dx, c.y + o.dy, c.z + o.dz);
    a = fma(J[(long)(25 + k) * n + g], xv[h], a);
    b = fma(J[(long)(32 + k) * n + g], xv[h], b);
  }
  b = fma(J[39L * n + g], xu[g], b);
  yu = a;
  yv = b;
}

// y = J^T x: slot k of row r = c - o_k lands in column c; rows outside a Neumann
// domain do not exist.
ACCH_DEV void spmv3d_t_cell(const Phys &P, const double *__restrict__ J, const double *__restrict__ x, long n, long g,
                            double &yu, double &yv) {
  const C3 c = cell_of_index(P, g);
  const double *xu = x, *xv = x + n;
  auto row = [&](Off3 o, long &r) {
    const int rx = c.x - o.dx, ry = c.y - o.dy, rz = c.z - o.dz;
    r = gidx(P, rx, ry, rz);
    return P.periodic || (rx >= 0 && rx < P.nx && ry >= 0 && ry < P.ny && rz >= 0 && rz < P.nz);
  };
  double a = 0.0, b = 0.0;
#pragma unroll
  for (int k = 0; k < 25; ++k) {
    long r;
    const bool ok = row(uu3(k), r);
    const double t = J[(long)k * n + r] * xu[r];
    a += ok ? t : 0.0;
  }
  a = fma(J[39L * n + g], xv[g], a);
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    long r;
    const bool ok = row(star3(k), r);
    const double t = J[(long)(25 + k) * n + r] * xu[r] + J[(long)(32 + k) * n + r] * xv[r];
    b += ok ? t : 0.0;
  }
  yu = a;
  yv = b;
}

namespace {

template <bool TR>
__global__ __launch_bounds__(256) void k_spmv3d(Phys P, const double *__restrict__ J, const double *__restrict__ x,
                                                 double *__restrict__ y) {
  const long n = (long)P.nx * P.ny * P.nz;
  for (long g = blockIdx.x * 256L + threadIdx.x; g < n; g += (long)gridDim.x * 256) {
    double yu, yv;
    if constexpr (TR) spmv3d_t_cell(P, J, x, n, g, yu, yv);
    else spmv3d_cell(P, J, x, n, g, yu, yv);
    y[g] = yu;
    y[n + g] = yv;
  }
}

// w = J z_j (or J^T z_j) fused with the Gram–Schmidt dots, one instantiation per
// Arnoldi step (as k_spmv_dots2d).
template <int J, bool TR>
__global__ __launch_bounds__(256) void k_spmv_dots3d(Phys P, const double *__restrict__ Jm,
                                                      const double *__restrict__ Z, double *__restrict__ V,
                                                      long vstride, GmresState *st, RedBuf red) {
  if (st->done) return;
  constexpr int NV = pow2_at_least(J + 1);
  const long n = (long)P.nx * P.ny * P.nz;
  const double *z = Z + (long)J * vstride;
  double *w = V + (long)(J + 1) * vstride;
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  for (long g = blockIdx.x * 256L + threadIdx.x; g < n; g += (long)gridDim.x * 256) {
    double bu[J + 1], bv[J + 1];
#pragma unroll
    for (int i = 0; i <= J; ++i) {
      bu[i] = V[(long)i * vstride + g];
      bv[i] = V[(long)i * vstride + n + g];
    }
    double yu, yv;
    if constexpr (TR) spmv3d_t_cell(P, Jm, z, n, g, yu, yv);
    else spmv3d_cell(P, Jm, z, n, g, yu, yv);
    w[g] = yu;
    w[n + g] = yv;
#pragma unroll
    for (int i = 0; i <= J; ++i) acc[i] = fma(yu, bu[i], fma(yv, bv[i], acc[i]));
  }
  block_partial_multi<NV>(acc, red.partials, threadIdx.x, 256, blockIdx.x, gridDim.x, J + 1);
}

// ---- adjoint pieces (see adjoint2d.hip for the derivation) -------------------
__global__ __launch_bounds__(256) void k_adjoint_prev_a3d(Phys P, const double *__restrict__ X1,
                                                           const double *__restrict__ X0, double inv_dt,
                                                           const double *__restrict__ lam, double lam_scale,
                                                           double *__restrict__ bar, double *__restrict__ out,
                                                           RedBuf red) {
  const long n = (long)P.nx * P.ny * P.nz;
  const double hg = 0.5 * P.gamma;
  const Trial T{X1, nullptr, X0, 0.0, 0.0, n};
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (long g = blockIdx.x * 256L + threadIdx.x; g < n; g += (long)gridDim.x * 256) {
    const C3 c = cell_of_index(P, g);
    const double u1 = X1[g], v1 = X1[n + g], u0 = X0[g], v0 = X0[n + g];
    const double lu = lam_scale * lam[g], lv = lam_scale * lam[n + g];
    double phi, dphi1, dphi0, psi, dpsi1, dpsi0, cc, cu0, cv0;
    g2s_d01(u1 + v1, u0 + v0, P.S, phi, dphi1, dphi0);
    g2s_d01(u1 - v1, u0 - v0, P.S, psi, dpsi1, dpsi0);
    mobility_d0(P.mob, u1, v1, u0, v0, cc, cu0, cv0);
    const double lapu = lap3(X1, P, c.x, c.y, c.z) + lap3(X0, P, c.x, c.y, c.z);
    const double lapv = lap3(X1 + n, P, c.x, c.y, c.z) + lap3(X0 + n, P, c.x, c.y, c.z);
    const double mu = -0.5 * P.alpha * (u1 + u0 - 1.0) + P.theta * (phi + psi) - hg * lapu;
    const double nu = -0.5 * P.beta * (v1 + v0) + P.theta * (phi - psi) - hg * lapv;
    double mubar = 0.0, cbar = lv * nu / P.rho;
    for (int f = 0; f < 6; ++f) {
      if (!face3(P, c.x, c.y, c.z, f)) continue;
      const C3 nb = step(c, f);
      const Q3 qn = cell_q3(T, P, nb);
      const double lun = lam_scale * ld3(lam, P, nb.x, nb.y, nb.z);
      const double w = face_w(P, f);
      mubar += w * 0.5 * (cc + qn.c) * (lu - lun);
      cbar += 0.5 * w * (qn.mu - mu) * (lun - lu);
    }
    const double nubar = lv * cc / P.rho;
    const double mu_u0 = -0.5 * P.alpha + P.theta * (dphi0 + dpsi0), mu_v0 = P.theta * (dphi0 - dpsi0);
    const double nu_u0 = P.theta * (dphi0 - dpsi0), nu_v0 = -0.5 * P.beta + P.theta * (dphi0 + dpsi0);
    out[g] = -lu * inv_dt + mubar * mu_u0 + nubar * nu_u0 + cbar * cu0;
    out[n + g] = -lv * inv_dt + mubar * mu_v0 + nubar * nu_v0 + cbar * cv0;
    bar[g] = mubar;
    bar[n + g] = nubar;
    acc[0] = fma(mubar, -0.5 * (u1 + u0 - 1.0), acc[0]);
    acc[1] = fma(nubar, -0.5 * (v1 + v0), acc[1]);
    acc[2] += mubar * (phi + psi) + nubar * (phi - psi);
    acc[3] += -0.5 * (mubar * lapu + nubar * lapv);
  }
  block_partial<4>(acc, red.partials, threadIdx.x, 256, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(256) void k_adjoint_prev_b3d(Phys P, const double *__restrict__ bar,
                                                           double *__restrict__ out) {
  const long n = (long)P.nx * P.ny * P.nz;
  const double hg = 0.5 * P.gamma;
  for (long g = blockIdx.x * 256L + threadIdx.x; g < n; g += (long)gridDim.x * 256) {
    const C3 c = cell_of_index(P, g);
    out[g] -= hg * lap3(bar, P, c.x, c.y, c.z);
    out[n + g] -= hg * lap3(bar + n, P, c.x, c.y, c.z);
  }
}

__global__ __launch_bounds__(256) void k_energy_grad3d(Phys P, const double *__restrict__ X, double vol,
                                                        double *__restrict__ gout, RedBuf red) {
  const long n = (long)P.nx * P.ny * P.nz;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (long g = blockIdx.x * 256L + threadIdx.x; g < n; g += (long)gridDim.x * 256) {
    const C3 c = cell_of_index(P, g);
    const double u = X[g], v = X[n + g];
    const double p = u + v, q = u - v;
    const double dp = dPhi(p), dq = dPhi(q);
    gout[g] = vol * (0.5 * P.alpha * (1.0 - 2.0 * u) + P.theta * (dp + dq) - P.gamma * lap3(X, P, c.x, c.y, c.z));
    gout[n + g] = vol * (-P.beta * v + P.theta * (dp - dq) - P.gamma * lap3(X + n, P, c.x, c.y, c.z));
    double gd = 0.0;
    for (int fld = 0; fld < 2; ++fld) {
      const double *fp = X + fld * n;
      const double m = fp[g];
      for (int f = 0; f < 6; ++f) {
        const C3 nb = step(c, f);
        const double d = ld3(fp, P, nb.x, nb.y, nb.z) - m;
        gd += 0.5 * d * d * face_w(P, f);
      }
    }
    acc[0] = fma(0.5 * u, 1.0 - u, acc[0]);
    acc[1] = fma(-0.5 * v, v, acc[1]);
    acc[2] += Phi(p) + Phi(q);
    acc[3] = fma(0.5, gd, acc[3]);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) acc[k] *= vol;
  block_partial<4>(acc, red.partials, threadIdx.x, 256, blockIdx.x, gridDim.x);
}

int nblocks3(const Phys &P) { return reduce_blocks((long)P.nx * P.ny * P.nz); }

}  // namespace

hipError_t launch_residual3d(const BatchLaunch &bl, const double *X, const double *Sdir, double lam,
                             const GmresState *shift_st, const double *Xn, double dt, double *Xt, double *F,
                             double *Q, const RedBuf &red, hipStream_t s) {
  hipLaunchKernelGGL(k_cellq3d, dim3(nblocks3(bl.P0)), dim3(256), 0, s, bl.P0, X, Sdir, lam, shift_st, Xn, Q);
  hipLaunchKernelGGL(k_residual3d, dim3(bl.grid[kFamCell]), dim3(256), 0, s, bl.P0, X, Sdir, lam, shift_st, Xn,
                     1.0 / dt, (const double *)Q, Xt, F, red);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(kFinPlain, 2, red, bl, kFamCell, nullptr, FinalizeArgs{}, s);
}

hipError_t launch_energy3d(const BatchLaunch &bl, const double *X, const RedBuf &red, hipStream_t s) {
  hipLaunchKernelGGL(k_energy3d, dim3(bl.grid[kFamCell]), dim3(256), 0, s, bl.P0, X, red);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(kFinPlain, 2, red, bl, kFamCell, nullptr, FinalizeArgs{}, s);
}

hipError_t launch_jacobian3d(const BatchLaunch &bl, const double *X, const double *Xn, double dt, double *J,
                             double *Q, hipStream_t s) {
  hipLaunchKernelGGL(k_celld3d, dim3(nblocks3(bl.P0)), dim3(256), 0, s, bl.P0, X, Xn, Q);
  hipLaunchKernelGGL(k_jacobian3d, dim3(nblocks3(bl.P0)), dim3(256), 0, s, bl.P0, (const double *)Q, 1.0 / dt, J);
  return hipGetLastError();
}

hipError_t launch_spmv3d(const BatchLaunch &bl, const double *J, const double *x, double *y, int transpose,
                         hipStream_t s) {
  if (transpose)
    hipLaunchKernelGGL(k_spmv3d<true>, dim3(nblocks3(bl.P0)), dim3(256), 0, s, bl.P0, J, x, y);
  else
    hipLaunchKernelGGL(k_spmv3d<false>, dim3(nblocks3(bl.P0)), dim3(256), 0, s, bl.P0, J, x, y);
  return hipGetLastError();
}

template <int J, bool TR>
static hipError_t dots3_at(int j, const BatchLaunch &bl, const double *Jm, const double *Z, double *V, long vstride,
                           GmresState *st, const RedBuf &red, hipStream_t s) {
  if (j == J) {
    hipLaunchKernelGGL((k_spmv_dots3d<J, TR>), dim3(bl.grid[kFamCell]), dim3(256), 0, s, bl.P0, Jm, Z, V, vstride,
                       st, red);
    return hipGetLastError();
  }
  if constexpr (J + 1 < kMaxRestart) return dots3_at<J + 1, TR>(j, bl, Jm, Z, V, vstride, st, red, s);
  return hipErrorInvalidValue;
}

hipError_t launch_spmv_dots3d(const BatchLaunch &bl, const double *J, const double *Z, double *V, long vstride, int j,
                              int transpose, GmresState *st, const RedBuf &red, hipStream_t s) {
  if (j < 0 || j >= kMaxRestart) return hipErrorInvalidValue;
  hipError_t e = transpose ? dots3_at<0, true>(j, bl, J, Z, V, vstride, st, red, s)
                           : dots3_at<0, false>(j, bl, J, Z, V, vstride, st, red, s);
  return e;   // the dots are summed by the Gram–Schmidt kernel (k_gmres_orth)
}

hipError_t launch_adjoint_prev3d(const Phys &P, const double *X1, const double *X0, double dt, const double *lam,
                                 double lam_scale, double *bar, double *out, const RedBuf &red, hipStream_t s) {
  const int nb = nblocks3(P);
  hipLaunchKernelGGL(k_adjoint_prev_a3d, dim3(nb), dim3(256), 0, s, P, X1, X0, 1.0 / dt, lam, lam_scale, bar, out,
                     red);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  BatchLaunch bl = single_launch(P, 0);
  e = launch_finalize(kFinPlain, 4, red, bl, kFamCell, nullptr, FinalizeArgs{}, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_adjoint_prev_b3d, dim3(nb), dim3(256), 0, s, P, bar, out);
  return hipGetLastError();
}

hipError_t launch_energy_grad3d(const Phys &P, const double *X, double vol, double *g, const RedBuf &red,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_energy_grad3d, dim3(nblocks3(P)), dim3(256), 0, s, P, X, vol, g, red);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(kFinPlain, 4, red, single_launch(P, 0), kFamCell, nullptr, FinalizeArgs{}, s);
}

}  // namespace acch
