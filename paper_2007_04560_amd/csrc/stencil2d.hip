// 2D stencil kernels of scheme (2.20): residual, discrete energy and mass,
// analytic Jacobian assembly and the Jacobian product.
//
// Fields are FP64, x fastest; a state vector holds the u field then the v field.
// The residual and Jacobian kernels stage a (32+4) x (8+4) tile of the four
// fields in LDS (the radius-2 dependence of F_u), evaluate the cell quantities
// (mu, c, ...) once on the tile plus a one-cell halo, and then the face fluxes.
#include "kernels.h"
#include "physics.h"

namespace acch {
namespace {

constexpr int TX = 32, TY = 8;             // output tile, one cell per thread
constexpr int LX2 = TX + 4, LY2 = TY + 4;  // fields with halo 2
constexpr int LX1 = TX + 2, LY1 = TY + 2;  // cell quantities with halo 1

// Load the four fields of a tile with a 2-cell halo.  With Sdir the unknown state is
// the line-search trial X + lam (S - shift e_u).
ACCH_DEV void load_tile(const Phys &P, const double *__restrict__ X, const double *__restrict__ Sdir,
                        double lam, const double *shift_ptr, const double *__restrict__ Xn, int bx0, int by0,
                        int tid, double (*su1)[LX2], double (*sv1)[LX2], double (*su0)[LX2],
                        double (*sv0)[LX2]) {
  const long n = (long)P.nx * P.ny;
  const double shift = shift_ptr ? *shift_ptr : 0.0;
  for (int k = tid; k < LX2 * LY2; k += TX * TY) {
    const int ly = k / LX2, lx = k - ly * LX2;
    const int gx = wrap_index(bx0 + lx - 2, P.nx, P.periodic);
    const int gy = wrap_index(by0 + ly - 2, P.ny, P.periodic);
    const long g = (long)gy * P.nx + gx;
    double u1 = X[g], v1 = X[n + g];
    if (Sdir) {
      u1 = fma(lam, Sdir[g] - shift, u1);
      v1 = fma(lam, Sdir[n + g], v1);
    }
    su1[ly][lx] = u1;
    sv1[ly][lx] = v1;
    su0[ly][lx] = Xn[g];
    sv0[ly][lx] = Xn[n + g];
  }
}

ACCH_DEV double lap5(double (*s)[LX2], int cy, int cx, double wx, double wy) {
  const double c = s[cy][cx];
  return (s[cy][cx - 1] - c + (s[cy][cx + 1] - c)) * wx + (s[cy - 1][cx] - c + (s[cy + 1][cx] - c)) * wy;
}

// ---------------------------------------------------------------------------
// Residual F(X; Xn, dt), optional trial state, ||F||^2 and admissibility count.
// ---------------------------------------------------------------------------
// Tile origin of local tile lb (tiles of TX x TY cells, x fastest).
ACCH_DEV void tile_origin(const Phys &P, int lb, int &bx0, int &by0) {
  const int ntx = (P.nx + TX - 1) / TX;
  const int ty = lb / ntx;
  bx0 = (lb - ty * ntx) * TX;
  by0 = ty * TY;
}

// Batched launches: lam_b / shift_st (may be null) are per instance; the state
// vectors are offset by the instance's xoff.
__global__ __launch_bounds__(TX *TY) void k_residual2d(Phys P0, Batch bt, const double *__restrict__ X,
                                                        const double *__restrict__ Sdir, double lam0,
                                                        const double *__restrict__ lam_b,
                                                        const GmresState *shift_st, const double *__restrict__ Xn,
                                                        double inv_dt, double *__restrict__ Xt,
                                                        double *__restrict__ F, RedBuf red) {
  __shared__ double su1[LY2][LX2], sv1[LY2][LX2], su0[LY2][LX2], sv0[LY2][LX2];
  __shared__ double smu[LY1][LX1], sc[LY1][LX1], spm[LY1][LX1];
  const Loc L = locate(bt, kFamTile);
  if (!L.on) return;
  const Phys P = bt.map[kFamTile] ? bt.inst[L.b].P : P0;
  const long xo = bt.map[kFamTile] ? bt.inst[L.b].xoff : 0;
  X += xo;
  Xn += xo;
  F += xo;
  if (Sdir) Sdir += xo;
  if (Xt) Xt += xo;
  const double lam = lam_b ? lam_b[L.b] : lam0;
  const double *shift = shift_st ? &shift_st[L.b].shift : nullptr;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
  int bx0, by0;
  tile_origin(P, L.lb, bx0, by0);
  const long n = (long)P.nx * P.ny;
  load_tile(P, X, Sdir, lam, shift, Xn, bx0, by0, tid, su1, sv1, su0, sv0);
  __syncthreads();
  const double hg = 0.5 * P.gamma;
  for (int k = tid; k < LX1 * LY1; k += TX * TY) {
    const int ly = k / LX1, lx = k - ly * LX1;
    const int cy = ly + 1, cx = lx + 1;
    const double u1 = su1[cy][cx], v1 = sv1[cy][cx], u0 = su0[cy][cx], v0 = sv0[cy][cx];
    const double phi = g2s(u1 + v1, u0 + v0, P.S);
    const double psi = g2s(u1 - v1, u0 - v0, P.S);
    const double lap = lap5(su1, cy, cx, P.wx, P.wy) + lap5(su0, cy, cx, P.wx, P.wy);
    smu[ly][lx] = -0.5 * P.alpha * (u1 + u0 - 1.0) + P.theta * (phi + psi) - hg * lap;
    sc[ly][lx] = mobility_of(P.mob, u1, v1, u0, v0);
    spm[ly][lx] = P.theta * (phi - psi);
  }
  __syncthreads();
  const int gx = bx0 + tx, gy = by0 + ty;
  double acc[2] = {0.0, 0.0};
  if (gx < P.nx && gy < P.ny) {
    const int cy = ty + 2, cx = tx + 2, my = ty + 1, mx = tx + 1;
    const double u1 = su1[cy][cx], v1 = sv1[cy][cx], u0 = su0[cy][cx], v0 = sv0[cy][cx];
    const double lapv = lap5(sv1, cy, cx, P.wx, P.wy) + lap5(sv0, cy, cx, P.wx, P.wy);
    const double nu = -0.5 * P.beta * (v1 + v0) + spm[my][mx] - hg * lapv;
    const double ck = sc[my][mx], muk = smu[my][mx];
    const double Fv = (v1 - v0) * inv_dt + ck * nu / P.rho;
    double div = 0.0;
    if (face_exists(gx, -1, P.nx, P.periodic)) div += 0.5 * (ck + sc[my][mx - 1]) * (smu[my][mx - 1] - muk) * P.wx;
    if (face_exists(gx, 1, P.nx, P.periodic)) div += 0.5 * (ck + sc[my][mx + 1]) * (smu[my][mx + 1] - muk) * P.wx;
    if (face_exists(gy, -1, P.ny, P.periodic)) div += 0.5 * (ck + sc[my - 1][mx]) * (smu[my - 1][mx] - muk) * P.wy;
    if (face_exists(gy, 1, P.ny, P.periodic)) div += 0.5 * (ck + sc[my + 1][mx]) * (smu[my + 1][mx] - muk) * P.wy;
    const double Fu = (u1 - u0) * inv_dt - div;
    const long g = (long)gy * P.nx + gx;
    F[g] = Fu;
    F[n + g] = Fv;
    if (Xt) {
      Xt[g] = u1;
      Xt[n + g] = v1;
    }
    acc[0] = Fu * Fu + Fv * Fv;
    const double p = u1 + v1, q = u1 - v1;
    acc[1] = (p > 0.0 && p < 1.0 && q > 0.0 && q < 1.0) ? 0.0 : 1.0;
  }
  block_partial<2>(acc, red.partials, tid, TX * TY, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// Discrete energy (eqs. relations, freeenergy) with the exact Phi, and sum u.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_energy2d(Phys P0, Batch bt, const double *__restrict__ X, RedBuf red) {
  const Loc L = locate(bt, kFamCell);
  if (!L.on) return;
  const Phys P = bt.map[kFamCell] ? bt.inst[L.b].P : P0;
  if (bt.map[kFamCell]) X += bt.inst[L.b].xoff;
  const long n = (long)P.nx * P.ny;
  double acc[2] = {0.0, 0.0};
  for (long g = L.lb * 256L + threadIdx.x; g < n; g += (long)L.nb * 256) {
    const int gy = (int)(g / P.nx), gx = (int)(g - (long)gy * P.nx);
    const double u = X[g], v = X[n + g];
    double e = 0.5 * P.alpha * u * (1.0 - u) - 0.5 * P.beta * v * v + P.theta * (Phi(u + v) + Phi(u - v));
    const long gw = (long)gy * P.nx + wrap_index(gx - 1, P.nx, P.periodic);
    const long ge = (long)gy * P.nx + wrap_index(gx + 1, P.nx, P.periodic);
    const long gs = (long)wrap_index(gy - 1, P.ny, P.periodic) * P.nx + gx;
    const long gn = (long)wrap_index(gy + 1, P.ny, P.periodic) * P.nx + gx;
    double grad = 0.0;
    for (int c = 0; c < 2; ++c) {
      const double *f = X + c * n;
      const double fk = f[g];
      const double dw = fk - f[gw], de = f[ge] - fk, ds = fk - f[gs], dn = f[gn] - fk;
      grad += 0.5 * (dw * dw + de * de) * P.wx + 0.5 * (ds * ds + dn * dn) * P.wy;
    }
    e += 0.5 * P.gamma * grad;
    acc[0] += e;
    acc[1] += u;
  }
  block_partial<2>(acc, red.partials, threadIdx.x, 256, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// Analytic Jacobian, 24 slot arrays J[slot][cell] (slot table in include/acch.h).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(TX *TY) void k_jacobian2d(Phys P0, Batch bt, const double *__restrict__ X,
                                                        const double *__restrict__ Xn, double inv_dt,
                                                        double *__restrict__ J) {
  __shared__ double su1[LY2][LX2], sv1[LY2][LX2], su0[LY2][LX2], sv0[LY2][LX2];
  __shared__ double smu[LY1][LX1], sc[LY1][LX1], scu[LY1][LX1], scv[LY1][LX1], sAm[LY1][LX1], sav[LY1][LX1];
  const Loc L = locate(bt, kFamTile);
  if (!L.on) return;
  const Phys P = bt.map[kFamTile] ? bt.inst[L.b].P : P0;
  if (bt.map[kFamTile]) {
    X += bt.inst[L.b].xoff;
    Xn += bt.inst[L.b].xoff;
    J += bt.inst[L.b].joff;
  }
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
  int bx0, by0;
  tile_origin(P, L.lb, bx0, by0);
  const long n = (long)P.nx * P.ny;
  load_tile(P, X, nullptr, 0.0, nullptr, Xn, bx0, by0, tid, su1, sv1, su0, sv0);
  __syncthreads();
  const double hg = 0.5 * P.gamma;
  for (int k = tid; k < LX1 * LY1; k += TX * TY) {
    const int ly = k / LX1, lx = k - ly * LX1;
    const int cy = ly + 1, cx = lx + 1;
    const int gx = bx0 + lx - 1, gy = by0 + ly - 1;   // unwrapped; only the existence tests use it
    const double u1 = su1[cy][cx], v1 = sv1[cy][cx], u0 = su0[cy][cx], v0 = sv0[cy][cx];
    double phi, dphi, psi, dpsi, c, cu, cv;
    g2s_d(u1 + v1, u0 + v0, P.S, phi, dphi);
    g2s_d(u1 - v1, u0 - v0, P.S, psi, dpsi);
    mobility_d(P.mob, u1, v1, u0, v0, c, cu, cv);
    const double lap = lap5(su1, cy, cx, P.wx, P.wy) + lap5(su0, cy, cx, P.wx, P.wy);
    double wsum = 0.0;
    if (face_exists(gx, -1, P.nx, P.periodic)) wsum += P.wx;
    if (face_exists(gx, 1, P.nx, P.periodic)) wsum += P.wx;
    if (face_exists(gy, -1, P.ny, P.periodic)) wsum += P.wy;
    if (face_exists(gy, 1, P.ny, P.periodic)) wsum += P.wy;
    smu[ly][lx] = -0.5 * P.alpha * (u1 + u0 - 1.0) + P.theta * (phi + psi) - hg * lap;
    sc[ly][lx] = c;
    scu[ly][lx] = cu;
    scv[ly][lx] = cv;
    sAm[ly][lx] = -0.5 * P.alpha + P.theta * (dphi + dpsi) + hg * wsum;
    sav[ly][lx] = P.theta * (dphi - dpsi);
  }
  __syncthreads();
  const int gx = bx0 + tx, gy = by0 + ty;
  if (gx >= P.nx || gy >= P.ny) return;
  const int cy = ty + 2, cx = tx + 2, my = ty + 1, mx = tx + 1;
  const double u1 = su1[cy][cx], v1 = sv1[cy][cx], u0 = su0[cy][cx], v0 = sv0[cy][cx];
  double phi, dphi, psi, dpsi;
  g2s_d(u1 + v1, u0 + v0, P.S, phi, dphi);
  g2s_d(u1 - v1, u0 - v0, P.S, psi, dpsi);
  const double lapv = lap5(sv1, cy, cx, P.wx, P.wy) + lap5(sv0, cy, cx, P.wx, P.wy);
  const double nu = -0.5 * P.beta * (v1 + v0) + P.theta * (phi - psi) - hg * lapv;
  const bool eW = face_exists(gx, -1, P.nx, P.periodic), eE = face_exists(gx, 1, P.nx, P.periodic);
  const bool eS = face_exists(gy, -1, P.ny, P.periodic), eN = face_exists(gy, 1, P.ny, P.periodic);
  const double wsum = (eW ? P.wx : 0.0) + (eE ? P.wx : 0.0) + (eS ? P.wy : 0.0) + (eN ? P.wy : 0.0);
  const double Bnu = -0.5 * P.beta + P.theta * (dphi + dpsi) + hg * wsum;
  const double ck = sc[my][mx], muk = smu[my][mx], cuk = scu[my][mx], cvk = scv[my][mx];
  const double Amk = sAm[my][mx], avk = sav[my][mx];
  // faces W, E, S, N: neighbour (dy, dx) in the halo-1 arrays, weight, existence
  const int fdy[4] = {0, 0, -1, 1}, fdx[4] = {-1, 1, 0, 0};
  const double fw[4] = {P.wx, P.wx, P.wy, P.wy};
  const bool fe[4] = {eW, eE, eS, eN};
  double D[4], ct[4];
  double Wc = 0.0, sWD = 0.0, sW2c = 0.0;
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const int yy = my + fdy[f], xx = mx + fdx[f];
    D[f] = smu[yy][xx] - muk;
    ct[f] = 0.5 * (ck + sc[yy][xx]);
    if (fe[f]) {
      Wc += fw[f] * ct[f];
      sWD += fw[f] * D[f];
      sW2c += fw[f] * fw[f] * ct[f];
    }
  }
  double s[kNSlot2D];
  s[0] = inv_dt - 0.5 * cuk * sWD + Amk * Wc + hg * sW2c;
  // first neighbours (slots 1..4 = W, E, S, N)
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const int yy = my + fdy[f], xx = mx + fdx[f];
    s[1 + f] = fe[f] ? -fw[f] * (0.5 * scu[yy][xx] * D[f] + ct[f] * sAm[yy][xx] + hg * Wc) : 0.0;
    s[14 + f] = fe[f] ? -fw[f] * (0.5 * scv[yy][xx] * D[f] + ct[f] * sav[yy][xx]) : 0.0;
    s[19 + f] = fe[f] ? -ck * hg * fw[f] / P.rho : 0.0;
  }
  // second neighbours along the axes: (-2,0), (2,0), (0,-2), (0,2)
  s[5] = (eW && face_exists(gx - 1, -1, P.nx, P.periodic)) ? hg * P.wx * P.wx * ct[0] : 0.0;
  s[6] = (eE && face_exists(gx + 1, 1, P.nx, P.periodic)) ? hg * P.wx * P.wx * ct[1] : 0.0;
  s[7] = (eS && face_exists(gy - 1, -1, P.ny, P.periodic)) ? hg * P.wy * P.wy * ct[2] : 0.0;
  s[8] = (eN && face_exists(gy + 1, 1, P.ny, P.periodic)) ? hg * P.wy * P.wy * ct[3] : 0.0;
  // diagonal neighbours: two paths, through the x face and through the y face
  const double wxy = hg * P.wx * P.wy;
  s[9] = (eW && eS) ? wxy * (ct[0] + ct[2]) : 0.0;   // (-1,-1)
  s[10] = (eE && eS) ? wxy * (ct[1] + ct[2]) : 0.0;  // (1,-1)
  s[11] = (eW && eN) ? wxy * (ct[0] + ct[3]) : 0.0;  // (-1,1)
  s[12] = (eE && eN) ? wxy * (ct[1] + ct[3]) : 0.0;  // (1,1)
  s[13] = -0.5 * cvk * sWD + avk * Wc;
  s[18] = inv_dt + (cvk * nu + ck * Bnu) / P.rho;
  s[23] = (cuk * nu + ck * avk) / P.rho;
  const long g = (long)gy * P.nx + gx;
#pragma unroll
  for (int k = 0; k < kNSlot2D; ++k) J[k * n + g] = s[k];
}

// y = J x for the 24-slot layout.
ACCH_DEV void spmv_cell(const Phys &P, const double *__restrict__ J, const double *__restrict__ x, long n,
                        int gx, int gy, double &yu, double &yv) {
  const int xm2 = wrap_index(gx - 2, P.nx, P.periodic), xm1 = wrap_index(gx - 1, P.nx, P.periodic);
  const int xp1 = wrap_index(gx + 1, P.nx, P.periodic), xp2 = wrap_index(gx + 2, P.nx, P.periodic);
  const int ym2 = wrap_index(gy - 2, P.ny, P.periodic), ym1 = wrap_index(gy - 1, P.ny, P.periodic);
  const int yp1 = wrap_index(gy + 1, P.ny, P.periodic), yp2 = wrap_index(gy + 2, P.ny, P.periodic);
  const long r0 = (long)gy * P.nx, rm1 = (long)ym1 * P.nx, rp1 = (long)yp1 * P.nx;
  const long rm2 = (long)ym2 * P.nx, rp2 = (long)yp2 * P.nx;
  const long g = r0 + gx;
  const double *xu = x, *xv = x + n;
  const long iw = r0 + xm1, ie = r0 + xp1, is = rm1 + gx, in_ = rp1 + gx;
  double a = J[0 * n + g] * xu[g];
  a = fma(J[1 * n + g], xu[iw], a);
  a = fma(J[2 * n + g], xu[ie], a);
  a = fma(J[3 * n + g], xu[is], a);
  a = fma(J[4 * n + g], xu[in_], a);
  a = fma(J[5 * n + g], xu[r0 + xm2], a);
  a = fma(J[6 * n + g], xu[r0 + xp2], a);
  a = fma(J[7 * n + g], xu[rm2 + gx], a);
  a = fma(J[8 * n + g], xu[rp2 + gx], a);
  a = fma(J[9 * n + g], xu[rm1 + xm1], a);
  a = fma(J[10 * n + g], xu[rm1 + xp1], a);
  a = fma(J[11 * n + g], xu[rp1 + xm1], a);
  a = fma(J[12 * n + g], xu[rp1 + xp1], a);
  a = fma(J[13 * n + g], xv[g], a);
  a = fma(J[14 * n + g], xv[iw], a);
  a = fma(J[15 * n + g], xv[ie], a);
  a = fma(J[16 * n + g], xv[is], a);
  a = fma(J[17 * n + g], xv[in_], a);
  double b = J[18 * n + g] * xv[g];
  b = fma(J[19 * n + g], xv[iw], b);
  b = fma(J[20 * n + g], xv[ie], b);
  b = fma(J[21 * n + g], xv[is], b);
  b = fma(J[22 * n + g], xv[in_], b);
  b = fma(J[23 * n + g], xu[g], b);
  yu = a;
  yv = b;
}

// y = J^T x for the 24-slot layout: the entry of slot k (column offset o_k) of row
// r = c - o_k lands in column c.  Rows outside a Neumann domain do not exist; slots
// that point outside it are zero, so the two descriptions agree.
ACCH_DEV void spmv_t_cell(const Phys &P, const double *__restrict__ J, const double *__restrict__ x, long n,
                          int gx, int gy, double &yu, double &yv) {
  const double *xu = x, *xv = x + n;
  auto row = [&](int dx, int dy, long &r) -> bool {
    const int rx = gx + dx, ry = gy + dy;
    r = (long)wrap_index(ry, P.ny, P.periodic) * P.nx + wrap_index(rx, P.nx, P.periodic);
    return P.periodic || (rx >= 0 && rx < P.nx && ry >= 0 && ry < P.ny);
  };
  auto term = [&](int slot, int dx, int dy, const double *xf) -> double {
    long r;
    const bool ok = row(dx, dy, r);
    const double a = J[(long)slot * n + r] * xf[r];
    return ok ? a : 0.0;
  };
  double a = term(0, 0, 0, xu);
  a += term(1, 1, 0, xu);
  a += term(2, -1, 0, xu);
  a += term(3, 0, 1, xu);
  a += term(4, 0, -1, xu);
  a += term(5, 2, 0, xu);
  a += term(6, -2, 0, xu);
  a += term(7, 0, 2, xu);
  a += term(8, 0, -2, xu);
  a += term(9, 1, 1, xu);
  a += term(10, -1, 1, xu);
  a += term(11, 1, -1, xu);
  a += term(12, -1, -1, xu);
  a += term(23, 0, 0, xv);
  double b = term(13, 0, 0, xu);
  b += term(14, 1, 0, xu);
  b += term(15, -1, 0, xu);
  b += term(16, 0, 1, xu);
  b += term(17, 0, -1, xu);
  b += term(18, 0, 0, xv);
  b += term(19, 1, 0, xv);
  b += term(20, -1, 0, xv);
  b += term(21, 0, 1, xv);
  b += term(22, 0, -1, xv);
  yu = a;
  yv = b;
}

template <bool TR>
ACCH_DEV void matvec_cell(const Phys &P, const double *__restrict__ J, const double *__restrict__ x, long n, int gx,
                          int gy, double &yu, double &yv) {
  if constexpr (TR) spmv_t_cell(P, J, x, n, gx, gy, yu, yv);
  else spmv_cell(P, J, x, n, gx, gy, yu, yv);
}

// y = J x (TR = false) or J^T x (TR = true).
template <bool TR>
__global__ __launch_bounds__(256) void k_spmv2d(Phys P0, Batch bt, const double *__restrict__ J,
                                                 const double *__restrict__ x, double *__restrict__ y) {
  const Loc L = locate(bt, kFamCell);
  if (!L.on) return;
  const Phys P = bt.map[kFamCell] ? bt.inst[L.b].P : P0;
  if (bt.map[kFamCell]) {
    J += bt.inst[L.b].joff;
    x += bt.inst[L.b].xoff;
    y += bt.inst[L.b].xoff;
  }
  const long n = (long)P.nx * P.ny;
  for (long g = L.lb * 256L + threadIdx.x; g < n; g += (long)L.nb * 256) {
    const int gy = (int)(g / P.nx), gx = (int)(g - (long)gy * P.nx);
    double yu, yv;
    matvec_cell<TR>(P, J, x, n, gx, gy, yu, yv);
    y[g] = yu;
    y[n + g] = yv;
  }
}

// w = J z_j (J^T z_j when TR) written to the Arnoldi slot j+1, fused with the
// classical Gram–Schmidt dots h_ij = inv_norm_i <w, W_i>, i <= j.  One instantiation
// per Arnoldi step j (the host knows j: a cycle's steps are enqueued in order), so
// every basis load of a cell is issued before the first is used.  Skipped when the
// cycle is finished.
template <int J, bool TR>
__global__ __launch_bounds__(256) void k_spmv_dots2d(Phys P0, Batch bt, const double *__restrict__ Jm,
                                                      const double *__restrict__ Z, double *__restrict__ V,
                                                      long vstride, GmresState *st, RedBuf red) {
  const Loc L = locate(bt, kFamCell);
  if (!L.on || st[L.b].done) return;
  const Phys P = bt.map[kFamCell] ? bt.inst[L.b].P : P0;
  if (bt.map[kFamCell]) {
    Jm += bt.inst[L.b].joff;
    Z += bt.inst[L.b].xoff;
    V += bt.inst[L.b].xoff;
  }
  constexpr int NV = pow2_at_least(J + 1);
  const long n = (long)P.nx * P.ny;
  const double *z = Z + (long)J * vstride;
  double *w = V + (long)(J + 1) * vstride;
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  for (long g = L.lb * 256L + threadIdx.x; g < n; g += (long)L.nb * 256) {
    const int gy = (int)(g / P.nx), gx = (int)(g - (long)gy * P.nx);
    double bu[J + 1], bv[J + 1];
#pragma unroll
    for (int i = 0; i <= J; ++i) {
      bu[i] = V[(long)i * vstride + g];
      bv[i] = V[(long)i * vstride + n + g];
    }
    double yu, yv;
    matvec_cell<TR>(P, Jm, z, n, gx, gy, yu, yv);
    w[g] = yu;
    w[n + g] = yv;
#pragma unroll
    for (int i = 0; i <= J; ++i) acc[i] = fma(yu, bu[i], fma(yv, bv[i], acc[i]));
  }
  block_partial_multi<NV>(acc, red.partials, threadIdx.x, 256, blockIdx.x, gridDim.x, J + 1);
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
int reduce_blocks(long n) {
  long b = (n + 255) / 256;
  if (b > kRedBlocks) b = kRedBlocks;
  if (b < 1) b = 1;
  return (int)b;
}

void family_blocks(const Phys &P, int nsub, int (&nb)[kFamilies]) {
  const long n = (long)P.nx * P.ny * (P.nz > 0 ? P.nz : 1);
  nb[kFamTile] = ((P.nx + TX - 1) / TX) * ((P.ny + TY - 1) / TY);
  nb[kFamCell] = reduce_blocks(n);
  nb[kFamElem] = reduce_blocks(2 * n);
  nb[kFamSub] = nsub;
}

BatchLaunch single_launch(const Phys &P, int nsub) {
  BatchLaunch bl{};
  bl.P0 = P;
  bl.count = 1;
  bl.ncell = (long)P.nx * P.ny * (P.nz > 0 ? P.nz : 1);
  family_blocks(P, nsub, bl.grid);
  return bl;
}

hipError_t launch_residual2d(const BatchLaunch &bl, const double *X, const double *Sdir, double lam0,
                             const double *lam_b, const GmresState *shift_st, const double *Xn, double dt, double *Xt,
                             double *F, const RedBuf &red, hipStream_t s) {
  hipLaunchKernelGGL(k_residual2d, dim3(bl.grid[kFamTile]), dim3(TX, TY), 0, s, bl.P0, bl.bt, X, Sdir, lam0, lam_b,
                     shift_st, Xn, 1.0 / dt, Xt, F, red);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(kFinPlain, 2, red, bl, kFamTile, nullptr, FinalizeArgs{}, s);
}

hipError_t launch_energy2d(const BatchLaunch &bl, const double *X, const RedBuf &red, hipStream_t s) {
  hipLaunchKernelGGL(k_energy2d, dim3(bl.grid[kFamCell]), dim3(256), 0, s, bl.P0, bl.bt, X, red);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finalize(kFinPlain, 2, red, bl, kFamCell, nullptr, FinalizeArgs{}, s);
}

hipError_t launch_jacobian2d(const BatchLaunch &bl, const double *X, const double *Xn, double dt, double *J,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_jacobian2d, dim3(bl.grid[kFamTile]), dim3(TX, TY), 0, s, bl.P0, bl.bt, X, Xn, 1.0 / dt, J);
  return hipGetLastError();
}

hipError_t launch_spmv2d(const BatchLaunch &bl, const double *J, const double *x, double *y, int transpose,
                         hipStream_t s) {
  const dim3 grid(bl.grid[kFamCell]);
  if (transpose)
    hipLaunchKernelGGL(k_spmv2d<true>, grid, dim3(256), 0, s, bl.P0, bl.bt, J, x, y);
  else
    hipLaunchKernelGGL(k_spmv2d<false>, grid, dim3(256), 0, s, bl.P0, bl.bt, J, x, y);
  return hipGetLastError();
}

template <int J, bool TR>
static hipError_t spmv_dots_at(int j, const BatchLaunch &bl, const double *Jm, const double *Z, double *V,
                               long vstride, GmresState *st, const RedBuf &red, hipStream_t s) {
  if (j == J) {
    hipLaunchKernelGGL((k_spmv_dots2d<J, TR>), dim3(bl.grid[kFamCell]), dim3(256), 0, s, bl.P0, bl.bt, Jm, Z, V,
                       vstride, st, red);
    return hipGetLastError();
  }
  if constexpr (J + 1 < kMaxRestart) return spmv_dots_at<J + 1, TR>(j, bl, Jm, Z, V, vstride, st, red, s);
  return hipErrorInvalidValue;
}

hipError_t launch_spmv_dots2d(const BatchLaunch &bl, const double *J, const double *Z, double *V, long vstride, int j,
                              int transpose, GmresState *st, const RedBuf &red, hipStream_t s) {
  if (j < 0 || j >= kMaxRestart) return hipErrorInvalidValue;
  hipError_t e = transpose ? spmv_dots_at<0, true>(j, bl, J, Z, V, vstride, st, red, s)
                           : spmv_dots_at<0, false>(j, bl, J, Z, V, vstride, st, red, s);
  return e;   // the dots are summed by the Gram–Schmidt kernel (k_gmres_orth)
}

}  // namespace acch
