// Pointwise pieces of scheme (2.20): the truncated divided difference of Lemma 2.2,
// the mobility and their derivatives.  Device functions only.
#pragma once

#include "common.h"

namespace acch {

// a_m = 1/((2m+1)(2m)) and b_m = 1/(2m+1), m = 1..kMaxS (index 0 unused).
struct SeriesTable {
  double a[kMaxS + 1];
  double b[kMaxS + 1];
};

constexpr SeriesTable make_series_table() {
  SeriesTable t{};
  for (int m = 1; m <= kMaxS; ++m) {
    t.a[m] = 1.0 / ((2.0 * m + 1.0) * (2.0 * m));
    t.b[m] = 1.0 / (2.0 * m + 1.0);
  }
  return t;
}

static __constant__ SeriesTable c_series = make_series_table();

// f_S(x, s) = ln x - sum_{m=1}^{S} a_m (s/x)^{2m}   (Lemma 2.2, constant term dropped)
ACCH_DEV double f_series(double x, double s, int S) {
  const double r = s / x;
  const double t = r * r;
  double p = c_series.a[S];
  for (int m = S - 1; m >= 1; --m) p = fma(t, p, c_series.a[m]);
  return log(x) - t * p;
}

// f_S and its partial derivatives:
//   f_x = (1/x)(1 + sum_m r^{2m}/(2m+1)),   f_s = -(1/x) sum_m r^{2m-1}/(2m+1).
ACCH_DEV void f_series_d(double x, double s, int S, double &f, double &fx, double &fs) {
  const double ix = 1.0 / x;
  const double r = s * ix;
  const double t = r * r;
  double pa = c_series.a[S], pb = c_series.b[S];
  for (int m = S - 1; m >= 1; --m) {
    pa = fma(t, pa, c_series.a[m]);
    pb = fma(t, pb, c_series.b[m]);
  }
  f = log(x) - t * pa;
  fx = ix * fma(t, pb, 1.0);
  fs = -ix * r * pb;
}

// One component of G2^S (eq. D2-1): phi^S = f_S(z, s) - f_S(1 - z, s) with
// z = (x1 + x0)/2, s = (x1 - x0)/2 (the difference form, which tends to Phi'(z)).
ACCH_DEV double g2s(double x1, double x0, int S) {
  const double z = 0.5 * (x1 + x0);
  const double s = 0.5 * (x1 - x0);
  return f_series(z, s, S) - f_series(1.0 - z, s, S);
}

// phi^S and d phi^S / d x1 = 1/2 [f_x(z,s) + f_s(z,s) + f_x(1-z,s) - f_s(1-z,s)].
ACCH_DEV void g2s_d(double x1, double x0, int S, double &g, double &dg) {
  const double z = 0.5 * (x1 + x0);
  const double s = 0.5 * (x1 - x0);
  double f1, fx1, fs1, f2, fx2, fs2;
  f_series_d(z, s, S, f1, fx1, fs1);
  f_series_d(1.0 - z, s, S, f2, fx2, fs2);
  g = f1 - f2;
  dg = 0.5 * (fx1 + fs1 + fx2 - fs2);
}

// phi^S with both partial derivatives: d/dx1 as in g2s_d and
// d phi^S / d x0 = 1/2 [f_x(z,s) - f_s(z,s) + f_x(1-z,s) + f_s(1-z,s)].
ACCH_DEV void g2s_d01(double x1, double x0, int S, double &g, double &d1, double &d0) {
  const double z = 0.5 * (x1 + x0);
  const double s = 0.5 * (x1 - x0);
  double f1, fx1, fs1, f2, fx2, fs2;
  f_series_d(z, s, S, f1, fx1, fs1);
  f_series_d(1.0 - z, s, S, f2, fx2, fs2);
  g = f1 - f2;
  d1 = 0.5 * (fx1 + fs1 + fx2 - fs2);
  d0 = 0.5 * (fx1 - fs1 + fx2 + fs2);
}

// Mobility inside A~ and its derivatives with respect to (u1, v1).
ACCH_DEV double mobility_of(int mob, double u1, double v1, double u0, double v0) {
  if (mob == 0) {
    const double ub = 0.5 * (u1 + u0), vb = 0.5 * (v1 + v0);
    return ub * (1.0 - ub) * (0.25 - vb * vb);
  }
  if (mob == 1)
    return 0.5 * (u1 * (1.0 - u1) * (0.25 - v1 * v1) + u0 * (1.0 - u0) * (0.25 - v0 * v0));
  return u0 * (1.0 - u0) * (0.25 - v0 * v0);
}

ACCH_DEV void mobility_d(int mob, double u1, double v1, double u0, double v0, double &c,
                         double &cu, double &cv) {
  if (mob == 0) {
    const double ub = 0.5 * (u1 + u0), vb = 0.5 * (v1 + v0);
    c = ub * (1.0 - ub) * (0.25 - vb * vb);
    cu = 0.5 * (1.0 - 2.0 * ub) * (0.25 - vb * vb);
    cv = -ub * (1.0 - ub) * vb;
  } else if (mob == 1) {
    c = 0.5 * (u1 * (1.0 - u1) * (0.25 - v1 * v1) + u0 * (1.0 - u0) * (0.25 - v0 * v0));
    cu = 0.5 * (1.0 - 2.0 * u1) * (0.25 - v1 * v1);
    cv = -u1 * (1.0 - u1) * v1;
  } else {
    c = u0 * (1.0 - u0) * (0.25 - v0 * v0);
    cu = 0.0;
    cv = 0.0;
  }
}

// Mobility inside A~ and its derivatives with respect to the previous state (u0, v0).
ACCH_DEV void mobility_d0(int mob, double u1, double v1, double u0, double v0, double &c, double &cu,
                          double &cv) {
  if (mob == 0) {
    const double ub = 0.5 * (u1 + u0), vb = 0.5 * (v1 + v0);
    c = ub * (1.0 - ub) * (0.25 - vb * vb);
    cu = 0.5 * (1.0 - 2.0 * ub) * (0.25 - vb * vb);
    cv = -ub * (1.0 - ub) * vb;
  } else if (mob == 1) {
    c = 0.5 * (u1 * (1.0 - u1) * (0.25 - v1 * v1) + u0 * (1.0 - u0) * (0.25 - v0 * v0));
    cu = 0.5 * (1.0 - 2.0 * u0) * (0.25 - v0 * v0);
    cv = -u0 * (1.0 - u0) * v0;
  } else {
    c = u0 * (1.0 - u0) * (0.25 - v0 * v0);
    cu = (1.0 - 2.0 * u0) * (0.25 - v0 * v0);
    cv = -2.0 * u0 * (1.0 - u0) * v0;
  }
}

// Phi(z) = z ln z + (1-z) ln(1-z) (exact, for the energy diagnostic).
ACCH_DEV double Phi(double z) { return z * log(z) + (1.0 - z) * log(1.0 - z); }

// Phi'(z) = ln z - ln(1-z).
ACCH_DEV double dPhi(double z) { return log(z) - log(1.0 - z); }

}  // namespace acch
