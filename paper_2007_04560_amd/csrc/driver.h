// Host-side pieces shared by the single-instance and the batched drivers.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/acch.h"
#include "common.h"

namespace acch {

// Records the message returned by acch_last_error and returns code.
int fail(int code, const std::string &msg);

#define HIP_TRY(expr)                                                                              \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess)                                                                          \
      return ::acch::fail(ACCH_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));       \
  } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Split n cells into `parts` pieces, the larger ones first (shared reading with the
// oracle's decomposition).
inline void split(int n, int parts, std::vector<int> &start, std::vector<int> &len) {
  start.resize(parts);
  len.resize(parts);
  const int base = n / parts, rem = n % parts;
  int s = 0;
  for (int k = 0; k < parts; ++k) {
    start[k] = s;
    len[k] = base + (k < rem ? 1 : 0);
    s += len[k];
  }
}

// Subdomain boxes of one grid.
struct Geometry {
  long ncell = 0;
  BoxGeom G{};
  std::vector<SubInfo> subs;
  std::vector<int> lvl;  // nlev + 1 prefix counts
  std::vector<int> cells;  // 3D: box cells (i | j << 10 | k << 20) in level order, then
                           // the windowed apply's column lists (when G.wmax > 0)
  std::vector<int> own;  // owner subdomain of each grid column (nx), then of each row (ny)
  int min_part = 0;      // smallest owned width / height
  int tile_blocks = 0;
};

// The backtracking line search (the reading of the unspecified line search shared
// with the oracle): Armijo test on ||F||^2/2 with alpha = 1e-4 and slope -||F||^2,
// a quadratic model on the first backtrack and a cubic one after, each new lambda
// clamped to [0.1, 0.5] lambda; an inadmissible or non-finite trial halves lambda;
// failure below lambda = 1e-8.  The caller evaluates ||F(X + lam S)||^2 and the
// inadmissible count for `lam` and passes them to trial().
struct LineSearch {
  enum { kSearching = 0, kAccepted = 1, kFailed = 2 };
  double lam = 1.0, f0 = 0.0, slope = 0.0, lp = 0.0, fp = 0.0, f2 = 0.0;
  bool have_prev = false;
  int state = kSearching;

  void start(double fnorm) {
    f0 = 0.5 * fnorm * fnorm;
    slope = -2.0 * f0;
    lam = 1.0;
    have_prev = false;
    lp = fp = 0.0;
    state = kSearching;
  }

  void trial(double f2_trial, double bad) {
    constexpr double alpha = 1e-4, lam_min = 1e-8;
    if (bad > 0.0 || !(f2_trial == f2_trial) || std::isinf(f2_trial)) {
      lam *= 0.5;
      if (lam < lam_min) state = kFailed;
      return;
    }
    const double ft = 0.5 * f2_trial;
    if (ft <= f0 + alpha * lam * slope) {
      f2 = f2_trial;
      state = kAccepted;
      return;
    }
    double nl;
    if (!have_prev) {
      nl = -slope * lam * lam / (2.0 * (ft - f0 - slope * lam));
    } else {
      const double t1 = ft - f0 - slope * lam, t2 = fp - f0 - slope * lp;
      const double a = (t1 / (lam * lam) - t2 / (lp * lp)) / (lam - lp);
      const double b = (-lp * t1 / (lam * lam) + lam * t2 / (lp * lp)) / (lam - lp);
      if (a == 0.0) {
        nl = -slope / (2.0 * b);
      } else {
        const double disc = b * b - 3.0 * a * slope;
        nl = disc >= 0.0 ? (-b + std::sqrt(disc)) / (3.0 * a) : 0.5 * lam;
      }
    }
    if (!std::isfinite(nl)) nl = 0.5 * lam;
    nl = std::min(std::max(nl, 0.1 * lam), 0.5 * lam);
    have_prev = true;
    lp = lam;
    fp = ft;
    lam = nl;
    if (lam < lam_min) state = kFailed;
  }
};

int validate_params(const acch_params &p);
// The stencil kernels' description of a grid and its coefficients (validated params).
Phys phys_of(const acch_params &p);
int build_geometry(const acch_params &p, Geometry &geo);

}  // namespace acch
