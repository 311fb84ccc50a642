// acch_residual_noalloc: the residual of scheme (2.20) with its norm for callers that
// cannot allocate device memory.  No context and no workspace: the two-kernel norm
// reduction keeps its block partials and its result in `scratch`, a static device array
// of the library (one copy per GPU, held until the process ends).  Its address on each
// device is taken once, with hipGetSymbolAddress, the first time the entry point runs
// on that device; host code uses only that address, never the array's name.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/acch.h"
#include "driver.h"
#include "kernels.h"

namespace {

constexpr size_t kScratchBytes = (size_t)1 << 20;   // 1 MiB per GPU
constexpr int kOutDoubles = 64;                       // finalize output, then the partials
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (taken once per device).
int scratch_address(double **out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return acch::fail(ACCH_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return acch::fail(ACCH_EDEVICE, "no device address for the scratch array");
    g_scratch_ptr[dev] = ptr;
  }
  *out = (double *)g_scratch_ptr[dev];
  return ACCH_OK;
}

}  // namespace

extern "C" int acch_residual_noalloc(const acch_params *pin, const double *X, const double *Xn, double dt, double *F,
                                     double *fnorm2, int *inadmissible) {
  using namespace acch;
  if (!pin || !X || !Xn || !F || !(dt > 0)) return fail(ACCH_EINVAL, "bad arguments");
  acch_params p = *pin;
  acch_params_default(&p);
  int rc = validate_params(p);
  if (rc) return rc;
  if (p.dim != 2) return fail(ACCH_EUNSUPPORTED, "acch_residual_noalloc is 2D");
  const Phys P = phys_of(p);
  const BatchLaunch bl = single_launch(P, 1);
  const size_t need = (size_t)(kOutDoubles + 2 * (size_t)bl.grid[kFamTile]) * sizeof(double);
  if (need > kScratchBytes)
    return fail(ACCH_EINVAL, "grid too large for the 1 MiB scratch array (at most 65504 tiles of 32 x 8 cells)");
  double *sp = nullptr;
  rc = scratch_address(&sp);
  if (rc) return rc;
  RedBuf red{};
  red.out = sp;
  red.counter = nullptr;   // not used by these reductions
  red.partials = sp + kOutDoubles;
  hipStream_t s = (hipStream_t)p.stream;
  HIP_TRY(launch_residual2d(bl, X, nullptr, 0.0, nullptr, nullptr, Xn, dt, nullptr, F, red, s));
  double vals[2] = {0.0, 0.0};
  HIP_TRY(hipMemcpyAsync(vals, sp, sizeof(vals), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (fnorm2) *fnorm2 = vals[0];
  if (inadmissible) *inadmissible = (int)vals[1];
  return ACCH_OK;
}
