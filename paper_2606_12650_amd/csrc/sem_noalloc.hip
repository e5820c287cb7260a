// vec_dot_noalloc: the deterministic dot product of vec_dot (the two-stage
// tree reduction of paper Sec. VIII-B) for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops).  The
// per-tile partials live in a fixed library-owned array of device memory
// instead of a caller workspace; the kernels are vec_dot's, so the result is
// bitwise that of vec_dot.
//
// The array is a file-scope device symbol.  Its host-side name is only a
// stand-in for the symbol, never a device address: on the first call on a
// device (with that device current) the address of that device's copy is
// looked up once with hipGetSymbolAddress and kept per device; every launch
// takes that address.  Each GPU holds its own copy until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "sem_error.h"
#include "sem_internal.h"

namespace semk {

namespace {

// Partials the array holds: one double per streaming tile of kVecTile
// entries, so vectors of up to kNoAllocMaxN entries (512 KiB of device
// memory per GPU).
constexpr int64_t kNoAllocPartials = 65536;
constexpr int64_t kNoAllocMaxN = kNoAllocPartials * kVecTile;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kNoAllocPartials];

std::mutex g_scratch_mu;
double *g_scratch_dev[kMaxDevices] = {};  // device address of `scratch`, per device

// The address of the current device's copy of `scratch` (looked up once).
hipError_t scratch_for(int dev, double **out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_dev[dev] = (double *)p;
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}

}  // namespace

}  // namespace semk

extern "C" {

int vec_dot_noalloc(int64_t n, const double *x, const double *y, const double *wt, double *out,
                    void *stream) {
  using namespace semk;
  if (n < 0) return set_error(SEM_ERR_ARG, "vec_dot_noalloc: n < 0");
  if (n > kNoAllocMaxN)
    return set_error(SEM_ERR_ARG, "vec_dot_noalloc: n = " + std::to_string(n) + " exceeds the maximum " +
                                      std::to_string(kNoAllocMaxN) + " of the built-in scratch");
  if (n > 0 && (!x || !y)) return set_error(SEM_ERR_ARG, "vec_dot_noalloc: null vector");
  if (!out) return set_error(SEM_ERR_ARG, "vec_dot_noalloc: null output");
  hipStream_t s = (hipStream_t)stream;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_hip_error(e, "vec_dot_noalloc: hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return set_error(SEM_ERR_ARG, "vec_dot_noalloc: device index out of range");
  if (s != nullptr) {
    hipDevice_t sdev = -1;
    e = hipStreamGetDevice(s, &sdev);
    if (e != hipSuccess) return set_hip_error(e, "vec_dot_noalloc: hipStreamGetDevice");
    if (sdev != dev) return set_error(SEM_ERR_ARG, "vec_dot_noalloc: the stream belongs to another device than the current one");
  }
  double *part = nullptr;
  e = scratch_for(dev, &part);
  if (e != hipSuccess) return set_hip_error(e, "vec_dot_noalloc: hipGetSymbolAddress");
  // every partial the final stage reads is written by the first stage of
  // this call, so nothing in the array needs clearing
  e = launch_dot(n, x, y, wt, out, part, s);
  if (e != hipSuccess) return set_hip_error(e, "vec_dot_noalloc: launch");
  return SEM_OK;
}

}  // extern "C"
