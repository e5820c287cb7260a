// Run-time specialisation of the per-order kernels for orders outside the
// built set (the analogue of the paper's jit clause, Sec. IV: values known
// only at run time become compile-time constants of generated code).  The
// kernels of sem_kernels.h are compiled with hipRTC for one order and the
// device's architecture, loaded as a module and launched with the shapes
// the built kernels use.  FP64 only, matrix-core element tile only.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "sem_types.h"

namespace semk {

// Orders served at run time.
inline bool rtc_order(int N) { return N > kMaxOrder && N <= kMaxRtcOrder; }

// Compile (once per process and architecture; also cached on disk) and load
// (once per device) the kernels of order N for the current device.  On
// failure *why holds the reason (the compiler log for a compile error).
hipError_t rtc_prepare(int N, std::string *why);

// gfx950, with or without a target-feature suffix: the one architecture the
// kernels are written for.
bool rtc_arch_supported(const char *arch);

// Compile the kernels of order N for `arch` (e.g. "gfx950") without a GPU;
// *code_bytes receives the code object size.
hipError_t rtc_build(int N, const char *arch, size_t *code_bytes, std::string *why);

// Launches for an order prepared above (same arguments and grids as the
// built kernels' launchers).
hipError_t rtc_setup_geom(const Box &b, double amp, const double *D, const double *nodes, double *G,
                          double *diag, hipStream_t s);
hipError_t rtc_ax_f64(const Box &b, const double *D, const double *G, double *u, double *w,
                      const double *r, const double *minv, double *x, CgState *cg, double *part,
                      hipStream_t s);
hipError_t rtc_gather(const Box &b, const double *wl, double *out, int mode, hipStream_t s);
hipError_t rtc_cg_init(const Box &b, const double *bvec, double *x, double *r, double *p,
                       const double *minv, double *part_a, double *part_b, hipStream_t s);
hipError_t rtc_cg_update(const Box &b, double *r, const double *w, const double *minv, CgState *st,
                         double *part_rr, double *part_rz, hipStream_t s);
hipError_t rtc_fill_c(const Box &b, double *c, hipStream_t s);

}  // namespace semk
