// Launches of the element kernels of the spectral-element Poisson operator
// on gfx950 (the kernels are in sem_kernels.h): the metric setup and the
// operator w = A_L u (paper Sec. VIII-B, the "ax" kernel, with N fixed at
// compile time as its jit clause does) in FP64, FP32 and BF16 mode.  Orders
// 1..12 launch the kernels built here; orders 13..15 launch the same kernels
// compiled at run time (sem_rtc.hip).
#include <hip/hip_runtime.h>

#include "sem_device.h"
#include "sem_internal.h"
#include "sem_kernels.h"
#include "sem_rtc.h"

namespace semk {

namespace {

// Rounded copy of G for a low-precision operator.
template <class P>
__global__ void __launch_bounds__(256)
    convert_g_kernel(int64_t n, const double *__restrict__ src, typename P::TG *__restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  if constexpr (P::kBf16) {
    dst[i] = bf16_bits((float)src[i]);
  } else {
    dst[i] = (typename P::TG)src[i];
  }
}

template <int N1, class P>
hipError_t ax_dispatch(const Box &b, const void *D, const void *G, void *u, void *w, const void *r,
                       const void *minv, void *x, CgState *cg, double *part, hipStream_t s) {
  using C = OpCfg<N1>;
  using TV = typename P::TV;
  using TG = typename P::TG;
  using TC = typename P::TC;
  const int64_t blocks = (b.E() + C::EPB - 1) / C::EPB;
  if (blocks == 0) return hipSuccess;
  if (cg)
    hipLaunchKernelGGL((ax_kernel<N1, P, true>), dim3((unsigned)blocks), dim3(C::THREADS), 0, s,
                       b.E(), (const TC *)D, (const TG *)G, (TV *)u, (TV *)w, (const TV *)r,
                       (const TV *)minv, (TV *)x, cg, part);
  else
    hipLaunchKernelGGL((ax_kernel<N1, P, false>), dim3((unsigned)blocks), dim3(C::THREADS), 0, s,
                       b.E(), (const TC *)D, (const TG *)G, (TV *)u, (TV *)w, (const TV *)r,
                       (const TV *)minv, (TV *)x, cg, part);
  return hipGetLastError();
}

template <int N1, class P>
hipError_t mfma_dispatch(const Box &b, const void *D, const void *G, void *u, void *w, const void *r,
                         const void *minv, void *x, CgState *cg, double *part, hipStream_t s,
                         bool stream_w) {
  using C = MfmaCfg<N1>;
  using TV = typename P::TV;
  using TG = typename P::TG;
  using TC = typename P::TC;
  const int64_t blocks = (b.E() + C::EPB - 1) / C::EPB;
  if (blocks == 0) return hipSuccess;
  if (cg)
    hipLaunchKernelGGL((ax_mfma_kernel<N1, P, true>), dim3((unsigned)blocks), dim3(C::THREADS), 0, s,
                       b.E(), (const TC *)D, (const TG *)G, (TV *)u, (TV *)w, (const TV *)r,
                       (const TV *)minv, (TV *)x, cg, part);
  else if (stream_w)
    hipLaunchKernelGGL((ax_mfma_local_kernel<N1, P>), dim3((unsigned)blocks), dim3(C::THREADS), 0, s,
                       b.E(), (const TC *)D, (const TG *)G, (TV *)u, (TV *)w);
  else
    hipLaunchKernelGGL((ax_mfma_kernel<N1, P, false>), dim3((unsigned)blocks), dim3(C::THREADS), 0,
                       s, b.E(), (const TC *)D, (const TG *)G, (TV *)u, (TV *)w, (const TV *)r,
                       (const TV *)minv, (TV *)x, cg, part);
  return hipGetLastError();
}

template <int N1>
hipError_t setup_dispatch(const Box &b, double amp, const double *D, const double *nodes,
                          double *G, double *diag, hipStream_t s) {
  using C = AxCfg<N1>;
  const int64_t blocks = (b.E() + C::EPB - 1) / C::EPB;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL((setup_geom_kernel<N1>), dim3((unsigned)blocks), dim3(C::THREADS), 0, s, b,
                     amp, D, nodes, G, diag);
  return hipGetLastError();
}

}  // namespace

#define SEM_FOR_EACH_ORDER(X) \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12)

int ax_elements_per_block(int N) {
  switch (N) {
#define CASE(n) \
  case n:       \
    return AxCfg<n + 1>::EPB;
    SEM_FOR_EACH_ORDER(CASE)
#undef CASE
    default:
      return 1;
  }
}

int64_t ax_num_blocks(const Box &b) {
  const int epb = ax_elements_per_block(b.N);
  return (b.E() + epb - 1) / epb;
}

// Operator launch for precision P (class cls): the matrix-core tile or the
// vector-unit one, by OpImpl.
template <class P>
hipError_t ax_launch(const Box &b, int cls, int impl, const void *D, const void *G, void *u, void *w,
                     const void *r, const void *minv, void *x, CgState *cg, double *part,
                     hipStream_t s, bool stream_w) {
  const bool mfma = impl == kImplMfma || (impl == kImplDefault && op_uses_mfma(cls, b.N));
  switch (b.N) {
#define CASE(n)                                                                      \
  case n:                                                                            \
    return mfma ? mfma_dispatch<n + 1, P>(b, D, G, u, w, r, minv, x, cg, part, s, stream_w) \
                : ax_dispatch<n + 1, P>(b, D, G, u, w, r, minv, x, cg, part, s);
    SEM_FOR_EACH_ORDER(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_ax_f64(const Box &b, int impl, const double *D, const double *G, double *u,
                         double *w, const double *r, const double *minv, double *x, CgState *cg,
                         double *part, hipStream_t s, bool stream_w) {
  if (rtc_order(b.N))  // run-time kernels: the matrix-core tile only
    return impl == kImplValu ? hipErrorInvalidValue : rtc_ax_f64(b, D, G, u, w, r, minv, x, cg, part, s);
  return ax_launch<PrecF64>(b, 0, impl, D, G, u, w, r, minv, x, cg, part, s, stream_w);
}

hipError_t launch_ax_lowp(const Box &b, int prec, int impl, const float *D, const void *G, float *u,
                          float *w, const float *r, const float *minv, float *x, CgState *cg,
                          double *part, hipStream_t s, bool stream_w) {
  if (prec == SEM_F32)
    return ax_launch<PrecF32>(b, 1, impl, D, G, u, w, r, minv, x, cg, part, s, stream_w);
  if (prec == SEM_BF16)
    return ax_launch<PrecBF16>(b, 2, impl, D, G, u, w, r, minv, x, cg, part, s, stream_w);
  return hipErrorInvalidValue;
}

hipError_t launch_convert_g(int prec, int64_t n, const double *src, void *dst, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (prec == SEM_F32)
    hipLaunchKernelGGL(convert_g_kernel<PrecF32>, dim3(blocks), dim3(256), 0, s, n, src, (float *)dst);
  else if (prec == SEM_BF16)
    hipLaunchKernelGGL(convert_g_kernel<PrecBF16>, dim3(blocks), dim3(256), 0, s, n, src,
                       (uint16_t *)dst);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_setup_geom(const Box &b, double amp, const double *D, const double *nodes,
                             double *G, double *diag, hipStream_t s) {
  if (rtc_order(b.N)) return rtc_setup_geom(b, amp, D, nodes, G, diag, s);
  switch (b.N) {
#define CASE(n) \
  case n:       \
    return setup_dispatch<n + 1>(b, amp, D, nodes, G, diag, s);
    SEM_FOR_EACH_ORDER(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace semk
