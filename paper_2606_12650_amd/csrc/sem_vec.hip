// Gather-scatter, streaming updates and reductions of the Jacobi-PCG on gfx950
// (paper Sec. V-B "gs" kernel and the Sec. VIII-B streaming and tree-
// reduction kernels).
//
// Streaming kernels: one thread per 8 entries of an element-local vector,
// 256 threads per work-group, every access a full-wave coalesced load or
// store.  The gather-scatter fuses into the kernel that consumes the
// assembled vector instead of making a pass of its own: on element-column
// tiles (copies paired across faces, sem_cg_dev.h) or, on linear tiles, as a
// pull where each node reads the copies of itself held by neighbouring
// elements.
//
// Reductions are deterministic: a work-group sums a fixed tile (wave64
// butterfly, then its waves in order) and a second one-group launch sums the
// partials in tile order.  Results depend only on the data and the sizes.
#include <hip/hip_runtime.h>

#include "sem_cg_dev.h"
#include "sem_device.h"
#include "sem_internal.h"
#include "sem_kernels.h"
#include "sem_rtc.h"

namespace semk {
namespace {

__global__ void __launch_bounds__(kFinThreads)
    cg_init_finish_kernel(CgState *st, const double *__restrict__ part_rz,
                          const double *__restrict__ part_bb, int64_t n) {
  __shared__ double sred[2 * (kFinThreads / 64)];
  cg_init_step(st, part_rz, part_bb, n, sred);
}

__global__ void __launch_bounds__(kFinThreads)
    cg_alpha_kernel(CgState *st, const double *__restrict__ part, int64_t n) {
  __shared__ double sred[2 * (kFinThreads / 64)];
  cg_alpha_step(st, part, n, sred);
}

__global__ void __launch_bounds__(kFinThreads)
    cg_beta_kernel(CgState *st, const double *__restrict__ part_rr,
                   const double *__restrict__ part_rz, int64_t n) {
  __shared__ double sred[2 * (kFinThreads / 64)];
  cg_beta_step(st, part_rr, part_rz, n, sred);
}

__global__ void __launch_bounds__(kFinThreads)
    outer_finish_kernel(CgState *st, const double *__restrict__ part, int64_t n) {
  __shared__ double sred[2 * (kFinThreads / 64)];
  outer_finish_step(st, part, n, sred);
}

// The last x += alpha p of a solve (the operator kernel folds it into the
// next iteration's prologue, and there is no next iteration).
__global__ void __launch_bounds__(kVecThreads)
    cg_finish_kernel(int64_t L, double *__restrict__ x, const double *__restrict__ p,
                     const CgState *__restrict__ st) {
  if (st->done == kRunning || st->done_stage != 2) return;
  const double alpha = st->alpha;
  const int64_t base = (int64_t)blockIdx.x * kVecTile + threadIdx.x;
#pragma unroll
  for (int u = 0; u < kVecItems; ++u) {
    const int64_t idx = base + (int64_t)u * kVecThreads;
    if (idx < L) x[idx] += alpha * p[idx];
  }
}

// ------------------------------------------------------------ inner-outer CG
template <int N1>
__global__ void __launch_bounds__(kVecThreads)
    inner_start_kernel(Box b, int64_t L, int64_t ntiles, const double *__restrict__ r64,
                       const CgState *__restrict__ outer, float *__restrict__ rin,
                       float *__restrict__ e, float *__restrict__ p,
                       const float *__restrict__ minv32, double *__restrict__ part_rz,
                       double *__restrict__ part_rr) {
  __shared__ double sred[2 * (kVecThreads / 64)];
  const double inv_s = 1.0 / sqrt(outer->rnorm2);
  const int64_t tile = xcd_tile(ntiles);
  TileSums t{0.0, 0.0};
  if (tile < ntiles) t = inner_start_tile<N1>(b, L, tile, r64, inv_s, rin, e, p, minv32, sred);
  if (threadIdx.x == 0) {
    part_rz[tile] = t.a;
    part_rr[tile] = t.b;
  }
}

__global__ void __launch_bounds__(kFinThreads)
    inner_init_kernel(CgState *st, const double *__restrict__ part_rz,
                      const double *__restrict__ part_rr, int64_t n, double rtol2, int max_iter) {
  __shared__ double sred[2 * (kFinThreads / 64)];
  inner_init_step(st, part_rz, part_rr, n, rtol2, max_iter, sred);
}

// e += alpha_in p_in (if the inner solve's last update ran), x += ||r||_c e.
__global__ void __launch_bounds__(kVecThreads)
    outer_correct_kernel(int64_t L, double *__restrict__ x, float *__restrict__ e,
                         const float *__restrict__ p, const CgState *__restrict__ inner,
                         const CgState *__restrict__ outer) {
  if (outer->done != kRunning) return;
  const bool add_p = inner->done != kRunning && inner->done_stage == 2;
  outer_correct_tile(L, blockIdx.x, x, e, p, (float)inner->alpha, add_p, sqrt(outer->rnorm2));
}

// True residual r = mask o (b - QQ^T w_L) with w_L = A_L x (FP64) and the
// partials of ||r||_c^2.
template <int N1>
__global__ void __launch_bounds__(kVecThreads)
    residual_kernel(Box b, int64_t L, int64_t ntiles, const double *__restrict__ bvec,
                    const double *__restrict__ wl, double *__restrict__ r,
                    const CgState *__restrict__ outer, double *__restrict__ part) {
  __shared__ double sred[2 * (kVecThreads / 64)];
  const int done = outer->done;
  const int64_t tile = xcd_tile(ntiles);
  double rr = 0.0;
  if (tile < ntiles && done == kRunning) rr = residual_tile<N1>(b, L, tile, bvec, wl, r, sred);
  if (threadIdx.x == 0) part[tile] = rr;
}

// ------------------------------------------------------------ generic vectors
// Full tiles issue every load before the first use (the loads of all items
// are in flight together); the last, partial tile takes the entry-by-entry
// path.  Both read x and y once: non-temporal.
__global__ void __launch_bounds__(kVecThreads)
    axpy_kernel(int64_t n, double alpha, const double *__restrict__ x, double *__restrict__ y) {
  const int64_t base = (int64_t)blockIdx.x * kVecTile + threadIdx.x;
  if ((int64_t)(blockIdx.x + 1) * kVecTile <= n) {
    double xv[kVecItems], yv[kVecItems];
#pragma unroll
    for (int u = 0; u < kVecItems; ++u) {
      xv[u] = ld_once(x + base + (int64_t)u * kVecThreads);
      yv[u] = ld_once(y + base + (int64_t)u * kVecThreads);
    }
#pragma unroll
    for (int u = 0; u < kVecItems; ++u) st_once(y + base + (int64_t)u * kVecThreads, fma(alpha, xv[u], yv[u]));
    return;
  }
#pragma unroll
  for (int u = 0; u < kVecItems; ++u) {
    const int64_t idx = base + (int64_t)u * kVecThreads;
    if (idx < n) y[idx] = fma(alpha, x[idx], y[idx]);
  }
}

// Per-thread sums in item order (the same order on both paths), then the
// block tree.
template <bool W>
__global__ void __launch_bounds__(kVecThreads)
    dot_partial_kernel(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                       const double *__restrict__ wt, double *__restrict__ part) {
  __shared__ double sred[2 * (kVecThreads / 64)];
  const int64_t base = (int64_t)blockIdx.x * kVecTile + threadIdx.x;
  double acc = 0.0;
  if ((int64_t)(blockIdx.x + 1) * kVecTile <= n) {
    double xv[kVecItems], yv[kVecItems], wv[kVecItems];
#pragma unroll
    for (int u = 0; u < kVecItems; ++u) {
      const int64_t idx = base + (int64_t)u * kVecThreads;
      xv[u] = ld_once(x + idx);
      yv[u] = ld_once(y + idx);
      wv[u] = W ? ld_once(wt + idx) : 1.0;
    }
#pragma unroll
    for (int u = 0; u < kVecItems; ++u) {
      const double v = xv[u] * yv[u];
      acc += W ? wv[u] * v : v;
    }
  } else {
#pragma unroll
    for (int u = 0; u < kVecItems; ++u) {
      const int64_t idx = base + (int64_t)u * kVecThreads;
      if (idx < n) {
        const double v = x[idx] * y[idx];
        acc += W ? wt[idx] * v : v;
      }
    }
  }
  const double t = block_sum<kVecThreads>(acc, sred);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void __launch_bounds__(kFinThreads)
    dot_final_kernel(const double *__restrict__ part, int64_t n, double *__restrict__ out) {
  __shared__ double sred[2 * (kFinThreads / 64)];
  const double t = sum_partials<kFinThreads>(part, n, sred);
  if (threadIdx.x == 0) *out = t;
}

inline dim3 vec_grid(int64_t n) { return dim3((unsigned)vec_num_blocks(n)); }

// The update of order N1 - 1 with tile shape V (upd_shape).
template <int N1, typename TV, int V>
hipError_t update_launch(const Box &b, TV *r, const TV *w, const TV *minv, CgState *st,
                         double *part_rr, double *part_rz, hipStream_t s) {
  constexpr bool f64 = sizeof(TV) == 8;
  if constexpr (!upd_variant_exists(N1, f64, V)) {
    return hipErrorInvalidValue;
  } else {
    hipLaunchKernelGGL((cg_update_kernel<N1, TV, V>), dim3((unsigned)upd_grid_blocks(b, f64, V)),
                       dim3(UpdTile<N1, TV, V>::BLOCK), 0, s, b, upd_num_tiles(b, f64, V), r, w,
                       minv, st, part_rr, part_rz);
    return hipGetLastError();
  }
}

template <typename TV>
hipError_t update_typed(const Box &b, int variant, TV *r, const TV *w, const TV *minv, CgState *st,
                        double *part_rr, double *part_rz, hipStream_t s) {
  if (b.E() == 0) return hipSuccess;
  switch (b.N) {
#define UCASE(n_)                                                                                \
  case n_:                                                                                       \
    switch (variant) {                                                                           \
      case 0: return update_launch<n_ + 1, TV, 0>(b, r, w, minv, st, part_rr, part_rz, s);       \
      case 1: return update_launch<n_ + 1, TV, 1>(b, r, w, minv, st, part_rr, part_rz, s);       \
      case 2: return update_launch<n_ + 1, TV, 2>(b, r, w, minv, st, part_rr, part_rz, s);       \
      case 3: return update_launch<n_ + 1, TV, 3>(b, r, w, minv, st, part_rr, part_rz, s);       \
      default: return hipErrorInvalidValue;                                                      \
    }
    UCASE(1) UCASE(2) UCASE(3) UCASE(4) UCASE(5) UCASE(6)
    UCASE(7) UCASE(8) UCASE(9) UCASE(10) UCASE(11) UCASE(12)
#undef UCASE
    default:
      return hipErrorInvalidValue;
  }
}
static_assert(kUpdVariants == 4, "update_typed dispatches four candidate shapes");
inline dim3 xcd_vec_grid(int64_t n) { return dim3((unsigned)vec_grid_blocks(n)); }

}  // namespace

#define DISPATCH_N(b, KERNEL, ...)                                      \
  switch ((b).N) {                                                      \
    case 1: hipLaunchKernelGGL(KERNEL<2>, __VA_ARGS__); break;          \
    case 2: hipLaunchKernelGGL(KERNEL<3>, __VA_ARGS__); break;          \
    case 3: hipLaunchKernelGGL(KERNEL<4>, __VA_ARGS__); break;          \
    case 4: hipLaunchKernelGGL(KERNEL<5>, __VA_ARGS__); break;          \
    case 5: hipLaunchKernelGGL(KERNEL<6>, __VA_ARGS__); break;          \
    case 6: hipLaunchKernelGGL(KERNEL<7>, __VA_ARGS__); break;          \
    case 7: hipLaunchKernelGGL(KERNEL<8>, __VA_ARGS__); break;          \
    case 8: hipLaunchKernelGGL(KERNEL<9>, __VA_ARGS__); break;          \
    case 9: hipLaunchKernelGGL(KERNEL<10>, __VA_ARGS__); break;         \
    case 10: hipLaunchKernelGGL(KERNEL<11>, __VA_ARGS__); break;        \
    case 11: hipLaunchKernelGGL(KERNEL<12>, __VA_ARGS__); break;        \
    case 12: hipLaunchKernelGGL(KERNEL<13>, __VA_ARGS__); break;        \
    default: return hipErrorInvalidValue;                               \
  }

#define DISPATCH_N_MODE(b, MODE, KERNEL, ...)                           \
  switch ((b).N) {                                                      \
    case 1: hipLaunchKernelGGL((KERNEL<2, MODE>), __VA_ARGS__); break;  \
    case 2: hipLaunchKernelGGL((KERNEL<3, MODE>), __VA_ARGS__); break;  \
    case 3: hipLaunchKernelGGL((KERNEL<4, MODE>), __VA_ARGS__); break;  \
    case 4: hipLaunchKernelGGL((KERNEL<5, MODE>), __VA_ARGS__); break;  \
    case 5: hipLaunchKernelGGL((KERNEL<6, MODE>), __VA_ARGS__); break;  \
    case 6: hipLaunchKernelGGL((KERNEL<7, MODE>), __VA_ARGS__); break;  \
    case 7: hipLaunchKernelGGL((KERNEL<8, MODE>), __VA_ARGS__); break;  \
    case 8: hipLaunchKernelGGL((KERNEL<9, MODE>), __VA_ARGS__); break;  \
    case 9: hipLaunchKernelGGL((KERNEL<10, MODE>), __VA_ARGS__); break; \
    case 10: hipLaunchKernelGGL((KERNEL<11, MODE>), __VA_ARGS__); break;\
    case 11: hipLaunchKernelGGL((KERNEL<12, MODE>), __VA_ARGS__); break;\
    case 12: hipLaunchKernelGGL((KERNEL<13, MODE>), __VA_ARGS__); break;\
    default: return hipErrorInvalidValue;                               \
  }

// The gather on the tiles the CG update of this order and precision uses.
template <int N1, int MODE, typename T>
void gather_launch(const Box &b, const T *wl, T *out, hipStream_t s) {
  if constexpr (UpdTile<N1, T>::LINEAR) {
    const int64_t L = b.L();
    hipLaunchKernelGGL((gather_kernel<N1, MODE, T>), xcd_vec_grid(L), dim3(kVecThreads), 0, s, b, L,
                       vec_num_blocks(L), wl, out);
  } else {
    const bool f64 = sizeof(T) == 8;
    hipLaunchKernelGGL((gather_col_kernel<N1, MODE, T>), dim3((unsigned)upd_grid_blocks(b, f64)),
                       dim3(UpdTile<N1, T>::BLOCK), 0, s, b, upd_num_tiles(b, f64), wl, out);
  }
}

template <typename T>
hipError_t gather_typed(const Box &b, const T *wl, T *out, int mode, hipStream_t s) {
  if (b.L() == 0) return hipSuccess;
  if (mode != kGatherAssembled && mode != kGatherMasked && mode != kGatherInverse)
    return hipErrorInvalidValue;
  switch (b.N) {
#define GCASE(n_)                                                                 \
  case n_:                                                                        \
    if (mode == kGatherAssembled) gather_launch<n_ + 1, kGatherAssembled, T>(b, wl, out, s); \
    else if (mode == kGatherMasked) gather_launch<n_ + 1, kGatherMasked, T>(b, wl, out, s);  \
    else gather_launch<n_ + 1, kGatherInverse, T>(b, wl, out, s);                   \
    break;
    GCASE(1) GCASE(2) GCASE(3) GCASE(4) GCASE(5) GCASE(6)
    GCASE(7) GCASE(8) GCASE(9) GCASE(10) GCASE(11) GCASE(12)
#undef GCASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gather(const Box &b, const double *wl, double *out, int mode, hipStream_t s) {
  if (rtc_order(b.N)) return b.L() == 0 ? hipSuccess : rtc_gather(b, wl, out, mode, s);
  return gather_typed<double>(b, wl, out, mode, s);
}

hipError_t launch_gather_f32(const Box &b, const float *wl, float *out, int mode, hipStream_t s) {
  return gather_typed<float>(b, wl, out, mode, s);
}

hipError_t launch_cg_init(const Box &b, const double *bvec, double *x, double *r, double *p,
                          const double *minv, CgState *st, double *part_a, double *part_b,
                          hipStream_t s) {
  const int64_t L = b.L();
  const int64_t nt = vec_num_blocks(L);
  hipError_t e;
  if (rtc_order(b.N)) {
    e = rtc_cg_init(b, bvec, x, r, p, minv, part_a, part_b, s);
  } else {
    DISPATCH_N(b, cg_init_kernel, xcd_vec_grid(L), dim3(kVecThreads), 0, s, b, L, nt, bvec, x, r, p,
               minv, part_a, part_b);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(cg_init_finish_kernel, dim3(1), dim3(kFinThreads), 0, s, st, part_a, part_b,
                     vec_grid_blocks(L));
  return hipGetLastError();
}

hipError_t launch_cg_alpha(CgState *st, const double *part_pap, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(cg_alpha_kernel, dim3(1), dim3(kFinThreads), 0, s, st, part_pap, n);
  return hipGetLastError();
}

hipError_t launch_cg_beta(CgState *st, const double *part_rr, const double *part_rz, int64_t n,
                          hipStream_t s) {
  hipLaunchKernelGGL(cg_beta_kernel, dim3(1), dim3(kFinThreads), 0, s, st, part_rr, part_rz, n);
  return hipGetLastError();
}

hipError_t launch_cg_update(const Box &b, int variant, double *r, const double *w, const double *minv,
                            CgState *st, double *part_rr, double *part_rz, hipStream_t s) {
  if (rtc_order(b.N)) {
    if (variant != 0) return hipErrorInvalidValue;
    return b.E() == 0 ? hipSuccess : rtc_cg_update(b, r, w, minv, st, part_rr, part_rz, s);
  }
  return update_typed<double>(b, variant, r, w, minv, st, part_rr, part_rz, s);
}

hipError_t launch_cg_update_f32(const Box &b, int variant, float *r, const float *w, const float *minv,
                                CgState *st, double *part_rr, double *part_rz, hipStream_t s) {
  return update_typed<float>(b, variant, r, w, minv, st, part_rr, part_rz, s);
}

hipError_t launch_cg_finish(const Box &b, double *x, const double *p, const CgState *st,
                            hipStream_t s) {
  const int64_t L = b.L();
  hipLaunchKernelGGL(cg_finish_kernel, vec_grid(L), dim3(kVecThreads), 0, s, L, x, p, st);
  return hipGetLastError();
}

hipError_t launch_inner_start(const Box &b, const double *r64, CgState *outer, CgState *inner,
                              double rtol2, int max_iter, float *rin, float *e, float *p,
                              const float *minv32, double *part_a, double *part_b, hipStream_t s) {
  const int64_t L = b.L();
  const int64_t nt = vec_num_blocks(L);
  DISPATCH_N(b, inner_start_kernel, xcd_vec_grid(L), dim3(kVecThreads), 0, s, b, L, nt, r64, outer,
             rin, e, p, minv32, part_a, part_b);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(inner_init_kernel, dim3(1), dim3(kFinThreads), 0, s, inner, part_a, part_b,
                     vec_grid_blocks(L), rtol2, max_iter);
  return hipGetLastError();
}

hipError_t launch_outer_correct(const Box &b, double *x, float *e, const float *p,
                                const CgState *inner, const CgState *outer, hipStream_t s) {
  const int64_t L = b.L();
  hipLaunchKernelGGL(outer_correct_kernel, vec_grid(L), dim3(kVecThreads), 0, s, L, x, e, p, inner,
                     outer);
  return hipGetLastError();
}

hipError_t launch_outer_step(const Box &b, const double *bvec, const double *w64, double *r64,
                             CgState *outer, double *part, hipStream_t s) {
  const int64_t L = b.L();
  const int64_t nt = vec_num_blocks(L);
  DISPATCH_N(b, residual_kernel, xcd_vec_grid(L), dim3(kVecThreads), 0, s, b, L, nt, bvec, w64, r64,
             outer, part);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(outer_finish_kernel, dim3(1), dim3(kFinThreads), 0, s, outer, part,
                     vec_grid_blocks(L));
  return hipGetLastError();
}

hipError_t launch_fill_c(const Box &b, double *c, hipStream_t s) {
  const int64_t L = b.L();
  if (L == 0) return hipSuccess;
  if (rtc_order(b.N)) return rtc_fill_c(b, c, s);
  DISPATCH_N(b, fill_c_kernel, vec_grid(L), dim3(kVecThreads), 0, s, b, L, c);
  return hipGetLastError();
}

hipError_t launch_axpy(int64_t n, double alpha, const double *x, double *y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(axpy_kernel, vec_grid(n), dim3(kVecThreads), 0, s, n, alpha, x, y);
  return hipGetLastError();
}

hipError_t launch_dot(int64_t n, const double *x, const double *y, const double *wt, double *out,
                      double *partials, hipStream_t s) {
  const int64_t nb = vec_num_blocks(n);
  if (nb > 0) {
    if (wt)
      hipLaunchKernelGGL(dot_partial_kernel<true>, vec_grid(n), dim3(kVecThreads), 0, s, n, x, y,
                         wt, partials);
    else
      hipLaunchKernelGGL(dot_partial_kernel<false>, vec_grid(n), dim3(kVecThreads), 0, s, n, x,
                         y, wt, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(kFinThreads), 0, s, partials, nb, out);
  return hipGetLastError();
}

}  // namespace semk
