// Batched Jacobi-PCG: many independent solves of different sizes and orders
// advance together, one CG iteration per batched step, in seven launches that
// cover every solve.
//
// The two streaming launches and the two operator launches (FP64 and low-
// precision work) are persistent kernels over work lists of (solve, tile) items; the three per-solve launches run one
// work-group per solve.  Every item is computed by the same device functions
// as a single solve (sem_ax_tile.h, sem_cg_dev.h) on the same tiles, and each
// solve's reductions are summed in the same order, so an FP64 solve gives the
// same bits alone and in a batch.  A mixed-precision solve moves through the
// inner-outer phases (SlotPhase) on the device; the host only polls.
#include <hip/hip_runtime.h>

#include "sem_ax_tile.h"
#include "sem_cg_dev.h"
#include "sem_device.h"
#include "sem_internal.h"

namespace semk {

namespace {

constexpr int kOpThreads = 256;

constexpr int align16(int v) { return (v + 15) / 16 * 16; }

// LDS of the operator launches: the largest supported FP64 tile, and the
// largest low-precision one (FP32 values).
constexpr int kLdsBytes = 61 * 1024;
constexpr int kLdsBytesLowp = 31 * 1024;

// LDS needed by one operator tile (reduction buffer, D, two element tiles).
template <int N1, int EPB, class P>
constexpr int tile_lds_bytes() {
  using TC = typename P::TC;
  return align16(kOpThreads * 8) + align16(N1 * N1 * (int)sizeof(TC)) +
         AxTile<N1>::kTiles * align16(EPB * AxTile<N1>::TILE * (int)sizeof(TC));
}

template <int N1, int EPB, class P, bool CG>
__device__ __forceinline__ void op_tile(const BatchSlot &S, int e0, unsigned char *smem,
                                        typename P::TV *u, typename P::TV *w,
                                        const typename P::TV *r, const typename P::TV *minv,
                                        typename P::TV *x, const typename P::TC *D,
                                        const typename P::TG *G, double alpha, double beta) {
  static_assert(tile_lds_bytes<N1, EPB, P>() <= (sizeof(typename P::TC) == 8 ? kLdsBytes : kLdsBytesLowp),
                "operator tile exceeds the LDS budget");
  static_assert(N1 * N1 * EPB <= kOpThreads, "operator tile exceeds the work-group");
  using TC = typename P::TC;
  double *sred = (double *)smem;
  TC *sD = (TC *)(smem + align16(kOpThreads * 8));
  TC *s1 = (TC *)((unsigned char *)sD + align16(N1 * N1 * (int)sizeof(TC)));
  TC *s2 = (TC *)((unsigned char *)s1 + align16(EPB * AxTile<N1>::TILE * (int)sizeof(TC)));
  TC *s3 = (TC *)((unsigned char *)s2 + align16(EPB * AxTile<N1>::TILE * (int)sizeof(TC)));
  ax_tile<N1, EPB, P, CG>(S.E, e0, D, G, u, w, r, minv, x, alpha, beta, S.part_el, sD, s1, s2, s3,
                          sred);
}

// FP64 work of an operator item: a CG iteration of an FP64 solve, or the
// true-residual operator of a mixed solve's outer step.
template <int N1, int EPB>
__device__ __forceinline__ void op_item_f64(const BatchSlot &S, int e0, unsigned char *smem) {
  if (S.mixed == 0) {
    if (S.phase != kPhaseFp64 || S.st->done != kRunning) return;
    op_tile<N1, EPB, PrecF64, true>(S, e0, smem, S.p, S.w, S.r, S.minv, S.x, S.D, S.G,
                                    S.st->alpha, S.st->beta);
  } else if (S.phase == kPhaseOuterOp) {
    op_tile<N1, EPB, PrecF64, false>(S, e0, smem, S.x, S.w, nullptr, nullptr, nullptr, S.D, S.G,
                                     0.0, 0.0);
  }
}

// Low-precision work of an operator item: an inner iteration of a mixed solve.
template <int N1, int EPB>
__device__ __forceinline__ void op_item_lowp(const BatchSlot &S, int e0, unsigned char *smem) {
  if (S.mixed == 0 || S.phase != kPhaseInner || S.st_in->done != kRunning) return;
  if (S.mixed == SEM_F32)
    op_tile<N1, EPB, PrecF32, true>(S, e0, smem, S.pin, S.win, S.rin, S.minv32, S.e, S.Dlo,
                                    (const float *)S.Glo, S.st_in->alpha, S.st_in->beta);
  else
    op_tile<N1, EPB, PrecBF16, true>(S, e0, smem, S.pin, S.win, S.rin, S.minv32, S.e, S.Dlo,
                                     (const uint16_t *)S.Glo, S.st_in->alpha, S.st_in->beta);
}

// Supported (order, elements per item) pairs, orders 1..11: the single-solve
// kernel's tile and a larger one that fits 256 threads and the LDS budget.
#define SEM_BATCH_TILES(X)                                                    \
  X(1, 32) X(1, 64) X(2, 14) X(2, 28) X(3, 8) X(3, 16) X(4, 5) X(4, 10)      \
  X(5, 3) X(5, 7) X(6, 2) X(6, 5) X(7, 2) X(7, 4) X(8, 1) X(8, 2) X(9, 1)   \
  X(9, 2) X(10, 1) X(11, 1)

// Two persistent operator launches per batched iteration, one per
// arithmetic class, so that the FP64 variants' register count does not
// lower the occupancy of the low-precision inner iterations.
template <bool F64>
__global__ void __launch_bounds__(kOpThreads)
    batch_op_kernel(const BatchSlot *__restrict__ slots, const BatchItem *__restrict__ items,
                    const int *__restrict__ counts) {
  __shared__ __align__(16) unsigned char smem[F64 ? kLdsBytes : kLdsBytesLowp];
  const int n = counts[0];
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const BatchItem item = items[it];
    const BatchSlot &S = slots[item.slot];
    if (!S.active) continue;
    if (F64 ? (S.mixed != 0 && S.phase != kPhaseOuterOp) : (S.mixed == 0 || S.phase != kPhaseInner))
      continue;
#define OPCASE(n_, epb_)                                  \
    if (S.N == n_ && S.epb == epb_) {                     \
      if (F64)                                            \
        op_item_f64<n_ + 1, epb_>(S, item.first, smem);   \
      else                                                \
        op_item_lowp<n_ + 1, epb_>(S, item.first, smem);  \
      continue;                                           \
    }
    SEM_BATCH_TILES(OPCASE)
#undef OPCASE
  }
}

// Streaming items are walked so that each XCD takes one contiguous range of
// the list (tiles of one solve are contiguous in it).
__device__ inline void xcd_range(int n, int *start, int *end, int *step) {
  const int per_xcd_blocks = gridDim.x / kNumXcd;
  const int xcd = blockIdx.x % kNumXcd;
  const int chunk = (n + kNumXcd - 1) / kNumXcd;
  *start = xcd * chunk + blockIdx.x / kNumXcd;
  *end = min(n, (xcd + 1) * chunk);
  *step = per_xcd_blocks;
}

template <int N1>
__device__ __forceinline__ void update_item(const BatchSlot &S, int tile, double *sred) {
  if (S.mixed == 0) {
    if (S.phase != kPhaseFp64 || S.st->done != kRunning) return;
    const TileSums t = cg_update_tile<N1, double>(S.box, S.L, tile, S.r, S.w, S.minv,
                                                  S.st->alpha, sred);
    if (threadIdx.x == 0) {
      S.part_rr[tile] = t.a;
      S.part_rz[tile] = t.b;
    }
  } else if (S.phase == kPhaseInner) {
    if (S.st_in->done != kRunning) return;
    const TileSums t = cg_update_tile<N1, float>(S.box, S.L, tile, S.rin, S.win, S.minv32,
                                                 S.st_in->alpha, sred);
    if (threadIdx.x == 0) {
      S.part_rr[tile] = t.a;
      S.part_rz[tile] = t.b;
    }
  } else if (S.phase == kPhaseOuterOp) {
    const double rr = residual_tile<N1>(S.box, S.L, tile, S.b, S.w, S.r, sred);
    if (threadIdx.x == 0) S.part_rr[tile] = rr;
  }
}

__global__ void __launch_bounds__(kVecThreads)
    batch_update_kernel(const BatchSlot *__restrict__ slots, const BatchItem *__restrict__ items,
                        const int *__restrict__ counts) {
  __shared__ double sred[kVecThreads / 64];
  int start, end, step;
  xcd_range(counts[1], &start, &end, &step);
  for (int it = start; it < end; it += step) {
    const BatchItem item = items[it];
    const BatchSlot &S = slots[item.slot];
    if (!S.active) continue;
    switch (S.N) {
#define UCASE(n_) \
  case n_:        \
    update_item<n_ + 1>(S, item.first, sred); \
    break;
      UCASE(1) UCASE(2) UCASE(3) UCASE(4) UCASE(5) UCASE(6)
      UCASE(7) UCASE(8) UCASE(9) UCASE(10) UCASE(11)
#undef UCASE
      default:
        break;
    }
  }
}

// Second streaming launch: the end of an FP64 solve (x += alpha p), the
// correction of a mixed solve (e += alpha p, x += ||r|| e) and the inner
// restart (r_in = r / ||r||, e = p = 0 and the partials of its scalars).
template <int N1>
__device__ __forceinline__ void finish_item(const BatchSlot &S, int tile, double *sred) {
  if (S.phase == kPhaseFp64Done) {
    if (S.st->done_stage != 2) return;
    const double alpha = S.st->alpha;
    const int64_t base = (int64_t)tile * kVecTile + threadIdx.x;
#pragma unroll
    for (int u = 0; u < kVecItems; ++u) {
      const int64_t idx = base + (int64_t)u * kVecThreads;
      if (idx < S.L) S.x[idx] += alpha * S.p[idx];
    }
  } else if (S.phase == kPhaseInnerDone) {
    const bool add_p = S.st_in->done_stage == 2;
    outer_correct_tile(S.L, tile, S.x, S.e, S.pin, (float)S.st_in->alpha, add_p,
                       sqrt(S.st->rnorm2));
  } else if (S.phase == kPhaseRestart) {
    const TileSums t = inner_start_tile<N1>(S.box, S.L, tile, S.r, 1.0 / sqrt(S.st->rnorm2), S.rin,
                                            S.e, S.pin, S.minv32, sred);
    if (threadIdx.x == 0) {
      S.part_rz[tile] = t.a;
      S.part_rr[tile] = t.b;
    }
  }
}

__global__ void __launch_bounds__(kVecThreads)
    batch_finish_kernel(const BatchSlot *__restrict__ slots, const BatchItem *__restrict__ items,
                        const int *__restrict__ counts) {
  __shared__ double sred[kVecThreads / 64];
  int start, end, step;
  xcd_range(counts[1], &start, &end, &step);
  for (int it = start; it < end; it += step) {
    const BatchItem item = items[it];
    const BatchSlot &S = slots[item.slot];
    if (!S.active) continue;
    switch (S.N) {
#define FCASE(n_) \
  case n_:        \
    finish_item<n_ + 1>(S, item.first, sred); \
    break;
      FCASE(1) FCASE(2) FCASE(3) FCASE(4) FCASE(5) FCASE(6)
      FCASE(7) FCASE(8) FCASE(9) FCASE(10) FCASE(11)
#undef FCASE
      default:
        break;
    }
  }
}

// Per-solve launches: one work-group of kFinThreads per slot.
__global__ void __launch_bounds__(kFinThreads)
    batch_alpha_kernel(const BatchSlot *__restrict__ slots) {
  __shared__ double sred[kFinThreads / 64];
  const BatchSlot &S = slots[blockIdx.x];
  if (!S.active) return;
  if (S.mixed == 0 && S.phase == kPhaseFp64)
    cg_alpha_step(S.st, S.part_el, S.E, sred);
  else if (S.mixed != 0 && S.phase == kPhaseInner)
    cg_alpha_step(S.st_in, S.part_el, S.E, sred);
}

__global__ void __launch_bounds__(kFinThreads)
    batch_beta_kernel(BatchSlot *__restrict__ slots) {
  __shared__ double sred[kFinThreads / 64];
  BatchSlot &S = slots[blockIdx.x];
  if (!S.active) return;
  const int phase = S.phase;
  if (S.mixed == 0) {
    if (phase != kPhaseFp64) return;
    cg_beta_step(S.st, S.part_rr, S.part_rz, S.ntiles, sred);
    if (threadIdx.x == 0 && S.st->done != kRunning) S.phase = kPhaseFp64Done;
  } else if (phase == kPhaseInner) {
    cg_beta_step(S.st_in, S.part_rr, S.part_rz, S.ntiles, sred);
    if (threadIdx.x == 0 && S.st_in->done != kRunning) {
      S.inner_total += S.st_in->iter;
      if (S.st_in->iter == 0) {  // the inner solver made no progress
        S.st->done = kBreakdown;
        S.phase = kPhaseFinished;
      } else {
        S.phase = kPhaseInnerDone;
      }
    }
  } else if (phase == kPhaseOuterOp) {
    outer_finish_step(S.st, S.part_rr, S.ntiles, sred);
    if (threadIdx.x == 0) S.phase = S.st->done != kRunning ? kPhaseFinished : kPhaseRestart;
  }
}

__global__ void __launch_bounds__(kFinThreads)
    batch_phase_kernel(BatchSlot *__restrict__ slots, BatchStatus *__restrict__ status) {
  __shared__ double sred[kFinThreads / 64];
  BatchSlot &S = slots[blockIdx.x];
  if (!S.active) return;
  const int phase = S.phase;
  if (phase == kPhaseRestart) {
    inner_init_step(S.st_in, S.part_rz, S.part_rr, S.ntiles, S.eta2, S.inner_max, sred);
    if (threadIdx.x == 0) S.phase = S.st_in->done == kRunning ? kPhaseInner : kPhaseInnerDone;
  }
  if (threadIdx.x == 0) {
    if (phase == kPhaseFp64Done) S.phase = kPhaseFinished;
    if (phase == kPhaseInnerDone) S.phase = kPhaseOuterOp;
    BatchStatus st;
    st.phase = S.phase;
    st.done = S.st->done;
    st.iters = S.mixed ? S.inner_total : S.st->iter;
    st.outer_iters = S.mixed ? S.st->iter : 0;
    st.rnorm2 = S.st->rnorm2;
    st.bnorm2 = S.st->bnorm2;
    status[blockIdx.x] = st;
  }
}

}  // namespace

int batch_default_epb(int N) {
  const int n1 = N + 1;
  return n1 * n1 >= 128 ? 1 : 128 / (n1 * n1);
}

bool batch_epb_supported(int N, int epb) {
#define SCASE(n_, epb_) \
  if (N == n_ && epb == epb_) return true;
  SEM_BATCH_TILES(SCASE)
#undef SCASE
  return false;
}

hipError_t launch_batch_iteration(BatchSlot *slots, int max_slots, const BatchItem *op_items,
                                  const BatchItem *vec_items, const int *counts,
                                  BatchStatus *status, hipStream_t s) {
  hipLaunchKernelGGL(batch_op_kernel<true>, dim3(kBatchOpBlocks), dim3(kOpThreads), 0, s, slots,
                     op_items, counts);
  hipLaunchKernelGGL(batch_op_kernel<false>, dim3(kBatchOpBlocks), dim3(kOpThreads), 0, s, slots,
                     op_items, counts);
  hipLaunchKernelGGL(batch_alpha_kernel, dim3(max_slots), dim3(kFinThreads), 0, s, slots);
  hipLaunchKernelGGL(batch_update_kernel, dim3(kBatchVecBlocks), dim3(kVecThreads), 0, s, slots,
                     vec_items, counts);
  hipLaunchKernelGGL(batch_beta_kernel, dim3(max_slots), dim3(kFinThreads), 0, s, slots);
  hipLaunchKernelGGL(batch_finish_kernel, dim3(kBatchVecBlocks), dim3(kVecThreads), 0, s, slots,
                     vec_items, counts);
  hipLaunchKernelGGL(batch_phase_kernel, dim3(max_slots), dim3(kFinThreads), 0, s, slots, status);
  return hipGetLastError();
}

}  // namespace semk
