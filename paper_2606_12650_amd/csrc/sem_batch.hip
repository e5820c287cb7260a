// Batched Jacobi-PCG: many independent solves of different sizes and orders
// advance together, one CG iteration per batched step.
//
// Every batched iteration starts with a one-work-group schedule kernel that
// reads the solves' phases on the device and writes compact work lists: for
// each (arithmetic class, order) bin the solves with operator work in it and
// the prefix sums of their item counts, and the same for the streaming tiles
// of every unfinished solve.  The operator work then runs in one persistent
// launch per bin, each compiled for its order (work-group size, LDS and
// registers of the single-solve kernel of that order), so a bin of small
// elements is not held to the resources of the largest order.  Each work-group
// takes a contiguous range of its bin's items and finds their solves by
// searching the prefix sums; finished solves and idle phases take no items.
// The per-solve scalars run one work-group per solve, the streaming launches
// walk the streaming list in XCD-contiguous ranges.
//
// Every item is computed by the same device functions as a single solve
// (sem_ax_tile.h, sem_cg_dev.h) and each solve's reductions are summed in
// the same order (per-element and per-tile partials, fixed trees), so an FP64
// solve gives the same bits alone and in a batch, for any tile size.  A
// mixed-precision solve moves through the inner-outer phases (SlotPhase) on
// the device; the host only polls.
#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <mutex>
#include <type_traits>

#include "sem_ax_mfma.h"
#include "sem_ax_tile.h"
#include "sem_cg_dev.h"
#include "sem_device.h"
#include "sem_internal.h"

namespace semk {

namespace {

constexpr int kSchedThreads = 1024;

// Orders a batch takes.
#define SEM_BATCH_ORDERS(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11)

// Operator tiles compiled for batches (order, elements per work-group).  An
// order uses the vector-unit tiles or the matrix-core ones of its class, as
// its single solves do (op_uses_mfma): the single-solve tile first, then a
// larger one where the FP64 LDS stays within 64 KiB and the work-group within
// 512 (vector) or 1024 (matrix-core) threads.
#define SEM_BATCH_TILES_VALU(X)                                               \
  X(1, 32) X(1, 64) X(2, 14) X(2, 28) X(3, 8) X(3, 16) X(4, 5) X(4, 10)      \
  X(5, 3) X(5, 6) X(6, 2) X(6, 4) X(7, 2) X(7, 4) X(8, 1) X(8, 2) X(9, 1)   \
  X(9, 2) X(10, 1) X(11, 1)
#define SEM_BATCH_TILES_MFMA(X) X(7, 2) X(7, 4) X(8, 1) X(8, 2) X(9, 1) X(10, 1) X(11, 1)

template <int CLS>
struct ClassPrec;
template <>
struct ClassPrec<0> {
  using P = PrecF64;
};
template <>
struct ClassPrec<1> {
  using P = PrecF32;
};
template <>
struct ClassPrec<2> {
  using P = PrecBF16;
};
template <>
struct ClassPrec<3> {
  using P = PrecF64;
};

template <int N1, int EPB, bool MFMA>
struct OpCfg {
  static constexpr int THREADS =
      MFMA ? 64 * MfmaTile<N1>::W * EPB : (AxTile<N1>::TPE * EPB + 63) / 64 * 64;
  static constexpr int kTiles = MFMA ? 3 : AxTile<N1>::kTiles;
  static constexpr int SRED = MFMA ? THREADS / 64 : THREADS;
};

// Largest k in [0, cnt) with pre[k] <= w, for 1 <= cnt <= 4096 and
// pre[0] = 0 <= w, pre strictly increasing.  Called by whole waves (all 64
// lanes, uniform arguments); two rounds of one load per lane.
__device__ inline int find_slot(const int *__restrict__ pre, int cnt, int w) {
  const int lane = threadIdx.x & 63;
  int base = 0, span = cnt;
  if (cnt > 64) {
    const int step = (cnt + 63) / 64;
    const int idx = lane * step;
    const unsigned long long m = __ballot(idx < cnt && pre[idx] <= w);
    base = (63 - __clzll((long long)m)) * step;
    span = min(step, cnt - base);
  }
  const unsigned long long m = __ballot(lane < span && pre[base + lane] <= w);
  return base + 63 - __clzll((long long)m);
}

// [w0, w1): this work-group's contiguous share of n items.
__device__ inline void block_range(int n, int *w0, int *w1) {
  const int per = (n + (int)gridDim.x - 1) / (int)gridDim.x;
  *w0 = (int)blockIdx.x * per;
  *w1 = min(n, *w0 + per);
}

// Streaming items: each XCD takes one contiguous eighth of the list (the
// neighbour copies that the gather-scatter reads then sit in its L2), and each
// work-group a contiguous range of its XCD's eighth.  gridDim is a multiple
// of kNumXcd.
__device__ inline void xcd_block_range(int n, int *w0, int *w1) {
  const int blocks = (int)gridDim.x / kNumXcd;
  const int xcd = (int)blockIdx.x % kNumXcd, j = (int)blockIdx.x / kNumXcd;
  const int xper = (n + kNumXcd - 1) / kNumXcd;
  const int xs = xcd * xper, xe = min(n, xs + xper);
  const int per = (max(0, xe - xs) + blocks - 1) / blocks;
  *w0 = xs + j * per;
  *w1 = min(xe, *w0 + per);
}

// ------------------------------------------------------------- schedule

// Operator bin of a slot in this iteration (-1: no operator work).
__device__ inline int slot_bin(const BatchSlot &S) {
  if (!S.active || S.phase == kPhaseFinished) return -1;
  int cls = -1;
  if (S.mixed == 0) {
    if (S.phase == kPhaseFp64 && S.st->done == kRunning) cls = 0;
  } else if (S.phase == kPhaseOuterOp) {
    cls = 3;
  } else if (S.phase == kPhaseInner && S.st_in->done == kRunning) {
    cls = S.mixed == SEM_F32 ? 1 : 2;
  }
  return cls < 0 ? -1 : batch_bin(cls, S.N);
}

// Ordered compaction of one work list by one wave: the slots q < ms with
// count(q) > 0 in ascending order, the exclusive prefix sums of their counts
// (ballots and a wave scan) and [count, total].
template <class C>
__device__ inline void build_list(const BatchSched &sc, int b, int ms, C count) {
  const int lane = threadIdx.x & 63;
  int off = 0, run = 0;
  for (int c = 0; c < ms; c += 64) {
    const int q = c + lane;
    const int n = q < ms ? count(q) : 0;
    const bool in = n > 0;
    const unsigned long long m = __ballot(in);
    const int pos = __popcll(m & ((1ull << lane) - 1ull));
    int x = n;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int y = __shfl_up(x, d);
      if (lane >= d) x += y;
    }
    if (in) {
      sc.slot[b * ms + off + pos] = q;
      sc.prefix[b * (ms + 1) + off + pos] = run + x - n;
    }
    off += __popcll(m);
    run += __shfl(x, 63);
  }
  if (lane == 0) {
    sc.prefix[b * (ms + 1) + off] = run;
    sc.meta[2 * b] = off;
    sc.meta[2 * b + 1] = run;
  }
}

__global__ void __launch_bounds__(kSchedThreads)
    batch_schedule_kernel(const BatchSlot *__restrict__ slots, BatchSched sc, BatchTiles tiles) {
  __shared__ int s_bin[kBatchMaxSlots];
  __shared__ int s_cnt[kBatchMaxSlots];
  const int ms = sc.max_slots;
  for (int q = threadIdx.x; q < ms; q += blockDim.x) {
    const BatchSlot &S = slots[q];
    const int b = slot_bin(S);
    s_bin[q] = b;
    const int epb = b < 0 ? 1 : tiles.epb[b / kBatchOrders][S.N];
    s_cnt[q] = b < 0 ? 0 : (int)((S.E + epb - 1) / epb);
  }
  __syncthreads();
  // one wave per list
  const int wave = threadIdx.x >> 6;
  for (int b = wave; b < kBatchLists; b += kSchedThreads / 64) {
    if (b >= kBatchUpdLists) {
      // update tiles of the slots in the operator bins of this family and order
      const int fam = (b - kBatchUpdLists) / kBatchOrders;
      const int N = b - kBatchUpdLists - fam * kBatchOrders + 1;
      build_list(sc, b, ms, [&](int q) {
        const int sb = s_bin[q];
        const bool in_fam = fam == 0 ? sb == batch_bin(0, N)
                                     : (sb == batch_bin(1, N) || sb == batch_bin(2, N));
        return in_fam ? slots[q].utiles : 0;
      });
    } else if (b == kBatchResidList) {
      // streaming tiles of the slots whose outer operator runs (class 3)
      build_list(sc, b, ms, [&](int q) {
        const int sb = s_bin[q];
        return (sb >= 0 && sb / kBatchOrders == 3) ? slots[q].vtiles : 0;
      });
    } else if (b < kBatchBins) {
      build_list(sc, b, ms, [&](int q) { return s_bin[q] == b ? s_cnt[q] : 0; });
    }
  }
}

// The two finishing lists, rebuilt after the beta launch has set this
// iteration's phases: FP64 solves that stopped (x owes alpha p) and mixed
// solves whose inner solve ended or whose inner solve restarts.
__global__ void __launch_bounds__(128)
    batch_fin_schedule_kernel(const BatchSlot *__restrict__ slots, BatchSched sc) {
  const int wave = threadIdx.x >> 6;
  if (wave == 0) {
    build_list(sc, kBatchFinList, sc.max_slots, [&](int q) {
      const BatchSlot &S = slots[q];
      return (S.active && S.mixed == 0 && S.phase == kPhaseFp64Done && S.st->done_stage == 2)
                 ? S.vtiles : 0;
    });
  } else {
    build_list(sc, kBatchFinList + 1, sc.max_slots, [&](int q) {
      const BatchSlot &S = slots[q];
      return (S.active && S.mixed != 0 &&
              (S.phase == kPhaseInnerDone || S.phase == kPhaseRestart)) ? S.vtiles : 0;
    });
  }
}

// ------------------------------------------------------------- operator

// The element tile of a batched operator item: the matrix-core one or the
// vector-unit one, as the single solves of this class and order run.
template <int N1, int EPB, class P, bool CG, bool MFMA>
__device__ __forceinline__ void batch_tile(int64_t E, int64_t e0, const typename P::TC *D,
                                           const typename P::TG *G, typename P::TV *u,
                                           typename P::TV *w, const typename P::TV *r,
                                           const typename P::TV *minv, typename P::TV *x,
                                           double alpha, double beta, double *part,
                                           typename P::TC *sD, typename P::TC *s1,
                                           typename P::TC *s2, typename P::TC *s3, double *sred) {
  if constexpr (MFMA)
    ax_tile_mfma<N1, EPB, P, CG, true>(E, e0, D, G, u, w, r, minv, x, alpha, beta, part, sD, s1, s2, s3,
                                 sred);
  else
    ax_tile<N1, EPB, P, CG, true>(E, e0, D, G, u, w, r, minv, x, alpha, beta, part, sD, s1, s2, s3,
                                  sred);
}

template <int N1, int EPB, int CLS, bool MFMA>
__global__ void __launch_bounds__((OpCfg<N1, EPB, MFMA>::THREADS))
    batch_op_kernel(const BatchSlot *__restrict__ slots, BatchSched sc, int bin) {
  using P = typename ClassPrec<CLS>::P;
  using TC = typename P::TC;
  using T = AxTile<N1>;
  using C = OpCfg<N1, EPB, MFMA>;
  static_assert((int)sizeof(TC) * (N1 * N1 + C::kTiles * EPB * T::TILE) + 8 * C::SRED <= 64 * 1024,
                "batched operator tile exceeds 64 KiB of LDS");
  static_assert(C::THREADS <= (MFMA ? 1024 : 512), "batched operator tile exceeds its work-group");
  __shared__ TC sD[N1 * N1];
  __shared__ TC s1[EPB * T::TILE];
  __shared__ TC s2[EPB * T::TILE];
  __shared__ TC s3[C::kTiles == 3 ? EPB * T::TILE : 1];
  __shared__ double sred[C::SRED];
  const int cnt = sc.meta[2 * bin], total = sc.meta[2 * bin + 1];
  int w0, w1;
  block_range(total, &w0, &w1);
  if (w0 >= w1) return;
  const int *pre = sc.prefix + bin * (sc.max_slots + 1);
  const int *sl = sc.slot + bin * sc.max_slots;
  // the walk is uniform over the work-group: keep it in scalar registers
  int k = __builtin_amdgcn_readfirstlane(find_slot(pre, cnt, w0));
  int first = __builtin_amdgcn_readfirstlane(pre[k]);
  int next = __builtin_amdgcn_readfirstlane(pre[k + 1]);
#pragma unroll 1
  for (int w = w0; w < w1; ++w) {
    while (w >= next) {
      ++k;
      first = next;
      next = __builtin_amdgcn_readfirstlane(pre[k + 1]);
    }
    const BatchSlot &S = slots[__builtin_amdgcn_readfirstlane(sl[k])];
    const int64_t e0 = (int64_t)(w - first) * EPB;
    if constexpr (CLS == 0) {
      batch_tile<N1, EPB, PrecF64, true, MFMA>(S.E, e0, S.D, S.G, S.p, S.w, S.r, S.minv, S.x,
                                               S.st->alpha, S.st->beta, S.part_el, sD, s1, s2, s3,
                                               sred);
    } else if constexpr (CLS == 3) {  // true-residual operator of a mixed solve's outer step
      batch_tile<N1, EPB, PrecF64, false, MFMA>(S.E, e0, S.D, S.G, S.x, S.w, nullptr, nullptr,
                                                nullptr, 0.0, 0.0, S.part_el, sD, s1, s2, s3, sred);
    } else {
      batch_tile<N1, EPB, P, true, MFMA>(S.E, e0, S.Dlo, (const typename P::TG *)S.Glo, S.pin,
                                         S.win, S.rin, S.minv32, S.e, S.st_in->alpha,
                                         S.st_in->beta, S.part_el, sD, s1, s2, s3, sred);
    }
  }
}

// ------------------------------------------------------------- streaming

// The per-item functions below return false when the slot has no work of
// their kind in this iteration (the walk then skips its remaining items).

// The FP64 true residual of a mixed solve's outer step on one streaming tile.
template <int N1>
__device__ __forceinline__ bool residual_item(const BatchSlot &S, int tile, double *sred) {
  if (S.phase != kPhaseOuterOp || tile >= S.vtiles) return false;
  const double rr = residual_tile<N1>(S.box, S.L, tile, S.b, S.w, S.r, sred);
  if (threadIdx.x == 0) S.part_rr[tile] = rr;
  return true;
}

// The end of an FP64 solve (x += alpha p), the correction of a mixed solve
// (e += alpha p, x += ||r|| e) and the inner restart (r_in = r / ||r||,
// e = p = 0 and the partials of its scalars); these phases are set by the
// beta launch of the same iteration.
template <int N1, bool MIXED>
__device__ __forceinline__ bool finish_item(const BatchSlot &S, int tile, double *sred) {
  if constexpr (!MIXED) {
    if (S.phase != kPhaseFp64Done || S.st->done_stage != 2) return false;
    const double alpha = S.st->alpha;
    const int64_t base = (int64_t)tile * kVecTile + threadIdx.x;
#pragma unroll
    for (int u = 0; u < kVecItems; ++u) {
      const int64_t idx = base + (int64_t)u * kVecThreads;
      if (idx < S.L) S.x[idx] += alpha * S.p[idx];
    }
  } else {
    if (S.phase == kPhaseInnerDone) {
      const bool add_p = S.st_in->done_stage == 2;
      outer_correct_tile(S.L, tile, S.x, S.e, S.pin, (float)S.st_in->alpha, add_p,
                         sqrt(S.st->rnorm2));
    } else if (S.phase == kPhaseRestart) {
      const TileSums t = inner_start_tile<N1>(S.box, S.L, tile, S.r, 1.0 / sqrt(S.st->rnorm2),
                                              S.rin, S.e, S.pin, S.minv32, sred);
      if (threadIdx.x == 0) {
        S.part_rz[tile] = t.a;
        S.part_rr[tile] = t.b;
      }
    } else {
      return false;
    }
  }
  return true;
}

// A persistent walk over the items of one work list: each work-group takes
// a contiguous range of its XCD's share and calls f(slot, item) per item;
// when f returns false the slot has nothing to do in this launch and the
// walk jumps to the next slot.
template <class F>
__device__ __forceinline__ void walk_list(const BatchSlot *__restrict__ slots, const BatchSched &sc,
                                          int list, F f) {
  const int cnt = sc.meta[2 * list], total = sc.meta[2 * list + 1];
  int w0, w1;
  xcd_block_range(total, &w0, &w1);
  if (w0 >= w1) return;
  const int *pre = sc.prefix + list * (sc.max_slots + 1);
  const int *sl = sc.slot + list * sc.max_slots;
  // the walk is uniform over the work-group: keep it in scalar registers
  int k = __builtin_amdgcn_readfirstlane(find_slot(pre, cnt, w0));
  int first = __builtin_amdgcn_readfirstlane(pre[k]);
  int next = __builtin_amdgcn_readfirstlane(pre[k + 1]);
#pragma unroll 1
  for (int w = w0; w < w1; ++w) {
    while (w >= next) {
      ++k;
      first = next;
      next = __builtin_amdgcn_readfirstlane(pre[k + 1]);
    }
    if (!f(slots[__builtin_amdgcn_readfirstlane(sl[k])], w - first)) w = next - 1;
  }
}

// The CG update of one order and family (its own launch: the update tile's
// registers depend on the order).
template <int N1, bool MIXED>
using BatchUpd = UpdTile<N1, typename std::conditional<MIXED, float, double>::type>;

template <int N1, bool MIXED>
__global__ void __launch_bounds__((BatchUpd<N1, MIXED>::BLOCK))
    batch_upd_kernel(const BatchSlot *__restrict__ slots, BatchSched sc, int list) {
  using TV = typename std::conditional<MIXED, float, double>::type;
  __shared__ double sred[2 * (BatchUpd<N1, MIXED>::BLOCK / 64)];
  __shared__ double sA[BatchUpd<N1, MIXED>::LDS];
  const int cnt = sc.meta[2 * list], total = sc.meta[2 * list + 1];
  int w0, w1;
  xcd_block_range(total, &w0, &w1);
  if (w0 >= w1) return;
  const int *pre = sc.prefix + list * (sc.max_slots + 1);
  const int *sl = sc.slot + list * sc.max_slots;
  int k = __builtin_amdgcn_readfirstlane(find_slot(pre, cnt, w0));
  int first = __builtin_amdgcn_readfirstlane(pre[k]);
  int next = __builtin_amdgcn_readfirstlane(pre[k + 1]);
  // the slot's operands and state, loaded once per slot (not once per item)
  int cur = -1, active = 0, ut = 0;
  Box box;
  TV *r = nullptr;
  const TV *wv = nullptr, *minv = nullptr;
  double alpha = 0.0;
  double *prr = nullptr, *prz = nullptr;
#pragma unroll 1
  for (int w = w0; w < w1; ++w) {
    while (w >= next) {
      ++k;
      first = next;
      next = __builtin_amdgcn_readfirstlane(pre[k + 1]);
    }
    if (k != cur) {
      cur = k;
      const BatchSlot &S = slots[__builtin_amdgcn_readfirstlane(sl[k])];
      const CgState *st = MIXED ? S.st_in : S.st;
      active = __builtin_amdgcn_readfirstlane(
          (S.phase == (MIXED ? kPhaseInner : kPhaseFp64) && st->done == kRunning) ? 1 : 0);
      ut = S.utiles;
      box = S.box;
      alpha = st->alpha;
      prr = S.part_rr;
      prz = S.part_rz;
      if constexpr (MIXED) {
        r = S.rin; wv = S.win; minv = S.minv32;
      } else {
        r = S.r; wv = S.w; minv = S.minv;
      }
    }
    if (!active) {  // the slot has no update in this iteration: skip its items
      w = next - 1;
      continue;
    }
    const int tile = w - first;
    if (tile >= ut) continue;
    const TileSums t = cg_update_tile<N1, TV>(box, tile, r, wv, minv, alpha, sA, sred,
                                              (int)threadIdx.x);
    if (threadIdx.x == 0) {
      prr[tile] = t.a;
      prz[tile] = t.b;
    }
  }
}

// The outer steps' true residuals of the mixed solves (every order).
__global__ void __launch_bounds__(kVecThreads)
    batch_resid_kernel(const BatchSlot *__restrict__ slots, BatchSched sc) {
  __shared__ double sred[2 * (kVecThreads / 64)];
  walk_list(slots, sc, kBatchResidList, [&](const BatchSlot &S, int tile) {
    switch (S.N) {
#define RCASE(n_) \
  case n_:        \
    return residual_item<n_ + 1>(S, tile, sred);
      RCASE(1) RCASE(2) RCASE(3) RCASE(4) RCASE(5) RCASE(6)
      RCASE(7) RCASE(8) RCASE(9) RCASE(10) RCASE(11)
#undef RCASE
      default:
        return false;
    }
  });
}

// The phases that end an iteration, one launch per family: FP64 solves
// (MIXED = false) or mixed solves, so that each compiles only its own paths.
template <bool MIXED>
__global__ void __launch_bounds__(kVecThreads)
    batch_fin_kernel(const BatchSlot *__restrict__ slots, BatchSched sc) {
  __shared__ double sred[2 * (kVecThreads / 64)];
  walk_list(slots, sc, kBatchFinList + (MIXED ? 1 : 0), [&](const BatchSlot &S, int tile) {
    switch (S.N) {
#define FCASE(n_) \
  case n_:        \
    return finish_item<n_ + 1, MIXED>(S, tile, sred);
      FCASE(1) FCASE(2) FCASE(3) FCASE(4) FCASE(5) FCASE(6)
      FCASE(7) FCASE(8) FCASE(9) FCASE(10) FCASE(11)
#undef FCASE
      default:
        return false;
    }
  });
}

// ------------------------------------------------------------- scalars

// Per-solve launches: one work-group of kFinThreads per slot.
__global__ void __launch_bounds__(kFinThreads)
    batch_alpha_kernel(const BatchSlot *__restrict__ slots) {
  __shared__ double sred[2 * (kFinThreads / 64)];
  const BatchSlot &S = slots[blockIdx.x];
  if (!S.active) return;
  if (S.mixed == 0 && S.phase == kPhaseFp64)
    cg_alpha_step(S.st, S.part_el, S.E, sred);
  else if (S.mixed != 0 && S.phase == kPhaseInner)
    cg_alpha_step(S.st_in, S.part_el, S.E, sred);
}

__global__ void __launch_bounds__(kFinThreads)
    batch_beta_kernel(BatchSlot *__restrict__ slots) {
  __shared__ double sred[2 * (kFinThreads / 64)];
  BatchSlot &S = slots[blockIdx.x];
  if (!S.active) return;
  const int phase = S.phase;
  if (S.mixed == 0) {
    if (phase != kPhaseFp64) return;
    cg_beta_step(S.st, S.part_rr, S.part_rz, S.utiles, sred);
    if (threadIdx.x == 0 && S.st->done != kRunning) S.phase = kPhaseFp64Done;
  } else if (phase == kPhaseInner) {
    cg_beta_step(S.st_in, S.part_rr, S.part_rz, S.utiles, sred);
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
    outer_finish_step(S.st, S.part_rr, S.vtiles, sred);
    if (threadIdx.x == 0) S.phase = S.st->done != kRunning ? kPhaseFinished : kPhaseRestart;
  }
}

__global__ void __launch_bounds__(kFinThreads)
    batch_phase_kernel(BatchSlot *__restrict__ slots, BatchStatus *__restrict__ status) {
  __shared__ double sred[2 * (kFinThreads / 64)];
  BatchSlot &S = slots[blockIdx.x];
  if (!S.active) return;
  const int phase = S.phase;
  if (phase == kPhaseRestart) {
    inner_init_step(S.st_in, S.part_rz, S.part_rr, S.vtiles, S.eta2, S.inner_max, sred);
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

// ------------------------------------------------------------- launch sizes

// Resident work-groups of each persistent kernel on a device: the occupancy
// the compiler's resource use allows, times the compute units.
struct BatchGrids {
  int op[kBatchClasses][kBatchOrders + 1][65];  // [class][order][elements per item]
  int upd[2][kBatchOrders + 1];                 // [FP64, inner][order]
  int resid;
  int fin[2];                                   // [FP64, mixed]
};
std::mutex g_grid_mu;
std::map<int, BatchGrids> g_grids;

template <class K>
int resident_blocks(K kernel, int threads, int cus, int mult = 1) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(kernel),
                                                   threads, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return per_cu * cus * mult;
}
// The operator and update launches take 16 times the resident work-groups,
// each a sixteenth of the range: a work-group that moves on to its next item
// first waits for its previous item's stores (one counter covers vector loads
// and stores), while a fresh work-group starts loading at once.  Measured on
// MI355X: one 32.8 M-point N = 9 solve batched took 2.10 s at 1x, 1.86 s at
// 16x (1.67 s as a single solve); 64x and 256x were slower again.
#ifndef SEM_BATCH_GRID_MULT
#define SEM_BATCH_GRID_MULT 16
#endif

const BatchGrids *current_grids() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lock(g_grid_mu);
  auto it = g_grids.find(dev);
  return it == g_grids.end() ? nullptr : &it->second;
}

// Grid sizes of the operator kernels of one tile in every class that runs it.
template <int N1, int EPB, bool MFMA>
void fill_grid(BatchGrids &g, int cus) {
  constexpr int N = N1 - 1;
  constexpr int T = OpCfg<N1, EPB, MFMA>::THREADS;
  if constexpr (op_uses_mfma(0, N) == MFMA)
    g.op[0][N][EPB] = resident_blocks(batch_op_kernel<N1, EPB, 0, MFMA>, T, cus, SEM_BATCH_GRID_MULT);
  if constexpr (op_uses_mfma(1, N) == MFMA)
    g.op[1][N][EPB] = resident_blocks(batch_op_kernel<N1, EPB, 1, MFMA>, T, cus, SEM_BATCH_GRID_MULT);
  if constexpr (op_uses_mfma(2, N) == MFMA)
    g.op[2][N][EPB] = resident_blocks(batch_op_kernel<N1, EPB, 2, MFMA>, T, cus, SEM_BATCH_GRID_MULT);
  if constexpr (op_uses_mfma(3, N) == MFMA)
    g.op[3][N][EPB] = resident_blocks(batch_op_kernel<N1, EPB, 3, MFMA>, T, cus, SEM_BATCH_GRID_MULT);
}

template <int N1, int EPB, bool MFMA>
bool launch_op(int cls, const BatchGrids &g, const BatchSlot *slots, const BatchSched &sc, int bin,
               hipStream_t s) {
  constexpr int N = N1 - 1;
  if (op_uses_mfma(cls, N) != MFMA) return false;
  const dim3 grid(g.op[cls][N][EPB]), threads(OpCfg<N1, EPB, MFMA>::THREADS);
  if constexpr (op_uses_mfma(0, N) == MFMA)
    if (cls == 0) hipLaunchKernelGGL((batch_op_kernel<N1, EPB, 0, MFMA>), grid, threads, 0, s, slots, sc, bin);
  if constexpr (op_uses_mfma(1, N) == MFMA)
    if (cls == 1) hipLaunchKernelGGL((batch_op_kernel<N1, EPB, 1, MFMA>), grid, threads, 0, s, slots, sc, bin);
  if constexpr (op_uses_mfma(2, N) == MFMA)
    if (cls == 2) hipLaunchKernelGGL((batch_op_kernel<N1, EPB, 2, MFMA>), grid, threads, 0, s, slots, sc, bin);
  if constexpr (op_uses_mfma(3, N) == MFMA)
    if (cls == 3) hipLaunchKernelGGL((batch_op_kernel<N1, EPB, 3, MFMA>), grid, threads, 0, s, slots, sc, bin);
  return true;
}

}  // namespace

int batch_default_epb(int cls, int N) {
  const int n1 = N + 1;
  if (op_uses_mfma(cls, N)) {
    const int nw = mfma_waves(n1);
    return nw >= 8 ? 1 : 8 / nw;
  }
  return n1 * n1 >= 128 ? 1 : 128 / (n1 * n1);
}

bool batch_epb_supported(int cls, int N, int epb) {
  if (cls < 0 || cls >= kBatchClasses) return false;
  const bool mfma = op_uses_mfma(cls, N);
#define SCASE_V(n_, epb_) \
  if (!mfma && N == n_ && epb == epb_) return true;
#define SCASE_M(n_, epb_) \
  if (mfma && N == n_ && epb == epb_) return true;
  SEM_BATCH_TILES_VALU(SCASE_V)
  SEM_BATCH_TILES_MFMA(SCASE_M)
#undef SCASE_V
#undef SCASE_M
  return false;
}

hipError_t batch_prepare() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  {
    std::lock_guard<std::mutex> lock(g_grid_mu);
    if (g_grids.count(dev)) return hipSuccess;
  }
  int cus = 0;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  BatchGrids g;
  std::memset(&g, 0, sizeof(g));
#define GCASE_V(n_, epb_) fill_grid<n_ + 1, epb_, false>(g, cus);
#define GCASE_M(n_, epb_) fill_grid<n_ + 1, epb_, true>(g, cus);
  SEM_BATCH_TILES_VALU(GCASE_V)
  SEM_BATCH_TILES_MFMA(GCASE_M)
#undef GCASE_V
#undef GCASE_M
#define UCASE(n_)                                                                     \
  g.upd[0][n_] = xcd_grid(                                                              \
      resident_blocks(batch_upd_kernel<n_ + 1, false>, BatchUpd<n_ + 1, false>::BLOCK, cus, SEM_BATCH_GRID_MULT));  \
  g.upd[1][n_] = xcd_grid(                                                              \
      resident_blocks(batch_upd_kernel<n_ + 1, true>, BatchUpd<n_ + 1, true>::BLOCK, cus, SEM_BATCH_GRID_MULT));
  SEM_BATCH_ORDERS(UCASE)
#undef UCASE
  g.resid = xcd_grid(resident_blocks(batch_resid_kernel, kVecThreads, cus));
  g.fin[0] = xcd_grid(resident_blocks(batch_fin_kernel<false>, kVecThreads, cus));
  g.fin[1] = xcd_grid(resident_blocks(batch_fin_kernel<true>, kVecThreads, cus));
  (void)hipGetLastError();
  std::lock_guard<std::mutex> lock(g_grid_mu);
  g_grids[dev] = g;
  return hipSuccess;
}

hipError_t launch_batch_iteration(BatchSlot *slots, int max_slots, const BatchSched &sched,
                                  const BatchTiles &tiles, uint64_t bins, BatchStatus *status,
                                  hipStream_t s) {
  const BatchGrids *g = current_grids();
  if (!g) return hipErrorNotInitialized;
  hipLaunchKernelGGL(batch_schedule_kernel, dim3(1), dim3(kSchedThreads), 0, s, slots, sched, tiles);
  for (int cls = 0; cls < kBatchClasses; ++cls)
    for (int N = 1; N <= kBatchOrders; ++N) {
      const int bin = batch_bin(cls, N);
      if (!((bins >> bin) & 1u)) continue;
      const int epb = tiles.epb[cls][N];
      bool launched = false;
#define LCASE_V(n_, epb_)                                                         \
  if (!launched && N == n_ && epb == epb_)                                        \
    launched = launch_op<n_ + 1, epb_, false>(cls, *g, slots, sched, bin, s);
#define LCASE_M(n_, epb_)                                                         \
  if (!launched && N == n_ && epb == epb_)                                        \
    launched = launch_op<n_ + 1, epb_, true>(cls, *g, slots, sched, bin, s);
      SEM_BATCH_TILES_VALU(LCASE_V)
      SEM_BATCH_TILES_MFMA(LCASE_M)
#undef LCASE_V
#undef LCASE_M
      if (!launched) return hipErrorInvalidValue;
    }
  hipLaunchKernelGGL(batch_alpha_kernel, dim3(max_slots), dim3(kFinThreads), 0, s, slots);
  const bool f64 = (bins >> kBatchBins) & 1u, mix = (bins >> (kBatchBins + 1)) & 1u;
  auto in_use = [&](int cls, int N) { return ((bins >> batch_bin(cls, N)) & 1u) != 0; };
#define UCASE(n_)                                                                              \
  if (in_use(0, n_))                                                                           \
    hipLaunchKernelGGL((batch_upd_kernel<n_ + 1, false>), dim3(g->upd[0][n_]),                 \
                       dim3(BatchUpd<n_ + 1, false>::BLOCK), 0, s, slots, sched,              \
                       batch_upd_list(0, n_));                                                 \
  if (in_use(1, n_) || in_use(2, n_))                                                          \
    hipLaunchKernelGGL((batch_upd_kernel<n_ + 1, true>), dim3(g->upd[1][n_]),                  \
                       dim3(BatchUpd<n_ + 1, true>::BLOCK), 0, s, slots, sched,               \
                       batch_upd_list(1, n_));
  SEM_BATCH_ORDERS(UCASE)
#undef UCASE
  if (mix)
    hipLaunchKernelGGL(batch_resid_kernel, dim3(g->resid), dim3(kVecThreads), 0, s, slots, sched);
  hipLaunchKernelGGL(batch_beta_kernel, dim3(max_slots), dim3(kFinThreads), 0, s, slots);
  hipLaunchKernelGGL(batch_fin_schedule_kernel, dim3(1), dim3(128), 0, s, slots, sched);
  if (f64)
    hipLaunchKernelGGL((batch_fin_kernel<false>), dim3(g->fin[0]), dim3(kVecThreads), 0, s, slots,
                       sched);
  if (mix)
    hipLaunchKernelGGL((batch_fin_kernel<true>), dim3(g->fin[1]), dim3(kVecThreads), 0, s, slots,
                       sched);
  hipLaunchKernelGGL(batch_phase_kernel, dim3(max_slots), dim3(kFinThreads), 0, s, slots, status);
  return hipGetLastError();
}

}  // namespace semk
