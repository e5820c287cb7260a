// Types and launch-shape rules of libsem that device code sees: mesh and
// solver state, tile shapes, batch records.  Nothing here names the HIP
// runtime API, so the run-time compiled kernels (orders outside the
// compiled set) include it as the built kernels do.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "sem.h"

namespace semk {

constexpr int kMinOrder = 1;
constexpr int kMaxOrder = 12;     // orders whose kernels are built with the library
constexpr int kMaxRtcOrder = 15;  // orders compiled at run time (one MFMA row block: N + 1 <= 16)

// Unsigned division by a runtime constant d >= 1 as a multiply and shift
// (Granlund-Montgomery): q = (n * M) >> k with k = 32 + ceil(log2 d) and
// M = ceil(2^k / d) < 2^33; exact for every n < 2^31.
struct FastDiv {
  uint64_t M;
  uint32_t k;
  uint32_t d;
  static FastDiv make(uint32_t d) {
    uint32_t sh = 0;
    while ((1ull << sh) < d) ++sh;
    FastDiv f;
    f.k = 32 + sh;
    f.M = ((1ull << f.k) + d - 1) / d;
    f.d = d;
    return f;
  }
  __host__ __device__ uint32_t div(uint32_t n) const { return (uint32_t)(((uint64_t)n * M) >> k); }
};

// Box mesh dimensions and polynomial order (fdx, fdy divide by nx, ny).
struct Box {
  int nx, ny, nz, N;
  FastDiv fdx, fdy;
  static Box make(int nx, int ny, int nz, int N) {
    Box b;
    b.nx = nx; b.ny = ny; b.nz = nz; b.N = N;
    b.fdx = FastDiv::make((uint32_t)nx);
    b.fdy = FastDiv::make((uint32_t)ny);
    return b;
  }
  __host__ __device__ int n1() const { return N + 1; }
  __host__ __device__ int64_t E() const { return (int64_t)nx * ny * nz; }
  __host__ __device__ int64_t np() const { return (int64_t)(N + 1) * (N + 1) * (N + 1); }
  __host__ __device__ int64_t L() const { return E() * np(); }
};

// Status of a device-resident CG solve.
enum CgDone : int { kRunning = 0, kConverged = 1, kBreakdown = 2, kMaxIter = 3 };

// Scalars of the CG recurrence, kept in device memory so that no iteration
// needs the host.  `done` is first so that a single aligned load checks it.
struct CgState {
  int done;
  int iter;
  int max_iter;
  int done_stage;  // 2 when the last finished iteration updated r (x still owes alpha p)
  double rho;     // <r, Minv r>_c
  double alpha;
  double beta;
  double pap;     // <p, A p>_c
  double rnorm2;  // <r, r>_c
  double bnorm2;  // <b, b>_c
  double rtol2;   // rtol^2 (< 0: fixed-iteration mode, never converges)
  double tol2;    // rtol2 * bnorm2
};

// Launch shapes of the element kernels (shared by host sizing code).
int ax_elements_per_block(int N);
int64_t ax_num_blocks(const Box &b);
constexpr int kVecThreads = 256;
constexpr int kVecItems = 8;   // entries per thread of the streaming kernels
constexpr int64_t kVecTile = (int64_t)kVecThreads * kVecItems;
inline int64_t vec_num_blocks(int64_t n) { return (n + kVecTile - 1) / kVecTile; }
// Launch size (and partial count) of the element-local streaming kernels:
// tiles padded to a multiple of the XCD count.
inline int64_t vec_grid_blocks(int64_t n) { return 8 * ((vec_num_blocks(n) + 7) / 8); }

// Tiles of the CG update (the gather-scatter pulled into r -= alpha w) are
// element-aligned: upd_ept consecutive elements with upd_ks threads per
// (i, j) column over all planes.  Up to order 7 a tile fills 256 threads; at
// order 8 it holds two FP64 elements or one FP32 element with three threads
// per column; at orders 9 and 10 the FP32 tile holds two elements with one
// thread per column.  The FP64 update from order 9 and the FP32 update from
// order 11 keep linear streaming tiles of kVecTile entries.  All of these
// are the candidates (upd_shape) that measured fastest per CG iteration on
// MI355X.
__host__ __device__ constexpr int upd_ks(int n1, bool f64) { return n1 == 9 ? 3 : 1; }
__host__ __device__ constexpr int upd_ept(int n1, bool f64) {
  return n1 == 9 ? (f64 ? 2 : 1) : n1 >= 10 ? 2 : kVecThreads / (n1 * n1);
}
__host__ __device__ constexpr bool upd_linear(int n1, bool f64) { return n1 >= (f64 ? 10 : 12); }

// Candidate update tiles for tuning: shape v of an order and vector type
// (threads per column, elements per tile, plane ranges per element).  v = 0
// is the default above ({0, 0, 0}: the linear streaming tile); v = 1 ..
// kUpdVariants - 1 are alternatives compiled beside it for orders 1..12:
// more elements per tile, more threads per column (fewer planes per thread),
// fewer elements per tile, or plane ranges.  Every candidate stays within
// 512 threads and 32 KiB of LDS.  ks = -1 marks a missing candidate (the
// orders compiled at run time have the default only).
struct UpdShape {
  int ks, ept, kp;
};
constexpr int kUpdVariants = 4;
__host__ __device__ constexpr UpdShape upd_shape(int n1, bool f64, int v) {
  if (v == 0)
    return upd_linear(n1, f64) ? UpdShape{0, 0, 0} : UpdShape{upd_ks(n1, f64), upd_ept(n1, f64), 1};
  if (v < 0 || v >= kUpdVariants) return UpdShape{-1, 0, 0};
  switch (n1) {
    case 2: return v == 1 ? UpdShape{1, 128, 1} : v == 2 ? UpdShape{1, 32, 1} : UpdShape{2, 32, 1};
    case 3: return v == 1 ? UpdShape{1, 56, 1} : v == 2 ? UpdShape{1, 14, 1} : UpdShape{3, 18, 1};
    case 4: return v == 1 ? UpdShape{1, 32, 1} : v == 2 ? UpdShape{1, 8, 1} : UpdShape{2, 16, 1};
    case 5: return v == 1 ? UpdShape{1, 20, 1} : v == 2 ? UpdShape{1, 5, 1} : UpdShape{2, 10, 1};
    case 6: return v == 1 ? UpdShape{1, 14, 1} : v == 2 ? UpdShape{2, 3, 1} : UpdShape{2, 7, 1};
    case 7: return v == 1 ? UpdShape{1, 10, 1} : v == 2 ? UpdShape{2, 2, 1} : UpdShape{2, 5, 1};
    case 8: return v == 1 ? UpdShape{1, 8, 1} : v == 2 ? UpdShape{2, 2, 1} : UpdShape{2, 4, 1};
    case 9:
      if (f64) return v == 1 ? UpdShape{1, 4, 1} : v == 2 ? UpdShape{1, 2, 1} : UpdShape{3, 1, 1};
      return v == 1 ? UpdShape{1, 4, 1} : v == 2 ? UpdShape{1, 2, 1} : UpdShape{3, 2, 1};
    case 10:
      if (f64) return v == 1 ? UpdShape{2, 2, 1} : v == 2 ? UpdShape{2, 1, 1} : UpdShape{1, 4, 1};
      return v == 1 ? UpdShape{2, 2, 1} : v == 2 ? UpdShape{2, 1, 1} : UpdShape{1, 4, 1};
    case 11:
      if (f64) return v == 1 ? UpdShape{2, 2, 1} : v == 2 ? UpdShape{2, 1, 1} : UpdShape{1, 2, 1};
      return v == 1 ? UpdShape{2, 2, 1} : v == 2 ? UpdShape{2, 1, 1} : UpdShape{4, 1, 1};
    case 12:
      if (f64) return v == 1 ? UpdShape{1, 2, 2} : v == 2 ? UpdShape{2, 1, 1} : UpdShape{3, 1, 1};
      return v == 1 ? UpdShape{3, 1, 1} : v == 2 ? UpdShape{2, 1, 1} : UpdShape{2, 1, 2};
    case 13:
      if (f64) return v == 1 ? UpdShape{1, 2, 2} : v == 2 ? UpdShape{2, 1, 1} : UpdShape{3, 1, 1};
      return v == 1 ? UpdShape{2, 1, 1} : v == 2 ? UpdShape{3, 1, 1} : UpdShape{1, 1, 2};
    default: return UpdShape{-1, 0, 0};
  }
}
__host__ __device__ constexpr bool upd_variant_exists(int n1, bool f64, int v) {
  return v >= 0 && v < kUpdVariants && upd_shape(n1, f64, v).ks >= 0;
}
// Update tiles of shape v on box b (one partial per tile).
inline int64_t upd_num_tiles(const Box &b, bool f64, int v = 0) {
  const UpdShape sh = upd_shape(b.N + 1, f64, v);
  if (sh.ks == 0) return vec_num_blocks(b.L());
  return (b.E() + sh.ept - 1) / sh.ept * sh.kp;
}
// Launch size of the update (a multiple of the XCD count).
inline int64_t upd_grid_blocks(const Box &b, bool f64, int v = 0) {
  return 8 * ((upd_num_tiles(b, f64, v) + 7) / 8);
}
// Partials a solve's streaming reductions need room for (every candidate
// update tile of both vector types).
inline int64_t stream_partials(const Box &b) {
  int64_t v = vec_grid_blocks(b.L());
  for (int f = 0; f < 2; ++f)
    for (int k = 0; k < kUpdVariants; ++k)
      if (upd_variant_exists(b.N + 1, f == 1, k)) {
        const int64_t u = upd_grid_blocks(b, f == 1, k);
        if (u > v) v = u;
      }
  return v;
}

// What the gather kernel writes at a node: the sum of its copies
// (assembled), the same with box-boundary nodes zeroed (masked), or the
// Jacobi inverse 1/sum with boundary nodes zeroed (inverse).
enum GatherMode : int { kGatherAssembled = 0, kGatherMasked = 1, kGatherInverse = 2 };

// ---------------------------------------------------------------- operator
// Which element tile an operator runs by default, per arithmetic class (0 and
// 3 FP64, 1 FP32, 2 BF16) and order N: the matrix-core tile (sem_ax_mfma.h)
// where it measured faster on MI355X than the vector-unit tiles
// (sem_ax_tile.h) inside the CG, i.e. from N = 7 in FP64 and FP32 and from
// N = 9 in BF16.
__host__ __device__ constexpr bool op_uses_mfma(int cls, int N) {
  return (cls == 0 || cls == 3 || cls == 1) ? N >= 7 : N >= 9;
}

// Operator implementation request: the default above, or forced.
enum OpImpl : int { kImplDefault = 0, kImplMfma = 1, kImplValu = 2 };

// ---------------------------------------------------------------- batches
// Phase of a solve inside a batch (advanced on the device).
enum SlotPhase : int {
  kPhaseFp64 = 0,       // FP64 Jacobi-PCG iterations
  kPhaseFp64Done = 1,   // FP64 solve stopped: the last x += alpha p is pending
  kPhaseInner = 2,      // inner low-precision PCG iterations
  kPhaseInnerDone = 3,  // inner solve stopped: x += ||r|| (e + alpha p) pending
  kPhaseOuterOp = 4,    // FP64 true residual of the corrected x
  kPhaseRestart = 5,    // inner restart r_in = r / ||r|| pending
  kPhaseFinished = 6,   // nothing left to do
};

// One solve of a batch: the operator data of its sem_ctx plus its vectors.
struct BatchSlot {
  Box box;
  int N;
  int vtiles;  // streaming tiles (vec_num_blocks(L)); partials of the streaming phases
  int mixed;   // 0: FP64, else the low-precision copy's sem_prec
  int active;
  int phase;  // SlotPhase, written by the device
  int inner_total;
  int inner_max;
  int utiles;  // update tiles of its CG update (upd_num_tiles); partials of that update
  double eta2;
  int64_t E, L;
  const double *D, *G, *b;
  double *minv, *r, *p, *w, *x;
  const float *Dlo;
  const void *Glo;
  float *minv32, *e, *rin, *pin, *win;
  CgState *st, *st_in;
  double *part_el, *part_rr, *part_rz;
};

// Compact per-slot status the host polls (written by the device).
struct BatchStatus {
  int phase;
  int done;
  int iters;        // FP64 iterations, or total inner iterations (mixed)
  int outer_iters;  // mixed: outer steps
  double rnorm2, bnorm2;
};

// Operator work of a batched iteration is binned by class and order: class 0
// is the FP64 CG iterations of FP64 solves, classes 1 and 2 the FP32 and BF16
// inner iterations of mixed solves, class 3 the FP64 true-residual operator
// of their outer steps.  Lists kBatchFinList and kBatchFinList + 1 hold the
// streaming tiles of the FP64 and mixed solves whose phase ends this
// iteration (rebuilt after the beta launch), kBatchResidList those of the
// mixed solves computing an outer true residual; after them come the update
// tiles of the CG update, per order, of the FP64 solves (family 0, the slots
// of bin (0, N)) and of the inner solves (family 1, bins (1, N) and (2, N)).
constexpr int kBatchOrders = 11;  // batches take orders 1..11
constexpr int kBatchClasses = 4;
constexpr int kBatchBins = kBatchClasses * kBatchOrders;
constexpr int kBatchFinList = kBatchBins;
constexpr int kBatchResidList = kBatchBins + 2;
constexpr int kBatchUpdLists = kBatchBins + 3;
constexpr int kBatchLists = kBatchUpdLists + 2 * kBatchOrders;
constexpr int kBatchMaxSlots = 4096;
__host__ __device__ inline int batch_bin(int cls, int N) { return cls * kBatchOrders + (N - 1); }
__host__ __device__ inline int batch_upd_list(int fam, int N) {
  return kBatchUpdLists + fam * kBatchOrders + (N - 1);
}

// Work lists that the schedule kernel rebuilds on the device at the start of
// every batched iteration (kBatchLists lists, max_slots entries each): the
// slots with work in the bin in ascending order, the exclusive prefix sums of
// their item counts (one more entry: the total), and [count, total].
struct BatchSched {
  int *meta;
  int *slot;
  int *prefix;
  int max_slots;
};

// Elements per operator item, by class and order (index 1..11).
struct BatchTiles {
  int epb[kBatchClasses][kBatchOrders + 1];
};

}  // namespace semk
