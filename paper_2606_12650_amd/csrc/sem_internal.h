// Internal declarations of libsem: workspace layout, device CG state and the
// kernel launchers shared by the C-ABI translation unit and the kernel units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "sem.h"

namespace semk {

constexpr int kMinOrder = 1;
constexpr int kMaxOrder = 12;

// Box mesh dimensions and polynomial order.
struct Box {
  int nx, ny, nz, N;
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
  int pad;
  double rho;     // <r, Minv r>_c
  double alpha;
  double beta;
  double pap;     // <p, A p>_c
  double rnorm2;  // <r, r>_c
  double bnorm2;  // <b, b>_c
  double rtol2;   // rtol^2 (< 0: fixed-iteration mode, never converges)
  double tol2;    // rtol2 * bnorm2
};

// Skeleton categories for the gather-scatter: nodes whose lattice index is a
// multiple of N in the directions of the bit set c (bit 0 = x, 1 = y, 2 = z).
// start[c-1] .. start[c]-1 are the thread ids of category c (c = 1..7).
struct Skeleton {
  int64_t start[8];
};
Skeleton make_skeleton(const Box &b);

// Launch shapes of the element kernels (shared by host sizing code).
int ax_elements_per_block(int N);
int64_t ax_num_blocks(const Box &b);
constexpr int kVecThreads = 256;
constexpr int kVecItems = 8;   // entries per thread of the streaming kernels
constexpr int64_t kVecTile = (int64_t)kVecThreads * kVecItems;
inline int64_t vec_num_blocks(int64_t n) { return (n + kVecTile - 1) / kVecTile; }

// ---------------------------------------------------------------- launchers
// All return the hipError_t of the launch (hipGetLastError after it).

// G (E x 6 x np) and the element-local Jacobi diagonal (L) of box b.
hipError_t launch_setup_geom(const Box &b, double amp, const double *D, const double *nodes,
                             double *G, double *diag_local, hipStream_t s);
// In place: d <- (interior node) ? 1/d : 0.
hipError_t launch_invert_diag(const Box &b, double *d, hipStream_t s);
// Inverse multiplicity c as an L-vector.
hipError_t launch_fill_c(const Box &b, double *c, hipStream_t s);

// w = A_L u.  With cg != null the CG prologue p <- Minv r + beta p runs first
// (u is p, updated in place) and per-block partial sums of p.w go to part.
hipError_t launch_ax_f64(const Box &b, const double *D, const double *G, double *u, double *w,
                         const double *r, const double *minv, const CgState *cg, double *part,
                         hipStream_t s);

// Gather-scatter over copies of shared nodes; masked != 0 zeroes boundary
// nodes.  Skipped when *done != 0 (done may be null).
hipError_t launch_dssum(const Box &b, const Skeleton &sk, double *w, int masked, const int *done,
                        hipStream_t s);

// CG pieces (all skip when the state's done flag is set).
hipError_t launch_cg_init(const Box &b, const double *bvec, double *x, double *r, double *p,
                          const double *minv, double *part_rz, double *part_bb, hipStream_t s);
hipError_t launch_cg_finalize_init(CgState *st, const double *part_rz, const double *part_bb,
                                   int64_t nparts, hipStream_t s);
hipError_t launch_cg_finalize_alpha(CgState *st, const double *part_pw, int64_t nparts,
                                    hipStream_t s);
hipError_t launch_cg_update(const Box &b, double *x, const double *p, double *r, const double *w,
                            const double *minv, const CgState *st, double *part_rr,
                            double *part_rz, hipStream_t s);
hipError_t launch_cg_finalize_beta(CgState *st, const double *part_rr, const double *part_rz,
                                   int64_t nparts, hipStream_t s);

// Generic vectors.
hipError_t launch_axpy(int64_t n, double alpha, const double *x, double *y, hipStream_t s);
hipError_t launch_dot(int64_t n, const double *x, const double *y, const double *wt,
                      double *out, double *partials, hipStream_t s);

}  // namespace semk
