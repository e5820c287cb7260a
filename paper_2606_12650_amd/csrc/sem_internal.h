// Internal declarations of libsem: the kernel launchers shared by the C-ABI
// translation unit and the kernel units (types in sem_types.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "sem_types.h"

namespace semk {

// Operator tiles compiled for batches, per class and order: elements per
// work-group of the default tile of that class and order (its single-solve
// size first).
int batch_default_epb(int cls, int N);
bool batch_epb_supported(int cls, int N, int epb);
// Resident work-groups of every batched kernel on the current device
// (queried once per process; call before graph capture).
hipError_t batch_prepare();

// One batched iteration over every active slot: the schedule, one operator
// launch per bin set in `bins` (bit cls * 11 + N - 1), the per-solve scalar
// launches and the streaming launches of the FP64 and mixed solves (bits
// kBatchBins and kBatchBins + 1 of `bins`: which families are present).
hipError_t launch_batch_iteration(BatchSlot *slots, int max_slots, const BatchSched &sched,
                                  const BatchTiles &tiles, uint64_t bins, BatchStatus *status,
                                  hipStream_t s);

// ---------------------------------------------------------------- launchers
// All return the hipError_t of the launch (hipGetLastError after it).

// G (E x 6 x np) and the element-local Jacobi diagonal (L) of box b.
hipError_t launch_setup_geom(const Box &b, double amp, const double *D, const double *nodes,
                             double *G, double *diag_local, hipStream_t s);
// Inverse multiplicity c as an L-vector.
hipError_t launch_fill_c(const Box &b, double *c, hipStream_t s);

// w = A_L u.  With cg != null (a CG iteration) a prologue first finishes the
// previous iteration, x += alpha p, then forms p <- Minv r + beta p (u is p,
// updated in place), and the per-element sums of p.w go to part (E of them).
// impl: an OpImpl.  stream_w: w goes to the caller as it is (no gather reads
// it next), so the matrix-core tile writes it with non-temporal stores (the
// orders compiled at run time keep plain stores).
hipError_t launch_ax_f64(const Box &b, int impl, const double *D, const double *G, double *u,
                         double *w, const double *r, const double *minv, double *x, CgState *cg,
                         double *part, hipStream_t s, bool stream_w = false);

// Low-precision operator (prec SEM_F32 or SEM_BF16): FP32 vectors, G stored
// as float or bfloat16 bits, D as float (bfloat16-rounded in BF16 mode),
// FP32 accumulation; the CG variant mirrors launch_ax_f64 (x is the inner
// correction e).  impl: an OpImpl.
hipError_t launch_ax_lowp(const Box &b, int prec, int impl, const float *D, const void *G, float *u,
                          float *w, const float *r, const float *minv, float *x, CgState *cg,
                          double *part, hipStream_t s, bool stream_w = false);
// dst[i] = src[i] rounded to float (SEM_F32) or to bfloat16 bits (SEM_BF16).
hipError_t launch_convert_g(int prec, int64_t n, const double *src, void *dst, hipStream_t s);

// out = the copies of every node of wl summed (GatherMode); wl != out.
hipError_t launch_gather(const Box &b, const double *wl, double *out, int mode, hipStream_t s);
hipError_t launch_gather_f32(const Box &b, const float *wl, float *out, int mode, hipStream_t s);

// CG start: x = 0, r = mask o b, p = 0, partials of <r, Minv r>_c and
// ||b||_c^2; then a one-group launch sets rho, ||b||_c and the tolerance.
hipError_t launch_cg_init(const Box &b, const double *bvec, double *x, double *r, double *p,
                          const double *minv, CgState *st, double *part_a, double *part_b,
                          hipStream_t s);
// CG update with the gather of w fused in: r -= alpha mask o QQ^T w,
// partials of ||r||_c^2 and <r, Minv r>_c (upd_num_tiles(b, f64, variant) of
// each).  Skipped when done.  variant: the update tile shape (upd_shape; the
// orders compiled at run time have shape 0 only).
hipError_t launch_cg_update(const Box &b, int variant, double *r, const double *w, const double *minv,
                            CgState *st, double *part_rr, double *part_rz, hipStream_t s);
// One-group launches that finish the reductions and advance the scalars:
// alpha = rho / <p, A p> (breakdown check), and after the update
// iteration count, ||r||_c, rho, beta and the done flag.
hipError_t launch_cg_alpha(CgState *st, const double *part_pap, int64_t n, hipStream_t s);
hipError_t launch_cg_beta(CgState *st, const double *part_rr, const double *part_rz, int64_t n,
                          hipStream_t s);
// After the last iteration: x += alpha p if that iteration's update ran.
hipError_t launch_cg_finish(const Box &b, double *x, const double *p, const CgState *st,
                            hipStream_t s);
// FP32 update for the inner solver of the inner-outer CG.
hipError_t launch_cg_update_f32(const Box &b, int variant, float *r, const float *w, const float *minv,
                                CgState *st, double *part_rr, double *part_rz, hipStream_t s);

// Inner-outer CG steps.  inner_start: r_in = r / ||r||_c in FP32, e = p = 0,
// then the inner state: tolerance rtol2 = eta^2 (relative), iteration cap,
// rho.  outer_correct: e += alpha_in p_in (if the inner solve's last update
// ran), x += ||r||_c e.  outer_step (after w64 = A_L x): r = mask o (b -
// QQ^T w64), ||r||_c^2, the outer count and the done flag.
hipError_t launch_inner_start(const Box &b, const double *r64, CgState *outer, CgState *inner,
                              double rtol2, int max_iter, float *rin, float *e, float *p,
                              const float *minv32, double *part_a, double *part_b, hipStream_t s);
hipError_t launch_outer_correct(const Box &b, double *x, float *e, const float *p,
                                const CgState *inner, const CgState *outer, hipStream_t s);
hipError_t launch_outer_step(const Box &b, const double *bvec, const double *w64, double *r64,
                             CgState *outer, double *part, hipStream_t s);

// Non-specialised kernels of the specialisation study (sem_generic.hip):
// the operator with N a run-time argument (orders 1..kGenericMaxN1 - 1),
// axpy and dot with the work-group size `block` chosen at launch (a power of
// two in [64, 1024]) and a looped in-group tree.  The dot's partials hold
// generic_dot_groups(n, block) doubles.
constexpr int kGenericMaxN1 = 12;
constexpr int64_t kGenericMaxGrid = 65536;
int generic_ax_epb(int N);
int64_t generic_dot_groups(int64_t n, int block);
hipError_t launch_ax_generic(const Box &b, const double *D, const double *G, const double *u,
                             double *w, hipStream_t s);
hipError_t launch_axpy_generic(int64_t n, double alpha, const double *x, double *y, int block,
                               hipStream_t s);
hipError_t launch_dot_generic(int64_t n, const double *x, const double *y, const double *wt,
                              double *out, double *partials, int block, hipStream_t s);

// Generic vectors.
hipError_t launch_axpy(int64_t n, double alpha, const double *x, double *y, hipStream_t s);
hipError_t launch_dot(int64_t n, const double *x, const double *y, const double *wt,
                      double *out, double *partials, hipStream_t s);

}  // namespace semk
