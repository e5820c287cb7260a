// Device pieces of the Jacobi-PCG (paper Sec. VIII-A) shared by the single-
// solve kernels and the batched persistent kernels: the same functions give
// the same bits on both paths.
//
// *_tile functions process one streaming tile (kVecTile consecutive entries
// of one element-local vector) with a work-group of kVecThreads and return
// the tile's block sums in thread 0.  *_step functions finish a reduction
// over a solve's partials with a work-group of kFinThreads and advance the
// solve's scalars (thread 0 writes).
#pragma once

#include <hip/hip_runtime.h>

#include "sem_device.h"
#include "sem_internal.h"

namespace semk {

constexpr int kFinThreads = 1024;

struct TileSums {
  double a, b;
};

// CG start: x = 0, r = mask o b, p = 0; sums <r, Minv r>_c and ||r||_c^2.
template <int N1>
__device__ inline TileSums cg_init_tile(const Box &b, int64_t L, int64_t tile,
                                        const double *__restrict__ bvec, double *__restrict__ x,
                                        double *__restrict__ r, double *__restrict__ p,
                                        const double *__restrict__ minv, double *sred) {
  double rz = 0.0, bb = 0.0;
  const int64_t base = tile * kVecTile + threadIdx.x;
#pragma unroll
  for (int u = 0; u < kVecItems; ++u) {
    const int64_t idx = base + (int64_t)u * kVecThreads;
    if (idx < L) {
      const Node<N1> n = node_at<N1>(b, idx);
      const double c = n.inv_mult();
      const double rv = n.boundary ? 0.0 : bvec[idx];
      x[idx] = 0.0;
      r[idx] = rv;
      p[idx] = 0.0;
      rz += c * rv * (minv[idx] * rv);
      bb += c * rv * rv;
    }
  }
  TileSums t;
  t.a = block_sum<kVecThreads>(rz, sred);
  t.b = block_sum<kVecThreads>(bb, sred);
  return t;
}

// CG update with the gather-scatter pulled in: r -= alpha mask o QQ^T w;
// sums ||r||_c^2 and <r, Minv r>_c (FP64 even for FP32 vectors).  FP64
// vectors: entry by entry, missing copies masked.  FP32 vectors: all loads of
// the thread's entries are issued first (clamped, branch-free addresses),
// then the arithmetic and the predicated stores; this measured 1.7x faster
// for FP32 and slower for FP64 (register pressure).
template <int N1, typename TV>
__device__ inline TileSums cg_update_tile(const Box &b, int64_t L, int64_t tile, TV *__restrict__ r,
                                          const TV *__restrict__ w, const TV *__restrict__ minv,
                                          double alpha, double *sred) {
  double rr = 0.0, rz = 0.0;
  const int64_t base = tile * kVecTile + threadIdx.x;
  if constexpr (sizeof(TV) == 8) {
#pragma unroll
    for (int u = 0; u < kVecItems; ++u) {
      const int64_t idx = base + (int64_t)u * kVecThreads;
      if (idx < L) {
        const Node<N1> n = node_at<N1>(b, idx);
        if (!n.boundary) {
          const double wa = gather_copies<N1>(w, b, n, idx);
          const TV rt = (TV)((double)ld_once(r + idx) - alpha * wa);
          r[idx] = rt;
          const double rv = (double)rt;
          const double c = n.inv_mult();
          rr += c * rv * rv;
          rz += c * rv * ((double)ld_once(minv + idx) * rv);
        }
      }
    }
    TileSums t;
    t.a = block_sum<kVecThreads>(rr, sred);
    t.b = block_sum<kVecThreads>(rz, sred);
    return t;
  }
  constexpr int GS = 4;
#pragma unroll
  for (int g0 = 0; g0 < kVecItems; g0 += GS) {
    Copies<N1> cp[GS];
    TV wv[GS][8], rv[GS], mv[GS];
    bool on[GS];
    double c[GS];
#pragma unroll
    for (int u = 0; u < GS; ++u) {
      const int64_t idx0 = base + (int64_t)(g0 + u) * kVecThreads;
      const int64_t idx = idx0 < L ? idx0 : L - 1;
      const Node<N1> n = node_at<N1>(b, idx);
      on[u] = idx0 < L && !n.boundary;
      c[u] = n.inv_mult();
      cp[u] = copies_of<N1>(b, n, idx);
      load_copies<N1, TV>(w, cp[u], wv[u]);
      rv[u] = ld_once(r + idx);
      mv[u] = ld_once(minv + idx);
    }
#pragma unroll
    for (int u = 0; u < GS; ++u) {
      if (on[u]) {
        const double wa = sum_copies<N1, TV>(cp[u], wv[u]);
        const TV rt = (TV)((double)rv[u] - alpha * wa);
        r[base + (int64_t)(g0 + u) * kVecThreads] = rt;
        const double rd = (double)rt;
        rr += c[u] * rd * rd;
        rz += c[u] * rd * ((double)mv[u] * rd);
      }
    }
  }
  TileSums t;
  t.a = block_sum<kVecThreads>(rr, sred);
  t.b = block_sum<kVecThreads>(rz, sred);
  return t;
}

// Inner start of the inner-outer CG: r_in = r / ||r||_c in FP32, e = 0,
// p = 0; sums <r_in, Minv r_in>_c and ||r_in||_c^2.
template <int N1>
__device__ inline TileSums inner_start_tile(const Box &b, int64_t L, int64_t tile,
                                            const double *__restrict__ r64, double inv_s,
                                            float *__restrict__ rin, float *__restrict__ e,
                                            float *__restrict__ p, const float *__restrict__ minv32,
                                            double *sred) {
  double rz = 0.0, rr = 0.0;
  const int64_t base = tile * kVecTile + threadIdx.x;
#pragma unroll
  for (int u = 0; u < kVecItems; ++u) {
    const int64_t idx = base + (int64_t)u * kVecThreads;
    if (idx < L) {
      const Node<N1> n = node_at<N1>(b, idx);
      const float rv = (float)(r64[idx] * inv_s);
      rin[idx] = rv;
      e[idx] = 0.0f;
      p[idx] = 0.0f;
      const double c = n.inv_mult();
      rz += c * (double)rv * ((double)minv32[idx] * (double)rv);
      rr += c * (double)rv * (double)rv;
    }
  }
  TileSums t;
  t.a = block_sum<kVecThreads>(rz, sred);
  t.b = block_sum<kVecThreads>(rr, sred);
  return t;
}

// True residual of the inner-outer CG: r = mask o (b - QQ^T w_L) with
// w_L = A_L x in FP64; sum ||r||_c^2.
template <int N1>
__device__ inline double residual_tile(const Box &b, int64_t L, int64_t tile,
                                       const double *__restrict__ bvec,
                                       const double *__restrict__ wl, double *__restrict__ r,
                                       double *sred) {
  double rr = 0.0;
  const int64_t base = tile * kVecTile + threadIdx.x;
#pragma unroll
  for (int u = 0; u < kVecItems; ++u) {
    const int64_t idx = base + (int64_t)u * kVecThreads;
    if (idx < L) {
      const Node<N1> n = node_at<N1>(b, idx);
      double rv = 0.0;
      if (!n.boundary) rv = bvec[idx] - gather_copies<N1>(wl, b, n, idx);
      r[idx] = rv;
      rr += rv * rv * n.inv_mult();
    }
  }
  return block_sum<kVecThreads>(rr, sred);
}

// Finish the inner solve and correct the outer iterate on one tile:
// e += alpha_in p_in (when the inner solve's last update ran), then
// x += s e with s = ||r||_c of the outer step.
__device__ inline void outer_correct_tile(int64_t L, int64_t tile, double *__restrict__ x,
                                          float *__restrict__ e, const float *__restrict__ p,
                                          float alpha, bool add_p, double s) {
  const int64_t base = tile * kVecTile + threadIdx.x;
#pragma unroll
  for (int u = 0; u < kVecItems; ++u) {
    const int64_t idx = base + (int64_t)u * kVecThreads;
    if (idx < L) {
      float ev = e[idx];
      if (add_p) {
        ev += alpha * p[idx];
        e[idx] = ev;
      }
      x[idx] += s * (double)ev;
    }
  }
}

// ---------------------------------------------------------------- steps
// rho, ||b||_c and the tolerance after cg_init_tile.
__device__ inline void cg_init_step(CgState *st, const double *__restrict__ part_rz,
                                    const double *__restrict__ part_bb, int64_t n, double *sred) {
  const double rho = sum_partials<kFinThreads>(part_rz, n, sred);
  const double bn = sum_partials<kFinThreads>(part_bb, n, sred);
  if (threadIdx.x == 0) {
    st->rho = rho;
    st->bnorm2 = bn;
    st->rnorm2 = bn;
    st->beta = 0.0;
    st->alpha = 0.0;
    st->iter = 0;
    st->tol2 = st->rtol2 * bn;
    st->done = (bn == 0.0) ? kConverged : kRunning;
    if (!isfinite(bn) || !isfinite(rho)) st->done = kBreakdown;
  }
}

// alpha = rho / <p, A p>_c (or breakdown) from the per-element partials.
__device__ inline void cg_alpha_step(CgState *st, const double *__restrict__ part, int64_t n,
                                     double *sred) {
  // the state loads are independent of the partial sums: issue them first
  const int done = st->done;
  const double rho = st->rho;
  const double pap = sum_partials<kFinThreads>(part, n, sred);
  if (threadIdx.x == 0 && done == kRunning) {
    st->pap = pap;
    if (!(pap > 0.0) || !isfinite(pap)) {
      st->done = kBreakdown;
      st->done_stage = 1;
    } else {
      st->alpha = rho / pap;
    }
  }
}

// Iteration count, ||r||_c, beta, rho and the done flag from the update's
// tile partials.
__device__ inline void cg_beta_step(CgState *st, const double *__restrict__ part_rr,
                                    const double *__restrict__ part_rz, int64_t n, double *sred) {
  const int done = st->done;
  const int it = st->iter + 1;
  const int max_iter = st->max_iter;
  const double rho = st->rho, tol2 = st->tol2;
  const double rrt = sum_partials<kFinThreads>(part_rr, n, sred);
  const double rzt = sum_partials<kFinThreads>(part_rz, n, sred);
  if (threadIdx.x == 0 && done == kRunning) {
    st->iter = it;
    st->rnorm2 = rrt;
    const double beta = rzt / rho;
    st->beta = beta;
    st->rho = rzt;
    if (!isfinite(rrt) || !isfinite(beta)) {
      st->done = kBreakdown;
    } else if (tol2 >= 0.0 && rrt <= tol2) {
      st->done = kConverged;
    } else if (it >= max_iter) {
      st->done = kMaxIter;
    }
    st->done_stage = 2;
  }
}

// Outer step of the inner-outer CG: ||r||_c^2 of the true residual, the outer
// count and the done flag.
__device__ inline void outer_finish_step(CgState *st, const double *__restrict__ part, int64_t n,
                                         double *sred) {
  const int done = st->done;
  const int it = st->iter + 1;
  const int max_iter = st->max_iter;
  const double tol2 = st->tol2;
  const double rr = sum_partials<kFinThreads>(part, n, sred);
  if (threadIdx.x == 0 && done == kRunning) {
    st->iter = it;
    st->rnorm2 = rr;
    if (!isfinite(rr)) {
      st->done = kBreakdown;
    } else if (rr <= tol2) {
      st->done = kConverged;
    } else if (it >= max_iter) {
      st->done = kMaxIter;
    }
  }
}

// Inner solve reset and start: tolerance eta^2 ||r_in||^2, cap, rho.
__device__ inline void inner_init_step(CgState *st, const double *__restrict__ part_rz,
                                       const double *__restrict__ part_rr, int64_t n, double rtol2,
                                       int max_iter, double *sred) {
  const double rho = sum_partials<kFinThreads>(part_rz, n, sred);
  const double rr = sum_partials<kFinThreads>(part_rr, n, sred);
  if (threadIdx.x == 0) {
    st->max_iter = max_iter;
    st->rtol2 = rtol2;
    st->done_stage = 0;
    st->rho = rho;
    st->bnorm2 = rr;
    st->rnorm2 = rr;
    st->beta = 0.0;
    st->alpha = 0.0;
    st->iter = 0;
    st->tol2 = rtol2 * rr;
    st->done = (rr == 0.0) ? kConverged : kRunning;
    if (!isfinite(rr) || !isfinite(rho)) st->done = kBreakdown;
  }
}

}  // namespace semk
