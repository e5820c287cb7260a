// The per-order kernels of libsem (N fixed at compile time, as the jit clause
// of the paper's "ax" kernel fixes it, Sec. VIII-B): the metric setup, the
// element operator (vector-ALU and matrix-core tiles), the gather-scatter
// forms, the CG start and the CG update.  The library builds them for orders
// 1..12 (sem_ax.hip, sem_vec.hip); for orders 13..15 the same text is
// compiled at run time (sem_rtc.hip), so both paths run the same kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "sem_ax_mfma.h"
#include "sem_ax_tile.h"
#include "sem_cg_dev.h"
#include "sem_device.h"
#include "sem_types.h"

namespace semk {

template <int N1>
struct AxCfg {
  // elements per work-group of the per-order kernels: about 128 threads of
  // one (i, j) column each
  static constexpr int EPB = (N1 * N1 >= 128) ? 1 : (128 / (N1 * N1));
  static constexpr int THREADS = N1 * N1 * EPB;
};

// The operator kernels: the same elements per work-group, AxTile<N1>::TPE
// threads per element.
#ifndef SEM_OP_MIN_WAVES_SPLIT
#define SEM_OP_MIN_WAVES_SPLIT 1
#endif
#ifndef SEM_OP_MIN_WAVES_COL
#define SEM_OP_MIN_WAVES_COL 1
#endif
template <int N1>
struct OpCfg {
  static constexpr int EPB = AxCfg<N1>::EPB;
  static constexpr int THREADS = AxTile<N1>::TPE * EPB;
  static constexpr int MIN_WAVES = AxTile<N1>::kSplit ? SEM_OP_MIN_WAVES_SPLIT : SEM_OP_MIN_WAVES_COL;
};

template <int N1, class P, bool CG>
__global__ void __launch_bounds__(OpCfg<N1>::THREADS, OpCfg<N1>::MIN_WAVES)
    ax_kernel(int64_t E, const typename P::TC *__restrict__ Dg, const typename P::TG *__restrict__ G,
              typename P::TV *u, typename P::TV *__restrict__ w, const typename P::TV *__restrict__ r,
              const typename P::TV *__restrict__ minv, typename P::TV *__restrict__ x,
              CgState *__restrict__ st, double *__restrict__ part) {
  using C = OpCfg<N1>;
  using TC = typename P::TC;
  __shared__ TC sD[N1 * N1];
  __shared__ TC s1[C::EPB * AxTile<N1>::TILE];
  __shared__ TC s2[C::EPB * AxTile<N1>::TILE];
  __shared__ TC s3[AxTile<N1>::kTiles == 3 ? C::EPB * AxTile<N1>::TILE : 1];
  __shared__ double sred[CG ? C::THREADS : 1];
  double alpha = 0.0, beta = 0.0;
  if (CG) {
    if (st->done) return;  // uniform: converged solves skip all work
    alpha = st->alpha;
    beta = st->beta;
  }
  ax_tile<N1, C::EPB, P, CG>(E, (int64_t)blockIdx.x * C::EPB, Dg, G, u, w, r, minv, x, alpha, beta,
                             part, sD, s1, s2, s3, sred);
}

// The operator with the D contractions on the matrix cores (sem_ax_mfma.h):
// ceil((N+1)^2 / 16) waves per element.
template <int N1, class P, bool CG, bool SW>
__device__ __forceinline__ void ax_mfma_body(int64_t E, const typename P::TC *__restrict__ Dg,
                                             const typename P::TG *__restrict__ G,
                                             typename P::TV *u, typename P::TV *__restrict__ w,
                                             const typename P::TV *__restrict__ r,
                                             const typename P::TV *__restrict__ minv,
                                             typename P::TV *__restrict__ x,
                                             CgState *__restrict__ st, double *__restrict__ part) {
  using C = MfmaCfg<N1>;
  using TC = typename P::TC;
  __shared__ TC sD[N1 * N1];
  __shared__ TC s1[C::EPB * AxTile<N1>::TILE];
  __shared__ TC s2[C::EPB * AxTile<N1>::TILE];
  __shared__ TC s3[C::EPB * AxTile<N1>::TILE];
  __shared__ double sred[C::THREADS / 64];
  double alpha = 0.0, beta = 0.0;
  if (CG) {
    if (st->done) return;  // uniform: converged solves skip all work
    alpha = st->alpha;
    beta = st->beta;
  }
  ax_tile_mfma<N1, C::EPB, P, CG, false, SW>(E, (int64_t)blockIdx.x * C::EPB, Dg, G, u, w, r, minv,
                                             x, alpha, beta, part, sD, s1, s2, s3, sred);
}

template <int N1, class P, bool CG>
__global__ void __launch_bounds__(MfmaCfg<N1>::THREADS, (mfma_waves_per_simd<N1, P, CG>()))
    ax_mfma_kernel(int64_t E, const typename P::TC *__restrict__ Dg,
                   const typename P::TG *__restrict__ G, typename P::TV *u,
                   typename P::TV *__restrict__ w, const typename P::TV *__restrict__ r,
                   const typename P::TV *__restrict__ minv, typename P::TV *__restrict__ x,
                   CgState *__restrict__ st, double *__restrict__ part) {
  ax_mfma_body<N1, P, CG, false>(E, Dg, G, u, w, r, minv, x, st, part);
}

// The element-local sem_ax, whose result goes to the caller as it is (no
// gather reads it next): the same kernel with w written by non-temporal
// stores.
template <int N1, class P>
__global__ void __launch_bounds__(MfmaCfg<N1>::THREADS, (mfma_waves_per_simd<N1, P, false>()))
    ax_mfma_local_kernel(int64_t E, const typename P::TC *__restrict__ Dg,
                         const typename P::TG *__restrict__ G, typename P::TV *u,
                         typename P::TV *__restrict__ w) {
  ax_mfma_body<N1, P, false, true>(E, Dg, G, u, w, nullptr, nullptr, nullptr, nullptr, nullptr);
}

// Metric setup: coordinates of the (deformed) box mesh, isoparametric
// Jacobian by D along r, s, t, G = w_i w_j w_k det(J) J^-1 J^-T, then the
// diagonal of the element operator.
template <int N1>
__global__ void __launch_bounds__(AxCfg<N1>::THREADS)
    setup_geom_kernel(Box b, double amp, const double *__restrict__ Dg,
                      const double *__restrict__ nodes, double *__restrict__ G,
                      double *__restrict__ diag) {
  using C = AxCfg<N1>;
  using T = AxTile<N1>;
  constexpr int NP = T::NP;
  constexpr int PL = N1 * N1;
  constexpr int N = N1 - 1;
  __shared__ double sD[N1 * N1];
  __shared__ double sx[3][C::EPB * T::TILE];

  const int tid = threadIdx.x;
  const int el = tid / PL;
  const int ij = tid - el * PL;
  const int i = ij % N1;
  const int j = ij / N1;
  const int64_t e = (int64_t)blockIdx.x * C::EPB + el;
  const bool active = e < b.E();
  for (int t = tid; t < N1 * N1; t += C::THREADS) sD[t] = Dg[t];

  const int64_t ee = active ? e : 0;
  const int ex = (int)(ee % b.nx);
  const int ey = (int)((ee / b.nx) % b.ny);
  const int ez = (int)(ee / ((int64_t)b.nx * b.ny));
  const double xi_i = nodes[i], xi_j = nodes[j];
  const double X0 = (ex + 0.5 * (xi_i + 1.0)) / b.nx;
  const double Y0 = (ey + 0.5 * (xi_j + 1.0)) / b.ny;
  double *SX = sx[0] + el * T::TILE;
  double *SY = sx[1] + el * T::TILE;
  double *SZ = sx[2] + el * T::TILE;
  const double twopi = 2.0 * M_PI;
  for (int k = 0; k < N1; ++k) {
    const double Z0 = (ez + 0.5 * (nodes[k] + 1.0)) / b.nz;
    double bump = 0.0;
    if (amp != 0.0) bump = amp * sin(twopi * X0) * sin(twopi * Y0) * sin(twopi * Z0);
    const int o = k * T::PLANE + j * T::P + i;
    SX[o] = X0 + bump;
    SY[o] = Y0 + bump;
    SZ[o] = Z0 + bump;
  }
  __syncthreads();

  const double wij = nodes[N1 + i] * nodes[N1 + j];
  const int64_t base = e * NP + ij;
  double grr[N1], gss[N1], gtt[N1], grs[N1], grt[N1], gst[N1];
  for (int k = 0; k < N1; ++k) {
    double J[3][3];
    double *S[3] = {SX, SY, SZ};
    for (int d = 0; d < 3; ++d) {
      double a = 0.0, bb = 0.0, c = 0.0;
      for (int l = 0; l < N1; ++l) {
        a += sD[i * N1 + l] * S[d][k * T::PLANE + j * T::P + l];
        bb += sD[j * N1 + l] * S[d][k * T::PLANE + l * T::P + i];
        c += sD[k * N1 + l] * S[d][l * T::PLANE + j * T::P + i];
      }
      J[d][0] = a;
      J[d][1] = bb;
      J[d][2] = c;
    }
    // cofactors; inv[m][d] = cof[d][m] / det
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double c10 = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    const double c11 = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    const double c12 = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    const double c20 = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    const double c21 = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    const double c22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    // rows of J^-1: R_m[d] = cof[d][m] / det
    const double inv = 1.0 / det;
    const double R0[3] = {c00 * inv, c10 * inv, c20 * inv};
    const double R1[3] = {c01 * inv, c11 * inv, c21 * inv};
    const double R2[3] = {c02 * inv, c12 * inv, c22 * inv};
    const double sc = wij * nodes[N1 + k] * det;
    grr[k] = sc * (R0[0] * R0[0] + R0[1] * R0[1] + R0[2] * R0[2]);
    grs[k] = sc * (R0[0] * R1[0] + R0[1] * R1[1] + R0[2] * R1[2]);
    grt[k] = sc * (R0[0] * R2[0] + R0[1] * R2[1] + R0[2] * R2[2]);
    gss[k] = sc * (R1[0] * R1[0] + R1[1] * R1[1] + R1[2] * R1[2]);
    gst[k] = sc * (R1[0] * R2[0] + R1[1] * R2[1] + R1[2] * R2[2]);
    gtt[k] = sc * (R2[0] * R2[0] + R2[1] * R2[1] + R2[2] * R2[2]);
    if (active) {
      double *Ge = G + e * 6 * NP + ij + k * PL;
      Ge[0 * NP] = grr[k];
      Ge[1 * NP] = grs[k];
      Ge[2 * NP] = grt[k];
      Ge[3 * NP] = gss[k];
      Ge[4 * NP] = gst[k];
      Ge[5 * NP] = gtt[k];
    }
  }
  __syncthreads();
  for (int k = 0; k < N1; ++k) {
    const int o = k * T::PLANE + j * T::P + i;
    SX[o] = grr[k];
    SY[o] = gss[k];
    SZ[o] = gtt[k];
  }
  __syncthreads();
  const double Dii = sD[i * N1 + i], Djj = sD[j * N1 + j];
  for (int k = 0; k < N1; ++k) {
    double d = 0.0;
    for (int l = 0; l < N1; ++l) {
      const double a = sD[l * N1 + i], bb = sD[l * N1 + j], c = sD[l * N1 + k];
      d += a * a * SX[k * T::PLANE + j * T::P + l];
      d += bb * bb * SY[k * T::PLANE + l * T::P + i];
      d += c * c * SZ[l * T::PLANE + j * T::P + i];
    }
    const double Dkk = sD[k * N1 + k];
    d += 2.0 * Dii * Djj * grs[k] + 2.0 * Dii * Dkk * grt[k] + 2.0 * Djj * Dkk * gst[k];
    if (active) diag[base + k * PL] = d;
  }
  (void)N;
}

// ------------------------------------------------------------ gather-scatter
template <int N1, int MODE, typename T>
__global__ void __launch_bounds__(kVecThreads)
    gather_kernel(Box b, int64_t L, int64_t ntiles, const T *__restrict__ wl, T *__restrict__ out) {
  const int64_t tile = xcd_tile(ntiles);
  if (tile >= ntiles) return;
  const int64_t base = tile * kVecTile + threadIdx.x;
#pragma unroll
  for (int u = 0; u < kVecItems; ++u) {
    const int64_t idx = base + (int64_t)u * kVecThreads;
    if (idx < L) {
      const Node<N1> n = node_at<N1>(b, idx);
      double v;
      if (MODE != kGatherAssembled && n.boundary) {
        v = 0.0;
      } else {
        v = gather_copies<N1>(wl, b, n, idx);
        if (MODE == kGatherInverse) v = 1.0 / v;
      }
      out[idx] = (T)v;
    }
  }
}

// The same gather on element-column tiles (copies paired across faces, as
// in the CG update), used where that tile is the update's tile.
template <int N1, int MODE, typename T>
__global__ void __launch_bounds__((UpdTile<N1, T>::BLOCK))
    gather_col_kernel(Box b, int64_t ntiles, const T *__restrict__ wl, T *__restrict__ out) {
  using U = UpdTile<N1, T>;
  __shared__ double sA[U::LDS];
  const int64_t tile = xcd_tile(ntiles);
  if (tile >= ntiles) return;
  const ColumnPos<N1, T> p(b, tile, (int)threadIdx.x);
  double S[U::KN];
  column_copy_sums<N1, T>(p, wl, sA, S);
#pragma unroll
  for (int kk = 0; kk < U::KN; ++kk) {
    const int k = p.kb + kk;
    if (p.live && k < p.kend) {
      double v = S[kk];
      if (MODE != kGatherAssembled && p.boundary(b, k))
        v = 0.0;
      else if (MODE == kGatherInverse)
        v = 1.0 / v;
      out[p.col0 + (int64_t)k * U::COLS] = (T)v;
    }
  }
}

// ------------------------------------------------------------ CG kernels
template <int N1>
__global__ void __launch_bounds__(kVecThreads)
    cg_init_kernel(Box b, int64_t L, int64_t ntiles, const double *__restrict__ bvec,
                   double *__restrict__ x, double *__restrict__ r, double *__restrict__ p,
                   const double *__restrict__ minv, double *__restrict__ part_rz,
                   double *__restrict__ part_bb) {
  __shared__ double sred[2 * (kVecThreads / 64)];
  const int64_t tile = xcd_tile(ntiles);
  TileSums t{0.0, 0.0};
  if (tile < ntiles) t = cg_init_tile<N1>(b, L, tile, bvec, x, r, p, minv, sred);
  if (threadIdx.x == 0) {
    part_rz[tile] = t.a;
    part_bb[tile] = t.b;
  }
}

// V: the update tile shape (upd_shape), one kernel per candidate.
template <int N1, typename TV, int V = 0>
__global__ void __launch_bounds__((UpdTile<N1, TV, V>::BLOCK))
    cg_update_kernel(Box b, int64_t ntiles, TV *__restrict__ r, const TV *__restrict__ w,
                     const TV *__restrict__ minv, CgState *__restrict__ st,
                     double *__restrict__ part_rr, double *__restrict__ part_rz) {
  __shared__ double sred[2 * (UpdTile<N1, TV, V>::BLOCK / 64)];
  __shared__ double sA[UpdTile<N1, TV, V>::LDS];
  if (st->done) return;
  const double alpha = st->alpha;
  const int64_t tile = xcd_tile(ntiles);
  TileSums t{0.0, 0.0};
  if (tile < ntiles)
    t = cg_update_tile<N1, TV, V>(b, tile, r, w, minv, alpha, sA, sred, (int)threadIdx.x);
  if (threadIdx.x == 0) {
    part_rr[tile] = t.a;
    part_rz[tile] = t.b;
  }
}

// ------------------------------------------------------------ setup helpers
template <int N1>
__global__ void __launch_bounds__(kVecThreads)
    fill_c_kernel(Box b, int64_t L, double *__restrict__ c) {
  const int64_t base = (int64_t)blockIdx.x * kVecTile + threadIdx.x;
#pragma unroll
  for (int u = 0; u < kVecItems; ++u) {
    const int64_t idx = base + (int64_t)u * kVecThreads;
    if (idx < L) c[idx] = node_at<N1>(b, idx).inv_mult();
  }
}

}  // namespace semk
