// The element operator on one tile of elements, shared by the per-order
// kernels and the batched persistent kernel (same code, same bits).
//
// Mapping (one element per (N+1)^2 threads): thread (i, j) of an element owns
// the column of nodes (i, j, 0..N) in registers.  The contraction along t runs
// in registers; the contractions along r and s read the element's tile from
// LDS.  Every HBM access is a full-wave coalesced load or store of a k-plane
// of the element (element-major layout, i fastest).
#pragma once

#include <hip/hip_runtime.h>

#include "sem_device.h"
#include "sem_types.h"

namespace semk {

template <int N1>
struct AxTile {
  static constexpr int P = N1 + 1;      // padded row (LDS bank spread)
  static constexpr int PLANE = N1 * P;  // one k-plane of the padded tile
  static constexpr int TILE = N1 * PLANE;
  static constexpr int NP = N1 * N1 * N1;
  static constexpr int kTiles = N1 > 8 ? 3 : 2;  // LDS tiles per element
  // Orders N >= 8 split each (i, j) column over two threads (k halves): a
  // whole column of FP64 values no longer fits the register budget of more
  // than one wave per SIMD.
  static constexpr bool kSplit = N1 >= 9;
  static constexpr int TPE = (kSplit ? 2 : 1) * N1 * N1;  // threads per element
};

// The operator on one tile of EPB consecutive elements starting at e0,
// computed by the first N1*N1*EPB threads of the work-group (any others
// only join the barriers).  Shared by the per-order kernels below and the
// batched persistent kernel, so both produce the same bits.
//   CG: prologue x += alpha p_old, p = Minv r + beta p_old (u is p), and the
//   per-element sums of p.(A_L p) go to part_el[e] (summed in a fixed tree).
// sD: N1*N1, s1/s2 (and s3 when AxTile<N1>::kTiles == 3): EPB *
// AxTile<N1>::TILE values of TC each, sred: blockDim doubles, all in LDS.
template <int N1, int EPB, class P, bool CG, bool OPQ = false>
__device__ __forceinline__ void ax_tile_col(int64_t E, int64_t e0, const typename P::TC *__restrict__ Dg,
                                        const typename P::TG *__restrict__ G, typename P::TV *u,
                                        typename P::TV *__restrict__ w,
                                        const typename P::TV *__restrict__ r,
                                        const typename P::TV *__restrict__ minv,
                                        typename P::TV *__restrict__ x, double alpha_d, double beta_d,
                                        double *__restrict__ part_el, typename P::TC *sD,
                                        typename P::TC *s1, typename P::TC *s2,
                                        typename P::TC *s3, double *sred) {
  using T = AxTile<N1>;
  using TV = typename P::TV;
  using TC = typename P::TC;
  constexpr int NP = T::NP;
  constexpr int PL = N1 * N1;
  const int tid = OPQ ? opaque_tid() : (int)threadIdx.x;
  const int el = tid / PL;
  const int ij = tid - el * PL;
  const int i = ij % N1;
  const int j = ij / N1;
  const int64_t e = e0 + el;
  const bool active = el < EPB && e < E;

  for (int t = tid; t < N1 * N1; t += blockDim.x) sD[t] = Dg[t];

  const int64_t base = e * NP + ij;
  // G is loaded for the whole column up front (all its latency overlaps) up to
  // N = 7; beyond, one k-plane at a time keeps the register count in bounds.
  constexpr bool kPrefetchG = N1 <= 8;
  const typename P::TG *Ge = G + (active ? e : 0) * 6 * NP + ij;
  TC uk[N1];  // the operand (p in CG), in the contraction type
  TC g[6][kPrefetchG ? N1 : 1];
  if (active) {
    if (CG) {
      const TV beta = (TV)beta_d, alpha = (TV)alpha_d;
#pragma unroll
      for (int k = 0; k < N1; ++k) {
        const int64_t idx = base + k * PL;
        const TV pold = ld_once(u + idx);
        st_once(x + idx, ld_once(x + idx) + alpha * pold);
        const TV v = minv_at(minv, r, idx) * ld_once(r + idx) + beta * pold;
        uk[k] = (TC)v;
        st_once(u + idx, v);
      }
    } else {
#pragma unroll
      for (int k = 0; k < N1; ++k) uk[k] = (TC)ld_once(u + base + k * PL);
    }
    if constexpr (kPrefetchG) {
#pragma unroll
      for (int q = 0; q < 6; ++q)
#pragma unroll
        for (int k = 0; k < N1; ++k) g[q][k] = load_g<P>(Ge + q * NP + k * PL);
    }
  } else {
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      uk[k] = (TC)0;
      if constexpr (kPrefetchG) {
#pragma unroll
        for (int q = 0; q < 6; ++q) g[q][k] = (TC)0;
      }
    }
  }

  TC uc[N1];  // contraction input (rounded to bfloat16 in that mode)
#pragma unroll
  for (int k = 0; k < N1; ++k) uc[k] = contraction_input<P>(uk[k]);

  // Large orders write the weighted gradient's r and s parts straight to two
  // more LDS tiles as they are formed, so they need not stay in registers
  // across the barrier; small orders reuse the operand tile.
  constexpr bool kWideCol = N1 > 8;
  const int slot = el < EPB ? el : 0;  // idle threads alias slot 0 but never write
  TC *S1 = s1 + slot * T::TILE;
  TC *S2 = s2 + slot * T::TILE;
  TC *S3 = kWideCol ? s3 + slot * T::TILE : nullptr;
  if (el < EPB) {
#pragma unroll
    for (int k = 0; k < N1; ++k) S1[k * T::PLANE + j * T::P + i] = uc[k];
  }
  __syncthreads();

  TC Da[N1], Db[N1];
#pragma unroll
  for (int l = 0; l < N1; ++l) {
    Da[l] = sD[i * N1 + l];
    Db[l] = sD[j * N1 + l];
  }
  TC wr[kWideCol ? 1 : N1], ws[kWideCol ? 1 : N1], wt[N1];
#pragma unroll
  for (int k = 0; k < N1; ++k) {
    TC ur = 0, us = 0, ut = 0;
#pragma unroll
    for (int l = 0; l < N1; ++l) {
      ur += Da[l] * S1[k * T::PLANE + j * T::P + l];
      us += Db[l] * S1[k * T::PLANE + l * T::P + i];
      ut += sD[k * N1 + l] * uc[l];
    }
    TC gk[6];
    if constexpr (kPrefetchG) {
#pragma unroll
      for (int q = 0; q < 6; ++q) gk[q] = g[q][k];
    } else {
#pragma unroll
      for (int q = 0; q < 6; ++q) gk[q] = active ? load_g<P>(Ge + q * NP + k * PL) : (TC)0;
    }
    const TC a = contraction_input<P>(gk[0] * ur + gk[1] * us + gk[2] * ut);
    const TC c = contraction_input<P>(gk[1] * ur + gk[3] * us + gk[4] * ut);
    wt[k] = contraction_input<P>(gk[2] * ur + gk[4] * us + gk[5] * ut);
    if constexpr (kWideCol) {
      if (el < EPB) {
        S2[k * T::PLANE + j * T::P + i] = a;
        S3[k * T::PLANE + j * T::P + i] = c;
      }
    } else {
      wr[k] = a;
      ws[k] = c;
    }
  }
  __syncthreads();
  TC *SR = S1, *SS = S2;
  if constexpr (kWideCol) {
    SR = S2;
    SS = S3;
  } else {
    if (el < EPB) {
#pragma unroll
      for (int k = 0; k < N1; ++k) {
        S1[k * T::PLANE + j * T::P + i] = wr[k];
        S2[k * T::PLANE + j * T::P + i] = ws[k];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int l = 0; l < N1; ++l) {
    Da[l] = sD[l * N1 + i];
    Db[l] = sD[l * N1 + j];
  }
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < N1; ++k) {
    TC v = 0;
#pragma unroll
    for (int l = 0; l < N1; ++l) {
      v += Da[l] * SR[k * T::PLANE + j * T::P + l];
      v += Db[l] * SS[k * T::PLANE + l * T::P + i];
      v += sD[l * N1 + k] * wt[l];
    }
    if (active) w[base + k * PL] = (TV)v;
    acc += (double)uk[k] * (double)v;
  }
  if (CG) {
    // per-element sum of p.(A_L p): fixed tree over the element's threads
    sred[tid] = acc;
    __syncthreads();
    constexpr int P2 = next_pow2(PL);
    const int lt = ij;
#pragma unroll
    for (int s = P2 / 2; s > 0; s >>= 1) {
      if (el < EPB && lt < s && lt + s < PL) sred[tid] += sred[tid + s];
      __syncthreads();
    }
    if (active && lt == 0) part_el[e] = sred[tid];
  }
  __syncthreads();  // LDS is free for the next tile
}

// The same operator with two threads per (i, j) column (orders N >= 8):
// thread (i, j, h) owns nodes (i, j, k) for k in its half h of 0..N.  All
// three gradient contractions read the operand tile in LDS (the t one across
// the two halves); the weighted gradient goes to LDS as it is formed (r and s
// parts to s2 and s3, the t part to s1 once the operand is no longer read),
// and the transposed contractions read it back.  LDS as ax_tile with three
// tiles; sred: blockDim doubles.
template <int N1, int EPB, class P, bool CG, bool OPQ = false>
__device__ __forceinline__ void ax_tile_split(int64_t E, int64_t e0, const typename P::TC *__restrict__ Dg,
                                              const typename P::TG *__restrict__ G, typename P::TV *u,
                                              typename P::TV *__restrict__ w,
                                              const typename P::TV *__restrict__ r,
                                              const typename P::TV *__restrict__ minv,
                                              typename P::TV *__restrict__ x, double alpha_d,
                                              double beta_d, double *__restrict__ part_el,
                                              typename P::TC *sD, typename P::TC *s1,
                                              typename P::TC *s2, typename P::TC *s3, double *sred) {
  using T = AxTile<N1>;
  using TV = typename P::TV;
  using TC = typename P::TC;
  constexpr int NP = T::NP;
  constexpr int PL = N1 * N1;
  constexpr int KH = (N1 + 1) / 2;  // k values of the first half; the second has N1 - KH
  const int tid = OPQ ? opaque_tid() : (int)threadIdx.x;
  const int el = tid / T::TPE;
  const int rr = tid - el * T::TPE;
  const int h = rr / PL;
  const int ij = rr - h * PL;
  const int i = ij % N1;
  const int j = ij / N1;
  const int k0 = h * KH;
  const int nk = h ? N1 - KH : KH;
  const int64_t e = e0 + el;
  const bool mine = el < EPB;
  const bool active = mine && e < E;

  for (int t = tid; t < N1 * N1; t += blockDim.x) sD[t] = Dg[t];

  const int64_t base = e * NP + ij;
  const int slot = mine ? el : 0;  // idle threads alias slot 0 but never write
  TC *S1 = s1 + slot * T::TILE;
  TC *S2 = s2 + slot * T::TILE;
  TC *S3 = s3 + slot * T::TILE;
  // Loads are issued unconditionally (entry 0 for lanes without a node, the
  // value dropped) so that they are all in flight together; stores are
  // predicated.  kc clamps the shorter second half of an odd order.
  TC uk[KH];  // this half of the operand (p in CG)
  int64_t idx[KH];
  TV pv[KH], xv[KH], mv[KH], rv[KH];
#pragma unroll
  for (int kk = 0; kk < KH; ++kk) {
    const int kc = min(k0 + kk, N1 - 1);
    idx[kk] = (active && kk < nk) ? base + (int64_t)kc * PL : 0;
    pv[kk] = ld_once(u + idx[kk]);
    if (CG) {
      xv[kk] = ld_once(x + idx[kk]);
      mv[kk] = minv_at(minv, r, idx[kk]);
      rv[kk] = ld_once(r + idx[kk]);
    }
  }
#pragma unroll
  for (int kk = 0; kk < KH; ++kk) {
    const int kc = min(k0 + kk, N1 - 1);
    const bool ok = active && kk < nk;
    TV v = pv[kk];
    if (CG) {
      const TV xn = xv[kk] + (TV)alpha_d * pv[kk];
      v = mv[kk] * rv[kk] + (TV)beta_d * pv[kk];
      if (ok) {
        st_once(x + idx[kk], xn);
        st_once(u + idx[kk], v);
      }
    }
    uk[kk] = ok ? (TC)v : (TC)0;
    if (mine && kk < nk) S1[kc * T::PLANE + j * T::P + i] = contraction_input<P>(uk[kk]);
  }
  __syncthreads();

  const typename P::TG *Ge = G + (active ? e : 0) * 6 * NP + ij;
  TC Da[N1], Db[N1];
#pragma unroll
  for (int l = 0; l < N1; ++l) {
    Da[l] = sD[i * N1 + l];
    Db[l] = sD[j * N1 + l];
  }
  TC wt[KH];
#pragma unroll
  for (int kk = 0; kk < KH; ++kk) {
    const int k = min(k0 + kk, N1 - 1);
    TC gk[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const TC gv = load_g<P>(Ge + q * NP + k * PL);
      gk[q] = active ? gv : (TC)0;
    }
    TC ur = 0, us = 0, ut = 0;
#pragma unroll
    for (int l = 0; l < N1; ++l) {
      ur += Da[l] * S1[k * T::PLANE + j * T::P + l];
      us += Db[l] * S1[k * T::PLANE + l * T::P + i];
      ut += sD[k * N1 + l] * S1[l * T::PLANE + j * T::P + i];
    }
    const TC a = contraction_input<P>(gk[0] * ur + gk[1] * us + gk[2] * ut);
    const TC c = contraction_input<P>(gk[1] * ur + gk[3] * us + gk[4] * ut);
    wt[kk] = contraction_input<P>(gk[2] * ur + gk[4] * us + gk[5] * ut);
    if (mine && kk < nk) {
      S2[k * T::PLANE + j * T::P + i] = a;
      S3[k * T::PLANE + j * T::P + i] = c;
    }
  }
  __syncthreads();  // the operand tile is read for the last time above
  if (mine) {
#pragma unroll
    for (int kk = 0; kk < KH; ++kk)
      if (kk < nk) S1[(k0 + kk) * T::PLANE + j * T::P + i] = wt[kk];
  }
  __syncthreads();
#pragma unroll
  for (int l = 0; l < N1; ++l) {
    Da[l] = sD[l * N1 + i];
    Db[l] = sD[l * N1 + j];
  }
  double acc = 0.0;
#pragma unroll
  for (int kk = 0; kk < KH; ++kk) {
    const int k = min(k0 + kk, N1 - 1);
    TC v = 0;
#pragma unroll
    for (int l = 0; l < N1; ++l) {
      v += Da[l] * S2[k * T::PLANE + j * T::P + l];
      v += Db[l] * S3[k * T::PLANE + l * T::P + i];
      v += sD[l * N1 + k] * S1[l * T::PLANE + j * T::P + i];
    }
    if (kk < nk) {
      if (active) w[base + (int64_t)k * PL] = (TV)v;
      acc += (double)uk[kk] * (double)v;
    }
  }
  if (CG) {
    // per-element sum of p.(A_L p): fixed tree over the element's threads
    sred[tid] = acc;
    __syncthreads();
    constexpr int P2 = next_pow2(T::TPE);
#pragma unroll
    for (int st = P2 / 2; st > 0; st >>= 1) {
      if (mine && rr < st && rr + st < T::TPE) sred[tid] += sred[tid + st];
      __syncthreads();
    }
    if (active && rr == 0) part_el[e] = sred[tid];
  }
  __syncthreads();  // LDS is free for the next tile
}

// The element operator on a tile of EPB elements: AxTile<N1>::TPE threads per
// element (the first EPB * TPE threads of the work-group; any others only
// join the barriers).  Same contract for both layouts.  OPQ: the caller loops
// over tiles in a persistent kernel (see opaque_tid).
template <int N1, int EPB, class P, bool CG, bool OPQ = false>
__device__ __forceinline__ void ax_tile(int64_t E, int64_t e0, const typename P::TC *__restrict__ Dg,
                                        const typename P::TG *__restrict__ G, typename P::TV *u,
                                        typename P::TV *__restrict__ w,
                                        const typename P::TV *__restrict__ r,
                                        const typename P::TV *__restrict__ minv,
                                        typename P::TV *__restrict__ x, double alpha_d, double beta_d,
                                        double *__restrict__ part_el, typename P::TC *sD,
                                        typename P::TC *s1, typename P::TC *s2,
                                        typename P::TC *s3, double *sred) {
  if constexpr (AxTile<N1>::kSplit)
    ax_tile_split<N1, EPB, P, CG, OPQ>(E, e0, Dg, G, u, w, r, minv, x, alpha_d, beta_d, part_el, sD, s1,
                                  s2, s3, sred);
  else
    ax_tile_col<N1, EPB, P, CG, OPQ>(E, e0, Dg, G, u, w, r, minv, x, alpha_d, beta_d, part_el, sD, s1,
                                s2, s3, sred);
}

}  // namespace semk
