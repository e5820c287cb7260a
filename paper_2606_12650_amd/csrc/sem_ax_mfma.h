// The low-precision element operator with its D contractions on the matrix
// cores (gfx950 MFMA, FP32 accumulation): the same tile contract as ax_tile
// (sem_ax_tile.h) for PrecF32 and PrecBF16.
//
// Each directional contraction of an element is a GEMM
//     C[m][n] = sum_c A[m][c] B[c][n]
// with A = D (gradient) or D^T (transposed contraction), c the contracted
// 1-D index, m the output 1-D index (N+1 of the 16 MFMA rows) and n a pair of
// the two other indices (N1*N1 pairs, 16 per MFMA column tile).  FP32 uses
// v_mfma_f32_16x16x4f32 over ceil(N1/4) steps of K, BF16 one
// v_mfma_f32_16x16x32_bf16 (K padded with zeros).  Operand B and the results
// go through LDS; the metric product between the two contractions and the
// final sum of the three directions run one thread per (i, j) column as in
// ax_tile.  Work-groups must be whole waves (MFMA runs on all 64 lanes).
//
// Lane layouts of the two instructions (lane l of the wave):
//   A[m][c]: m = l % 16, c = 4 s + l / 16 (f32, step s) or 8 (l / 16) + q (bf16)
//   B[c][n]: c as for A, n = l % 16
//   C[m][n] in result register v: m = 4 (l / 16) + v, n = l % 16
#pragma once

#include <hip/hip_runtime.h>

#include "sem_ax_tile.h"
#include "sem_device.h"
#include "sem_internal.h"

namespace semk {

typedef float mfma_v4f __attribute__((ext_vector_type(4)));
typedef __bf16 mfma_v8bf __attribute__((ext_vector_type(8)));

template <int N1>
struct MfmaTile {
  static_assert(N1 <= 16, "one MFMA row block per 1-D index");
  static constexpr int PAIRS = N1 * N1;
  static constexpr int NT = (PAIRS + 15) / 16;  // column tiles per contraction
  static constexpr int KS = (N1 + 3) / 4;       // f32 K steps
  static constexpr int kTiles = 6;              // LDS tiles per element
};

// LDS offset of the point with contracted/output index c and pair index q in
// direction d (0: r contracts i, 1: s contracts j, 2: t contracts k).
template <int N1>
__device__ __forceinline__ int mfma_point(int d, int c, int q) {
  using T = AxTile<N1>;
  const int a = q % N1, b = q / N1;
  int i, j, k;
  if (d == 0) { i = c; j = a; k = b; }
  else if (d == 1) { j = c; i = a; k = b; }
  else { k = c; i = a; j = b; }
  return k * T::PLANE + j * T::P + i;
}

// One column tile of one directional contraction of one element:
// out(point) = sum_c Dm[m][c] in(point(c, q)) for the tile's 16 pairs.
// transpose = false: Dm = D (gradient); true: Dm = D^T.
template <int N1, class P>
__device__ __forceinline__ void mfma_contract(const typename P::TC *sD, const float *in, float *out,
                                              int d, int tile, bool transpose) {
  using M = MfmaTile<N1>;
  const int l = threadIdx.x & 63;
  const int n = l & 15;
  const int q = tile * 16 + n;  // pair index of this lane's column
  const bool qok = q < M::PAIRS;
  mfma_v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
  const int m = l & 15;
  if constexpr (P::kBf16) {
    mfma_v8bf a, b;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int c = 8 * (l >> 4) + s;
      const bool cok = c < N1;
      const float av = (m < N1 && cok) ? (float)(transpose ? sD[c * N1 + m] : sD[m * N1 + c]) : 0.0f;
      const float bv = (qok && cok) ? in[mfma_point<N1>(d, c, q)] : 0.0f;
      a[s] = (__bf16)av;  // exact: D and the operand are bfloat16 values already
      b[s] = (__bf16)bv;
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
  } else {
#pragma unroll
    for (int s = 0; s < M::KS; ++s) {
      const int c = 4 * s + (l >> 4);
      const bool cok = c < N1;
      const float av = (m < N1 && cok) ? (float)(transpose ? sD[c * N1 + m] : sD[m * N1 + c]) : 0.0f;
      const float bv = (qok && cok) ? in[mfma_point<N1>(d, c, q)] : 0.0f;
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int mo = 4 * (l >> 4) + v;
    if (mo < N1 && qok) out[mfma_point<N1>(d, mo, q)] = acc[v];
  }
}

// Same contract as ax_tile<N1, EPB, P, CG> (P = PrecF32 or PrecBF16) with
// blockDim a multiple of 64.  LDS: sD N1*N1 TC, tiles 6 * EPB * TILE floats,
// sred blockDim doubles.
template <int N1, int EPB, class P, bool CG>
__device__ __forceinline__ void ax_tile_mfma(int64_t E, int64_t e0, const typename P::TC *__restrict__ Dg,
                                             const typename P::TG *__restrict__ G, float *u,
                                             float *__restrict__ w, const float *__restrict__ r,
                                             const float *__restrict__ minv, float *__restrict__ x,
                                             double alpha_d, double beta_d,
                                             double *__restrict__ part_el, float *sD, float *tiles,
                                             double *sred) {
  static_assert(sizeof(typename P::TC) == 4, "MFMA operator is for the FP32 / BF16 modes");
  using T = AxTile<N1>;
  using M = MfmaTile<N1>;
  constexpr int NP = T::NP;
  constexpr int PL = N1 * N1;
  const int tid = threadIdx.x;
  const int el = tid / PL;
  const int ij = tid - el * PL;
  const int i = ij % N1;
  const int j = ij / N1;
  const int64_t e = e0 + el;
  const bool active = el < EPB && e < E;
  const int slot = el < EPB ? el : 0;
  float *U = tiles + (slot * 6 + 0) * T::TILE;
  float *R = tiles + (slot * 6 + 1) * T::TILE;
  float *S = tiles + (slot * 6 + 2) * T::TILE;
  float *Tt = tiles + (slot * 6 + 3) * T::TILE;
  float *X1 = tiles + (slot * 6 + 4) * T::TILE;
  float *X2 = tiles + (slot * 6 + 5) * T::TILE;

  for (int t = tid; t < N1 * N1; t += blockDim.x) sD[t] = Dg[t];

  // prologue and operand, one thread per (i, j) column
  const int64_t base = e * NP + ij;
  float uk[N1];
  if (active) {
    if (CG) {
      const float beta = (float)beta_d, alpha = (float)alpha_d;
#pragma unroll
      for (int k = 0; k < N1; ++k) {
        const int64_t idx = base + k * PL;
        const float pold = ld_once(u + idx);
        st_once(x + idx, ld_once(x + idx) + alpha * pold);
        const float v = ld_once(minv + idx) * ld_once(r + idx) + beta * pold;
        uk[k] = v;
        st_once(u + idx, v);
      }
    } else {
#pragma unroll
      for (int k = 0; k < N1; ++k) uk[k] = ld_once(u + base + k * PL);
    }
  } else {
#pragma unroll
    for (int k = 0; k < N1; ++k) uk[k] = 0.0f;
  }
  if (el < EPB) {
#pragma unroll
    for (int k = 0; k < N1; ++k) U[k * T::PLANE + j * T::P + i] = contraction_input<P>(uk[k]);
  }
  __syncthreads();

  // gradient: 3 directions x NT column tiles per element, spread over waves
  const int nwaves = blockDim.x >> 6;
  const int wave = tid >> 6;
  constexpr int ITEMS = EPB * 3 * M::NT;
  for (int it = wave; it < ITEMS; it += nwaves) {
    const int es = it / (3 * M::NT);
    const int d = (it / M::NT) % 3;
    const int tile = it % M::NT;
    float *in = tiles + (es * 6 + 0) * T::TILE;
    float *out = tiles + (es * 6 + 1 + d) * T::TILE;
    mfma_contract<N1, P>((const typename P::TC *)sD, in, out, d, tile, false);
  }
  __syncthreads();

  // metric product at each node of the column (the weighted gradient is
  // rounded to bfloat16 in that mode, as it feeds the next contraction)
  const typename P::TG *Ge = G + (active ? e : 0) * 6 * NP + ij;
  if (el < EPB) {
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      const int o = k * T::PLANE + j * T::P + i;
      float gk[6];
#pragma unroll
      for (int qq = 0; qq < 6; ++qq) gk[qq] = active ? load_g<P>(Ge + qq * NP + k * PL) : 0.0f;
      const float ur = R[o], us = S[o], ut = Tt[o];
      R[o] = contraction_input<P>(gk[0] * ur + gk[1] * us + gk[2] * ut);
      S[o] = contraction_input<P>(gk[1] * ur + gk[3] * us + gk[4] * ut);
      Tt[o] = contraction_input<P>(gk[2] * ur + gk[4] * us + gk[5] * ut);
    }
  }
  __syncthreads();

  // transposed contractions: r -> U, s -> X1, t -> X2
  for (int it = wave; it < ITEMS; it += nwaves) {
    const int es = it / (3 * M::NT);
    const int d = (it / M::NT) % 3;
    const int tile = it % M::NT;
    float *in = tiles + (es * 6 + 1 + d) * T::TILE;
    float *out = tiles + (es * 6 + (d == 0 ? 0 : 3 + d)) * T::TILE;
    mfma_contract<N1, P>((const typename P::TC *)sD, in, out, d, tile, true);
  }
  __syncthreads();

  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < N1; ++k) {
    const int o = k * T::PLANE + j * T::P + i;
    const float v = (U[o] + X1[o]) + X2[o];
    if (active) w[base + k * PL] = v;
    acc += (double)uk[k] * (double)v;
  }
  if (CG) {
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
  __syncthreads();
}

}  // namespace semk
