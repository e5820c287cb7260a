// The element operator with its D contractions on the matrix cores (gfx950
// MFMA): the same tile contract as ax_tile (sem_ax_tile.h) for PrecF64
// (v_mfma_f64_16x16x4f64), PrecF32 (v_mfma_f32_16x16x4f32) and PrecBF16
// (v_mfma_f32_16x16x16bf16_1k, FP32 accumulation).
//
// Each directional contraction of an element is a GEMM
//     C[m][n] = sum_c A[m][c] B[c][n]
// with A = D (gradient) or D^T (divergence), c the contracted 1-D index, m the
// output 1-D index (N+1 of the 16 MFMA rows) and n a pair of the two other
// indices: N+1 squared pairs in column tiles of 16.  An element has
// ceil((N+1)^2 / 16) waves; wave w of an element takes column tile w of all
// three directions.  The element's waves are its column tiles rounded up to
// a multiple of four, or 16 (mfma_waves); the waves beyond the last tile take
// no part in the matrix-core phases but share the element's loads and stores.
//
// HBM loads and stores run in a flat layout (64 consecutive nodes per wave
// and instruction); the MFMA results go through three LDS tiles.  Per
// element:
//   prologue: load the operand (CG: update x and p first) and G into
//             registers, operand to LDS tile U
//   gradient: r and s results to R and S; the t result to U once every wave
//             has read the operand
//   metric:   at the flat-layout nodes (G from registers), the weighted
//             gradient back to R, S and U
//   divergence: r, s and t in place in R, S and U (a wave reads and writes
//             only its own column tile's pairs)
//   result:   w = (R + S) + U at the flat-layout nodes, stored to HBM.
//
// Lane layouts of the three instructions (lane l, g = l / 16):
//   f64/f32 16x16x4 step s: A[m = l % 16][c = 4 s + g], B[c = 4 s + g][n = l % 16]
//   bf16 16x16x16:          A[m = l % 16][c = 4 g + q], B[c = 4 g + q][n = l % 16]
//   result register v:      f64: m = 4 v + g;  f32 and bf16: m = 4 g + v;  n = l % 16
#pragma once

#include <hip/hip_runtime.h>

#include "sem_ax_tile.h"
#include "sem_device.h"
#include "sem_types.h"

namespace semk {

typedef double mfma_v4d __attribute__((ext_vector_type(4)));
typedef float mfma_v4f __attribute__((ext_vector_type(4)));
typedef short mfma_v4s __attribute__((ext_vector_type(4)));

// Waves per element: the column tiles, rounded up to a multiple of four
// above two, and 16 above eight.  A work-group's waves are spread over a CU's
// four SIMDs; with nine waves (N = 11) one SIMD held three of each group, so
// at seven waves per SIMD only two groups fit (measured: 14 of 27 possible
// waves resident per CU).  With a multiple of four every SIMD holds the same
// share; 16 waves at N = 11 also leave two nodes per thread instead of three
// in the flat layout.  Measured at N = 11 (32^3 box): FP32 / BF16 CG operator
// 529 / 482 -> 475 / 419 us, A.u 364 / 334 -> 336 / 296 us; FP64 unchanged.
__host__ __device__ constexpr int mfma_waves(int n1) {
  return ((n1 * n1 + 15) / 16) <= 2 ? (n1 * n1 + 15) / 16
         : ((n1 * n1 + 15) / 16) > 8 ? 16
                                      : ((n1 * n1 + 15) / 16 + 3) / 4 * 4;
}

template <int N1>
struct MfmaTile {
  static_assert(N1 <= 16, "one MFMA row block per 1-D index");
  static constexpr int PL = N1 * N1;
  static constexpr int NT = (PL + 15) / 16;  // column tiles
  static constexpr int W = mfma_waves(N1);   // waves per element (>= NT)
  static constexpr int KS = (N1 + 3) / 4;    // 16x16x4 steps
  static constexpr int kTiles = 3;           // LDS tiles per element: U, R, S
};

// Work-group of the matrix-core operator: EPB elements of W waves each
// (at least eight waves per work-group).
template <int N1>
struct MfmaCfg {
  static constexpr int W = MfmaTile<N1>::W;
  static constexpr int EPB = W >= 8 ? 1 : 8 / W;
  static constexpr int THREADS = 64 * W * EPB;
};

template <class P>
struct MfmaOps {
  using Acc = mfma_v4f;
  static constexpr bool kF64 = false;
};
template <>
struct MfmaOps<PrecF64> {
  using Acc = mfma_v4d;
  static constexpr bool kF64 = true;
};

// Where the FP64 tile loads G (ax_tile_mfma): with the operand, or from N = 8
// after the gradient, which keeps the kernel's registers down.  The A.u alone
// (no CG prologue) at N = 11 loads G with the operand and is held to eight
// waves per SIMD (64 VGPRs, two 16-wave work-groups per CU; the compiler
// spills three values): measured on MI355X, 32^3 box, 694 -> 649 us.  At
// N = 8, 9, 10 and 12 the same change measured 6 % faster to 80 % slower
// (296 -> 314, 388 -> 384, 525 -> 709, 644 -> 1159 us: spills), so those
// orders keep the late loads.
template <int N1, class P, bool CG>
constexpr bool mfma_late_g() {
  return MfmaOps<P>::kF64 && N1 >= 9 && (CG || N1 != 12);
}
template <int N1, class P, bool CG>
constexpr int mfma_waves_per_simd() {
  return (MfmaOps<P>::kF64 && N1 == 12 && !CG) ? 8 : 1;
}

// Result row of register v in lane group g.
template <class P>
__device__ __forceinline__ int mfma_row(int g, int v) {
  return MfmaOps<P>::kF64 ? 4 * v + g : 4 * g + v;
}

// LDS offset of the node with contracted/result index c and pair index q in
// direction d (0: r, c = i; 1: s, c = j; 2: t, c = k).
template <int N1>
__device__ __forceinline__ int mfma_point(int d, int c, int q) {
  using T = AxTile<N1>;
  const int a = q % N1, b = q / N1;
  const int i = d == 0 ? c : a;
  const int j = d == 1 ? c : (d == 0 ? a : b);
  const int k = d == 2 ? c : b;
  return k * T::PLANE + j * T::P + i;
}

__device__ __forceinline__ short mfma_bf16_bits(float v) {
  return (short)(__float_as_uint(v) >> 16);  // exact: v is a bfloat16 value
}

// The A operand of one lane: D (transpose = false) or D^T, zero-padded.
template <int N1, class P>
struct MfmaA {
  using TC = typename P::TC;
  TC a[P::kBf16 ? 1 : MfmaTile<N1>::KS];
  mfma_v4s ab;
  __device__ __forceinline__ void load(const TC *sD, bool transpose, int l) {
    const int m = l & 15, g = l >> 4;
    if constexpr (P::kBf16) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = 4 * g + q;
        const float v = (m < N1 && c < N1) ? (transpose ? sD[c * N1 + m] : sD[m * N1 + c]) : 0.0f;
        ab[q] = mfma_bf16_bits(v);
      }
    } else {
#pragma unroll
      for (int s = 0; s < MfmaTile<N1>::KS; ++s) {
        const int c = 4 * s + g;
        a[s] = (m < N1 && c < N1) ? (transpose ? sD[c * N1 + m] : sD[m * N1 + c]) : (TC)0;
      }
    }
  }
};

// Column tile `tile` of direction d: the four result rows of this lane for
// pair q = 16 tile + l % 16, from the LDS tile `in`.
template <int N1, class P>
__device__ __forceinline__ typename MfmaOps<P>::Acc mfma_contract(const MfmaA<N1, P> &A,
                                                                 const typename P::TC *in, int d,
                                                                 int tile, int l) {
  using M = MfmaTile<N1>;
  using TC = typename P::TC;
  const int g = l >> 4;
  const int q = tile * 16 + (l & 15);
  const bool qok = q < M::PL;
  typename MfmaOps<P>::Acc acc = {0, 0, 0, 0};
  if constexpr (P::kBf16) {
    mfma_v4s b;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = 4 * g + u;
      const bool ok = qok && c < N1;
      const float v = in[ok ? mfma_point<N1>(d, c, q) : 0];
      b[u] = mfma_bf16_bits(ok ? v : 0.0f);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A.ab, b, acc, 0, 0, 0);
  } else {
    TC b[M::KS];
#pragma unroll
    for (int s = 0; s < M::KS; ++s) {
      const int c = 4 * s + g;
      const bool ok = qok && c < N1;
      const TC v = in[ok ? mfma_point<N1>(d, c, q) : 0];
      b[s] = ok ? v : (TC)0;
    }
#pragma unroll
    for (int s = 0; s < M::KS; ++s) {
      if constexpr (MfmaOps<P>::kF64)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A.a[s], b[s], acc, 0, 0, 0);
      else
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A.a[s], b[s], acc, 0, 0, 0);
    }
  }
  return acc;
}

// Store the lane's result rows of a column tile to `out` (rows < N1 only).
template <int N1, class P>
__device__ __forceinline__ void mfma_store(typename P::TC *out, const typename MfmaOps<P>::Acc &acc,
                                           int d, int tile, int l) {
  const int g = l >> 4;
  const int q = tile * 16 + (l & 15);
  if (q >= MfmaTile<N1>::PL) return;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int m = mfma_row<P>(g, v);
    if (m < N1) out[mfma_point<N1>(d, m, q)] = (typename P::TC)acc[v];
  }
}

// Same contract as ax_tile<N1, EPB, P, CG, OPQ> with blockDim = MfmaCfg<N1>::THREADS
// (EPB = MfmaCfg<N1>::EPB).  LDS: sD N1*N1 TC, s1/s2/s3 EPB * AxTile<N1>::TILE
// TC each, sred blockDim / 64 doubles.  SW (without CG): w is written with
// non-temporal stores.
//
// HBM traffic runs in the flat layout: the element's 64 NT threads take its
// nodes in index order (thread t: nodes t, t + 64 NT, ...), so every load and
// store is a run of 64 consecutive values.  The t-direction results pass
// through LDS to meet that layout.
template <int N1, int EPB, class P, bool CG, bool OPQ = false, bool SW = false>
__device__ __forceinline__ void ax_tile_mfma(int64_t E, int64_t e0, const typename P::TC *__restrict__ Dg,
                                             const typename P::TG *__restrict__ G, typename P::TV *u,
                                             typename P::TV *__restrict__ w,
                                             const typename P::TV *__restrict__ r,
                                             const typename P::TV *__restrict__ minv,
                                             typename P::TV *__restrict__ x, double alpha_d,
                                             double beta_d, double *__restrict__ part_el,
                                             typename P::TC *sD, typename P::TC *s1,
                                             typename P::TC *s2, typename P::TC *s3,
                                             double *sred) {
  using T = AxTile<N1>;
  using M = MfmaTile<N1>;
  using TV = typename P::TV;
  using TC = typename P::TC;
  using Acc = typename MfmaOps<P>::Acc;
  constexpr int NP = T::NP;
  constexpr int PL = M::PL;
  constexpr int NTT = 64 * M::W;               // threads per element
  constexpr int PPT = (NP + NTT - 1) / NTT;    // nodes per thread in the flat layout
  const int tid = OPQ ? opaque_tid() : (int)threadIdx.x;
  const int wave = tid >> 6;
  const int el = wave / M::W;
  const int tile = wave - el * M::W;  // this wave's column tile in every direction
  const bool tiled = tile < M::NT;    // (the waves beyond the last tile have none)
  const int l = tid & 63;
  const int lt = tid - el * NTT;       // thread index within the element
  const int64_t e = e0 + el;
  const bool mine = el < EPB;
  const bool active = mine && e < E;
  const int slot = mine ? el : 0;
  TC *U = s1 + slot * T::TILE;
  TC *R = s2 + slot * T::TILE;
  TC *S = s3 + slot * T::TILE;

  for (int t = tid; t < N1 * N1; t += blockDim.x) sD[t] = Dg[t];

  // prologue in the flat layout.  Every load is issued unconditionally (lanes
  // without a node read entry 0 and drop the value) so that all are in flight
  // together; only the stores are predicated.
  int off[PPT];
  bool okv[PPT];
  int64_t idx[PPT];
#pragma unroll
  for (int m = 0; m < PPT; ++m) {
    const int pt = lt + NTT * m;
    okv[m] = active && pt < NP;
    idx[m] = okv[m] ? e * NP + pt : 0;
    const int pc = pt < NP ? pt : 0;
    off[m] = (pc / PL) * T::PLANE + ((pc % PL) / N1) * T::P + pc % N1;
  }
  TV pv[PPT], xv[PPT], mv[PPT], rv[PPT];
#pragma unroll
  for (int m = 0; m < PPT; ++m) {
    pv[m] = ld_once(u + idx[m]);
    if (CG) {
      xv[m] = ld_once(x + idx[m]);
      mv[m] = minv_at(minv, r, idx[m]);
      rv[m] = ld_once(r + idx[m]);
    }
  }
  // G with the prologue's loads, or in FP64 from N = 8 (LATE_G, mfma_late_g)
  // after the gradient, so that the gradient's MFMA accumulators and G are
  // never live together: the N = 11 CG operator then holds 70 instead of 98
  // VGPRs (measured on MI355X: CG iteration 466 -> 408 us; at N = 7 and for
  // FP32 / BF16 the early loads were faster).
  constexpr bool LATE_G = mfma_late_g<N1, P, CG>();
  TC gk[PPT][6];
  auto load_gk = [&]() {
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
      const int64_t gi = okv[m] ? e * 6 * NP + (idx[m] - e * NP) : 0;
#pragma unroll
      for (int c = 0; c < 6; ++c) gk[m][c] = load_g<P>(G + gi + (okv[m] ? (int64_t)c * NP : 0));
    }
  };
  if constexpr (!LATE_G) load_gk();
  TC uk[PPT];
#pragma unroll
  for (int m = 0; m < PPT; ++m) {
    TV val = pv[m];
    if (CG) {
      const TV xn = xv[m] + (TV)alpha_d * pv[m];
      val = mv[m] * rv[m] + (TV)beta_d * pv[m];
      if (okv[m]) {
        st_once(x + idx[m], xn);
        st_once(u + idx[m], val);
      }
    }
    uk[m] = okv[m] ? (TC)val : (TC)0;
    if (mine && lt + NTT * m < NP) U[off[m]] = contraction_input<P>(uk[m]);
  }
  __syncthreads();

  // gradient: r and s to LDS, t kept until the operand tile is free
  MfmaA<N1, P> A;
  A.load(sD, false, l);
  Acc ut = {0, 0, 0, 0};
  if (mine && tiled) {
    const Acc ur = mfma_contract<N1, P>(A, U, 0, tile, l);
    const Acc us = mfma_contract<N1, P>(A, U, 1, tile, l);
    ut = mfma_contract<N1, P>(A, U, 2, tile, l);
    mfma_store<N1, P>(R, ur, 0, tile, l);
    mfma_store<N1, P>(S, us, 1, tile, l);
  }
  __syncthreads();  // every wave has read the operand tile
  if (mine && tiled) mfma_store<N1, P>(U, ut, 2, tile, l);
  if constexpr (LATE_G) load_gk();
  __syncthreads();

  // metric at the flat-layout nodes; the weighted gradient is the next
  // contraction's input
  if (mine) {
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
      if (lt + NTT * m < NP) {
        const int o = off[m];
        const TC ur = R[o], us = S[o], utv = U[o];
        R[o] = contraction_input<P>(gk[m][0] * ur + gk[m][1] * us + gk[m][2] * utv);
        S[o] = contraction_input<P>(gk[m][1] * ur + gk[m][3] * us + gk[m][4] * utv);
        U[o] = contraction_input<P>(gk[m][2] * ur + gk[m][4] * us + gk[m][5] * utv);
      }
    }
  }
  __syncthreads();

  // divergence, in place: each wave reads and writes only its own column
  // tile's pairs in R (r), S (s) and U (t)
  A.load(sD, true, l);
  if (mine && tiled) {
    const Acc vr = mfma_contract<N1, P>(A, R, 0, tile, l);
    const Acc vs = mfma_contract<N1, P>(A, S, 1, tile, l);
    const Acc vt = mfma_contract<N1, P>(A, U, 2, tile, l);
    mfma_store<N1, P>(R, vr, 0, tile, l);
    mfma_store<N1, P>(S, vs, 1, tile, l);
    mfma_store<N1, P>(U, vt, 2, tile, l);
  }
  __syncthreads();

  double acc = 0.0;
  if (mine) {
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
      if (lt + NTT * m < NP) {
        const int o = off[m];
        const TC val = (R[o] + S[o]) + U[o];
        if (okv[m]) {
          // a result the caller takes as it is (SEM_AX_LOCAL) is streamed
          // past the caches; one a gather reads next is kept there
          if constexpr (!CG && SW)
            st_once(w + idx[m], (TV)val);
          else
            w[idx[m]] = (TV)val;
        }
        acc += (double)uk[m] * (double)val;
      }
    }
  }
  if (CG) {
    // per-element sum of p.(A_L p): wave sums, then the element's waves in order
    acc = wave_sum(acc);
    if (l == 0) sred[wave] = acc;
    __syncthreads();
    if (mine && tile == 0 && l == 0 && e < E) {
      double sum = 0.0;
      for (int t = 0; t < M::W; ++t) sum += sred[el * M::W + t];
      part_el[e] = sum;
    }
  }
  __syncthreads();  // LDS is free for the next tile
}

}  // namespace semk
