// Device pieces of the Jacobi-PCG (paper Sec. VIII-A) shared by the single-
// solve kernels and the batched persistent kernels: the same functions give
// the same bits on both paths.
//
// *_tile functions process one streaming tile (kVecTile consecutive entries
// of one element-local vector) with a work-group of kVecThreads and return
// the tile's block sums in thread 0; the CG update's tiles are element-aligned
// instead (UpdTile below).  *_step functions finish a reduction
// over a solve's partials with a work-group of kFinThreads and advance the
// solve's scalars (thread 0 writes).
#pragma once

#include <hip/hip_runtime.h>

#include "sem_device.h"
#include "sem_types.h"

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
      rz += c * rv * ((minv ? minv[idx] : 1.0) * rv);
      bb += c * rv * rv;
    }
  }
  TileSums t;
  block_sum2<kVecThreads>(rz, bb, sred, &t.a, &t.b);
  return t;
}

// CG update with the gather-scatter pulled in: r -= alpha mask o QQ^T w;
// sums ||r||_c^2 and <r, Minv r>_c (FP64 even for FP32 vectors).
//
// The tile is element-aligned (UpdTile): each thread owns KN planes of one
// (i, j) column of an element, so every load of w, r and Minv is a
// coalesced run of a plane, and the copies of a node that sit in other
// elements are reached in pairs along one direction at a time:
//   P = w(node) + w(y copy)                  pair across a y face,
//   A = P(this z level) + P(other z level)   pair across a z face,
//   S = A(this column) + A(x copy column)    pair across an x face.
// Each pair is one commutative addition of the same two numbers for every
// copy of the node (a missing copy leaves the other operand alone), so all
// copies get the same bits.  The A of the x copy column comes from LDS when
// that column is in the tile and is recomputed from w otherwise.  A missing
// copy is not loaded and adds an exact zero.
// The work-group has BLOCK threads; tid is threadIdx.x.  LINEAR tiles (FP64
// from order 9, FP32 from order 11) take kVecTile consecutive entries
// instead, each node summing its copies in ascending element-local order with
// missing copies masked.
// V selects one of the candidate shapes of upd_shape (0: the default).
template <int N1, typename TV, int V = 0>
struct UpdTile {
  static constexpr UpdShape SH = upd_shape(N1, sizeof(TV) == 8, V);
  static_assert(SH.ks >= 0, "update tile shape not among the candidates of this order");
  static constexpr bool LINEAR = SH.ks == 0;
  static constexpr int N = N1 - 1;
  static constexpr int COLS = N1 * N1;
  static constexpr int NP = COLS * N1;
  static constexpr int KS = LINEAR ? 1 : SH.ks;    // threads per column
  static constexpr int EPT = LINEAR ? 1 : SH.ept;  // elements per tile
  static constexpr int KP = LINEAR ? 1 : SH.kp;    // tiles per element (plane ranges)
  static constexpr int KT = (N1 + KP - 1) / KP;  // planes per tile
  static constexpr int KN = (KT + KS - 1) / KS;  // planes per thread
  static constexpr int THREADS = EPT * KS * COLS;
  static constexpr int BLOCK = LINEAR ? kVecThreads : 64 * ((THREADS + 63) / 64);
  // LDS: the A values of every plane slot of the tile (EPT > 1 only)
  static constexpr int LDS = (!LINEAR && EPT > 1) ? EPT * KS * KN * COLS : 1;
  static_assert(BLOCK <= 512, "update tile larger than its work-group");
  static_assert(8 * LDS <= 32 * 1024, "update tile LDS above 32 KiB");
};

// The w values a column's pair sums read: its planes kb .. kb + KN - 1 (own),
// their y copies and the z neighbours of planes 0 and N (with their y
// copies).  A copy the node does not have is not loaded and reads as zero
// (its lane's load is switched off, so it costs no memory request).
template <int KN, typename TV>
struct ColumnW {
  TV own[KN], yv[KN];
  TV zl, zyl, zh, zyh;
};

template <int N1, int KN, typename TV>
__device__ __forceinline__ void upd_column_load(const TV *__restrict__ w, int64_t col0, int kb,
                                                bool hy, int64_t yoff, bool z_lo, bool z_hi,
                                                int64_t dz, ColumnW<KN, TV> &c) {
  constexpr int N = N1 - 1, COLS = N1 * N1;
#pragma unroll
  for (int kk = 0; kk < KN; ++kk) {
    const int64_t a = col0 + (int64_t)min(kb + kk, N) * COLS;
    c.own[kk] = w[a];
    c.yv[kk] = hy ? w[a + yoff] : (TV)0;
  }
  const int64_t lo = col0 - dz + (int64_t)N * COLS, hi = col0 + dz;
  c.zl = z_lo ? w[lo] : (TV)0;
  c.zyl = z_lo && hy ? w[lo + yoff] : (TV)0;
  c.zh = z_hi ? w[hi] : (TV)0;
  c.zyh = z_hi && hy ? w[hi + yoff] : (TV)0;
}

// The A values (y and z pairs) of a loaded column, added in type AT.  A
// missing copy adds an exact zero.  Callers issue every load of the tile
// (upd_column_load) before the first call, so that all of them are in flight
// together: one HBM round trip per tile.
template <int N1, int KN, typename TV, typename AT = double>
__device__ __forceinline__ void upd_column_sum(const ColumnW<KN, TV> &c, int kb, AT (&A)[KN]) {
  constexpr int N = N1 - 1;
  const AT pl = (AT)c.zl + (AT)c.zyl;
  const AT ph = (AT)c.zh + (AT)c.zyh;
#pragma unroll
  for (int kk = 0; kk < KN; ++kk) {
    AT a = (AT)c.own[kk] + (AT)c.yv[kk];
    if (kb + kk == 0) a = a + pl;
    if (kb + kk == N) a = a + ph;
    A[kk] = a;
  }
}

// Linear tile: the items of a thread are taken kLinGroup at a time, all
// loads of a group (r, Minv and every present copy of w) before any sum, so
// a group costs one HBM round trip.
constexpr int kLinGroup = 4;

// Neighbour bits of element (ex, ey, ez): bit 0 / 1 a neighbour below /
// above in x, bits 2 / 3 in y, bits 4 / 5 in z.
__host__ __device__ __forceinline__ uint32_t elem_nb_bits(const Box &b, uint32_t ex, uint32_t ey,
                                                          uint32_t ez) {
  return (ex > 0 ? 1u : 0u) | (ex + 1 < (uint32_t)b.nx ? 2u : 0u) | (ey > 0 ? 4u : 0u) |
         (ey + 1 < (uint32_t)b.ny ? 8u : 0u) | (ez > 0 ? 16u : 0u) |
         (ez + 1 < (uint32_t)b.nz ? 32u : 0u);
}

// Where the items of a thread of the linear tile sit.  The index arithmetic
// is 32-bit (L < 2^32) and done once per thread where it can be: a thread's
// items lie kVecThreads apart, so they span its first element and at most
// the two after it, whose neighbour bits are found up front.  A node's face
// bits (bit 0 / 1: i = 0 / N, 2 / 3: j, 4 / 5: k) against its element's
// neighbour bits give everything else: a face bit with no neighbour is the
// box boundary, one with a neighbour a shared copy (mult = 2^(shared
// faces)), and copy q of the node sits a fixed, uniform step (off[q]) from
// its lowest copy lo.
template <int N1>
struct LinItems {
  static constexpr int N = N1 - 1;
  static constexpr uint32_t NP = (uint32_t)N1 * N1 * N1;
  static constexpr uint32_t dx = NP - N;  // to the same face node of the next element in x
  static_assert(kVecThreads * (kVecItems - 1) < 2 * NP, "a thread's items span at most three elements");
  uint32_t L, raw0, loc0, dy, dz;
  uint32_t nbs;  // neighbour bits of the first element and the two after it, 6 bits each
  struct Item {
    uint32_t raw;  // the item's index (may lie past L)
    uint32_t idx;  // raw, clamped into [0, L)
    uint32_t sh;   // faces shared with a neighbour (0 past L)
    uint32_t lo;   // the lowest copy of the node
    bool live;     // raw < L
    bool upd;      // live and not on the box boundary
  };
  __host__ __device__ LinItems(const Box &b, int64_t tile, int tid) {
    L = (uint32_t)b.L();
    dy = (uint32_t)b.nx * NP - (uint32_t)(N * N1);
    dz = (uint32_t)b.nx * (uint32_t)b.ny * NP - (uint32_t)(N * N1 * N1);
    raw0 = (uint32_t)(tile * kVecTile) + (uint32_t)tid;
    const uint32_t e0 = raw0 / NP;
    loc0 = raw0 - e0 * NP;
    const uint32_t eyz = b.fdx.div(e0);
    uint32_t ex = e0 - eyz * (uint32_t)b.nx;
    const uint32_t ezz = b.fdy.div(eyz);
    uint32_t ey = eyz - ezz * (uint32_t)b.ny, ez = ezz;
    nbs = elem_nb_bits(b, ex, ey, ez);
    next_element(b, ex, ey, ez);
    nbs |= elem_nb_bits(b, ex, ey, ez) << 6;
    next_element(b, ex, ey, ez);
    nbs |= elem_nb_bits(b, ex, ey, ez) << 12;
  }
  __host__ __device__ static void next_element(const Box &b, uint32_t &ex, uint32_t &ey, uint32_t &ez) {
    const bool wx = ex + 1 == (uint32_t)b.nx;
    ex = wx ? 0u : ex + 1;
    const bool wy = wx && ey + 1 == (uint32_t)b.ny;
    ey = wy ? 0u : ey + (wx ? 1u : 0u);
    ez += wy ? 1u : 0u;
  }
  __host__ __device__ uint32_t off(int q) const {
    return ((q & 1) ? dx : 0u) + ((q & 2) ? dy : 0u) + ((q & 4) ? dz : 0u);
  }
  __host__ __device__ Item item(int u) const {
    Item t;
    t.raw = raw0 + (uint32_t)(u * kVecThreads);
    t.live = t.raw < L;
    t.idx = t.live ? t.raw : L - 1;
    uint32_t loc = loc0 + (uint32_t)(u * kVecThreads);
    const uint32_t steps = (loc >= NP ? 1u : 0u) + (loc >= 2 * NP ? 1u : 0u);
    loc -= steps * NP;
    const uint32_t enb = (nbs >> (6u * steps)) & 63u;
    const uint32_t i = loc % N1, j = (loc / N1) % N1, k = loc / (N1 * N1);
    const uint32_t fb = (i == 0 ? 1u : 0u) | (i == (uint32_t)N ? 2u : 0u) | (j == 0 ? 4u : 0u) |
                        (j == (uint32_t)N ? 8u : 0u) | (k == 0 ? 16u : 0u) |
                        (k == (uint32_t)N ? 32u : 0u);
    t.sh = t.live ? (fb & enb) : 0u;
    t.upd = t.live && (fb & ~enb) == 0u;
    t.lo = t.idx - ((t.sh & 1u) ? dx : 0u) - ((t.sh & 4u) ? dy : 0u) - ((t.sh & 16u) ? dz : 0u);
    return t;
  }
  // copy q of the node exists
  __host__ __device__ static bool has_copy(uint32_t sh, int q) {
    return (!(q & 1) || (sh & 3u)) && (!(q & 2) || (sh & 12u)) && (!(q & 4) || (sh & 48u));
  }
};

template <int N1, typename TV>
__device__ inline TileSums cg_update_tile_linear(const Box &b, int64_t tile, TV *__restrict__ r,
                                                 const TV *__restrict__ w,
                                                 const TV *__restrict__ minv, double alpha,
                                                 double *sred, int tid) {
  static_assert(kVecItems % kLinGroup == 0, "linear update groups must tile the items");
  const LinItems<N1> P(b, tile, tid);
  const TV alpha_v = (TV)alpha;
  double rr = 0.0, rz = 0.0;
  // the new r of every item is stored at the end: a store issued between
  // two groups held the next group's loads back until it had completed
  TV rnew[kVecItems];
  bool upd[kVecItems];
#pragma unroll
  for (int g = 0; g < kVecItems; g += kLinGroup) {
    TV rv[kLinGroup], mv[kLinGroup], v[kLinGroup][8];
    double c[kLinGroup];
#pragma unroll
    for (int u = 0; u < kLinGroup; ++u) {
      const typename LinItems<N1>::Item t = P.item(g + u);
      upd[g + u] = t.upd;
      // 1 / mult: the exponent of 2^-(shared faces) set directly
      c[u] = __hiloint2double((int)((1023u - (uint32_t)__builtin_popcount(t.sh)) << 20), 0);
      rv[u] = ld_once(r + t.idx);
      mv[u] = minv_at(minv, r, (int64_t)t.idx);
#pragma unroll
      for (int q = 0; q < 8; ++q)
        v[u][q] = LinItems<N1>::has_copy(t.sh, q) ? w[t.lo + P.off(q)] : (TV)0;
    }
#pragma unroll
    for (int u = 0; u < kLinGroup; ++u) {
      // the copies in ascending element-local order (a missing one adds +0),
      // and r, in the vector type; the reductions in FP64
      TV wa = (TV)0;
#pragma unroll
      for (int q = 0; q < 8; ++q) wa += v[u][q];
      const TV rt = rv[u] - alpha_v * wa;
      rnew[g + u] = rt;
      if (upd[g + u]) {
        const double rd = (double)rt;
        rr += c[u] * rd * rd;
        rz += c[u] * rd * ((double)mv[u] * rd);
      }
    }
    // the next group's loads stay after this group's sums (all groups'
    // loads at once would need registers for every copy of every item):
    // an empty asm that takes the sums and orders memory accesses
#pragma unroll
    for (int u = 0; u < kLinGroup; ++u) asm volatile("" : "+v"(rnew[g + u]) : : "memory");
    asm volatile("" : "+v"(rr), "+v"(rz) : : "memory");
  }
#pragma unroll
  for (int u = 0; u < kVecItems; ++u)
    if (upd[u]) r[P.raw0 + (uint32_t)(u * kVecThreads)] = rnew[u];
  TileSums t;
  block_sum2<kVecThreads>(rr, rz, sred, &t.a, &t.b);
  return t;
}

// Where a thread of an element-column tile sits: its element, its (i, j)
// column, its planes kb .. kb + KN - 1 (those below kend are its own: the
// last thread of a plane range can reach past it when KS does not divide the
// range) and the copies its nodes have.
template <int N1, typename TV, int V = 0>
struct ColumnPos {
  using U = UpdTile<N1, TV, V>;
  static constexpr int N = U::N, COLS = U::COLS, NP = U::NP, KN = U::KN;
  bool live, hy, z_lo, z_hi, hx, x_in;
  int el, ks, col, i, j, kb, kend, ex, ey, ez;
  int64_t yoff, dz, col0;
  __host__ __device__ ColumnPos(const Box &b, int64_t tile, int tid) {
    const bool act = tid < U::THREADS;
    const int t = act ? tid : 0;
    el = t / (U::KS * COLS);
    const int rem = t - el * (U::KS * COLS);
    ks = rem / COLS;
    col = rem - ks * COLS;
    i = col % N1;
    j = col / N1;
    const int64_t grp = tile / U::KP;
    const int part = (int)(tile - grp * U::KP);
    kb = part * U::KT + ks * KN;
    kend = (part + 1) * U::KT < N1 ? (part + 1) * U::KT : N1;
    const int64_t E = b.E();
    const int64_t e_raw = grp * U::EPT + el;
    live = act && e_raw < E;
    const uint32_t e = (uint32_t)(e_raw < E ? e_raw : E - 1);
    const uint32_t eyz = b.fdx.div(e);
    ex = (int)(e - eyz * (uint32_t)b.nx);
    const uint32_t ezz = b.fdy.div(eyz);
    ey = (int)(eyz - ezz * (uint32_t)b.ny);
    ez = (int)ezz;
    const int64_t dy = (int64_t)b.nx * NP;
    dz = dy * b.ny;
    hy = (j == 0 && ey > 0) || (j == N && ey < b.ny - 1);
    yoff = j == 0 ? (int64_t)N * N1 - dy : dy - (int64_t)N * N1;
    z_lo = kb == 0 && ez > 0;
    z_hi = kb <= N && kb + KN > N && ez < b.nz - 1;
    hx = (i == 0 && ex > 0) || (i == N && ex < b.nx - 1);
    x_in = U::EPT > 1 && hx && (i == 0 ? el > 0 : el < U::EPT - 1);
    col0 = (int64_t)e * NP + col;
  }
  // Plane k (of this thread) is a node on the box boundary.
  __host__ __device__ bool boundary(const Box &b, int k) const {
    return (i == 0 && ex == 0) || (i == N && ex == b.nx - 1) || (j == 0 && ey == 0) ||
           (j == N && ey == b.ny - 1) || (k == 0 && ez == 0) || (k == N && ez == b.nz - 1);
  }
  // 1 / multiplicity of the node at plane k.
  __host__ __device__ double inv_mult(const Box &b, int k) const {
    const bool hz = (k == 0 && ez > 0) || (k == N && ez < b.nz - 1);
    const int m = (hx ? 2 : 1) * (hy ? 2 : 1) * (hz ? 2 : 1);
    return m == 1 ? 1.0 : (m == 2 ? 0.5 : (m == 4 ? 0.25 : 0.125));
  }
};

// S = the sum of all copies of each of the thread's nodes, as the pair tree
// above, added in type AT (the pairs and their order are the same in any
// type, so every copy of a node gets the same bits).  With several elements
// per tile this holds a work-group barrier: every thread of the work-group
// calls it.
template <int N1, typename TV, int V = 0, typename AT = double>
__device__ inline void column_copy_sums(const ColumnPos<N1, TV, V> &p, const TV *__restrict__ w,
                                        double *sA, AT (&S)[UpdTile<N1, TV, V>::KN]) {
  using U = UpdTile<N1, TV, V>;
  constexpr int N = U::N, COLS = U::COLS, NP = U::NP, KN = U::KN;
  // every load first (own column, then the x copy column where it lies in
  // another tile), so that both are in flight together; the branch holds
  // loads only (zeros where the column has no x copy there)
  ColumnW<KN, TV> cw, cx;
  upd_column_load<N1, KN, TV>(w, p.col0, p.kb, p.hy, p.yoff, p.z_lo, p.z_hi, p.dz, cw);
  if (p.hx && !p.x_in) {
    const int64_t xc = p.i == 0 ? p.col0 - NP + N : p.col0 + NP - N;
    upd_column_load<N1, KN, TV>(w, xc, p.kb, p.hy, p.yoff, p.z_lo, p.z_hi, p.dz, cx);
  } else {
#pragma unroll
    for (int kk = 0; kk < KN; ++kk) cx.own[kk] = cx.yv[kk] = (TV)0;
    cx.zl = cx.zyl = cx.zh = cx.zyh = (TV)0;
  }
  AT A[KN], X[KN];
  upd_column_sum<N1, KN, TV, AT>(cw, p.kb, A);
  upd_column_sum<N1, KN, TV, AT>(cx, p.kb, X);
  if constexpr (U::EPT > 1) {
    // slot (element, thread's plane range, plane, column)
#pragma unroll
    for (int kk = 0; kk < KN; ++kk) sA[((p.el * U::KS + p.ks) * KN + kk) * COLS + p.col] = (double)A[kk];
    __syncthreads();
    if (p.x_in) {
      const int xo =
          ((p.i == 0 ? p.el - 1 : p.el + 1) * U::KS + p.ks) * KN * COLS + p.j * N1 + (N - p.i);
#pragma unroll
      for (int kk = 0; kk < KN; ++kk) X[kk] = (AT)sA[xo + kk * COLS];  // exact: an AT value
    }
  }
#pragma unroll
  for (int kk = 0; kk < KN; ++kk) S[kk] = p.hx ? A[kk] + X[kk] : A[kk];
}

template <int N1, typename TV, int V = 0>
__device__ inline TileSums cg_update_tile(const Box &b, int64_t tile, TV *__restrict__ r,
                                          const TV *__restrict__ w, const TV *__restrict__ minv,
                                          double alpha, double *sA, double *sred,
                                          int tid) {
  using U = UpdTile<N1, TV, V>;
  if constexpr (U::LINEAR)
    return cg_update_tile_linear<N1, TV>(b, tile, r, w, minv, alpha, sred, tid);
  constexpr int N = U::N, COLS = U::COLS, KN = U::KN;
  const ColumnPos<N1, TV, V> p(b, tile, tid);
  // the copies of w are summed, and r updated, in the vector type (FP64, or
  // FP32 in the inner solve of the mixed CG); the reductions in FP64
  TV rv[KN], mv[KN];
#pragma unroll
  for (int kk = 0; kk < KN; ++kk) {
    const int64_t a = p.col0 + (int64_t)min(p.kb + kk, N) * COLS;
    rv[kk] = ld_once(r + a);
    mv[kk] = minv_at(minv, r, a);
  }
  TV S[KN];
  column_copy_sums<N1, TV, V, TV>(p, w, sA, S);
  const TV alpha_v = (TV)alpha;
  double rr = 0.0, rz = 0.0;
#pragma unroll
  for (int kk = 0; kk < KN; ++kk) {
    const int k = p.kb + kk;
    if (p.live && k < p.kend && !p.boundary(b, k)) {
      const TV rt = rv[kk] - alpha_v * S[kk];
      r[p.col0 + (int64_t)k * COLS] = rt;
      const double c = p.inv_mult(b, k);
      const double rd = (double)rt;
      rr += c * rd * rd;
      rz += c * rd * ((double)mv[kk] * rd);
    }
  }
  TileSums ts;
  block_sum2<U::BLOCK>(rr, rz, sred, &ts.a, &ts.b);
  return ts;
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
  block_sum2<kVecThreads>(rz, rr, sred, &t.a, &t.b);
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
  double rho, bn;
  sum_partials2<kFinThreads>(part_rz, part_bb, n, sred, &rho, &bn);
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
  double rrt, rzt;
  sum_partials2<kFinThreads>(part_rr, part_rz, n, sred, &rrt, &rzt);
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
  double rho, rr;
  sum_partials2<kFinThreads>(part_rz, part_rr, n, sred, &rho, &rr);
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
