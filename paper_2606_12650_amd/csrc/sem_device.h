// Device helpers shared by the kernel translation units: wave64 and block
// reductions, XCD-aware tile order and the per-node facts of element-local
// storage.
#pragma once

#include <hip/hip_runtime.h>

#include "sem_types.h"

namespace semk {

// ---------------------------------------------------------------- precisions
// Storage and arithmetic of one operator variant: vectors TV, geometric
// factors TG, contractions in TC.  BF16 keeps G as bfloat16 bits and rounds
// both contraction inputs (u and the G-weighted gradient) to bfloat16, so
// every product is exact in FP32 and only the FP32 accumulation rounds.
struct PrecF64 {
  using TV = double;
  using TG = double;
  using TC = double;
  static constexpr bool kBf16 = false;
};
struct PrecF32 {
  using TV = float;
  using TG = float;
  using TC = float;
  static constexpr bool kBf16 = false;
};
struct PrecBF16 {
  using TV = float;
  using TG = uint16_t;
  using TC = float;
  static constexpr bool kBf16 = true;
};

// Round an FP32 value to the nearest bfloat16 (ties to even); finite inputs.
__host__ __device__ inline uint16_t bf16_bits(float f) {
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf16_value(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}
__device__ inline float round_bf16(float f) { return bf16_value(bf16_bits(f)); }

// Loads of streams that a kernel reads once (G, the CG vectors) carry the
// non-temporal hint, so those lines leave the caches first and do not
// displace lines that are reused (the neighbour copies that the
// gather-scatter reads, the operator result that the next kernel reads).  On
// gfx950 this raises the operator's read-7-write-1 stream from 5.4 to
// 6.2 TB/s.  Stores get the hint only for vectors that are not read again
// before the next iteration (x and p in the operator prologue).
template <typename T>
__device__ __forceinline__ T ld_once(const T *p) {
  return __builtin_nontemporal_load(p);
}
template <typename T>
__device__ __forceinline__ void st_once(T *p, T v) {
  __builtin_nontemporal_store(v, p);
}

// threadIdx.x through an opaque register move.  A persistent kernel that
// loops over element tiles calls the tile with this: the compiler then
// recomputes the tile's thread-index arithmetic in each iteration instead of
// hoisting it out of the loop into registers held for the whole kernel,
// which had cost the batched operator kernels a third of their occupancy.
__device__ __forceinline__ int opaque_tid() {
  int t;
  asm volatile("v_mov_b32 %0, %1" : "=v"(t) : "v"((int)threadIdx.x));
  return t;
}

// The Jacobi inverse diagonal at idx, or 1 when the solve runs without a
// preconditioner (minv == nullptr, the plain CG).  Every masked node carries
// r = 0 throughout a solve, so 1 there gives z = r = mask o r as well.
// The load is issued in both cases, from `alt` (a vector of the same length
// that the caller loads at idx as well) when there is no minv: a load under
// the branch would split the tile's batch of loads, and the compiler then
// waits for each part in turn (the FP32 CG update at N = 7 took 87 instead
// of 55 us).
template <typename T>
__device__ __forceinline__ T minv_at(const T *minv, const T *alt, int64_t idx) {
  const T v = ld_once((minv ? minv : alt) + idx);
  return minv ? v : (T)1;
}

template <class P>
__device__ inline typename P::TC load_g(const typename P::TG *p) {
  if constexpr (P::kBf16) {
    return bf16_value(ld_once(p));
  } else {
    return (typename P::TC)ld_once(p);
  }
}
template <class P>
__device__ inline typename P::TC contraction_input(typename P::TC v) {
  if constexpr (P::kBf16) {
    return round_bf16(v);
  } else {
    return v;
  }
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over a block of T threads (T a multiple of 64); valid in thread 0.
// The order is fixed: butterfly inside each wave, then waves in index order.
template <int T>
__device__ inline double block_sum(double v, double *sred) {
  static_assert(T % 64 == 0, "block size must be a multiple of the wave size");
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sred[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < T / 64; ++q) t += sred[q];
  }
  __syncthreads();
  return t;
}

// Two block sums in one pass (one barrier instead of two), each value in the
// order of block_sum, so each result has block_sum's bits.  sred holds
// 2 * T / 64 doubles.  Valid in thread 0.
template <int T>
__device__ inline void block_sum2(double a, double b, double *sred, double *ta, double *tb) {
  static_assert(T % 64 == 0, "block size must be a multiple of the wave size");
  a = wave_sum(a);
  b = wave_sum(b);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    sred[wid] = a;
    sred[T / 64 + wid] = b;
  }
  __syncthreads();
  double x = 0.0, y = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < T / 64; ++q) x += sred[q];
#pragma unroll
    for (int q = 0; q < T / 64; ++q) y += sred[T / 64 + q];
  }
  __syncthreads();
  *ta = x;
  *tb = y;
}

constexpr int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Deterministic block sum through LDS for any block size T; valid in thread 0.
template <int T>
__device__ inline double block_sum_any(double v, double *sred) {
  sred[threadIdx.x] = v;
  __syncthreads();
  constexpr int P2 = next_pow2(T);
#pragma unroll
  for (int s = P2 / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s && (int)threadIdx.x + s < T) sred[threadIdx.x] += sred[threadIdx.x + s];
    __syncthreads();
  }
  const double t = sred[0];
  __syncthreads();
  return t;
}

// Sum of n partials in a fixed order by a block of T threads; valid in
// thread 0.  Each thread keeps eight running sums; the loads of four rounds
// (32 per thread) are issued together before they are added, so a sum of up
// to 32 T partials waits for memory once.
template <int T>
__device__ inline double sum_partials(const double *__restrict__ part, int64_t n, double *sred) {
  constexpr int R = 4;
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t q = threadIdx.x; q < n; q += (int64_t)R * 8 * T) {
    // rounds that hold any partial (the same for the whole block)
    const int64_t q0 = q - threadIdx.x;
    const int64_t left = (n - q0 + 8 * T - 1) / (8 * T);
    const int rounds = left < R ? (int)left : R;
    double v[R][8];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t idx = q + (int64_t)(r * 8 + u) * T;
        v[r][u] = (r < rounds && idx < n) ? part[idx] : 0.0;
      }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] += v[r][u];
  }
  const double t = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  return block_sum<T>(t, sred);
}

// sum_partials of two arrays of n partials at once: the loads of both are
// issued together (two rounds of eight per array and thread), so the pair
// waits for memory once.  Each array is summed in the order of sum_partials
// (a running sum per residue of the index modulo 8 T, in ascending index,
// however many rounds a pass holds), so each result has its bits.  sred
// holds 2 * T / 64 doubles.  Valid in thread 0.
template <int T>
__device__ inline void sum_partials2(const double *__restrict__ pa, const double *__restrict__ pb,
                                     int64_t n, double *sred, double *ta, double *tb) {
  constexpr int R = 2;
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double c[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t q = threadIdx.x; q < n; q += (int64_t)R * 8 * T) {
    const int64_t q0 = q - threadIdx.x;
    const int64_t left = (n - q0 + 8 * T - 1) / (8 * T);
    const int rounds = left < R ? (int)left : R;
    double va[R][8], vb[R][8];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t idx = q + (int64_t)(r * 8 + u) * T;
        const bool ok = r < rounds && idx < n;
        va[r][u] = ok ? pa[idx] : 0.0;
        vb[r][u] = ok ? pb[idx] : 0.0;
      }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        a[u] += va[r][u];
        c[u] += vb[r][u];
      }
  }
  const double x = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  const double y = ((c[0] + c[1]) + (c[2] + c[3])) + ((c[4] + c[5]) + (c[6] + c[7]));
  block_sum2<T>(x, y, sred, ta, tb);
}

// Work-groups are dispatched round-robin over the 8 XCDs; this maps the
// launch index to a tile so that each XCD walks one contiguous range of
// tiles in order (neighbouring elements then share that XCD's L2).
constexpr int kNumXcd = 8;
inline int64_t xcd_grid(int64_t ntiles) { return kNumXcd * ((ntiles + kNumXcd - 1) / kNumXcd); }
__device__ inline int64_t xcd_tile(int64_t ntiles) {
  const int64_t per = (ntiles + kNumXcd - 1) / kNumXcd;
  const int64_t b = blockIdx.x;
  return (b % kNumXcd) * per + b / kNumXcd;
}

// Position of an element-local node of a box mesh.
template <int N1>
struct Node {
  int i, j, k;
  int ex, ey, ez;
  bool boundary;  // on a face of the box (homogeneous Dirichlet)
  int mult;       // number of element-local copies (1, 2, 4 or 8)
  // 1 / mult, exactly (a power of two: no division)
  __device__ double inv_mult() const {
    return mult == 1 ? 1.0 : (mult == 2 ? 0.5 : (mult == 4 ? 0.25 : 0.125));
  }
};

// All index arithmetic is 32-bit: the element index is below 2^31 and the
// divisions by nx and ny are multiply-shifts.
template <int N1>
__device__ inline Node<N1> node_at(const Box &b, int64_t idx) {
  constexpr int N = N1 - 1;
  constexpr uint32_t NP = N1 * N1 * N1;
  // L < 2^32 (sem_setup refuses larger meshes): 32-bit division by a constant
  const uint32_t e = (uint32_t)idx / NP;
  const uint32_t loc = (uint32_t)idx - e * NP;
  Node<N1> n;
  n.i = (int)(loc % N1);
  n.j = (int)((loc / N1) % N1);
  n.k = (int)(loc / (N1 * N1));
  const uint32_t eyz = b.fdx.div(e);
  n.ex = (int)(e - eyz * (uint32_t)b.nx);
  const uint32_t ez = b.fdy.div(eyz);
  n.ey = (int)(eyz - ez * (uint32_t)b.ny);
  n.ez = (int)ez;
  n.boundary = (n.ex == 0 && n.i == 0) || (n.ex == b.nx - 1 && n.i == N) ||
               (n.ey == 0 && n.j == 0) || (n.ey == b.ny - 1 && n.j == N) ||
               (n.ez == 0 && n.k == 0) || (n.ez == b.nz - 1 && n.k == N);
  const int mx = ((n.i == 0 && n.ex > 0) || (n.i == N && n.ex < b.nx - 1)) ? 2 : 1;
  const int my = ((n.j == 0 && n.ey > 0) || (n.j == N && n.ey < b.ny - 1)) ? 2 : 1;
  const int mz = ((n.k == 0 && n.ez > 0) || (n.k == N && n.ez < b.nz - 1)) ? 2 : 1;
  n.mult = mx * my * mz;
  return n;
}

// Direct stiffness summation at one node: the sum of all element-local
// copies of the node in w, added in ascending element-local index order.
// Along each direction a node has one copy, or two when it sits on a face
// shared with the neighbouring element; the second copy is a fixed address
// step away (next element, local index N -> 0).  A missing copy adds +0.0,
// which leaves the sum unchanged.  load_copies issues all eight candidate
// loads unconditionally (a missing copy reads the node itself), so no branch
// separates them.  Every copy of a node computes the same sum in the same
// order: the result is exactly continuous.
template <int N1>
struct Copies {
  int64_t addr[8];
  bool valid[8];
};

template <int N1>
__device__ inline Copies<N1> copies_of(const Box &b, const Node<N1> &n, int64_t idx) {
  constexpr int N = N1 - 1;
  constexpr int64_t NP = (int64_t)N1 * N1 * N1;
  const int64_t dx = NP - N;
  const int64_t dy = (int64_t)b.nx * NP - (int64_t)N * N1;
  const int64_t dz = (int64_t)b.nx * b.ny * NP - (int64_t)N * N1 * N1;
  const bool sx = n.i == 0 && n.ex > 0, hx = sx || (n.i == N && n.ex < b.nx - 1);
  const bool sy = n.j == 0 && n.ey > 0, hy = sy || (n.j == N && n.ey < b.ny - 1);
  const bool sz = n.k == 0 && n.ez > 0, hz = sz || (n.k == N && n.ez < b.nz - 1);
  const int64_t lo = idx - (sx ? dx : 0) - (sy ? dy : 0) - (sz ? dz : 0);
  Copies<N1> c;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int d = q & 1, cc = (q >> 1) & 1, a = q >> 2;
    c.valid[q] = (d == 0 || hx) && (cc == 0 || hy) && (a == 0 || hz);
    c.addr[q] = c.valid[q] ? lo + (d ? dx : 0) + (cc ? dy : 0) + (a ? dz : 0) : idx;
  }
  return c;
}

template <int N1, typename T>
__device__ inline void load_copies(const T *__restrict__ w, const Copies<N1> &c, T (&v)[8]) {
#pragma unroll
  for (int q = 0; q < 8; ++q) v[q] = w[c.addr[q]];
}

template <int N1, typename T>
__device__ inline double sum_copies(const Copies<N1> &c, const T (&v)[8]) {
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q) s += c.valid[q] ? (double)v[q] : 0.0;
  return s;
}

// The same sum with the loads of missing copies masked off (fewer memory
// requests for interior nodes; the form the FP64 kernels measured fastest
// with).
template <int N1, typename T>
__device__ inline double gather_copies(const T *__restrict__ w, const Box &b, const Node<N1> &n,
                                       int64_t idx) {
  const Copies<N1> c = copies_of<N1>(b, n, idx);
  double v[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) v[q] = c.valid[q] ? (double)w[c.addr[q]] : 0.0;
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q) s += v[q];
  return s;
}

}  // namespace semk
