// Gather-scatter, streaming updates and reductions of the Jacobi-PCG on gfx950
// (paper Sec. V-B "gs" kernel and the Sec. VIII-B streaming and tree-
// reduction kernels).
//
// Reductions are deterministic: a block sums a fixed tile of 2048 entries
// (wave64 butterfly, then the block's waves in order); a single-block second
// stage sums the per-block partials in a fixed order.  Results depend only on
// the data and the vector length, never on scheduling.
#include <hip/hip_runtime.h>

#include "sem_internal.h"

namespace semk {
namespace {

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over a block of T threads (T a multiple of 64); valid in thread 0.
template <int T>
__device__ inline double block_sum(double v, double *sred) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sred[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < T / 64; ++q) t += sred[q];
  }
  return t;
}

// Per-node facts of element-local storage on a box mesh: Dirichlet flag and
// inverse multiplicity (1, 1/2, 1/4 or 1/8: exact).
template <int N1>
struct NodeInfo {
  bool boundary;
  double c;
};

template <int N1>
__device__ inline NodeInfo<N1> node_info(const Box &b, int64_t idx) {
  constexpr int N = N1 - 1;
  constexpr int NP = N1 * N1 * N1;
  const int64_t e = idx / NP;
  const int loc = (int)(idx - e * NP);
  const int i = loc % N1;
  const int j = (loc / N1) % N1;
  const int k = loc / (N1 * N1);
  const int ex = (int)(e % b.nx);
  const int64_t eyz = e / b.nx;
  const int ey = (int)(eyz % b.ny);
  const int ez = (int)(eyz / b.ny);
  NodeInfo<N1> r;
  r.boundary = (ex == 0 && i == 0) || (ex == b.nx - 1 && i == N) || (ey == 0 && j == 0) ||
               (ey == b.ny - 1 && j == N) || (ez == 0 && k == 0) || (ez == b.nz - 1 && k == N);
  const int mx = ((i == 0 && ex > 0) || (i == N && ex < b.nx - 1)) ? 2 : 1;
  const int my = ((j == 0 && ey > 0) || (j == N && ey < b.ny - 1)) ? 2 : 1;
  const int mz = ((k == 0 && ez > 0) || (k == N && ez < b.nz - 1)) ? 2 : 1;
  r.c = 1.0 / (double)(mx * my * mz);
  return r;
}

// ------------------------------------------------------------ gather-scatter
// One thread per skeleton node (a lattice node on at least one element face).
// It sums the node's copies in ascending element-local index order and writes
// the sum (or 0 on the box boundary when masked) back to every copy.
__global__ void __launch_bounds__(256)
    dssum_kernel(double *__restrict__ w, Box b, Skeleton sk, int masked,
                 const int *__restrict__ done) {
  if (done && *done) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= sk.start[7]) return;
  int c = 1;
  while (t >= sk.start[c]) ++c;
  int64_t q = t - sk.start[c - 1];
  const int N = b.N, N1 = b.N + 1;
  const int n[3] = {b.nx, b.ny, b.nz};
  int idx[3] = {0, 0, 0};
  // decode: directions off the face first (contiguous in memory), x before y
  for (int pass = 0; pass < 2; ++pass)
    for (int d = 0; d < 3; ++d) {
      const int face = (c >> d) & 1;
      if (face != pass) continue;
      const int64_t cnt = face ? (int64_t)n[d] + 1 : (int64_t)n[d] * (N - 1);
      idx[d] = (int)(q % cnt);
      q /= cnt;
    }
  int ncp[3], elc[3][2], loc[3][2];
  bool bnd = false;
  for (int d = 0; d < 3; ++d) {
    if ((c >> d) & 1) {
      const int m = idx[d];
      int k = 0;
      if (m > 0) { elc[d][k] = m - 1; loc[d][k] = N; ++k; }
      if (m < n[d]) { elc[d][k] = m; loc[d][k] = 0; ++k; }
      ncp[d] = k;
      bnd = bnd || m == 0 || m == n[d];
    } else {
      elc[d][0] = idx[d] / (N - 1);
      loc[d][0] = 1 + idx[d] % (N - 1);
      ncp[d] = 1;
    }
  }
  const int64_t np = (int64_t)N1 * N1 * N1;
  int64_t addr[8];
  int na = 0;
  double s = 0.0;
  for (int cz = 0; cz < ncp[2]; ++cz)
    for (int cy = 0; cy < ncp[1]; ++cy)
      for (int cx = 0; cx < ncp[0]; ++cx) {
        const int64_t e = elc[0][cx] + (int64_t)n[0] * (elc[1][cy] + (int64_t)n[1] * elc[2][cz]);
        const int64_t a = e * np + loc[0][cx] + N1 * (loc[1][cy] + N1 * loc[2][cz]);
        addr[na++] = a;
        s += w[a];
      }
  const double v = (masked && bnd) ? 0.0 : s;
  for (int a = 0; a < na; ++a) w[addr[a]] = v;
}

// ------------------------------------------------------------ CG kernels
template <int N1>
__global__ void __launch_bounds__(kVecThreads)
    cg_init_kernel(Box b, int64_t L, const double *__restrict__ bvec, double *__restrict__ x,
                   double *__restrict__ r, double *__restrict__ p,
                   const double *__restrict__ minv, double *__restrict__ part_rz,
                   double *__restrict__ part_bb) {
  __shared__ double sred[kVecThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kVecTile + threadIdx.x;
  double rz = 0.0, bb = 0.0;
#pragma unroll
  for (int u = 0; u < kVecItems; ++u) {
    const int64_t idx = base + (int64_t)u * kVecThreads;
    if (idx < L) {
      const NodeInfo<N1> ni = node_info<N1>(b, idx);
      const double rv = ni.boundary ? 0.0 : bvec[idx];
      x[idx] = 0.0;
      r[idx] = rv;
      p[idx] = 0.0;
      rz += ni.c * rv * (minv[idx] * rv);
      bb += ni.c * rv * rv;
    }
  }
  const double a = block_sum<kVecThreads>(rz, sred);
  __syncthreads();
  const double c = block_sum<kVecThreads>(bb, sred);
  if (threadIdx.x == 0) {
    part_rz[blockIdx.x] = a;
    part_bb[blockIdx.x] = c;
  }
}

template <int N1>
__global__ void __launch_bounds__(kVecThreads)
    cg_update_kernel(Box b, int64_t L, double *__restrict__ x, const double *__restrict__ p,
                     double *__restrict__ r, const double *__restrict__ w,
                     const double *__restrict__ minv, const CgState *__restrict__ st,
                     double *__restrict__ part_rr, double *__restrict__ part_rz) {
  __shared__ double sred[kVecThreads / 64];
  if (st->done) return;
  const double alpha = st->alpha;
  const int64_t base = (int64_t)blockIdx.x * kVecTile + threadIdx.x;
  double rr = 0.0, rz = 0.0;
#pragma unroll
  for (int u = 0; u < kVecItems; ++u) {
    const int64_t idx = base + (int64_t)u * kVecThreads;
    if (idx < L) {
      const double c = node_info<N1>(b, idx).c;
      x[idx] += alpha * p[idx];
      const double rv = r[idx] - alpha * w[idx];
      r[idx] = rv;
      rr += c * rv * rv;
      rz += c * rv * (minv[idx] * rv);
    }
  }
  const double a = block_sum<kVecThreads>(rr, sred);
  __syncthreads();
  const double c = block_sum<kVecThreads>(rz, sred);
  if (threadIdx.x == 0) {
    part_rr[blockIdx.x] = a;
    part_rz[blockIdx.x] = c;
  }
}

// Second stage of a reduction: one block sums `n` partials in a fixed order.
__device__ inline double sum_partials(const double *__restrict__ part, int64_t n, double *sred) {
  double t = 0.0;
  for (int64_t q = threadIdx.x; q < n; q += kVecThreads) t += part[q];
  return block_sum<kVecThreads>(t, sred);
}

__global__ void __launch_bounds__(kVecThreads)
    cg_finalize_init_kernel(CgState *st, const double *__restrict__ part_rz,
                            const double *__restrict__ part_bb, int64_t n) {
  __shared__ double sred[kVecThreads / 64];
  const double rz = sum_partials(part_rz, n, sred);
  __syncthreads();
  const double bb = sum_partials(part_bb, n, sred);
  if (threadIdx.x == 0) {
    st->rho = rz;
    st->bnorm2 = bb;
    st->rnorm2 = bb;
    st->beta = 0.0;
    st->alpha = 0.0;
    st->iter = 0;
    st->tol2 = st->rtol2 * bb;
    st->done = (bb == 0.0) ? kConverged : kRunning;
    if (!isfinite(bb) || !isfinite(rz)) st->done = kBreakdown;
  }
}

__global__ void __launch_bounds__(kVecThreads)
    cg_finalize_alpha_kernel(CgState *st, const double *__restrict__ part, int64_t n) {
  __shared__ double sred[kVecThreads / 64];
  if (st->done) return;
  const double pap = sum_partials(part, n, sred);
  if (threadIdx.x == 0) {
    st->pap = pap;
    if (!(pap > 0.0) || !isfinite(pap)) {
      st->done = kBreakdown;
    } else {
      st->alpha = st->rho / pap;
    }
  }
}

__global__ void __launch_bounds__(kVecThreads)
    cg_finalize_beta_kernel(CgState *st, const double *__restrict__ part_rr,
                            const double *__restrict__ part_rz, int64_t n) {
  __shared__ double sred[kVecThreads / 64];
  if (st->done) return;
  const double rr = sum_partials(part_rr, n, sred);
  __syncthreads();
  const double rz = sum_partials(part_rz, n, sred);
  if (threadIdx.x == 0) {
    const int it = st->iter + 1;
    st->iter = it;
    st->rnorm2 = rr;
    const double beta = rz / st->rho;
    st->beta = beta;
    st->rho = rz;
    if (!isfinite(rr) || !isfinite(beta)) {
      st->done = kBreakdown;
    } else if (st->tol2 >= 0.0 && rr <= st->tol2) {
      st->done = kConverged;
    } else if (it >= st->max_iter) {
      st->done = kMaxIter;
    }
  }
}

// ------------------------------------------------------------ setup helpers
template <int N1>
__global__ void __launch_bounds__(kVecThreads)
    invert_diag_kernel(Box b, int64_t L, double *__restrict__ d) {
  const int64_t base = (int64_t)blockIdx.x * kVecTile + threadIdx.x;
#pragma unroll
  for (int u = 0; u < kVecItems; ++u) {
    const int64_t idx = base + (int64_t)u * kVecThreads;
    if (idx < L) d[idx] = node_info<N1>(b, idx).boundary ? 0.0 : 1.0 / d[idx];
  }
}

template <int N1>
__global__ void __launch_bounds__(kVecThreads)
    fill_c_kernel(Box b, int64_t L, double *__restrict__ c) {
  const int64_t base = (int64_t)blockIdx.x * kVecTile + threadIdx.x;
#pragma unroll
  for (int u = 0; u < kVecItems; ++u) {
    const int64_t idx = base + (int64_t)u * kVecThreads;
    if (idx < L) c[idx] = node_info<N1>(b, idx).c;
  }
}

// ------------------------------------------------------------ generic vectors
__global__ void __launch_bounds__(kVecThreads)
    axpy_kernel(int64_t n, double alpha, const double *__restrict__ x, double *__restrict__ y) {
  const int64_t base = (int64_t)blockIdx.x * kVecTile + threadIdx.x;
#pragma unroll
  for (int u = 0; u < kVecItems; ++u) {
    const int64_t idx = base + (int64_t)u * kVecThreads;
    if (idx < n) y[idx] = fma(alpha, x[idx], y[idx]);
  }
}

template <bool W>
__global__ void __launch_bounds__(kVecThreads)
    dot_partial_kernel(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                       const double *__restrict__ wt, double *__restrict__ part) {
  __shared__ double sred[kVecThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kVecTile + threadIdx.x;
  double acc = 0.0;
#pragma unroll
  for (int u = 0; u < kVecItems; ++u) {
    const int64_t idx = base + (int64_t)u * kVecThreads;
    if (idx < n) {
      const double v = x[idx] * y[idx];
      acc += W ? wt[idx] * v : v;
    }
  }
  const double t = block_sum<kVecThreads>(acc, sred);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void __launch_bounds__(kVecThreads)
    dot_final_kernel(const double *__restrict__ part, int64_t n, double *__restrict__ out) {
  __shared__ double sred[kVecThreads / 64];
  const double t = sum_partials(part, n, sred);
  if (threadIdx.x == 0) *out = t;
}

#define SEM_FOR_EACH_ORDER(X) \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12)

inline dim3 vec_grid(int64_t n) { return dim3((unsigned)vec_num_blocks(n)); }

}  // namespace

Skeleton make_skeleton(const Box &b) {
  Skeleton sk;
  const int64_t n[3] = {b.nx, b.ny, b.nz};
  sk.start[0] = 0;
  for (int c = 1; c <= 7; ++c) {
    int64_t cnt = 1;
    for (int d = 0; d < 3; ++d) cnt *= ((c >> d) & 1) ? n[d] + 1 : n[d] * (b.N - 1);
    sk.start[c] = sk.start[c - 1] + cnt;
  }
  return sk;
}

hipError_t launch_dssum(const Box &b, const Skeleton &sk, double *w, int masked, const int *done,
                        hipStream_t s) {
  const int64_t total = sk.start[7];
  if (total == 0) return hipSuccess;
  const int64_t blocks = (total + 255) / 256;
  hipLaunchKernelGGL(dssum_kernel, dim3((unsigned)blocks), dim3(256), 0, s, w, b, sk, masked,
                     done);
  return hipGetLastError();
}

#define DISPATCH_N(b, KERNEL, ...)                                                      \
  switch ((b).N) {                                                                      \
    case 1: hipLaunchKernelGGL(KERNEL<2>, __VA_ARGS__); break;                          \
    case 2: hipLaunchKernelGGL(KERNEL<3>, __VA_ARGS__); break;                          \
    case 3: hipLaunchKernelGGL(KERNEL<4>, __VA_ARGS__); break;                          \
    case 4: hipLaunchKernelGGL(KERNEL<5>, __VA_ARGS__); break;                          \
    case 5: hipLaunchKernelGGL(KERNEL<6>, __VA_ARGS__); break;                          \
    case 6: hipLaunchKernelGGL(KERNEL<7>, __VA_ARGS__); break;                          \
    case 7: hipLaunchKernelGGL(KERNEL<8>, __VA_ARGS__); break;                          \
    case 8: hipLaunchKernelGGL(KERNEL<9>, __VA_ARGS__); break;                          \
    case 9: hipLaunchKernelGGL(KERNEL<10>, __VA_ARGS__); break;                         \
    case 10: hipLaunchKernelGGL(KERNEL<11>, __VA_ARGS__); break;                        \
    case 11: hipLaunchKernelGGL(KERNEL<12>, __VA_ARGS__); break;                        \
    case 12: hipLaunchKernelGGL(KERNEL<13>, __VA_ARGS__); break;                        \
    default: return hipErrorInvalidValue;                                               \
  }

hipError_t launch_cg_init(const Box &b, const double *bvec, double *x, double *r, double *p,
                          const double *minv, double *part_rz, double *part_bb, hipStream_t s) {
  const int64_t L = b.L();
  if (L == 0) return hipSuccess;
  DISPATCH_N(b, cg_init_kernel, vec_grid(L), dim3(kVecThreads), 0, s, b, L, bvec, x, r, p, minv,
             part_rz, part_bb);
  return hipGetLastError();
}

hipError_t launch_cg_update(const Box &b, double *x, const double *p, double *r, const double *w,
                            const double *minv, const CgState *st, double *part_rr,
                            double *part_rz, hipStream_t s) {
  const int64_t L = b.L();
  if (L == 0) return hipSuccess;
  DISPATCH_N(b, cg_update_kernel, vec_grid(L), dim3(kVecThreads), 0, s, b, L, x, p, r, w, minv,
             st, part_rr, part_rz);
  return hipGetLastError();
}

hipError_t launch_invert_diag(const Box &b, double *d, hipStream_t s) {
  const int64_t L = b.L();
  if (L == 0) return hipSuccess;
  DISPATCH_N(b, invert_diag_kernel, vec_grid(L), dim3(kVecThreads), 0, s, b, L, d);
  return hipGetLastError();
}

hipError_t launch_fill_c(const Box &b, double *c, hipStream_t s) {
  const int64_t L = b.L();
  if (L == 0) return hipSuccess;
  DISPATCH_N(b, fill_c_kernel, vec_grid(L), dim3(kVecThreads), 0, s, b, L, c);
  return hipGetLastError();
}

hipError_t launch_cg_finalize_init(CgState *st, const double *part_rz, const double *part_bb,
                                   int64_t nparts, hipStream_t s) {
  hipLaunchKernelGGL(cg_finalize_init_kernel, dim3(1), dim3(kVecThreads), 0, s, st, part_rz,
                     part_bb, nparts);
  return hipGetLastError();
}

hipError_t launch_cg_finalize_alpha(CgState *st, const double *part_pw, int64_t nparts,
                                    hipStream_t s) {
  hipLaunchKernelGGL(cg_finalize_alpha_kernel, dim3(1), dim3(kVecThreads), 0, s, st, part_pw,
                     nparts);
  return hipGetLastError();
}

hipError_t launch_cg_finalize_beta(CgState *st, const double *part_rr, const double *part_rz,
                                   int64_t nparts, hipStream_t s) {
  hipLaunchKernelGGL(cg_finalize_beta_kernel, dim3(1), dim3(kVecThreads), 0, s, st, part_rr,
                     part_rz, nparts);
  return hipGetLastError();
}

hipError_t launch_axpy(int64_t n, double alpha, const double *x, double *y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(axpy_kernel, vec_grid(n), dim3(kVecThreads), 0, s, n, alpha, x, y);
  return hipGetLastError();
}

hipError_t launch_dot(int64_t n, const double *x, const double *y, const double *wt, double *out,
                      double *partials, hipStream_t s) {
  const int64_t nb = vec_num_blocks(n);
  if (nb > 0) {
    if (wt)
      hipLaunchKernelGGL(dot_partial_kernel<true>, vec_grid(n), dim3(kVecThreads), 0, s, n, x, y,
                         wt, partials);
    else
      hipLaunchKernelGGL(dot_partial_kernel<false>, vec_grid(n), dim3(kVecThreads), 0, s, n, x,
                         y, wt, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(kVecThreads), 0, s, partials, nb, out);
  return hipGetLastError();
}

}  // namespace semk
