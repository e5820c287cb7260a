// The non-specialised forms of three hot-path kernels, for the paper's
// specialisation study (Sec. VIII-B, Tab. hip_vs_hip: the HIP-variable
// implementation against the one with run-time values fixed in the code).
// The solver never runs them.  Each computes what its specialised
// counterpart computes, with the run-time values that the specialised one
// knows at compile time left as kernel arguments:
//
//   ax_generic_kernel   w = A_L u with the order N a run-time argument: the
//                       same thread mapping as the vector-ALU column tile
//                       (one (i, j) column per thread, LDS tiles with padded
//                       rows), but every 1-D loop has a run-time bound, the
//                       tiles are sized at launch and no loop is unrolled
//                       for the order;
//   axpy_generic_kernel y += alpha x with the work-group size chosen at
//                       launch (grid-stride loop, one entry per step);
//   dot_generic_kernel  partial sums with the work-group size chosen at
//                       launch and the in-group tree reduction as a loop
//                       over halving strides with a barrier per level.
#include <hip/hip_runtime.h>

#include "sem_internal.h"

namespace semk {

namespace {

// LDS of one element: D (n1 x n1), the operand tile and the three weighted
// gradient tiles, each n1 planes of n1 padded rows of n1 + 1 values.
__host__ __device__ inline int generic_tile(int n1) { return n1 * n1 * (n1 + 1); }
inline size_t generic_lds_bytes(int n1, int epb) {
  return sizeof(double) * (size_t)(n1 * n1 + 4 * epb * generic_tile(n1));
}

__global__ void ax_generic_kernel(int n1, int epb, int64_t E, const double *__restrict__ Dg,
                                  const double *__restrict__ G, const double *__restrict__ u,
                                  double *__restrict__ w) {
  extern __shared__ double smem[];
  const int pl = n1 * n1, np = pl * n1, rs = n1 + 1, ps = n1 * rs, tile = generic_tile(n1);
  const int tid = threadIdx.x;
  const int el = tid / pl;
  const int ij = tid - el * pl;
  const int i = ij % n1, j = ij / n1;
  const int64_t e = (int64_t)blockIdx.x * epb + el;
  const bool active = el < epb && e < E;
  double *sD = smem;
  double *U = sD + pl + (el < epb ? el : 0) * 4 * tile;
  double *R = U + tile, *S = R + tile, *T = S + tile;
  for (int t = tid; t < pl; t += blockDim.x) sD[t] = Dg[t];
  if (active)
    for (int k = 0; k < n1; ++k) U[k * ps + j * rs + i] = u[e * np + k * pl + ij];
  __syncthreads();
  if (active) {
    const double *Ge = G + e * 6 * np + ij;
    for (int k = 0; k < n1; ++k) {
      double ur = 0.0, us = 0.0, ut = 0.0;
      for (int l = 0; l < n1; ++l) {
        ur += sD[i * n1 + l] * U[k * ps + j * rs + l];
        us += sD[j * n1 + l] * U[k * ps + l * rs + i];
        ut += sD[k * n1 + l] * U[l * ps + j * rs + i];
      }
      const int64_t g = (int64_t)k * pl;
      const double grr = Ge[g], grs = Ge[np + g], grt = Ge[2 * np + g];
      const double gss = Ge[3 * np + g], gst = Ge[4 * np + g], gtt = Ge[5 * np + g];
      const int o = k * ps + j * rs + i;
      R[o] = grr * ur + grs * us + grt * ut;
      S[o] = grs * ur + gss * us + gst * ut;
      T[o] = grt * ur + gst * us + gtt * ut;
    }
  }
  __syncthreads();
  if (active) {
    for (int k = 0; k < n1; ++k) {
      double v = 0.0;
      for (int l = 0; l < n1; ++l) {
        v += sD[l * n1 + i] * R[k * ps + j * rs + l];
        v += sD[l * n1 + j] * S[k * ps + l * rs + i];
        v += sD[l * n1 + k] * T[l * ps + j * rs + i];
      }
      w[e * np + k * pl + ij] = v;
    }
  }
}

__global__ void axpy_generic_kernel(int64_t n, double alpha, const double *__restrict__ x,
                                    double *__restrict__ y) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    y[i] = fma(alpha, x[i], y[i]);
}

// Sum of wt_i x_i y_i over this group's grid-stride entries (wt may be null;
// y null: the entries of x are summed), then the looped tree over blockDim.x
// (a power of two) threads.
__global__ void dot_generic_kernel(int64_t n, const double *__restrict__ x,
                                   const double *__restrict__ y, const double *__restrict__ wt,
                                   double *__restrict__ out) {
  extern __shared__ double sred[];
  const int tid = threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + tid; i < n; i += stride) {
    double v = y ? x[i] * y[i] : x[i];
    if (wt) v *= wt[i];
    acc += v;
  }
  sred[tid] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) sred[tid] += sred[tid + s];
    __syncthreads();
  }
  if (tid == 0) out[blockIdx.x] = sred[0];
}

}  // namespace

int generic_ax_epb(int N) {
  const int pl = (N + 1) * (N + 1);
  return pl >= 128 ? 1 : 128 / pl;
}

hipError_t launch_ax_generic(const Box &b, const double *D, const double *G, const double *u,
                             double *w, hipStream_t s) {
  const int n1 = b.N + 1;
  if (n1 < 2 || n1 > kGenericMaxN1) return hipErrorInvalidValue;
  const int epb = generic_ax_epb(b.N);
  const int64_t blocks = (b.E() + epb - 1) / epb;
  if (blocks == 0) return hipSuccess;
  const size_t lds = generic_lds_bytes(n1, epb);  // <= 61 KiB up to N = 11
  hipLaunchKernelGGL(ax_generic_kernel, dim3((unsigned)blocks), dim3(n1 * n1 * epb), lds, s, n1, epb,
                     b.E(), D, G, u, w);
  return hipGetLastError();
}

hipError_t launch_axpy_generic(int64_t n, double alpha, const double *x, double *y, int block,
                               hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t want = (n + block - 1) / block;
  const unsigned grid = (unsigned)(want < kGenericMaxGrid ? want : kGenericMaxGrid);
  hipLaunchKernelGGL(axpy_generic_kernel, dim3(grid), dim3(block), 0, s, n, alpha, x, y);
  return hipGetLastError();
}

int64_t generic_dot_groups(int64_t n, int block) {
  const int64_t want = (n + 8 * (int64_t)block - 1) / (8 * (int64_t)block);
  return want < 1 ? 1 : (want < kGenericMaxGrid ? want : kGenericMaxGrid);
}

hipError_t launch_dot_generic(int64_t n, const double *x, const double *y, const double *wt,
                              double *out, double *partials, int block, hipStream_t s) {
  const int64_t groups = generic_dot_groups(n, block);
  const size_t lds = sizeof(double) * (size_t)block;
  hipLaunchKernelGGL(dot_generic_kernel, dim3((unsigned)groups), dim3(block), lds, s, n, x, y, wt,
                     partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(dot_generic_kernel, dim3(1), dim3(block), lds, s, groups, partials,
                     (const double *)nullptr, (const double *)nullptr, out);
  return hipGetLastError();
}

}  // namespace semk
