// Generic gather-scatter on gfx950: the "gs" kernel of paper Sec. V-B in its
// own form, a loop over the unique ids of shared nodes with an inner loop over
// each id's copies, for any map of L-vector entries to global ids (periodic
// boxes, unstructured meshes).  The box mesh's CG does not use it: there the
// summation is fused into the operator and update kernels by index arithmetic.
//
// Layout (compressed rows, built once on the host):
//   offsets[r] .. offsets[r+1]-1  positions in ids of row r's copies
//   ids[q]                        an L-vector index
// Rows hold only ids with two or more copies, ascending id; a row's copies are
// in ascending L-index order, so consecutive rows of a box-like numbering
// touch neighbouring nodes and the loads of a wave fall on few cache lines.
//
// Kernel: two rows per thread.  A row's copies are loaded, summed in row
// order from 0 in FP64 and the sum is stored back to each copy.  Rows are
// disjoint, so no two threads touch one entry and no atomics are needed; the
// sum order is fixed, so the result does not depend on the launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "sem_gs.h"
#include "sem_internal.h"

namespace semk {

namespace {

constexpr int kGsThreads = 256;
// Copies a thread keeps in registers between the sum and the stores; longer
// rows (more than 8 copies cannot occur on a conforming hexahedral mesh) take
// a second pass over the vector.
constexpr int kGsRegCopies = 8;
// Rows per thread.  Each thread's work is the dependent chain offsets -> ids
// -> w -> store; giving a thread two rows whose loads are issued together
// doubles the loads in flight per wave at the same occupancy.
constexpr int kGsRowsPerThread = 2;

// Rows of work-group b: b*R*256 + t + 256*k for thread t and k < R, so each
// load instruction of a wave touches 64 consecutive rows.
template <int R>
__global__ __launch_bounds__(kGsThreads) void gs_rows_kernel(int32_t n_rows,
                                                             const int32_t *__restrict__ offsets,
                                                             const int32_t *__restrict__ ids,
                                                             int64_t n_copies, int64_t n,
                                                             double *__restrict__ w) {
  const int64_t base = (int64_t)blockIdx.x * (kGsThreads * R) + threadIdx.x;
  int32_t a[R], len[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int64_t r = base + (int64_t)k * kGsThreads;
    a[k] = 0;
    len[k] = 0;
    if (r < n_rows) {
      // a row whose copies do not lie inside ids[0 .. n_copies-1] is skipped
      const int32_t lo = offsets[r], hi = offsets[r + 1];
      if (lo >= 0 && hi >= lo && (int64_t)hi <= n_copies) {
        a[k] = lo;
        len[k] = hi - lo;
      }
    }
  }
  int32_t idx[R][kGsRegCopies];
#pragma unroll
  for (int k = 0; k < R; ++k)
#pragma unroll
    for (int q = 0; q < kGsRegCopies; ++q)
      idx[k][q] = (q < len[k] && len[k] <= kGsRegCopies) ? ids[a[k] + q] : -1;
  double val[R][kGsRegCopies];
#pragma unroll
  for (int k = 0; k < R; ++k)
#pragma unroll
    for (int q = 0; q < kGsRegCopies; ++q)
      val[k][q] = (idx[k][q] >= 0 && idx[k][q] < n) ? w[idx[k][q]] : 0.0;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    if (len[k] <= kGsRegCopies) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < kGsRegCopies; ++q)
        if (q < len[k]) s += val[k][q];
#pragma unroll
      for (int q = 0; q < kGsRegCopies; ++q)
        if (idx[k][q] >= 0 && idx[k][q] < n) w[idx[k][q]] = s;
    } else {
      double s = 0.0;
      for (int32_t q = a[k]; q < a[k] + len[k]; ++q) {
        const int32_t i = ids[q];
        if (i >= 0 && i < n) s += w[i];
      }
      for (int32_t q = a[k]; q < a[k] + len[k]; ++q) {
        const int32_t i = ids[q];
        if (i >= 0 && i < n) w[i] = s;
      }
    }
  }
}

}  // namespace

hipError_t launch_gs_rows(int32_t n_rows, const int32_t *offsets, const int32_t *ids,
                          int64_t n_copies, int64_t n, double *w, hipStream_t s) {
  if (n_rows <= 0) return hipSuccess;
  constexpr int per_block = kGsThreads * kGsRowsPerThread;
  const unsigned blocks = (unsigned)((n_rows + per_block - 1) / per_block);
  hipLaunchKernelGGL(gs_rows_kernel<kGsRowsPerThread>, dim3(blocks), dim3(kGsThreads), 0, s,
                     n_rows, offsets, ids, n_copies, n, w);
  return hipGetLastError();
}

int build_gs_csr(int64_t n, const int64_t *gid, int32_t *offsets, int64_t offsets_cap,
                 int32_t *ids, int64_t ids_cap, int32_t *n_rows, int64_t *n_copies,
                 const char **why) {
  // Sort keys (id, L index): ascending id, and within an id ascending L index.
  std::vector<uint64_t> key((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    if (gid[i] < 0 || gid[i] > INT32_MAX) {
      *why = "sem_gs_csr_build: a global id is negative or above 2^31-1";
      return SEM_ERR_ARG;
    }
    key[(size_t)i] = ((uint64_t)gid[i] << 32) | (uint64_t)i;
  }
  std::sort(key.begin(), key.end());
  int64_t rows = 0, copies = 0;
  for (int64_t q = 0; q < n;) {
    const uint64_t g = key[(size_t)q] >> 32;
    int64_t end = q + 1;
    while (end < n && (key[(size_t)end] >> 32) == g) ++end;
    if (end - q >= 2) {
      ++rows;
      copies += end - q;
    }
    q = end;
  }
  *n_rows = (int32_t)rows;
  *n_copies = copies;
  if (!offsets && !ids) return SEM_OK;  // size query
  if (!offsets || !ids) {
    *why = "sem_gs_csr_build: offsets and ids must both be given or both be NULL";
    return SEM_ERR_ARG;
  }
  if (offsets_cap < rows + 1 || ids_cap < copies) {
    *why = "sem_gs_csr_build: output capacity below the sizes of the rows";
    return SEM_ERR_NOMEM;
  }
  int64_t r = 0, c = 0;
  offsets[0] = 0;
  for (int64_t q = 0; q < n;) {
    const uint64_t g = key[(size_t)q] >> 32;
    int64_t end = q + 1;
    while (end < n && (key[(size_t)end] >> 32) == g) ++end;
    if (end - q >= 2) {
      for (int64_t t = q; t < end; ++t) ids[c++] = (int32_t)(key[(size_t)t] & 0xffffffffu);
      offsets[++r] = (int32_t)c;
    }
    q = end;
  }
  return SEM_OK;
}

}  // namespace semk
