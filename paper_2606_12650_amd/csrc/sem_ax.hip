// Element kernels of the spectral-element Poisson operator on gfx950:
// the metric setup and the FP64 operator w = A_L u (paper Sec. VIII-B, the
// "ax" kernel, with N fixed at compile time as its jit clause does).
//
// Mapping (one element per (N+1)^2 threads): thread (i, j) of an element owns
// the column of nodes (i, j, 0..N) in registers.  The contraction along t runs
// in registers; the contractions along r and s read the element's tile from
// LDS.  Every HBM access is a full-wave coalesced load or store of a k-plane
// of the element (element-major layout, i fastest).
#include <hip/hip_runtime.h>

#include "sem_ax_mfma.h"
#include "sem_ax_tile.h"
#include "sem_device.h"
#include "sem_internal.h"

namespace semk {

namespace {

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

}  // namespace

namespace {

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
template <int N1, class P, bool CG>
__global__ void __launch_bounds__(MfmaCfg<N1>::THREADS)
    ax_mfma_kernel(int64_t E, const typename P::TC *__restrict__ Dg,
                   const typename P::TG *__restrict__ G, typename P::TV *u,
                   typename P::TV *__restrict__ w, const typename P::TV *__restrict__ r,
                   const typename P::TV *__restrict__ minv, typename P::TV *__restrict__ x,
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
  ax_tile_mfma<N1, C::EPB, P, CG>(E, (int64_t)blockIdx.x * C::EPB, Dg, G, u, w, r, minv, x, alpha,
                                  beta, part, sD, s1, s2, s3, sred);
}

// Rounded copy of G for a low-precision operator.
template <class P>
__global__ void __launch_bounds__(256)
    convert_g_kernel(int64_t n, const double *__restrict__ src, typename P::TG *__restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  if constexpr (P::kBf16) {
    dst[i] = bf16_bits((float)src[i]);
  } else {
    dst[i] = (typename P::TG)src[i];
  }
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

template <int N1, class P>
hipError_t ax_dispatch(const Box &b, const void *D, const void *G, void *u, void *w, const void *r,
                       const void *minv, void *x, CgState *cg, double *part, hipStream_t s) {
  using C = OpCfg<N1>;
  using TV = typename P::TV;
  using TG = typename P::TG;
  using TC = typename P::TC;
  const int64_t blocks = (b.E() + C::EPB - 1) / C::EPB;
  if (blocks == 0) return hipSuccess;
  if (cg)
    hipLaunchKernelGGL((ax_kernel<N1, P, true>), dim3((unsigned)blocks), dim3(C::THREADS), 0, s,
                       b.E(), (const TC *)D, (const TG *)G, (TV *)u, (TV *)w, (const TV *)r,
                       (const TV *)minv, (TV *)x, cg, part);
  else
    hipLaunchKernelGGL((ax_kernel<N1, P, false>), dim3((unsigned)blocks), dim3(C::THREADS), 0, s,
                       b.E(), (const TC *)D, (const TG *)G, (TV *)u, (TV *)w, (const TV *)r,
                       (const TV *)minv, (TV *)x, cg, part);
  return hipGetLastError();
}

template <int N1, class P>
hipError_t mfma_dispatch(const Box &b, const void *D, const void *G, void *u, void *w, const void *r,
                         const void *minv, void *x, CgState *cg, double *part, hipStream_t s) {
  using C = MfmaCfg<N1>;
  using TV = typename P::TV;
  using TG = typename P::TG;
  using TC = typename P::TC;
  const int64_t blocks = (b.E() + C::EPB - 1) / C::EPB;
  if (blocks == 0) return hipSuccess;
  if (cg)
    hipLaunchKernelGGL((ax_mfma_kernel<N1, P, true>), dim3((unsigned)blocks), dim3(C::THREADS), 0, s,
                       b.E(), (const TC *)D, (const TG *)G, (TV *)u, (TV *)w, (const TV *)r,
                       (const TV *)minv, (TV *)x, cg, part);
  else
    hipLaunchKernelGGL((ax_mfma_kernel<N1, P, false>), dim3((unsigned)blocks), dim3(C::THREADS), 0,
                       s, b.E(), (const TC *)D, (const TG *)G, (TV *)u, (TV *)w, (const TV *)r,
                       (const TV *)minv, (TV *)x, cg, part);
  return hipGetLastError();
}

template <int N1>
hipError_t setup_dispatch(const Box &b, double amp, const double *D, const double *nodes,
                          double *G, double *diag, hipStream_t s) {
  using C = AxCfg<N1>;
  const int64_t blocks = (b.E() + C::EPB - 1) / C::EPB;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL((setup_geom_kernel<N1>), dim3((unsigned)blocks), dim3(C::THREADS), 0, s, b,
                     amp, D, nodes, G, diag);
  return hipGetLastError();
}

}  // namespace

#define SEM_FOR_EACH_ORDER(X) \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12)

int ax_elements_per_block(int N) {
  switch (N) {
#define CASE(n) \
  case n:       \
    return AxCfg<n + 1>::EPB;
    SEM_FOR_EACH_ORDER(CASE)
#undef CASE
    default:
      return 1;
  }
}

int64_t ax_num_blocks(const Box &b) {
  const int epb = ax_elements_per_block(b.N);
  return (b.E() + epb - 1) / epb;
}

// Operator launch for precision P (class cls): the matrix-core tile or the
// vector-unit one, by OpImpl.
template <class P>
hipError_t ax_launch(const Box &b, int cls, int impl, const void *D, const void *G, void *u, void *w,
                     const void *r, const void *minv, void *x, CgState *cg, double *part,
                     hipStream_t s) {
  const bool mfma = impl == kImplMfma || (impl == kImplDefault && op_uses_mfma(cls, b.N));
  switch (b.N) {
#define CASE(n)                                                                      \
  case n:                                                                            \
    return mfma ? mfma_dispatch<n + 1, P>(b, D, G, u, w, r, minv, x, cg, part, s)   \
                : ax_dispatch<n + 1, P>(b, D, G, u, w, r, minv, x, cg, part, s);
    SEM_FOR_EACH_ORDER(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_ax_f64(const Box &b, int impl, const double *D, const double *G, double *u,
                         double *w, const double *r, const double *minv, double *x, CgState *cg,
                         double *part, hipStream_t s) {
  return ax_launch<PrecF64>(b, 0, impl, D, G, u, w, r, minv, x, cg, part, s);
}

hipError_t launch_ax_lowp(const Box &b, int prec, int impl, const float *D, const void *G, float *u,
                          float *w, const float *r, const float *minv, float *x, CgState *cg,
                          double *part, hipStream_t s) {
  if (prec == SEM_F32) return ax_launch<PrecF32>(b, 1, impl, D, G, u, w, r, minv, x, cg, part, s);
  if (prec == SEM_BF16) return ax_launch<PrecBF16>(b, 2, impl, D, G, u, w, r, minv, x, cg, part, s);
  return hipErrorInvalidValue;
}

hipError_t launch_convert_g(int prec, int64_t n, const double *src, void *dst, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (prec == SEM_F32)
    hipLaunchKernelGGL(convert_g_kernel<PrecF32>, dim3(blocks), dim3(256), 0, s, n, src, (float *)dst);
  else if (prec == SEM_BF16)
    hipLaunchKernelGGL(convert_g_kernel<PrecBF16>, dim3(blocks), dim3(256), 0, s, n, src,
                       (uint16_t *)dst);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_setup_geom(const Box &b, double amp, const double *D, const double *nodes,
                             double *G, double *diag, hipStream_t s) {
  switch (b.N) {
#define CASE(n) \
  case n:       \
    return setup_dispatch<n + 1>(b, amp, D, nodes, G, diag, s);
    SEM_FOR_EACH_ORDER(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace semk
