// C-ABI entry points of libsem (declared in include/sem.h): argument checks,
// workspace layout, host-side basis construction and the device-resident CG
// driver (Jacobi PCG of paper Sec. VIII-A, iterations captured in a HIP graph).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "sem_device.h"
#include "sem_error.h"
#include "sem_gs.h"
#include "sem_internal.h"
#include "sem_rtc.h"

using semk::Box;
using semk::CgState;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return SEM_ERR_HIP;
}

#define SEM_HIP(call)                                     \
  do {                                                    \
    hipError_t e_ = (call);                               \
    if (e_ != hipSuccess) return hip_fail(e_, #call);     \
  } while (0)

constexpr size_t kAlign = 256;
// Inner iteration cap per outer step of the mixed solver when the caller
// gives none.  The inner solve normally stops at its tolerance first; at
// N = 11 in FP32 that takes about 1050 iterations, so the cap sits well above.
constexpr int kDefaultInnerMax = 5000;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Byte offsets of every buffer inside the caller's workspace.  The low-
// precision block (Dlo .. state_in) exists only when desc.lowprec != SEM_F64.
struct Layout {
  size_t D, nodes, G, minv, r, p, w, part_ax, part_rr, part_rz, state;
  size_t Dlo, Glo, minv32, e, rin, pin, win, state_in;
  size_t total;
};

// SEM_OK, or SEM_ERR_ARG for a malformed descriptor, or SEM_ERR_UNSUPPORTED
// for an order or precision no kernel serves: orders 1..12 are built with the
// library in every precision and element tile; orders 13..15 are compiled at
// run time in FP64 with the matrix-core tile.
int desc_check(const sem_mesh_desc *d, std::string *why) {
  if (!d) { *why = "null mesh descriptor"; return SEM_ERR_ARG; }
  if (d->nelx < 1 || d->nely < 1 || d->nelz < 1) { *why = "element counts must be >= 1"; return SEM_ERR_ARG; }
  if (d->order < semk::kMinOrder) { *why = "order N must be >= 1"; return SEM_ERR_ARG; }
  if (d->lowprec != SEM_F64 && d->lowprec != SEM_F32 && d->lowprec != SEM_BF16) {
    *why = "lowprec must be SEM_F64, SEM_F32 or SEM_BF16";
    return SEM_ERR_ARG;
  }
  if (d->flags != 0 && d->flags != SEM_FLAG_MFMA && d->flags != SEM_FLAG_VALU) {
    *why = "flags must be 0, SEM_FLAG_MFMA or SEM_FLAG_VALU";
    return SEM_ERR_ARG;
  }
  if (!std::isfinite(d->deform_amp)) { *why = "deform_amp must be finite"; return SEM_ERR_ARG; }
  if (d->order > semk::kMaxRtcOrder) {
    *why = "order N must be in [1, 15] (1..12 built, 13..15 compiled at run time)";
    return SEM_ERR_UNSUPPORTED;
  }
  if (semk::rtc_order(d->order) && (d->lowprec != SEM_F64 || d->flags == SEM_FLAG_VALU)) {
    *why = "orders 13..15 run in FP64 on the matrix-core tile only (lowprec SEM_F64, flags 0 or SEM_FLAG_MFMA)";
    return SEM_ERR_UNSUPPORTED;
  }
  const double L = (double)d->nelx * d->nely * d->nelz * std::pow(d->order + 1.0, 3);
  if (L > 4.0e9) { *why = "mesh too large (L > 4e9)"; return SEM_ERR_ARG; }
  return SEM_OK;
}

Box box_of(const sem_mesh_desc *d) { return Box::make(d->nelx, d->nely, d->nelz, d->order); }

Layout layout_of(const sem_mesh_desc *d) {
  const Box b = box_of(d);
  const size_t L = (size_t)b.L();
  const size_t n1 = (size_t)b.n1();
  Layout o;
  size_t at = 0;
  auto take = [&](size_t bytes) {
    const size_t off = at;
    at = align_up(at + bytes);
    return off;
  };
  o.D = take(n1 * n1 * sizeof(double));
  o.nodes = take(2 * n1 * sizeof(double));
  o.G = take(6 * L * sizeof(double));
  o.minv = take(L * sizeof(double));
  o.r = take(L * sizeof(double));
  o.p = take(L * sizeof(double));
  o.w = take(L * sizeof(double));
  o.part_ax = take((size_t)b.E() * sizeof(double));  // per-element p.Ap
  o.part_rr = take((size_t)semk::stream_partials(b) * sizeof(double));
  o.part_rz = take((size_t)semk::stream_partials(b) * sizeof(double));
  o.state = take(sizeof(CgState));
  o.Dlo = o.Glo = o.minv32 = o.e = o.rin = o.pin = o.win = o.state_in = 0;
  if (d->lowprec != SEM_F64) {
    const size_t gbytes = d->lowprec == SEM_BF16 ? 2 : 4;
    o.Dlo = take(n1 * n1 * sizeof(float));
    o.Glo = take(6 * L * gbytes);
    o.minv32 = take(L * sizeof(float));
    o.e = take(L * sizeof(float));
    o.rin = take(L * sizeof(float));
    o.pin = take(L * sizeof(float));
    o.win = take(L * sizeof(float));
    o.state_in = take(sizeof(CgState));
  }
  o.total = at;
  return o;
}

// ---------------------------------------------------------------- GLL basis
// Legendre P_N and P_N' at x by the three-term recurrence, in long double.
void legendre_pd(int N, long double x, long double *p, long double *dp) {
  long double p0 = 1.0L, p1 = x, d0 = 0.0L, d1 = 1.0L;
  if (N == 0) { *p = 1.0L; *dp = 0.0L; return; }
  for (int n = 1; n < N; ++n) {
    const long double p2 = ((2 * n + 1) * x * p1 - n * p0) / (n + 1);
    const long double d2 = d0 + (2 * n + 1) * p1;  // P'_{n+1} = P'_{n-1} + (2n+1) P_n
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  *p = p1;
  *dp = d1;
}

// GLL nodes (ascending) and weights.  Interior nodes: Newton on P_N' with
// P_N'' from Legendre's equation (1-x^2) P'' = 2x P' - N(N+1) P, started at
// the Chebyshev-Lobatto points; weights 2/(N(N+1) P_N(x)^2).
void gll_host(int N, std::vector<double> *xs, std::vector<double> *ws) {
  std::vector<long double> x(N + 1);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i <= N; ++i) x[i] = -cosl(pi * i / N);
  for (int i = 1; i < N; ++i) {
    long double v = x[i];
    for (int it = 0; it < 60; ++it) {
      long double p, dp;
      legendre_pd(N, v, &p, &dp);
      const long double d2 = (2.0L * v * dp - N * (N + 1.0L) * p) / (1.0L - v * v);
      const long double dv = dp / d2;
      v -= dv;
      if (fabsl(dv) < 1e-19L) break;
    }
    x[i] = v;
  }
  x[0] = -1.0L;
  x[N] = 1.0L;
  xs->assign(N + 1, 0.0);
  ws->assign(N + 1, 0.0);
  for (int i = 0; i <= N; ++i) {
    // symmetric node set: average the two mirrored estimates
    const long double v = 0.5L * (x[i] - x[N - i]);
    long double p, dp;
    legendre_pd(N, v, &p, &dp);
    (*xs)[i] = (double)v;
    (*ws)[i] = (double)(2.0L / (N * (N + 1.0L) * p * p));
  }
  if (N % 2 == 0) (*xs)[N / 2] = 0.0;
}

// D[a][b] = l_b'(x_a) = P_N(x_a) / (P_N(x_b) (x_a - x_b)) off the diagonal;
// -N(N+1)/4 and N(N+1)/4 at the two ends, 0 elsewhere on the diagonal.
void deriv_host(int N, const std::vector<double> &xs, std::vector<double> *D) {
  const int n1 = N + 1;
  D->assign((size_t)n1 * n1, 0.0);
  std::vector<long double> pn(n1);
  for (int a = 0; a < n1; ++a) {
    long double dp;
    legendre_pd(N, (long double)xs[a], &pn[a], &dp);
  }
  for (int a = 0; a < n1; ++a)
    for (int b = 0; b < n1; ++b)
      if (a != b)
        (*D)[a * n1 + b] = (double)(pn[a] / (pn[b] * ((long double)xs[a] - (long double)xs[b])));
  (*D)[0] = -N * (N + 1) / 4.0;
  (*D)[(size_t)N * n1 + N] = N * (N + 1) / 4.0;
}

}  // namespace

namespace semk {
int set_error(int code, const std::string &msg) { return fail(code, msg); }
int set_hip_error(hipError_t e, const char *what) { return hip_fail(e, what); }
}  // namespace semk

struct sem_ctx {
  sem_mesh_desc desc;
  Box box;
  Layout lay;
  char *ws;
  size_t ws_bytes;
  double *D, *nodes, *G, *minv, *r, *p, *w, *part_ax, *part_rr, *part_rz;
  CgState *st;
  // low-precision copy (null when desc.lowprec == SEM_F64)
  float *Dlo, *minv32, *e, *rin, *pin, *win;
  void *Glo;
  CgState *st_in;
  // partial counts: elements, streaming tiles, FP64 and FP32 update tiles
  int64_t n_ax_blocks, n_vec_blocks, n_upd_blocks, n_upd_blocks_in;
  // kernel variants (sem_set_knob): element tile (OpImpl) and update tile
  // shape (upd_shape), [0] for the FP64 iterations, [1] for the inner ones
  int op_impl[2];
  int upd_var[2];
  CgState host_state;  // staging for the state upload / status reads
  CgState host_inner;
  int in_batch;  // 1 while the context is a slot of a batch
  // Minv of the FP64 iterations of the running sem_cg call (null: plain CG)
  const double *cg_minv;
  // cached graphs: [0] FP64 CG iterations into graph_x, [1] inner iterations
  hipGraphExec_t graph[2];
  hipStream_t graph_stream[2];
  double *graph_x[2];
  const double *graph_minv[2];
  int graph_iters[2];
};

namespace {

// One Jacobi-PCG iteration: the operator kernel (its prologue finishes the
// previous iteration's x += alpha p and forms the new p; its epilogue leaves
// the partials of <p, A p>), a one-group alpha step, the update kernel (which
// pulls the assembled, masked A p from the element-local result) and a
// one-group step for beta, the residual and the done flag.
int enqueue_cg_iteration(sem_ctx *c, double *x, hipStream_t s) {
  const Box &b = c->box;
  SEM_HIP(semk::launch_ax_f64(b, c->op_impl[0], c->D, c->G, c->p, c->w, c->r, c->cg_minv, x, c->st, c->part_ax, s));
  SEM_HIP(semk::launch_cg_alpha(c->st, c->part_ax, c->n_ax_blocks, s));
  SEM_HIP(semk::launch_cg_update(b, c->upd_var[0], c->r, c->w, c->cg_minv, c->st, c->part_rr, c->part_rz, s));
  SEM_HIP(semk::launch_cg_beta(c->st, c->part_rr, c->part_rz, c->n_upd_blocks, s));
  return SEM_OK;
}

// One iteration of the inner (low-precision) Jacobi-PCG: the same four steps
// on FP32 vectors with the rounded operator; the inner correction e plays x.
int enqueue_inner_iteration(sem_ctx *c, double *, hipStream_t s) {
  const Box &b = c->box;
  SEM_HIP(semk::launch_ax_lowp(b, c->desc.lowprec, c->op_impl[1], c->Dlo, c->Glo,
                               c->pin, c->win, c->rin, c->minv32, c->e, c->st_in, c->part_ax, s));
  SEM_HIP(semk::launch_cg_alpha(c->st_in, c->part_ax, c->n_ax_blocks, s));
  SEM_HIP(semk::launch_cg_update_f32(b, c->upd_var[1], c->rin, c->win, c->minv32, c->st_in, c->part_rr,
                                     c->part_rz, s));
  SEM_HIP(semk::launch_cg_beta(c->st_in, c->part_rr, c->part_rz, c->n_upd_blocks_in, s));
  return SEM_OK;
}

typedef int (*enqueue_fn)(sem_ctx *, double *, hipStream_t);

void drop_graph(sem_ctx *c, int slot) {
  if (c->graph[slot]) (void)hipGraphExecDestroy(c->graph[slot]);
  c->graph[slot] = nullptr;
  c->graph_stream[slot] = nullptr;
  c->graph_x[slot] = nullptr;
  c->graph_minv[slot] = nullptr;
  c->graph_iters[slot] = 0;
}

// Capture `iters` iterations of `fn` on stream s into graph slot `slot`.
// Returns SEM_OK, or a positive value when capture is not possible (the
// caller then launches directly), or a negative error.
int capture_graph(sem_ctx *c, int slot, enqueue_fn fn, double *x, int iters, hipStream_t s) {
  if (c->graph[slot] && c->graph_stream[slot] == s && c->graph_x[slot] == x &&
      c->graph_minv[slot] == c->cg_minv && c->graph_iters[slot] == iters)
    return SEM_OK;
  drop_graph(c, slot);
  if (s == nullptr) return 1;  // the legacy null stream cannot be captured
  if (hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed) != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  int rc = SEM_OK;
  for (int it = 0; it < iters && rc == SEM_OK; ++it) rc = fn(c, x, s);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(s, &g);
  if (rc != SEM_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  c->graph[slot] = ex;
  c->graph_stream[slot] = s;
  c->graph_x[slot] = x;
  c->graph_minv[slot] = c->cg_minv;
  c->graph_iters[slot] = iters;
  return SEM_OK;
}

// Run iterations of `fn` (graph replays of `every`, or direct launches)
// until the device state `st` reports done; `host` receives the state.
int run_until_done(sem_ctx *c, int slot, enqueue_fn fn, double *x, CgState *st, CgState *host,
                   int every, int max_iter, hipStream_t s) {
  int rc = capture_graph(c, slot, fn, x, every, s);
  if (rc < 0) return rc;
  const bool use_graph = (rc == SEM_OK);
  int launched = 0;
  for (;;) {
    if (use_graph) {
      SEM_HIP(hipGraphLaunch(c->graph[slot], s));
    } else {
      for (int it = 0; it < every; ++it) {
        rc = fn(c, x, s);
        if (rc != SEM_OK) return rc;
      }
    }
    launched += every;
    SEM_HIP(hipMemcpyAsync(host, st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    SEM_HIP(hipStreamSynchronize(s));
    if (host->done != semk::kRunning) return SEM_OK;
    if (launched > max_iter + every) return fail(SEM_ERR_HIP, "sem_cg: device state stopped advancing");
  }
}

}  // namespace

extern "C" {

const char *sem_last_error(void) { return g_last_error.c_str(); }

size_t sem_workspace_bytes(const sem_mesh_desc *desc) {
  std::string why;
  if (desc_check(desc, &why) != SEM_OK) return 0;
  return layout_of(desc).total;
}

int sem_rtc_build(int order, const char *arch, size_t *code_bytes) {
  if (!arch || !*arch) return fail(SEM_ERR_ARG, "sem_rtc_build: null or empty architecture");
  if (order < semk::kMinOrder) return fail(SEM_ERR_ARG, "sem_rtc_build: order must be >= 1");
  if (!semk::rtc_order(order))
    return fail(SEM_ERR_UNSUPPORTED, "sem_rtc_build: orders 13..15 are compiled at run time (1..12 are built)");
  if (!semk::rtc_arch_supported(arch))
    return fail(SEM_ERR_UNSUPPORTED, std::string("sem_rtc_build: architecture ") + arch + " is not gfx950");
  std::string why;
  size_t bytes = 0;
  const hipError_t e = semk::rtc_build(order, arch, &bytes, &why);
  if (e != hipSuccess) return fail(SEM_ERR_HIP, "sem_rtc_build: " + why);
  if (code_bytes) *code_bytes = bytes;
  return SEM_OK;
}

int sem_setup(const sem_mesh_desc *desc, void *dev_ws, size_t ws_bytes, void *stream,
              sem_ctx **out) {
  std::string why;
  if (!out) return fail(SEM_ERR_ARG, "sem_setup: null output handle");
  *out = nullptr;
  const int dc = desc_check(desc, &why);
  if (dc != SEM_OK) return fail(dc, "sem_setup: " + why);
  if (!dev_ws) return fail(SEM_ERR_ARG, "sem_setup: null workspace");
  if (((uintptr_t)dev_ws) % kAlign != 0) return fail(SEM_ERR_ARG, "sem_setup: workspace not 256-byte aligned");
  const Layout lay = layout_of(desc);
  if (ws_bytes < lay.total)
    return fail(SEM_ERR_NOMEM, "sem_setup: workspace has " + std::to_string(ws_bytes) +
                                   " bytes, needs " + std::to_string(lay.total));
  if (semk::rtc_order(desc->order)) {
    // kernels of this order: compiled now (or taken from the cache) and loaded
    std::string rwhy;
    const hipError_t re = semk::rtc_prepare(desc->order, &rwhy);
    if (re != hipSuccess) return hip_fail(re, ("sem_setup: run-time kernels: " + rwhy).c_str());
  }
  hipStream_t s = (hipStream_t)stream;
  sem_ctx *c = new sem_ctx();
  c->desc = *desc;
  c->box = box_of(desc);
  c->lay = lay;
  c->ws = (char *)dev_ws;
  c->ws_bytes = ws_bytes;
  c->D = (double *)(c->ws + lay.D);
  c->nodes = (double *)(c->ws + lay.nodes);
  c->G = (double *)(c->ws + lay.G);
  c->minv = (double *)(c->ws + lay.minv);
  c->r = (double *)(c->ws + lay.r);
  c->p = (double *)(c->ws + lay.p);
  c->w = (double *)(c->ws + lay.w);
  c->part_ax = (double *)(c->ws + lay.part_ax);
  c->part_rr = (double *)(c->ws + lay.part_rr);
  c->part_rz = (double *)(c->ws + lay.part_rz);
  c->st = (CgState *)(c->ws + lay.state);
  c->n_ax_blocks = c->box.E();
  c->n_vec_blocks = semk::vec_grid_blocks(c->box.L());
  c->n_upd_blocks = semk::upd_num_tiles(c->box, true);
  c->n_upd_blocks_in = semk::upd_num_tiles(c->box, false);
  c->op_impl[0] = c->op_impl[1] = desc->flags;
  c->upd_var[0] = c->upd_var[1] = 0;
  c->in_batch = 0;
  for (int slot = 0; slot < 2; ++slot) {
    c->graph[slot] = nullptr;
    c->graph_stream[slot] = nullptr;
    c->graph_x[slot] = nullptr;
    c->graph_minv[slot] = nullptr;
    c->graph_iters[slot] = 0;
  }
  c->cg_minv = c->minv;
  const bool lowp = desc->lowprec != SEM_F64;
  c->Dlo = lowp ? (float *)(c->ws + lay.Dlo) : nullptr;
  c->Glo = lowp ? (void *)(c->ws + lay.Glo) : nullptr;
  c->minv32 = lowp ? (float *)(c->ws + lay.minv32) : nullptr;
  c->e = lowp ? (float *)(c->ws + lay.e) : nullptr;
  c->rin = lowp ? (float *)(c->ws + lay.rin) : nullptr;
  c->pin = lowp ? (float *)(c->ws + lay.pin) : nullptr;
  c->win = lowp ? (float *)(c->ws + lay.win) : nullptr;
  c->st_in = lowp ? (CgState *)(c->ws + lay.state_in) : nullptr;

  const int N = desc->order;
  std::vector<double> xs, wq, D;
  gll_host(N, &xs, &wq);
  deriv_host(N, xs, &D);
  std::vector<double> nodes(xs);
  nodes.insert(nodes.end(), wq.begin(), wq.end());
  auto bail = [&](int rc) {
    delete c;
    return rc;
  };
  hipError_t e;
  if ((e = hipMemcpyAsync(c->D, D.data(), D.size() * sizeof(double), hipMemcpyHostToDevice, s)) != hipSuccess)
    return bail(hip_fail(e, "sem_setup: upload D"));
  if ((e = hipMemcpyAsync(c->nodes, nodes.data(), nodes.size() * sizeof(double), hipMemcpyHostToDevice, s)) != hipSuccess)
    return bail(hip_fail(e, "sem_setup: upload nodes"));
  // element-local diagonal into r (scratch), then Minv = 1 / (sum of copies)
  if ((e = semk::launch_setup_geom(c->box, desc->deform_amp, c->D, c->nodes, c->G, c->r, s)) != hipSuccess)
    return bail(hip_fail(e, "sem_setup: geometry kernel"));
  if ((e = semk::launch_gather(c->box, c->r, c->minv, semk::kGatherInverse, s)) != hipSuccess)
    return bail(hip_fail(e, "sem_setup: diagonal gather-scatter"));
  // low-precision copy: D rounded on the host, G and Minv rounded on the GPU
  std::vector<float> Dlo(D.size());
  if (lowp) {
    for (size_t q = 0; q < D.size(); ++q) {
      const float f = (float)D[q];
      Dlo[q] = desc->lowprec == SEM_BF16 ? semk::bf16_value(semk::bf16_bits(f)) : f;
    }
    if ((e = hipMemcpyAsync(c->Dlo, Dlo.data(), Dlo.size() * sizeof(float), hipMemcpyHostToDevice, s)) != hipSuccess)
      return bail(hip_fail(e, "sem_setup: upload rounded D"));
    const int64_t L = c->box.L();
    if ((e = semk::launch_convert_g(desc->lowprec, 6 * L, c->G, c->Glo, s)) != hipSuccess)
      return bail(hip_fail(e, "sem_setup: round G"));
    if ((e = semk::launch_convert_g(SEM_F32, L, c->minv, c->minv32, s)) != hipSuccess)
      return bail(hip_fail(e, "sem_setup: round Minv"));
  }
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return bail(hip_fail(e, "sem_setup: synchronize"));
  *out = c;
  return SEM_OK;
}

int sem_destroy(sem_ctx *ctx) {
  if (!ctx) return fail(SEM_ERR_ARG, "sem_destroy: null handle");
  if (ctx->in_batch) return fail(SEM_ERR_ARG, "sem_destroy: remove the context from its batch first");
  drop_graph(ctx, 0);
  drop_graph(ctx, 1);
  delete ctx;
  return SEM_OK;
}

int64_t sem_nlocal(const sem_ctx *ctx) { return ctx ? ctx->box.L() : -1; }

int sem_ax(sem_ctx *ctx, const double *u, double *w, int mode, void *stream) {
  if (!ctx) return fail(SEM_ERR_ARG, "sem_ax: null handle");
  if (!u || !w) return fail(SEM_ERR_ARG, "sem_ax: null vector");
  if (u == w) return fail(SEM_ERR_ARG, "sem_ax: u and w must differ");
  if (mode != SEM_AX_LOCAL && mode != SEM_AX_ASSEMBLED && mode != SEM_AX_MASKED)
    return fail(SEM_ERR_ARG, "sem_ax: mode must be SEM_AX_LOCAL, SEM_AX_ASSEMBLED or SEM_AX_MASKED");
  hipStream_t s = (hipStream_t)stream;
  if (mode == SEM_AX_LOCAL) {  // the result goes to the caller: streamed stores
    SEM_HIP(semk::launch_ax_f64(ctx->box, ctx->op_impl[0], ctx->D, ctx->G, const_cast<double *>(u), w, nullptr,
                                nullptr, nullptr, nullptr, nullptr, s, true));
    return SEM_OK;
  }
  // element-local result into the workspace, then the gather-scatter pull
  SEM_HIP(semk::launch_ax_f64(ctx->box, ctx->op_impl[0], ctx->D, ctx->G, const_cast<double *>(u), ctx->w, nullptr,
                              nullptr, nullptr, nullptr, nullptr, s));
  SEM_HIP(semk::launch_gather(ctx->box, ctx->w, w,
                              mode == SEM_AX_MASKED ? semk::kGatherMasked : semk::kGatherAssembled, s));
  return SEM_OK;
}

int sem_cg(sem_ctx *ctx, const double *b, double *x, const sem_cg_opts *opts, sem_cg_info *info,
           void *stream) {
  if (!ctx) return fail(SEM_ERR_ARG, "sem_cg: null handle");
  if (!b || !x || !opts || !info) return fail(SEM_ERR_ARG, "sem_cg: null argument");
  if (ctx->in_batch) return fail(SEM_ERR_ARG, "sem_cg: the context is a slot of a batch");
  if (b == x) return fail(SEM_ERR_ARG, "sem_cg: b and x must differ");
  if (opts->mixed && ctx->desc.lowprec == SEM_F64)
    return fail(SEM_ERR_ARG, "sem_cg: mixed precision needs a mesh set up with lowprec SEM_F32 or SEM_BF16");
  if (opts->mixed && opts->fixed_iter > 0)
    return fail(SEM_ERR_ARG, "sem_cg: mixed precision runs in tolerance mode only");
  if (opts->fixed_iter <= 0 && !(opts->rtol > 0.0))
    return fail(SEM_ERR_ARG, "sem_cg: rtol must be > 0 unless fixed_iter > 0");
  if (opts->precond != SEM_PRECOND_JACOBI && opts->precond != SEM_PRECOND_NONE)
    return fail(SEM_ERR_ARG, "sem_cg: precond must be SEM_PRECOND_JACOBI or SEM_PRECOND_NONE");
  if (opts->precond == SEM_PRECOND_NONE && opts->mixed)
    return fail(SEM_ERR_ARG, "sem_cg: the plain CG (SEM_PRECOND_NONE) runs in FP64 only");
  hipStream_t s = (hipStream_t)stream;
  // plain CG: a null Minv makes every CG kernel take z = r
  ctx->cg_minv = opts->precond == SEM_PRECOND_NONE ? nullptr : ctx->minv;
  const int max_iter = opts->fixed_iter > 0 ? opts->fixed_iter : (opts->max_iter > 0 ? opts->max_iter : 20000);
  int every = opts->check_every > 0 ? opts->check_every : 25;

  CgState &h = ctx->host_state;
  std::memset(&h, 0, sizeof(h));
  h.max_iter = opts->mixed ? (opts->max_iter > 0 ? opts->max_iter : 50) : max_iter;
  h.rtol2 = opts->fixed_iter > 0 ? -1.0 : opts->rtol * opts->rtol;
  SEM_HIP(hipMemcpyAsync(ctx->st, &h, sizeof(CgState), hipMemcpyHostToDevice, s));
  SEM_HIP(semk::launch_cg_init(ctx->box, b, x, ctx->r, ctx->p, ctx->cg_minv, ctx->st, ctx->part_rz,
                               ctx->part_rr, s));
  int status = SEM_OK;
  if (!opts->mixed) {
    if (every > max_iter) every = max_iter;
    int rc = run_until_done(ctx, 0, enqueue_cg_iteration, x, ctx->st, &h, every, max_iter, s);
    if (rc != SEM_OK) return rc;
    SEM_HIP(semk::launch_cg_finish(ctx->box, x, ctx->p, ctx->st, s));
    SEM_HIP(hipStreamSynchronize(s));
    info->iters = h.iter;
    info->outer_iters = 0;
  } else {
    // Inner-outer refinement: inner Jacobi-PCG with the rounded operator on
    // FP32 vectors, outer FP64 true residual and update.
    // defaults measured on the 32^3, N = 7 mesh: restarts cost convergence,
    // so the inner solve runs to a moderate tolerance with a generous cap
    const double eta = opts->inner_rtol > 0.0 ? opts->inner_rtol
                                              : (ctx->desc.lowprec == SEM_BF16 ? 1e-2 : 1e-3);
    const int inner_max = opts->inner_max > 0 ? opts->inner_max : kDefaultInnerMax;
    if (every > inner_max) every = inner_max;
    const Box &bx = ctx->box;
    int inner_total = 0;
    SEM_HIP(hipMemcpyAsync(&h, ctx->st, sizeof(CgState), hipMemcpyDeviceToHost, s));
    SEM_HIP(hipStreamSynchronize(s));
    while (h.done == semk::kRunning) {
      SEM_HIP(semk::launch_inner_start(bx, ctx->r, ctx->st, ctx->st_in, eta * eta, inner_max, ctx->rin,
                                       ctx->e, ctx->pin, ctx->minv32, ctx->part_rz, ctx->part_rr, s));
      CgState &hi = ctx->host_inner;
      int rc = run_until_done(ctx, 1, enqueue_inner_iteration, nullptr, ctx->st_in, &hi, every,
                              inner_max, s);
      if (rc != SEM_OK) return rc;
      inner_total += hi.iter;
      SEM_HIP(semk::launch_outer_correct(bx, x, ctx->e, ctx->pin, ctx->st_in, ctx->st, s));
      SEM_HIP(semk::launch_ax_f64(bx, ctx->op_impl[0], ctx->D, ctx->G, x, ctx->w, nullptr, nullptr, nullptr, nullptr,
                                  nullptr, s));
      SEM_HIP(semk::launch_outer_step(bx, b, ctx->w, ctx->r, ctx->st, ctx->part_rr, s));
      SEM_HIP(hipMemcpyAsync(&h, ctx->st, sizeof(CgState), hipMemcpyDeviceToHost, s));
      SEM_HIP(hipStreamSynchronize(s));
      if (hi.iter == 0 && h.done == semk::kRunning) {
        h.done = semk::kBreakdown;  // the inner solver made no progress
        break;
      }
    }
    info->iters = inner_total;
    info->outer_iters = h.iter;
  }
  info->rel_res = h.bnorm2 > 0.0 ? std::sqrt(h.rnorm2 / h.bnorm2) : 0.0;
  if (h.done == semk::kBreakdown) status = SEM_ERR_BREAKDOWN;
  else if (h.done == semk::kMaxIter && opts->fixed_iter <= 0) status = SEM_ERR_NOTCONV;
  info->status = status;
  if (status == SEM_ERR_BREAKDOWN) g_last_error = "sem_cg: breakdown (p^T A p <= 0, non-finite, or no inner progress)";
  if (status == SEM_ERR_NOTCONV) g_last_error = "sem_cg: iteration cap reached";
  return status;
}

int sem_ax_lowp(sem_ctx *ctx, const float *u, float *w, int mode, void *stream) {
  if (!ctx) return fail(SEM_ERR_ARG, "sem_ax_lowp: null handle");
  if (ctx->desc.lowprec == SEM_F64)
    return fail(SEM_ERR_ARG, "sem_ax_lowp: the mesh was set up without a low-precision copy");
  if (!u || !w) return fail(SEM_ERR_ARG, "sem_ax_lowp: null vector");
  if (u == w) return fail(SEM_ERR_ARG, "sem_ax_lowp: u and w must differ");
  if (mode != SEM_AX_LOCAL && mode != SEM_AX_ASSEMBLED && mode != SEM_AX_MASKED)
    return fail(SEM_ERR_ARG, "sem_ax_lowp: mode must be SEM_AX_LOCAL, SEM_AX_ASSEMBLED or SEM_AX_MASKED");
  hipStream_t s = (hipStream_t)stream;
  float *dst = mode == SEM_AX_LOCAL ? w : ctx->win;
  SEM_HIP(semk::launch_ax_lowp(ctx->box, ctx->desc.lowprec, ctx->op_impl[1], ctx->Dlo,
                               ctx->Glo, const_cast<float *>(u), dst, nullptr, nullptr, nullptr, nullptr,
                               nullptr, s, mode == SEM_AX_LOCAL));
  if (mode != SEM_AX_LOCAL)
    SEM_HIP(semk::launch_gather_f32(ctx->box, ctx->win, w,
                                    mode == SEM_AX_MASKED ? semk::kGatherMasked : semk::kGatherAssembled, s));
  return SEM_OK;
}

int vec_axpy(int64_t n, double alpha, const double *x, double *y, void *stream) {
  if (n < 0) return fail(SEM_ERR_ARG, "vec_axpy: n < 0");
  if (n > 0 && (!x || !y)) return fail(SEM_ERR_ARG, "vec_axpy: null vector");
  SEM_HIP(semk::launch_axpy(n, alpha, x, y, (hipStream_t)stream));
  return SEM_OK;
}

int sem_gs_csr_build(int64_t n, const int64_t *gid, int32_t *offsets, int64_t offsets_cap,
                     int32_t *ids, int64_t ids_cap, int32_t *n_rows, int64_t *n_copies) {
  if (n < 0 || n > INT32_MAX) return fail(SEM_ERR_ARG, "sem_gs_csr_build: n must be in [0, 2^31-1]");
  if (n > 0 && !gid) return fail(SEM_ERR_ARG, "sem_gs_csr_build: null id array");
  if (!n_rows || !n_copies) return fail(SEM_ERR_ARG, "sem_gs_csr_build: null size output");
  const char *why = "";
  int rc;
  try {
    rc = semk::build_gs_csr(n, gid, offsets, offsets_cap, ids, ids_cap, n_rows, n_copies, &why);
  } catch (const std::bad_alloc &) {
    return fail(SEM_ERR_NOMEM, "sem_gs_csr_build: out of host memory for the sort keys");
  }
  return rc == SEM_OK ? SEM_OK : fail(rc, why);
}

int sem_gs(int32_t n_rows, const int32_t *offsets, const int32_t *ids, int64_t n_copies, int64_t n,
           double *w, void *stream) {
  if (n_rows < 0) return fail(SEM_ERR_ARG, "sem_gs: n_rows < 0");
  if (n < 0) return fail(SEM_ERR_ARG, "sem_gs: n < 0");
  if (n_copies < 0 || n_copies > INT32_MAX) return fail(SEM_ERR_ARG, "sem_gs: n_copies must be in [0, 2^31-1]");
  if (n_rows > 0 && (!offsets || !ids || !w)) return fail(SEM_ERR_ARG, "sem_gs: null pointer");
  SEM_HIP(semk::launch_gs_rows(n_rows, offsets, ids, n_copies, n, w, (hipStream_t)stream));
  return SEM_OK;
}

size_t vec_dot_workspace_bytes(int64_t n) {
  if (n < 0) return 0;
  const int64_t nb = semk::vec_num_blocks(n);
  return (size_t)(nb > 0 ? nb : 1) * sizeof(double);
}

int vec_dot(int64_t n, const double *x, const double *y, const double *wt, double *out,
            void *dev_ws, size_t ws_bytes, void *stream) {
  if (n < 0) return fail(SEM_ERR_ARG, "vec_dot: n < 0");
  if (n > 0 && (!x || !y)) return fail(SEM_ERR_ARG, "vec_dot: null vector");
  if (!out) return fail(SEM_ERR_ARG, "vec_dot: null output");
  if (!dev_ws) return fail(SEM_ERR_ARG, "vec_dot: null workspace");
  if (((uintptr_t)dev_ws) % sizeof(double) != 0) return fail(SEM_ERR_ARG, "vec_dot: workspace not 8-byte aligned");
  if (ws_bytes < vec_dot_workspace_bytes(n)) return fail(SEM_ERR_NOMEM, "vec_dot: workspace too small");
  SEM_HIP(semk::launch_dot(n, x, y, wt, out, (double *)dev_ws, (hipStream_t)stream));
  return SEM_OK;
}

// ------------------------------------------------------------ kernel knobs
namespace {
// Candidates of a knob for an order and precision family (0 when invalid).
int knob_count(int order, int prec, int knob) {
  if (order < semk::kMinOrder || order > semk::kMaxRtcOrder) return 0;
  if (prec != SEM_F64 && prec != SEM_F32 && prec != SEM_BF16) return 0;
  if (semk::rtc_order(order)) return (prec == SEM_F64 && (knob == SEM_KNOB_OP_TILE || knob == SEM_KNOB_UPDATE_TILE)) ? 1 : 0;
  if (knob == SEM_KNOB_OP_TILE) return 3;
  if (knob == SEM_KNOB_UPDATE_TILE) {
    int n = 0;
    while (n < semk::kUpdVariants && semk::upd_variant_exists(order + 1, prec == SEM_F64, n)) ++n;
    return n;
  }
  return 0;
}
}  // namespace

int sem_knob_count(int order, int prec, int knob) { return knob_count(order, prec, knob); }

int sem_set_knob(sem_ctx *ctx, int prec, int knob, int value) {
  if (!ctx) return fail(SEM_ERR_ARG, "sem_set_knob: null handle");
  if (ctx->in_batch) return fail(SEM_ERR_ARG, "sem_set_knob: the context is a slot of a batch");
  if (prec != SEM_F64 && prec != ctx->desc.lowprec)
    return fail(SEM_ERR_ARG, "sem_set_knob: prec must be SEM_F64 or the context's low-precision copy");
  if (knob != SEM_KNOB_OP_TILE && knob != SEM_KNOB_UPDATE_TILE)
    return fail(SEM_ERR_ARG, "sem_set_knob: knob must be SEM_KNOB_OP_TILE or SEM_KNOB_UPDATE_TILE");
  const int n = knob_count(ctx->box.N, prec, knob);
  if (value < 0 || value >= n)
    return fail(SEM_ERR_UNSUPPORTED, "sem_set_knob: value " + std::to_string(value) + " outside the " +
                                         std::to_string(n) + " candidates of this order and precision");
  const int fam = prec == SEM_F64 ? 0 : 1;
  if (knob == SEM_KNOB_OP_TILE) {
    ctx->op_impl[fam] = value;
  } else {
    ctx->upd_var[fam] = value;
    if (fam == 0) ctx->n_upd_blocks = semk::upd_num_tiles(ctx->box, true, value);
    else ctx->n_upd_blocks_in = semk::upd_num_tiles(ctx->box, false, value);
  }
  drop_graph(ctx, 0);  // captured iterations hold the old kernels
  drop_graph(ctx, 1);
  return SEM_OK;
}

int sem_get_knob(const sem_ctx *ctx, int prec, int knob, int *value) {
  if (!ctx || !value) return fail(SEM_ERR_ARG, "sem_get_knob: null argument");
  if (prec != SEM_F64 && prec != ctx->desc.lowprec)
    return fail(SEM_ERR_ARG, "sem_get_knob: prec must be SEM_F64 or the context's low-precision copy");
  const int fam = prec == SEM_F64 ? 0 : 1;
  if (knob == SEM_KNOB_OP_TILE) *value = ctx->op_impl[fam];
  else if (knob == SEM_KNOB_UPDATE_TILE) *value = ctx->upd_var[fam];
  else return fail(SEM_ERR_ARG, "sem_get_knob: knob must be SEM_KNOB_OP_TILE or SEM_KNOB_UPDATE_TILE");
  return SEM_OK;
}

// ------------------------------------------------- specialisation study
namespace {
bool generic_block_ok(int block) { return block >= 64 && block <= 1024 && (block & (block - 1)) == 0; }
}  // namespace

int sem_ax_generic(sem_ctx *ctx, const double *u, double *w, void *stream) {
  if (!ctx) return fail(SEM_ERR_ARG, "sem_ax_generic: null handle");
  if (!u || !w) return fail(SEM_ERR_ARG, "sem_ax_generic: null vector");
  if (u == w) return fail(SEM_ERR_ARG, "sem_ax_generic: u and w must differ");
  if (ctx->box.N + 1 > semk::kGenericMaxN1)
    return fail(SEM_ERR_UNSUPPORTED, "sem_ax_generic: orders above " + std::to_string(semk::kGenericMaxN1 - 1) +
                                         " are not served by the run-time-order kernel");
  SEM_HIP(semk::launch_ax_generic(ctx->box, ctx->D, ctx->G, u, w, (hipStream_t)stream));
  return SEM_OK;
}

int vec_axpy_generic(int64_t n, double alpha, const double *x, double *y, int block, void *stream) {
  if (n < 0) return fail(SEM_ERR_ARG, "vec_axpy_generic: n < 0");
  if (n > 0 && (!x || !y)) return fail(SEM_ERR_ARG, "vec_axpy_generic: null vector");
  if (!generic_block_ok(block)) return fail(SEM_ERR_ARG, "vec_axpy_generic: block must be a power of two in [64, 1024]");
  SEM_HIP(semk::launch_axpy_generic(n, alpha, x, y, block, (hipStream_t)stream));
  return SEM_OK;
}

size_t vec_dot_generic_workspace_bytes(int64_t n, int block) {
  if (n < 0 || !generic_block_ok(block)) return 0;
  return (size_t)semk::generic_dot_groups(n, block) * sizeof(double);
}

int vec_dot_generic(int64_t n, const double *x, const double *y, const double *wt, double *out,
                    void *dev_ws, size_t ws_bytes, int block, void *stream) {
  if (n < 0) return fail(SEM_ERR_ARG, "vec_dot_generic: n < 0");
  if (n > 0 && (!x || !y)) return fail(SEM_ERR_ARG, "vec_dot_generic: null vector");
  if (!out) return fail(SEM_ERR_ARG, "vec_dot_generic: null output");
  if (!generic_block_ok(block)) return fail(SEM_ERR_ARG, "vec_dot_generic: block must be a power of two in [64, 1024]");
  if (!dev_ws) return fail(SEM_ERR_ARG, "vec_dot_generic: null workspace");
  if (((uintptr_t)dev_ws) % sizeof(double) != 0) return fail(SEM_ERR_ARG, "vec_dot_generic: workspace not 8-byte aligned");
  if (ws_bytes < vec_dot_generic_workspace_bytes(n, block))
    return fail(SEM_ERR_NOMEM, "vec_dot_generic: workspace too small");
  SEM_HIP(semk::launch_dot_generic(n, x, y, wt, out, (double *)dev_ws, block, (hipStream_t)stream));
  return SEM_OK;
}

int sem_export(sem_ctx *ctx, int field, double *dst, void *stream) {
  if (!ctx) return fail(SEM_ERR_ARG, "sem_export: null handle");
  if (!dst) return fail(SEM_ERR_ARG, "sem_export: null destination");
  hipStream_t s = (hipStream_t)stream;
  const size_t L = (size_t)ctx->box.L();
  const size_t n1 = (size_t)ctx->box.n1();
  switch (field) {
    case SEM_FIELD_G:
      SEM_HIP(hipMemcpyAsync(dst, ctx->G, 6 * L * sizeof(double), hipMemcpyDeviceToDevice, s));
      break;
    case SEM_FIELD_MINV:
      SEM_HIP(hipMemcpyAsync(dst, ctx->minv, L * sizeof(double), hipMemcpyDeviceToDevice, s));
      break;
    case SEM_FIELD_D:
      SEM_HIP(hipMemcpyAsync(dst, ctx->D, n1 * n1 * sizeof(double), hipMemcpyDeviceToDevice, s));
      break;
    case SEM_FIELD_NODES:
      SEM_HIP(hipMemcpyAsync(dst, ctx->nodes, 2 * n1 * sizeof(double), hipMemcpyDeviceToDevice, s));
      break;
    case SEM_FIELD_C:
      SEM_HIP(semk::launch_fill_c(ctx->box, dst, s));
      break;
    default:
      return fail(SEM_ERR_ARG, "sem_export: unknown field");
  }
  return SEM_OK;
}

}  // extern "C"

// ====================================================================== batches

struct sem_batch {
  int max_slots;
  semk::BatchSlot *d_slots;
  semk::BatchSched sched;
  semk::BatchStatus *d_status;
  std::vector<semk::BatchSlot> slots;  // host copies as uploaded at add/remove
  std::vector<sem_ctx *> ctx;          // null for a free slot
  std::vector<semk::BatchStatus> status;
  semk::BatchTiles tiles;
  hipGraphExec_t graph;
  // what the captured graph was built for: stream, iterations, the operator
  // bins it launches and the tiles
  hipStream_t graph_stream;
  int graph_iters;
  uint64_t graph_bins;
  semk::BatchTiles graph_tiles;
};

namespace {

struct BatchLayout {
  size_t slots, meta, slot, prefix, status, total;
};

BatchLayout batch_layout(int max_slots) {
  BatchLayout o;
  size_t at = 0;
  auto take = [&](size_t bytes) {
    const size_t off = at;
    at = align_up(at + bytes);
    return off;
  };
  const size_t bins = semk::kBatchLists;
  o.slots = take((size_t)max_slots * sizeof(semk::BatchSlot));
  o.meta = take(bins * 2 * sizeof(int));
  o.slot = take(bins * (size_t)max_slots * sizeof(int));
  o.prefix = take(bins * ((size_t)max_slots + 1) * sizeof(int));
  o.status = take((size_t)max_slots * sizeof(semk::BatchStatus));
  o.total = at;
  return o;
}

// Operator bins the occupied slots can use: an FP64 solve its order's FP64
// CG bin, a mixed solve its low-precision bin and its outer operator bin.
uint64_t batch_bins(const sem_batch *B) {
  uint64_t m = 0;
  for (int q = 0; q < B->max_slots; ++q) {
    if (!B->ctx[q]) continue;
    const semk::BatchSlot &S = B->slots[q];
    if (S.mixed)
      m |= (1ull << semk::batch_bin(3, S.N)) | (1ull << semk::batch_bin(S.mixed == SEM_F32 ? 1 : 2, S.N)) |
           (1ull << (semk::kBatchBins + 1));
    else
      m |= (1ull << semk::batch_bin(0, S.N)) | (1ull << semk::kBatchBins);
  }
  return m;
}

}  // namespace

extern "C" {

size_t sem_batch_workspace_bytes(int max_slots) {
  if (max_slots < 1 || max_slots > semk::kBatchMaxSlots) return 0;
  return batch_layout(max_slots).total;
}

int sem_batch_create(int max_slots, void *dev_ws, size_t ws_bytes, void *stream, sem_batch **out) {
  if (!out) return fail(SEM_ERR_ARG, "sem_batch_create: null output handle");
  *out = nullptr;
  if (max_slots < 1 || max_slots > semk::kBatchMaxSlots)
    return fail(SEM_ERR_ARG, "sem_batch_create: max_slots out of range (1..4096)");
  if (!dev_ws || ((uintptr_t)dev_ws) % kAlign != 0)
    return fail(SEM_ERR_ARG, "sem_batch_create: workspace null or not 256-byte aligned");
  const BatchLayout lay = batch_layout(max_slots);
  if (ws_bytes < lay.total) return fail(SEM_ERR_NOMEM, "sem_batch_create: workspace too small");
  hipError_t e = semk::batch_prepare();
  if (e != hipSuccess) return hip_fail(e, "sem_batch_create: occupancy query");
  hipStream_t s = (hipStream_t)stream;
  sem_batch *B = new sem_batch();
  char *ws = (char *)dev_ws;
  B->max_slots = max_slots;
  B->d_slots = (semk::BatchSlot *)(ws + lay.slots);
  B->sched.meta = (int *)(ws + lay.meta);
  B->sched.slot = (int *)(ws + lay.slot);
  B->sched.prefix = (int *)(ws + lay.prefix);
  B->sched.max_slots = max_slots;
  B->d_status = (semk::BatchStatus *)(ws + lay.status);
  B->slots.assign(max_slots, semk::BatchSlot());
  for (auto &S : B->slots) std::memset(&S, 0, sizeof(S));
  B->ctx.assign(max_slots, nullptr);
  B->status.assign(max_slots, semk::BatchStatus());
  std::memset(&B->tiles, 0, sizeof(B->tiles));
  for (int c = 0; c < semk::kBatchClasses; ++c)
    for (int n = 1; n <= semk::kBatchOrders; ++n) B->tiles.epb[c][n] = semk::batch_default_epb(c, n);
  B->graph = nullptr;
  B->graph_stream = nullptr;
  B->graph_iters = 0;
  B->graph_bins = 0;
  std::memset(&B->graph_tiles, 0, sizeof(B->graph_tiles));
  e = hipMemcpyAsync(B->d_slots, B->slots.data(), max_slots * sizeof(semk::BatchSlot),
                     hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    std::vector<semk::BatchStatus> zero(max_slots);
    std::memset(zero.data(), 0, zero.size() * sizeof(semk::BatchStatus));
    e = hipMemcpyAsync(B->d_status, zero.data(), zero.size() * sizeof(semk::BatchStatus),
                       hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  if (e != hipSuccess) {
    delete B;
    return hip_fail(e, "sem_batch_create: initialise slot table");
  }
  *out = B;
  return SEM_OK;
}

int sem_batch_set_tile(sem_batch *B, int prec, int order, int elements_per_item) {
  if (!B) return fail(SEM_ERR_ARG, "sem_batch_set_tile: null handle");
  const int cls = prec == SEM_F64 ? 0 : prec == SEM_F32 ? 1 : prec == SEM_BF16 ? 2 : -1;
  if (cls < 0) return fail(SEM_ERR_ARG, "sem_batch_set_tile: prec must be SEM_F64, SEM_F32 or SEM_BF16");
  if (order < semk::kMinOrder || order > semk::kBatchOrders ||
      !semk::batch_epb_supported(cls, order, elements_per_item))
    return fail(SEM_ERR_UNSUPPORTED, "sem_batch_set_tile: tile not compiled for this order");
  B->tiles.epb[cls][order] = elements_per_item;
  if (cls == 0) B->tiles.epb[3][order] = elements_per_item;  // the outer steps' FP64 operator
  return SEM_OK;
}

int sem_batch_add(sem_batch *B, sem_ctx *ctx, const double *b, double *x, const sem_cg_opts *opts,
                  int *slot_out, void *stream) {
  if (!B || !ctx || !b || !x || !opts || !slot_out) return fail(SEM_ERR_ARG, "sem_batch_add: null argument");
  if (ctx->in_batch) return fail(SEM_ERR_ARG, "sem_batch_add: the context is already in a batch");
  if (b == x) return fail(SEM_ERR_ARG, "sem_batch_add: b and x must differ");
  if (opts->fixed_iter > 0) return fail(SEM_ERR_ARG, "sem_batch_add: batches run in tolerance mode");
  if (opts->precond != SEM_PRECOND_JACOBI)
    return fail(SEM_ERR_ARG, "sem_batch_add: batches run Jacobi-PCG (precond must be SEM_PRECOND_JACOBI)");
  if (!(opts->rtol > 0.0)) return fail(SEM_ERR_ARG, "sem_batch_add: rtol must be > 0");
  if (opts->mixed && ctx->desc.lowprec == SEM_F64)
    return fail(SEM_ERR_ARG, "sem_batch_add: mixed precision needs a low-precision copy");
  if (ctx->box.N > 11) return fail(SEM_ERR_UNSUPPORTED, "sem_batch_add: batches take orders 1..11");
  if (ctx->desc.flags != 0 || ctx->op_impl[0] != 0 || ctx->op_impl[1] != 0 || ctx->upd_var[0] != 0 ||
      ctx->upd_var[1] != 0)
    return fail(SEM_ERR_ARG, "sem_batch_add: batches run the default kernels (flags 0, no knob set)");
  int q = -1;
  for (int i = 0; i < B->max_slots; ++i)
    if (!B->ctx[i]) {
      q = i;
      break;
    }
  if (q < 0) return fail(SEM_ERR_NOMEM, "sem_batch_add: no free slot");
  hipStream_t s = (hipStream_t)stream;
  const Box &bx = ctx->box;
  // start the solve exactly as sem_cg does
  CgState &h = ctx->host_state;
  std::memset(&h, 0, sizeof(h));
  h.max_iter = opts->mixed ? (opts->max_iter > 0 ? opts->max_iter : 50)
                           : (opts->max_iter > 0 ? opts->max_iter : 20000);
  h.rtol2 = opts->rtol * opts->rtol;
  SEM_HIP(hipMemcpyAsync(ctx->st, &h, sizeof(CgState), hipMemcpyHostToDevice, s));
  SEM_HIP(semk::launch_cg_init(bx, b, x, ctx->r, ctx->p, ctx->minv, ctx->st, ctx->part_rz,
                               ctx->part_rr, s));
  SEM_HIP(hipMemcpyAsync(&h, ctx->st, sizeof(CgState), hipMemcpyDeviceToHost, s));
  SEM_HIP(hipStreamSynchronize(s));

  semk::BatchSlot S;
  std::memset(&S, 0, sizeof(S));
  S.box = bx;
  S.N = bx.N;
  S.vtiles = (int)semk::vec_num_blocks(bx.L());
  S.mixed = opts->mixed ? ctx->desc.lowprec : 0;
  S.active = 1;
  S.inner_total = 0;
  S.inner_max = opts->inner_max > 0 ? opts->inner_max : kDefaultInnerMax;
  const double eta = opts->inner_rtol > 0.0 ? opts->inner_rtol
                                            : (ctx->desc.lowprec == SEM_BF16 ? 1e-2 : 1e-3);
  S.eta2 = eta * eta;
  S.E = bx.E();
  S.L = bx.L();
  S.utiles = (int)semk::upd_num_tiles(bx, S.mixed == 0);
  S.D = ctx->D;
  S.G = ctx->G;
  S.b = b;
  S.minv = ctx->minv;
  S.r = ctx->r;
  S.p = ctx->p;
  S.w = ctx->w;
  S.x = x;
  S.Dlo = ctx->Dlo;
  S.Glo = ctx->Glo;
  S.minv32 = ctx->minv32;
  S.e = ctx->e;
  S.rin = ctx->rin;
  S.pin = ctx->pin;
  S.win = ctx->win;
  S.st = ctx->st;
  S.st_in = ctx->st_in;
  S.part_el = ctx->part_ax;
  S.part_rr = ctx->part_rr;
  S.part_rz = ctx->part_rz;
  if (h.done != semk::kRunning) S.phase = semk::kPhaseFinished;
  else S.phase = S.mixed ? semk::kPhaseRestart : semk::kPhaseFp64;
  semk::BatchStatus st0;
  std::memset(&st0, 0, sizeof(st0));
  st0.phase = S.phase;
  st0.done = h.done;
  st0.rnorm2 = h.rnorm2;
  st0.bnorm2 = h.bnorm2;
  SEM_HIP(hipMemcpyAsync(B->d_slots + q, &S, sizeof(S), hipMemcpyHostToDevice, s));
  SEM_HIP(hipMemcpyAsync(B->d_status + q, &st0, sizeof(st0), hipMemcpyHostToDevice, s));
  SEM_HIP(hipStreamSynchronize(s));
  B->slots[q] = S;
  B->ctx[q] = ctx;
  ctx->in_batch = 1;
  *slot_out = q;
  return SEM_OK;
}

int sem_batch_step(sem_batch *B, int iters, void *stream) {
  if (!B) return fail(SEM_ERR_ARG, "sem_batch_step: null handle");
  if (iters < 1) return fail(SEM_ERR_ARG, "sem_batch_step: iters must be >= 1");
  hipStream_t s = (hipStream_t)stream;
  const uint64_t bins = batch_bins(B);
  const bool same = B->graph && B->graph_stream == s && B->graph_iters == iters &&
                    B->graph_bins == bins &&
                    std::memcmp(&B->graph_tiles, &B->tiles, sizeof(B->tiles)) == 0;
  if (s != nullptr && !same) {
    if (B->graph) (void)hipGraphExecDestroy(B->graph);
    B->graph = nullptr;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed) == hipSuccess) {
      hipError_t e = hipSuccess;
      for (int it = 0; it < iters && e == hipSuccess; ++it)
        e = semk::launch_batch_iteration(B->d_slots, B->max_slots, B->sched, B->tiles, bins,
                                         B->d_status, s);
      hipGraph_t g = nullptr;
      hipError_t e2 = hipStreamEndCapture(s, &g);
      if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(e != hipSuccess ? e : e2, "sem_batch_step: capture");
      }
      hipGraphExec_t ex = nullptr;
      e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return hip_fail(e, "sem_batch_step: instantiate");
      B->graph = ex;
      B->graph_stream = s;
      B->graph_iters = iters;
      B->graph_bins = bins;
      B->graph_tiles = B->tiles;
    } else {
      (void)hipGetLastError();
    }
  }
  if (s != nullptr && B->graph && B->graph_stream == s && B->graph_iters == iters &&
      B->graph_bins == bins) {
    SEM_HIP(hipGraphLaunch(B->graph, s));
  } else {
    for (int it = 0; it < iters; ++it)
      SEM_HIP(semk::launch_batch_iteration(B->d_slots, B->max_slots, B->sched, B->tiles, bins,
                                           B->d_status, s));
  }
  return SEM_OK;
}

int sem_batch_poll(sem_batch *B, int *finished, int cap, int *n_finished, sem_cg_info *infos,
                   int *n_active, void *stream) {
  if (!B || !n_finished) return fail(SEM_ERR_ARG, "sem_batch_poll: null argument");
  if (cap > 0 && (!finished || !infos)) return fail(SEM_ERR_ARG, "sem_batch_poll: null output arrays");
  hipStream_t s = (hipStream_t)stream;
  SEM_HIP(hipMemcpyAsync(B->status.data(), B->d_status, B->max_slots * sizeof(semk::BatchStatus),
                         hipMemcpyDeviceToHost, s));
  SEM_HIP(hipStreamSynchronize(s));
  int nf = 0, na = 0;
  for (int q = 0; q < B->max_slots; ++q) {
    if (!B->ctx[q]) continue;
    ++na;
    const semk::BatchStatus &st = B->status[q];
    if (st.phase != semk::kPhaseFinished) continue;
    if (nf < cap) {
      finished[nf] = q;
      sem_cg_info &info = infos[nf];
      info.iters = st.iters;
      info.outer_iters = st.outer_iters;
      info.rel_res = st.bnorm2 > 0.0 ? std::sqrt(st.rnorm2 / st.bnorm2) : 0.0;
      info.status = st.done == semk::kBreakdown ? SEM_ERR_BREAKDOWN
                    : st.done == semk::kMaxIter ? SEM_ERR_NOTCONV : SEM_OK;
      info.reserved = 0;
    }
    ++nf;
  }
  *n_finished = nf < cap ? nf : (cap > 0 ? cap : 0);
  if (n_active) *n_active = na;
  return SEM_OK;
}

int sem_batch_remove(sem_batch *B, int slot, void *stream) {
  if (!B) return fail(SEM_ERR_ARG, "sem_batch_remove: null handle");
  if (slot < 0 || slot >= B->max_slots || !B->ctx[slot]) return fail(SEM_ERR_ARG, "sem_batch_remove: no such slot");
  hipStream_t s = (hipStream_t)stream;
  semk::BatchSlot S;
  std::memset(&S, 0, sizeof(S));
  SEM_HIP(hipMemcpyAsync(B->d_slots + slot, &S, sizeof(S), hipMemcpyHostToDevice, s));
  SEM_HIP(hipStreamSynchronize(s));
  B->slots[slot] = S;
  B->ctx[slot]->in_batch = 0;
  B->ctx[slot] = nullptr;
  return SEM_OK;
}

int sem_batch_destroy(sem_batch *B) {
  if (!B) return fail(SEM_ERR_ARG, "sem_batch_destroy: null handle");
  for (auto *c : B->ctx)
    if (c) c->in_batch = 0;
  if (B->graph) (void)hipGraphExecDestroy(B->graph);
  delete B;
  return SEM_OK;
}

}  // extern "C"
