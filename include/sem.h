/*
 * sem.h - C ABI of the MI355X spectral-element Poisson library (libsem.so).
 *
 * The library applies the matrix-free high-order spectral-element Poisson
 * operator of the Nekbone workload (paper Sec. VIII-A: a 3-D Poisson problem
 * on a box of E hexahedra with (N+1)^3 Gauss-Lobatto-Legendre nodes each,
 * solved by Jacobi-preconditioned CG; the operator is the "ax" kernel of
 * Sec. VIII-B, the assembly is the "gs" gather-scatter of Sec. V-B) and runs
 * that CG on one GPU.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Return value: 0 (SEM_OK) or a negative SEM_ERR_* code.  Nothing throws or
 *    aborts.  sem_last_error() returns a thread-local text for the last error.
 *  - Arguments are validated before any launch; on SEM_ERR_ARG nothing was
 *    enqueued.
 *  - Pointers named *_dev are device pointers (HBM).  The library allocates
 *    no device memory: every device buffer, including the workspace, belongs
 *    to the caller and must stay alive while work that uses it is pending.
 *    (The one library-owned buffer is the fixed partials array of
 *    vec_dot_noalloc, part of the library's code object.)
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls are asynchronous on that stream unless stated otherwise.
 *  - "L-vector": element-local storage of a nodal field, E*(N+1)^3 doubles,
 *    index  e*(N+1)^3 + i + (N+1)*(j + (N+1)*k)  with i (the r direction)
 *    fastest and  e = ex + nelx*(ey + nely*ez).  Node (i,j,k) of element
 *    (ex,ey,ez) is the global lattice point (ex*N+i, ey*N+j, ez*N+k); nodes
 *    on shared faces, edges and corners have one copy per element.
 *  - The mesh is the box [0,1]^3 split into nelx*nely*nelz equal hexahedra;
 *    deform_amp != 0 adds amp*sin(2 pi X)sin(2 pi Y)sin(2 pi Z) (at the
 *    undeformed point X) to all three coordinates.  Homogeneous Dirichlet
 *    conditions hold on every box face.
 */
#ifndef SEM_H
#define SEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum sem_status {
  SEM_OK = 0,
  SEM_ERR_ARG = -1,         /* invalid argument (null pointer, size, order)  */
  SEM_ERR_HIP = -2,         /* a HIP runtime call failed; text in last_error  */
  SEM_ERR_NOMEM = -3,       /* caller workspace smaller than required         */
  SEM_ERR_NOTCONV = -4,     /* CG hit its iteration cap before the tolerance  */
  SEM_ERR_BREAKDOWN = -5,   /* CG found p^T A p <= 0 or a non-finite scalar   */
  SEM_ERR_UNSUPPORTED = -6  /* order or precision outside the compiled set    */
};

/* Arithmetic of the optional low-precision operator copy. */
enum sem_prec { SEM_F64 = 0, SEM_F32 = 1, SEM_BF16 = 2 };

/* What sem_ax returns (the Poisson operator of Sec. VIII-B with or without
 * the gather-scatter of Sec. V-B):
 *   SEM_AX_LOCAL     w = A_L u           element-by-element operator only
 *   SEM_AX_ASSEMBLED w = Q Q^T A_L u     copies of a shared node summed
 *   SEM_AX_MASKED    w = mask o Q Q^T A_L u   (the A of the CG)             */
enum sem_ax_mode { SEM_AX_LOCAL = 0, SEM_AX_ASSEMBLED = 1, SEM_AX_MASKED = 3 };

/* Fields sem_export can copy out (setup results, for inspection). */
enum sem_field {
  SEM_FIELD_G = 0,     /* geometric factors, E x 6 x (N+1)^3 doubles, per element
                          the planes rr, rs, rt, ss, st, tt;
                          G = w_i w_j w_k det(J) J^-1 J^-T at each node          */
  SEM_FIELD_MINV = 1,  /* Jacobi inverse diagonal, L doubles (0 on the boundary) */
  SEM_FIELD_D = 2,     /* 1-D derivative matrix, (N+1)^2 doubles, D[a*(N+1)+b] =
                          l_b'(xi_a)                                            */
  SEM_FIELD_NODES = 3, /* GLL nodes xi_0..xi_N then weights w_0..w_N            */
  SEM_FIELD_C = 4      /* inverse multiplicity 1/mult, L doubles                */
};

typedef struct sem_ctx sem_ctx;  /* opaque host-side handle */

typedef struct {
  int32_t nelx, nely, nelz; /* elements per direction, each >= 1               */
  int32_t order;            /* polynomial order N: 1..12 (kernels built with the
                               library), 13..15 (kernels compiled at set-up
                               for the device, FP64 and the matrix-core tile
                               only); else SEM_ERR_UNSUPPORTED                 */
  double deform_amp;        /* 0 = affine elements                              */
  int32_t lowprec;          /* SEM_F64 (none), SEM_F32 or SEM_BF16: also keep a
                               rounded copy of G for the inner solver of the
                               mixed-precision CG                              */
  int32_t flags;            /* which element kernel the operators of this mesh
                               run (FP64 and the low-precision copy):
                               0: the faster one for the order and precision
                                  as measured on MI355X (matrix cores from
                                  N = 7 in FP64 and FP32 and from N = 9 in
                                  BF16, vector ALUs below);
                               SEM_FLAG_MFMA: always the matrix-core kernel
                                  (D contractions as f64 MFMA, or f32 / bf16
                                  MFMA with FP32 accumulation);
                               SEM_FLAG_VALU: always the vector-ALU kernel.
                               Results agree up to rounding order. */
} sem_mesh_desc;

enum { SEM_FLAG_MFMA = 1, SEM_FLAG_VALU = 2 };

/* Device bytes sem_setup needs for this mesh (0 if the descriptor is invalid
 * or unsupported): the problem data of Sec. VIII-A (G, the Jacobi diagonal,
 * D) plus the CG vectors and reduction scratch.  It is the footprint a
 * scheduler admits a solve by.  Host only. */
size_t sem_workspace_bytes(const sem_mesh_desc *desc);

/* Build the operator of `desc` in the caller's workspace (the set-up of the
 * Poisson problem, Sec. VIII-A: a box of E hexahedra with (N+1)^3 nodes each;
 * the derivative matrices that depend on N, Sec. III): GLL nodes and D on
 * the host, then on the GPU the mesh coordinates, the isoparametric metric G,
 * the Jacobi diagonal (summed over copies) and its inverse.  `dev_ws` must be
 * 256-byte aligned and hold sem_workspace_bytes(desc) bytes.  Synchronous:
 * returns after the stream has finished the setup.  For orders 13..15 the
 * per-order kernels are first compiled for the current device with hipRTC
 * (N a compile-time constant, as in the built kernels: the jit clause of
 * Sec. IV), or taken from the process's cache or the disk cache
 * ($SEM_RTC_CACHE, else $XDG_CACHE_HOME/libsem or $HOME/.cache/libsem); a
 * compile failure returns SEM_ERR_HIP with the compiler log in
 * sem_last_error().  Errors: SEM_ERR_ARG (malformed descriptor, null or
 * misaligned workspace), SEM_ERR_UNSUPPORTED (order or precision outside
 * what the kernels serve), SEM_ERR_NOMEM (workspace too small), SEM_ERR_HIP.
 * On success *out is a new handle (free with sem_destroy); the workspace
 * belongs to it until then. */
int sem_setup(const sem_mesh_desc *desc, void *dev_ws, size_t ws_bytes, void *stream,
              sem_ctx **out);

/* Compile and cache, without a GPU, the per-order kernels of an order in
 * 13..15 for the architecture `arch` ("gfx950", optionally with a feature
 * suffix such as ":sramecc+:xnack-"), as sem_setup does on first use of
 * that order; *code_bytes (may be NULL) receives the code object's size.
 * SEM_ERR_UNSUPPORTED for orders 1..12 (built with the library), above 15
 * and for any other architecture; SEM_ERR_HIP with the compiler log on a
 * compile failure. */
int sem_rtc_build(int order, const char *arch, size_t *code_bytes);

/* Free the host handle (and any captured CG graph).  Never frees dev_ws. */
int sem_destroy(sem_ctx *ctx);

/* L = E*(N+1)^3, or -1 for a null handle. */
int64_t sem_nlocal(const sem_ctx *ctx);

/* w = A u as selected by `mode` (enum sem_ax_mode), u and w L-vectors of
 * doubles on the device, u != w.  u may be discontinuous for SEM_AX_LOCAL. */
int sem_ax(sem_ctx *ctx, const double *u_dev, double *w_dev, int mode, void *stream);

/* w = A_lo u with the low-precision operator copy of a mesh set up with
 * desc.lowprec = SEM_F32 or SEM_BF16 (else SEM_ERR_ARG).  u and w are FP32
 * L-vectors on the device, u != w; `mode` as for sem_ax.  A_lo uses D and G
 * rounded to the copy's type (round to nearest even); in SEM_BF16 both
 * contraction inputs (u and the G-weighted gradient) are also rounded to
 * bfloat16, so products are exact and only the FP32 accumulation rounds.
 * This is the inner operator of the mixed-precision sem_cg. */
int sem_ax_lowp(sem_ctx *ctx, const float *u_dev, float *w_dev, int mode, void *stream);

/* Options of sem_cg. */
typedef struct {
  double rtol;         /* stop when ||r||_c <= rtol*||b||_c (tolerance mode)    */
  int32_t max_iter;    /* iteration cap in tolerance mode (<=0: 20000)          */
  int32_t fixed_iter;  /* > 0: run exactly this many iterations, no tolerance   */
  int32_t mixed;       /* 0: FP64 PCG.  1: inner-outer refinement: an inner
                          Jacobi-PCG with the low-precision operator copy on
                          FP32 vectors (needs desc.lowprec) solves
                          A_lo e = r/||r||_c to inner_rtol; then x += ||r||_c e
                          and r = b - A x in FP64; repeat until rtol.
                          max_iter then caps the outer steps (<=0: 50).     */
  int32_t check_every; /* iterations per captured graph replay (<=0: 25)        */
  double inner_rtol;   /* mixed: inner relative tolerance (<=0: 1e-3 for SEM_F32,
                          1e-2 for SEM_BF16)                                   */
  int32_t inner_max;   /* mixed: inner iteration cap per outer step (<=0: 5000) */
  int32_t precond;     /* SEM_PRECOND_JACOBI (0): z = Minv r with the inverse
                          diagonal of A.  SEM_PRECOND_NONE (1): plain CG, z = r
                          (the unpreconditioned CG of Sec. VIII-A); FP64 only
                          (SEM_ERR_ARG with mixed, and in batches)            */
} sem_cg_opts;

enum { SEM_PRECOND_JACOBI = 0, SEM_PRECOND_NONE = 1 };

typedef struct {
  int32_t iters;        /* CG iterations (mixed: total inner iterations)       */
  int32_t outer_iters;  /* mixed: outer refinement steps (else 0)              */
  int32_t status;       /* SEM_OK, SEM_ERR_NOTCONV or SEM_ERR_BREAKDOWN        */
  int32_t reserved;
  double rel_res;       /* final ||r||_c/||b||_c (recursive; mixed: true FP64) */
} sem_cg_info;

/* Jacobi-PCG (or plain CG, opts->precond) for A x = b (Sec. VIII-A) with x_0 = 0, c-weighted dots
 * <x,y>_c = sum_i x_i y_i / mult_i, scalars kept on the device.  b and x are
 * L-vectors (b continuous; boundary entries are ignored), x is overwritten.
 * Blocking: returns when the solve has finished; polls one small status word
 * every check_every iterations.  The return value equals info->status. */
int sem_cg(sem_ctx *ctx, const double *b_dev, double *x_dev, const sem_cg_opts *opts,
           sem_cg_info *info, void *stream);

/* y <- alpha*x + y over n doubles (a streaming update of CG, Sec. VIII-B).
 * n >= 0; x and y device pointers (may be null only when n == 0). */
int vec_axpy(int64_t n, double alpha, const double *x_dev, double *y_dev, void *stream);

/* Device scratch vec_dot needs for length n. */
size_t vec_dot_workspace_bytes(int64_t n);

/* *out_dev <- sum_i wt_i x_i y_i (wt_dev may be NULL: weight 1), a two-stage
 * tree reduction (Sec. VIII-B) in a fixed order: the result depends only on n
 * and the data, so repeated calls are bitwise identical.  out_dev is one
 * device double; dev_ws holds vec_dot_workspace_bytes(n) bytes. */
int vec_dot(int64_t n, const double *x_dev, const double *y_dev, const double *wt_dev,
            double *out_dev, void *dev_ws, size_t ws_bytes, void *stream);

/* vec_dot without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same kernels and the same summation order as vec_dot,
 * so the result is bitwise that of vec_dot on the same data.  The per-tile
 * partials live in a library-owned array of 512 KiB of device memory per
 * GPU (allocated with the library's code object, held until the process
 * ends); its address on the current device is looked up on the first call
 * there.  The call itself allocates nothing.
 * n <= 134217728 (65536 partials of 2048 entries), else SEM_ERR_ARG with
 * nothing enqueued.  The stream must belong to the current device (NULL:
 * the current device's null stream).  Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (different streams, or
 * different host threads) race and must be serialised by the caller.
 * Nothing in the array needs clearing between calls. */
int vec_dot_noalloc(int64_t n, const double *x_dev, const double *y_dev, const double *wt_dev,
                    double *out_dev, void *stream);

/* Generic gather-scatter (the "gs" kernel of paper Sec. V-B: a loop over the
 * unique ids of shared nodes, and for each an inner loop over its copies) for
 * any map of L-vector entries to global ids, e.g. a periodic box or an
 * unstructured mesh.  The box mesh's sem_ax and sem_cg do not need it.
 *
 * sem_gs_csr_build (host only, synchronous, no HIP call) turns n global ids
 * gid_host[0..n-1] (each in [0, 2^31-1], n <= 2^31-1, host memory) into
 * compressed rows: one row per id that occurs at least twice, rows in
 * ascending id order, a row's copies (L indices) in ascending order.
 * Row r's copies are ids_host[offsets_host[r] .. offsets_host[r+1]-1].
 * With offsets_host = ids_host = NULL it only sets *n_rows and *n_copies;
 * otherwise offsets_host holds offsets_cap >= *n_rows + 1 entries and
 * ids_host ids_cap >= *n_copies entries (else SEM_ERR_NOMEM).  All buffers
 * belong to the caller.  The sort takes 8 bytes of host memory per entry;
 * if that allocation fails the call returns SEM_ERR_NOMEM. */
int sem_gs_csr_build(int64_t n, const int64_t *gid_host, int32_t *offsets_host, int64_t offsets_cap,
                     int32_t *ids_host, int64_t ids_cap, int32_t *n_rows, int64_t *n_copies);

/* w <- Q Q^T w over the rows: every copy of a row receives the sum of the
 * row's copies, added in row order starting from 0 in FP64; entries in no
 * row are unchanged.  offsets_dev (n_rows + 1 int32) and ids_dev (n_copies
 * int32, n_copies = offsets[n_rows]) are device copies of what
 * sem_gs_csr_build produced; w_dev holds n doubles.  Rows must be disjoint
 * (as built): rows sharing an entry race.  Bad input is skipped, never
 * dereferenced: a row whose offsets fall outside [0, n_copies] (or decrease)
 * is left alone, and an id outside [0, n) is ignored.  Asynchronous on
 * stream; the result is bitwise independent of the launch. */
int sem_gs(int32_t n_rows, const int32_t *offsets_dev, const int32_t *ids_dev, int64_t n_copies,
           int64_t n, double *w_dev, void *stream);


/* ------------------------------------------------------------ kernel knobs
 * Tuning hooks (the launch-shape choices the paper's transformation scripts
 * make from the device context, Sec. V-B, Tab. context_params).  Each knob
 * has candidates 0 .. sem_knob_count() - 1, all compiled with the library;
 * 0 is the default (what measured fastest on MI355X).  They change the
 * kernels a context runs, not what it computes: results agree up to the
 * rounding order of the sums.
 *   SEM_KNOB_OP_TILE      the element operator's tile: 0 default, 1 the
 *                         matrix-core tile, 2 the vector-ALU tile (as
 *                         sem_mesh_desc.flags, per precision family);
 *   SEM_KNOB_UPDATE_TILE  the shape of the CG update tile (the gather-scatter
 *                         fused into r -= alpha A p): threads per (i, j)
 *                         column, elements per tile, plane ranges.
 * `prec` names the family: SEM_F64 for the FP64 operator and update (sem_ax,
 * the FP64 CG and the outer steps of the mixed one), SEM_F32 or SEM_BF16 for
 * the inner operator and update of the mixed CG.  Orders 13..15 have the
 * default only. */
enum sem_knob { SEM_KNOB_OP_TILE = 0, SEM_KNOB_UPDATE_TILE = 1 };

/* Number of candidates of `knob` for an order and precision family; 0 for
 * an invalid combination.  Host only. */
int sem_knob_count(int order, int prec, int knob);

/* Select candidate `value` of `knob` for the family `prec` of ctx (SEM_F64,
 * or ctx's low-precision copy).  The next sem_ax / sem_cg call runs it (a
 * captured CG graph is dropped).  SEM_ERR_UNSUPPORTED for a value outside
 * the candidates; SEM_ERR_ARG for a context in a batch (batches run the
 * defaults, and sem_batch_add refuses a context with a knob set). */
int sem_set_knob(sem_ctx *ctx, int prec, int knob, int value);

/* The current value of a knob. */
int sem_get_knob(const sem_ctx *ctx, int prec, int knob, int *value);

/* ------------------------------------------------- specialisation study
 * The paper compares kernels whose run-time values (the order N in the
 * Poisson operator, the work-group size of the streaming kernels, the
 * unrolled in-group reduction) are fixed in the generated code with a HIP
 * implementation that leaves them variable (Sec. VIII-B, Tab. hip_vs_hip).
 * These entry points are that variable form of three kernels, for timing
 * against sem_ax (SEM_AX_LOCAL), vec_axpy and vec_dot; the solver never
 * calls them.  Same results up to rounding order.
 *
 * sem_ax_generic: w = A_L u (element-local, as sem_ax with SEM_AX_LOCAL)
 * with one kernel for every order, N a kernel argument: the vector-ALU
 * column mapping with run-time loop bounds and LDS tiles sized at launch.
 * Orders 1..11 (else SEM_ERR_UNSUPPORTED); u != w, L-vectors of doubles. */
int sem_ax_generic(sem_ctx *ctx, const double *u_dev, double *w_dev, void *stream);

/* y <- alpha*x + y with the work-group size `block` (a power of two in
 * [64, 1024], else SEM_ERR_ARG) chosen at launch, one entry per thread and
 * grid-stride step. */
int vec_axpy_generic(int64_t n, double alpha, const double *x_dev, double *y_dev, int block,
                     void *stream);

/* Device scratch vec_dot_generic needs for (n, block); 0 if invalid. */
size_t vec_dot_generic_workspace_bytes(int64_t n, int block);

/* *out_dev <- sum_i wt_i x_i y_i with the work-group size `block` chosen at
 * launch and the in-group tree as a loop over halving strides (a barrier per
 * level); two launches (partials, then one group over them).  Deterministic
 * for fixed (n, block). */
int vec_dot_generic(int64_t n, const double *x_dev, const double *y_dev, const double *wt_dev,
                    double *out_dev, void *dev_ws, size_t ws_bytes, int block, void *stream);

/* Copy a setup field (enum sem_field) into dst_dev, which must hold the size
 * listed with the field. */
int sem_export(sem_ctx *ctx, int field, double *dst_dev, void *stream);

/* ------------------------------------------------------------------ batches
 * Many independent solves (different meshes, orders 1..11, FP64 or mixed
 * precision) advance together: each batched step runs one CG iteration of
 * every active solve.  A one-work-group schedule kernel first builds, on the
 * device, compact work lists of the solves that have operator work in each
 * (arithmetic class, order) bin, of their CG update tiles per order and of
 * the streaming tiles of the solves in an outer-residual phase; then one
 * persistent operator launch per bin in use and one update launch per order
 * and family in use (each compiled for its order), one work-group per solve
 * for the scalars, and the finishing launches over lists rebuilt after the
 * scalars have set each solve's phase.  Every solve's arithmetic and
 * reduction order are those of sem_cg, so an FP64 solve gives the same bits
 * in a batch as alone.
 * Solves join and leave between steps (continuous batching); the step's
 * graph is captured again only when the set of bins in use or the tiles
 * change.  The batch holds no memory of its own on the device beyond its
 * workspace; each solve keeps its state in its sem_ctx workspace.  Calls on
 * one batch must not overlap. */
typedef struct sem_batch sem_batch;

/* Workspace of a batch of up to max_slots solves (1..4096): slot table, the
 * work lists (69 lists of max_slots entries with prefix sums), status
 * records.  0 for an invalid max_slots. */
size_t sem_batch_workspace_bytes(int max_slots);

/* Create a batch in `dev_ws` (256-byte aligned).  Synchronous. */
int sem_batch_create(int max_slots, void *dev_ws, size_t ws_bytes, void *stream, sem_batch **out);

/* Elements per operator item for one precision (SEM_F64 for FP64 solves and
 * the outer steps of mixed ones, SEM_F32 / SEM_BF16 for inner iterations) and
 * order (autotuner hook; applies from the next step on, to every solve of
 * that order: the bits do not depend on it).  SEM_ERR_UNSUPPORTED for a tile
 * that is not compiled.  A batch runs the default element kernel of each
 * precision and order (see sem_mesh_desc.flags); sem_batch_add refuses a
 * context set up with a forced kernel. */
int sem_batch_set_tile(sem_batch *batch, int prec, int order, int elements_per_item);

/* Start the solve of A x = b on ctx (tolerance mode, opts as for sem_cg;
 * opts->mixed needs ctx's low-precision copy) in a free slot.  b and x must
 * stay valid until the slot is removed; x holds the solution once the slot
 * reports finished.  The context cannot run sem_cg or join another batch
 * until it is removed.  Synchronous.  *slot receives the slot index. */
int sem_batch_add(sem_batch *batch, sem_ctx *ctx, const double *b_dev, double *x_dev,
                  const sem_cg_opts *opts, int *slot, void *stream);

/* Run `iters` batched iterations (asynchronous; captured as a graph on a
 * non-null stream).  Finished solves cost nothing. */
int sem_batch_step(sem_batch *batch, int iters, void *stream);

/* Blocking status read: up to `cap` finished slots and their results into
 * finished[] / infos[] (*n_finished of them), and the number of occupied slots
 * into *n_active (may be NULL).  Finished slots stay until removed. */
int sem_batch_poll(sem_batch *batch, int *finished, int cap, int *n_finished, sem_cg_info *infos,
                   int *n_active, void *stream);

/* Free a slot (finished or not) and release its context.  Synchronous. */
int sem_batch_remove(sem_batch *batch, int slot, void *stream);

/* Free the host handle (the workspace stays the caller's). */
int sem_batch_destroy(sem_batch *batch);

/* Thread-local text of the last error ("" if none). */
const char *sem_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SEM_H */
