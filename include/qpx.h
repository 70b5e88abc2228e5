/*
 * qpx.h -- C-ABI of the batched single-precision differentiable
 * interior-point QP solver for MI355X (gfx950).
 *
 * Each QP in a batch is
 *
 *     minimize 1/2 x'Qx + q'x   subject to  A x = b,  G x <= h
 *
 * with x in R^n, G in R^{m x n} (m inequality rows), A in R^{p x n}
 * (p equality rows); paper section 2.1.  Multipliers: z (inequalities),
 * y (equalities); slacks s = h - Gx.
 *
 * Conventions for every entry point
 *  - All problem, solution and gradient arrays are DEVICE pointers, float32,
 *    batch-major and row-major (C-contiguous): Q[B][n][n], q[B][n],
 *    A[B][p][n], b[B][p], G[B][m][n], h[B][m], x[B][n], y[B][p], z[B][m],
 *    s[B][m].  Per-QP status/iteration arrays are int32[B].
 *  - The caller owns every buffer it passes.  The library never frees or
 *    keeps a caller pointer beyond the stream order of the call.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls enqueue work and return; results are valid once the stream
 *    reaches that point.
 *  - Return value: QPX_OK (0) or a negative QPX_ERR_* code.  Argument errors
 *    are detected on the host before anything is enqueued.  A per-QP
 *    numerical failure never fails the call: it is reported in status[].
 *  - Nothing here allocates per call except qp_solve / qp_backward's
 *    device workspace, which the context grows on demand and keeps.  The
 *    workspace is shared by the context's calls: a call on another stream
 *    than the previous workspace user waits for that stream on the host.
 *    Contexts are safe to use from several host threads.
 */
#ifndef QPX_H
#define QPX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define QPX_OK 0
#define QPX_PENDING 1            /* qp_serve_poll: result not ready yet       */
#define QPX_ERR_ARG (-1)         /* invalid argument (NULL, sizes, options)   */
#define QPX_ERR_OOM (-2)         /* device or host allocation failed          */
#define QPX_ERR_HIP (-3)         /* a HIP runtime call failed                 */
#define QPX_ERR_STATE (-4)       /* object used in the wrong state            */
#define QPX_ERR_UNSUPPORTED (-5) /* size beyond what the kernels support      */

/* ---- per-QP status (status[i] & 0xff) ----------------------------------- */
#define QPX_CONVERGED 0    /* scaled KKT residual < tol                       */
#define QPX_MAX_ITER 1     /* max_iter reached; last iterate returned         */
#define QPX_NONFINITE 2    /* a non-finite value appeared; see stage          */
#define QPX_FACTOR_FAIL 3  /* non-positive pivot in the KKT factorisation     */
/* (status[i] >> 8) & 0xff: first solver stage that produced a non-finite
 * value or failed factorisation (appendix D.4's trace groups):              */
#define QPX_STAGE_NONE 0
#define QPX_STAGE_SCALING 1    /* standard form: z/s scaling                  */
#define QPX_STAGE_PREDICTOR 2  /* (affine) predictor direction, incl. factor  */
#define QPX_STAGE_CENTERING 3  /* centering quantities (sigma, mu / kappa)    */
#define QPX_STAGE_CORRECTOR 4  /* corrector direction                         */
#define QPX_STAGE_LINESEARCH 5 /* step length                                 */
#define QPX_STAGE_RELAX 6      /* relaxation to kappa_relax (Algorithm 2),
                                  including the factorisation at the relaxed
                                  point that the gradients use               */
#define QPX_STAGE_BACKWARD 7   /* adjoint solve / gradients                   */
/* status[i] bits 16-17: precision events of the QP's run (informational;
 * the outcome is status[i] & 0xff):                                        */
#define QPX_USED_FP64_RESIDUAL (1 << 16) /* FP32 refinement stalled; FP64-
                                            accumulated residuals were used  */
#define QPX_ASM_FELL_BACK (1 << 17)      /* BF16x3 assembly switched to FP32 */

/* ---- formulations ------------------------------------------------------- */
#define QPX_BOUNDED 0   /* implicit complementarity, spectrally bounded system
                           (section 4, eq. implicit_partially_condensed)      */
#define QPX_STANDARD 1  /* standard explicit complementarity (section 3,
                           eq. explicit_partially_condensed); ablation arm    */
#define QPX_CONDENSED 2 /* implicit complementarity solved through the first
                           partially condensed form of appendix B.3: dv is
                           eliminated from every row, so the reduced matrix
                           Q + G' diag(z/s) G is unbounded as in the
                           standard form; no regularisation.  Negative
                           control of the ablation (expected to degrade in
                           FP32).                                             */

typedef struct qpx_ctx qpx_ctx;

typedef struct {
  int32_t B, n, m, p;   /* batch size and dimensions; m or p may be 0        */
  const float *Q, *q;   /* Q symmetric positive semidefinite                 */
  const float *A, *b;   /* may be NULL iff p == 0                            */
  const float *G, *h;   /* may be NULL iff m == 0                            */
} qp_batch;

typedef struct {
  int32_t form;          /* QPX_BOUNDED, QPX_STANDARD or QPX_CONDENSED       */
  int32_t max_iter;      /* Newton iterations of the solve (default 100)      */
  float tol;             /* stopping tolerance on scaled residuals (1e-5)     */
  float sigma;           /* fixed centering kappa_target = sigma kappa when
                            pc == 0 (Algorithm 1 as printed; default 0.1)     */
  int32_t pc;            /* 1: predictor-corrector centering (default)        */
  float kappa_relax;     /* central-path parameter of the backward (1e-4)     */
  int32_t relax_max_iter;/* Newton iterations of the relaxation (30)          */
  float relax_tol;       /* stopping tolerance of the relaxation (1e-6): the
                            gradient of a near-degenerate QP needs a relaxed
                            point tighter than the solve's tolerance; the
                            complementarity term of the implicit forms is
                            |kappa - kappa_relax| / kappa_relax             */
  int32_t kmax;          /* cap on bordered inequality rows of the bounded
                            factorisation; 0 = automatic: n when the factor
                            fits the workgroup's LDS, else every row (up to
                            m, within 1024 - n - p bordered-system rows)     */
  float delta_reg;       /* relative Tikhonov floor on the bordered block (0) */
  int32_t refine_steps;  /* iterative refinement steps of each KKT solve (0)  */
  int32_t block;         /* threads per QP: 0 = automatic, or 128/256/512     */
  int32_t assembly;      /* arithmetic of H = Q + G_I' diag(w) G_I, one of
                            QPX_ASM_* below (default QPX_ASM_AUTO)            */
  float backoff;         /* line-search back-off: step = min(1, backoff *
                            largest feasible step); 0 = the form's default:
                            1 (none) for the implicit forms, whose
                            retraction keeps s, z > 0 (eq. linesearch as
                            printed), 0.99 for the standard form           */
  int32_t fp64_residual; /* residual precision, one of QPX_RES_* below
                            (default QPX_RES_AUTO)                           */
} qp_opts;

/* Residual precision.  The method runs in single precision (sections 3
 * and 5); FP64 enters only as an accumulator of refinement residuals, and
 * by default only for QPs whose FP32 refinement stalls.
 *  QPX_RES_AUTO  stopping test and refinement residuals in FP32; a QP whose
 *                FP32 refinement contracts by less than 1/2 per step
 *                continues with FP64-accumulated refinement residuals (and
 *                FP64-accumulated stopping tests) for the rest of its
 *                solve.  Newton steps refine only regularised or
 *                split-product factors; the adjoint and equality-only
 *                solves are always refined (at least two steps).
 *  QPX_RES_FP64  every residual (stopping test, refinement) accumulated in
 *                FP64, and every adjoint solve refined twice.
 *  QPX_RES_FP32  FP32 residuals only; a stalled refinement just stops.     */
#define QPX_RES_AUTO 0
#define QPX_RES_FP64 1
#define QPX_RES_FP32 2

/* Assembly of the (1,1) block of the reduced KKT matrix.  The factorisation
 * and solves are FP32 in every mode (residuals: see QPX_RES_*).
 *  QPX_ASM_AUTO    QPX_ASM_MFMA_FP32 for the bounded form when n >= 96 and
 *                  the staging buffer fits the workgroup's LDS, else
 *                  QPX_ASM_FP32 (measured: the fastest choice on each side
 *                  of that size).
 *  QPX_ASM_FP32    FP32 fused multiply-adds on the vector ALUs.
 *  QPX_ASM_BF16X3  matrix cores: each operand split into two bfloat16 terms,
 *                  three products per pair accumulated in FP32 (relative
 *                  error about 2^-16 per product); every Newton and adjoint
 *                  solve then takes at least two steps of iterative
 *                  refinement against the exact operator, which restores
 *                  FP32 accuracy; a QP whose refinement contracts by less
 *                  than 1/2 per step switches to QPX_ASM_MFMA_FP32.
 *  QPX_ASM_MFMA_FP32  matrix cores with FP32 inputs.
 * An explicit matrix-core mode for sizes whose staging does not fit returns
 * QPX_ERR_UNSUPPORTED. */
#define QPX_ASM_AUTO 0
#define QPX_ASM_FP32 1
#define QPX_ASM_BF16X3 2
#define QPX_ASM_MFMA_FP32 3

typedef struct {
  float *x, *y, *z, *s;  /* [B][n], [B][p], [B][m], [B][m]; y may be NULL iff
                            p == 0, z and s may be NULL iff m == 0            */
  int32_t *status;       /* [B] per-QP status (see above); required           */
  int32_t *iters;        /* [B] Newton iterations used; may be NULL           */
  float *res;            /* [B] final scaled residual measure; may be NULL    */
  double *work;          /* [B] algorithmic flops of this QP's solve, counted
                            from the sizes of each iteration; may be NULL     */
} qp_out;

typedef struct {
  float *dQ, *dq, *dA, *db, *dG, *dh; /* same shapes as the problem; any may
                                         be NULL to skip writing it           */
} qp_grads;

/* Fill `o` with the defaults listed above.  Returns QPX_OK. */
int qp_default_opts(qp_opts *o);

/* Create a context bound to HIP device `device` (the device is made current
 * for the calls made through the context).  Returns QPX_ERR_HIP if the
 * device does not exist.  *ctx is NULL on failure. */
int qp_create(qpx_ctx **ctx, int device);

/* Release the context and its workspace.  NULL is accepted.  Work enqueued
 * through the context must be complete (the call synchronises the device). */
int qp_destroy(qpx_ctx *ctx);

/* Solve every QP of `batch` (Algorithm 1, implicit complementarity, or the
 * standard Mehrotra method when opts->form == QPX_STANDARD).  Writes
 * out->x, y, z, s, status and the optional arrays.  opts == NULL uses the
 * defaults.  Errors: QPX_ERR_ARG for NULL or inconsistent pointers, B < 0,
 * n < 1, m < 0, p < 0, p >= n, tol <= 0, max_iter < 1; QPX_ERR_UNSUPPORTED
 * if the sizes exceed what the kernels handle; QPX_ERR_OOM / QPX_ERR_HIP
 * from the runtime.  B == 0 is a no-op. */
int qp_solve(qpx_ctx *ctx, const qp_batch *batch, const qp_opts *opts,
             qp_out *out, void *stream);

/* Allocation-free qp_solve, for callers that cannot allocate device memory
 * (code under graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results and errors as qp_solve, computed by
 * the same kernels; the factor workspace of QPs whose bordered factor does
 * not fit LDS is a fixed per-device array of QPX_NOALLOC_SCRATCH_BYTES
 * (resolved by qp_create; held until the process ends) instead of the
 * context's growable workspace, and the call makes no allocation.
 * Errors: QPX_ERR_UNSUPPORTED if the batch needs more workspace than the
 * array holds (B x qp_plan.workspace_bytes > QPX_NOALLOC_SCRATCH_BYTES: split
 * the batch); QPX_ERR_STATE if the context's device has no array.  Every
 * call on one device shares that device's array: calls that overlap in
 * time on one device (different streams, threads or contexts) race and
 * must be ordered by the caller.  Nothing in the array needs to start at
 * zero: the kernels write each factor before reading it. */
#define QPX_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int qp_solve_noalloc(qpx_ctx *ctx, const qp_batch *batch, const qp_opts *opts,
                     qp_out *out, void *stream);

/* Backward pass at the relaxed point (sections 2.3 and 5):
 *  1. warm-start from the solution (x, y, z, s) given in `sol` (as written
 *     by qp_solve) and relax to kappa_relax (Algorithm 2);
 *  2. factor the reduced KKT system at the relaxed point and solve the
 *     adjoint system for the upstream gradient dl_dx [B][n] (Algorithm 3);
 *  3. write the parameter gradients dQ (symmetrised), dq, dA, db, dG, dh.
 * dl_dy [B][p] and dl_dz [B][m] may be NULL (zero upstream).  `relaxed`, if
 * not NULL, receives the relaxed point (its x, y, z, s, status, iters).
 * sol->status is read: QPs whose solve did not converge are still relaxed.
 * Errors as for qp_solve, plus QPX_ERR_ARG if kappa_relax <= 0. */
int qp_backward(qpx_ctx *ctx, const qp_batch *batch, const qp_opts *opts,
                const qp_out *sol, const float *dl_dx, const float *dl_dy,
                const float *dl_dz, qp_grads *grads, qp_out *relaxed,
                void *stream);

/* Human-readable name of a return code (QPX_OK, QPX_PENDING, QPX_ERR_*). */
const char *qp_status_string(int code);

/* Human-readable description of a per-QP status value (status[i] of
 * qp_out: the outcome in the low byte, the failing stage above it), e.g.
 * "non-finite value (stage: predictor)".  Never NULL. */
const char *qp_result_string(int32_t status);

/* Launch plan the library uses for one problem size (host only; no device
 * call, so it also answers on a machine without a GPU). */
typedef struct {
  int32_t threads;         /* threads per QP (one workgroup per QP)           */
  int32_t kb;              /* cap on bordered inequality rows                 */
  int32_t factor_in_lds;   /* 1: the factor lives in LDS; 0: in the context's
                              global workspace                                */
  int32_t assembly;        /* QPX_ASM_FP32, QPX_ASM_BF16X3 or QPX_ASM_MFMA_FP32 */
  size_t lds_bytes;        /* dynamic LDS per workgroup                       */
  size_t workspace_bytes;  /* global factor workspace per QP (0 if in LDS)   */
} qp_plan;

/* Fill *plan for n, m, p under opts (NULL = defaults).  Returns QPX_OK,
 * QPX_ERR_ARG (invalid sizes or options) or QPX_ERR_UNSUPPORTED (sizes the
 * kernels do not handle: bordered system above 1024 rows, m above 4096, or
 * an explicit matrix-core assembly whose staging does not fit). */
int qp_plan_query(int32_t n, int32_t m, int32_t p, const qp_opts *opts, qp_plan *plan);

/* ---- serving: continuous batching of single QPs ------------------------- */
typedef struct qpx_server qpx_server;

typedef struct {
  int32_t max_slots;       /* QPs resident on the device at once (256)        */
  int32_t iters_per_step;  /* Newton iterations per device step for the
                              largest size classes (4); systems of at most
                              64 / 128 rows run 4x / 2x as many             */
  int32_t n_max;           /* largest n accepted (256)                        */
  size_t arena_bytes;      /* device arena for resident QPs; admission is by
                              footprint (0 = 256 MiB)                          */
} qp_server_opts;

typedef struct {
  double t_submit, t_admit, t_done; /* seconds on the host monotonic clock    */
  int32_t status, iters;
} qp_timing;

/* Create a server that runs a scheduler thread on `ctx`'s device with its
 * own stream.  `opts`/`solver` may be NULL for defaults. */
int qp_server_create(qpx_ctx *ctx, const qp_server_opts *opts,
                     const qp_opts *solver, qpx_server **srv);

/* Submit one QP.  Q..h are HOST pointers (row-major float32, sizes as in
 * qp_batch with B = 1); they are copied before the call returns.  A/b may be
 * NULL iff p == 0, G/h iff m == 0.  *ticket identifies the request.
 * Errors: QPX_ERR_ARG (bad sizes, n > n_max, footprint > arena),
 * QPX_ERR_STATE (server stopped). */
int qp_serve_submit(qpx_server *srv, int32_t n, int32_t m, int32_t p,
                    const float *Q, const float *q, const float *A,
                    const float *b, const float *G, const float *h,
                    uint64_t *ticket);

/* Non-blocking.  Returns QPX_PENDING while the request is queued or on the
 * device; QPX_OK once done, after copying the solution into the HOST
 * buffers x[n], y[p], z[m], s[m] (any may be NULL) and filling *timing (may
 * be NULL).  A ticket can be collected once; QPX_ERR_ARG for an unknown or
 * already collected ticket. */
int qp_serve_poll(qpx_server *srv, uint64_t ticket, float *x, float *y,
                  float *z, float *s, qp_timing *timing);

/* Counters: requests admitted / completed, and the peak number of QPs that
 * were resident on the device together.  Any pointer may be NULL. */
int qp_serve_stats(qpx_server *srv, uint64_t *admitted, uint64_t *completed,
                   int32_t *peak_resident);

/* Stop the scheduler (finishing resident work) and free the server. */
int qp_server_destroy(qpx_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* QPX_H */
