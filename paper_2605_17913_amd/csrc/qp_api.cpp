// Host side of the C-ABI declared in include/qpx.h: argument validation,
// launch configuration, workspace management.  Every step of the solver runs
// in the HIP kernels of qp_kernel_impl.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "../../include/qpx.h"
#include "qp_internal.h"

namespace {

int set_device(const qpx_ctx *ctx) {
  return hipSetDevice(ctx->device) == hipSuccess ? QPX_OK : QPX_ERR_HIP;
}

// Make the workspace ready for a call on stream st: calls on another stream
// than the previous user of the workspace wait for that stream first (the
// workspace is shared by all calls of the context), and the buffer grows on
// demand (previous contents are not kept; the device is synchronised before
// a buffer that may still be in use is freed).
int ensure_ws(qpx_ctx *ctx, size_t bytes, hipStream_t st) {
  if (bytes == 0) return QPX_OK;
  if (ctx->ws_used && ctx->ws_stream != st &&
      hipStreamSynchronize(ctx->ws_stream) != hipSuccess)
    return QPX_ERR_HIP;
  ctx->ws_stream = st;
  ctx->ws_used = true;
  if (bytes <= ctx->ws_bytes) return QPX_OK;
  if (ctx->ws) {
    if (hipDeviceSynchronize() != hipSuccess) return QPX_ERR_HIP;
    hipFree(ctx->ws);
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
  }
  void *p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return QPX_ERR_OOM;
  ctx->ws = static_cast<float *>(p);
  ctx->ws_bytes = bytes;
  return QPX_OK;
}

// Global workspace of a launch: the factors when they do not fit LDS.
size_t ws_bytes(const qpk::Plan &pl, int B) {
  return pl.m_in_lds ? 0 : (size_t)B * pl.ws_stride * sizeof(float);
}

int check_batch(const qp_batch *bt) {
  if (!bt) return QPX_ERR_ARG;
  if (bt->B < 0 || bt->n < 1 || bt->m < 0 || bt->p < 0 || bt->p >= bt->n) return QPX_ERR_ARG;
  if (bt->B == 0) return QPX_OK;
  if (!bt->Q || !bt->q) return QPX_ERR_ARG;
  if (bt->p > 0 && (!bt->A || !bt->b)) return QPX_ERR_ARG;
  if (bt->m > 0 && (!bt->G || !bt->h)) return QPX_ERR_ARG;
  return QPX_OK;
}

int check_opts(const qp_opts &o) {
  if (o.form != QPX_BOUNDED && o.form != QPX_STANDARD && o.form != QPX_CONDENSED) return QPX_ERR_ARG;
  if (!(o.tol > 0.f) || o.max_iter < 1 || o.max_iter > 100000) return QPX_ERR_ARG;
  if (!(o.sigma > 0.f && o.sigma < 1.f)) return QPX_ERR_ARG;
  if (!(o.delta_reg >= 0.f)) return QPX_ERR_ARG;
  if (o.kmax < 0 || o.refine_steps < 0) return QPX_ERR_ARG;
  if (o.assembly < QPX_ASM_AUTO || o.assembly > QPX_ASM_MFMA_FP32) return QPX_ERR_ARG;
  if (!(o.backoff >= 0.f && o.backoff <= 1.f)) return QPX_ERR_ARG;
  if (o.fp64_residual < QPX_RES_AUTO || o.fp64_residual > QPX_RES_FP32) return QPX_ERR_ARG;
  return QPX_OK;
}

void fill_common(qpk::Params &P, const qp_batch *bt, const qp_opts &o, const qpk::Plan &pl,
                 qpx_ctx *ctx) {
  std::memset(&P, 0, sizeof(P));
  P.B = bt->B; P.n = bt->n; P.m = bt->m; P.p = bt->p;
  P.Q = bt->Q; P.q = bt->q; P.A = bt->A; P.b = bt->b; P.G = bt->G; P.h = bt->h;
  P.form = o.form; P.max_iter = o.max_iter; P.pc = o.pc; P.kb = pl.kb;
  P.relax_max_iter = o.relax_max_iter; P.refine = o.refine_steps;
  P.tol = o.tol; P.sigma = o.sigma; P.kappa_relax = o.kappa_relax;
  P.relax_tol = o.relax_tol; P.delta_reg = o.delta_reg;
  P.asm_mode = pl.amode;
  P.rmode = o.fp64_residual;
  P.backoff = o.backoff > 0.f ? o.backoff : (o.form == QPX_STANDARD ? 0.99f : 1.f);
  P.ws = pl.m_in_lds ? nullptr : ctx->ws;
  P.ws_stride = pl.ws_stride;
}


#ifdef QPK_PHASE_TIMING
// Profiling builds only: collect the per-phase cycle counters of one launch
// and print their sums over the batch to stderr.
static void phase_report(const char *what, qpk::Params &P, hipStream_t st, bool before) {
  static long long *buf = nullptr;
  static size_t cap = 0;
  const size_t need = (size_t)P.B * 16;
  if (before) {
    if (need > cap) {
      if (buf) (void)hipFree(buf);
      if (hipMalloc(&buf, need * sizeof(long long)) != hipSuccess) { buf = nullptr; cap = 0; return; }
      cap = need;
    }
    (void)hipMemsetAsync(buf, 0, need * sizeof(long long), st);
    P.phase = buf;
    return;
  }
  if (!buf) return;
  (void)hipStreamSynchronize(st);
  long long *h = new long long[need];
  (void)hipMemcpy(h, buf, need * sizeof(long long), hipMemcpyDeviceToHost);
  static const char *names[16] = {"init", "resid", "part", "asm", "fact", "rhs", "solve",
                                  "refine", "recover", "step", "bwd", "out", "", "", "", ""};
  double tot[16] = {0};
  for (size_t i = 0; i < (size_t)P.B; ++i)
    for (int k = 0; k < 15; ++k) tot[k] += (double)h[i * 16 + k];
  double all = 0;
  for (int k = 0; k < 15; ++k) all += tot[k];
  fprintf(stderr, "QPK_PHASES %s B=%d cycles/QP=%.0f", what, P.B, all / P.B);
  for (int k = 0; k < 12; ++k) fprintf(stderr, " %s=%.1f%%", names[k], 100.0 * tot[k] / all);
  fprintf(stderr, "\n");
  delete[] h;
}
#define QPK_PHASES(what, P, st, before) phase_report(what, P, st, before)
#else
#define QPK_PHASES(what, P, st, before) ((void)0)
#endif

}  // namespace

extern "C" {

int qp_default_opts(qp_opts *o) {
  if (!o) return QPX_ERR_ARG;
  o->form = QPX_BOUNDED;
  o->max_iter = 100;
  o->tol = 1e-5f;
  o->sigma = 0.1f;
  o->pc = 1;
  o->kappa_relax = 1e-4f;
  o->relax_max_iter = 30;
  o->relax_tol = 1e-6f;
  o->kmax = 0;
  o->delta_reg = 0.f;
  o->refine_steps = 0;
  o->block = 0;
  o->assembly = QPX_ASM_AUTO;
  o->backoff = 0.f;
  o->fp64_residual = QPX_RES_AUTO;
  return QPX_OK;
}

int qp_create(qpx_ctx **ctx, int device) {
  if (!ctx) return QPX_ERR_ARG;
  *ctx = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return QPX_ERR_HIP;
  // resolve this device's allocation-free workspace (qp_solve_noalloc) while
  // the device is current
  if (hipSetDevice(device) != hipSuccess) return QPX_ERR_HIP;
  int rc = qpk::noalloc_init(device);
  if (rc) return rc;
  qpx_ctx *c = new (std::nothrow) qpx_ctx();
  if (!c) return QPX_ERR_OOM;
  c->device = device;
  *ctx = c;
  return QPX_OK;
}

int qp_destroy(qpx_ctx *ctx) {
  if (!ctx) return QPX_OK;
  hipSetDevice(ctx->device);
  hipDeviceSynchronize();
  if (ctx->ws) hipFree(ctx->ws);
  delete ctx;
  return QPX_OK;
}

int qp_plan_query(int32_t n, int32_t m, int32_t p, const qp_opts *opts, qp_plan *plan) {
  if (!plan || n < 1 || m < 0 || p < 0 || p >= n) return QPX_ERR_ARG;
  qp_opts o;
  if (opts) o = *opts; else qp_default_opts(&o);
  int rc = check_opts(o);
  if (rc) return rc;
  qpk::Plan pl;
  if ((rc = qpk::make_plan(n, m, p, o, &pl))) return rc;
  plan->threads = pl.threads;
  plan->kb = pl.kb;
  plan->factor_in_lds = pl.m_in_lds ? 1 : 0;
  plan->assembly = pl.amode == 1 ? QPX_ASM_BF16X3 : (pl.amode == 2 ? QPX_ASM_MFMA_FP32 : QPX_ASM_FP32);
  plan->lds_bytes = pl.lds;
  plan->workspace_bytes = pl.m_in_lds ? 0 : (size_t)pl.ws_stride * sizeof(float);
  return QPX_OK;
}

// Checks shared by qp_solve and qp_solve_noalloc; fills the options and
// the launch plan.  Returns QPX_OK, an error, or QPX_PENDING for B == 0
// (nothing to do).
int prepare_solve(qpx_ctx *ctx, const qp_batch *bt, const qp_opts *opts, const qp_out *out,
                  qp_opts *o, qpk::Plan *pl) {
  if (!ctx || !out) return QPX_ERR_ARG;
  int rc = check_batch(bt);
  if (rc) return rc;
  if (opts) *o = *opts; else qp_default_opts(o);
  if ((rc = check_opts(*o))) return rc;
  if (bt->B == 0) return QPX_PENDING;
  if (!out->x || !out->status) return QPX_ERR_ARG;
  if (bt->p > 0 && !out->y) return QPX_ERR_ARG;
  if (bt->m > 0 && (!out->z || !out->s)) return QPX_ERR_ARG;
  return qpk::make_plan(bt->n, bt->m, bt->p, *o, pl);
}

int qp_solve(qpx_ctx *ctx, const qp_batch *bt, const qp_opts *opts, qp_out *out,
             void *stream) {
  qp_opts o;
  qpk::Plan pl;
  int rc = prepare_solve(ctx, bt, opts, out, &o, &pl);
  if (rc) return rc == QPX_PENDING ? QPX_OK : rc;
  if ((rc = set_device(ctx))) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lk(ctx->mu);
  if ((rc = ensure_ws(ctx, ws_bytes(pl, bt->B), st))) return rc;
  qpk::Params P;
  fill_common(P, bt, o, pl, ctx);
  P.x = out->x; P.y = out->y; P.z = out->z; P.s = out->s;
  P.status = out->status; P.iters = out->iters; P.res = out->res; P.work = out->work;
  P.mode = qpk::kSolve;
  QPK_PHASES("solve", P, st, true);
  const hipError_t e = qpk::launch(P, pl.threads, pl.m_in_lds, pl.lds, bt->B, st);
  QPK_PHASES("solve", P, st, false);
  return e == hipSuccess ? QPX_OK : QPX_ERR_HIP;
}

int qp_solve_noalloc(qpx_ctx *ctx, const qp_batch *bt, const qp_opts *opts, qp_out *out,
                     void *stream) {
  qp_opts o;
  qpk::Plan pl;
  int rc = prepare_solve(ctx, bt, opts, out, &o, &pl);
  if (rc) return rc == QPX_PENDING ? QPX_OK : rc;
  // the factors of QPs whose factor does not fit LDS go to this device's
  // fixed scratch array; a batch that needs more than it holds is refused
  const size_t need = ws_bytes(pl, bt->B);
  if (need > (size_t)QPX_NOALLOC_SCRATCH_BYTES) return QPX_ERR_UNSUPPORTED;
  float *scratch = qpk::noalloc_scratch(ctx->device);
  if (!scratch) return QPX_ERR_STATE;
  if ((rc = set_device(ctx))) return rc;
  qpk::Params P;
  fill_common(P, bt, o, pl, ctx);
  P.ws = pl.m_in_lds ? nullptr : scratch;
  P.x = out->x; P.y = out->y; P.z = out->z; P.s = out->s;
  P.status = out->status; P.iters = out->iters; P.res = out->res; P.work = out->work;
  P.mode = qpk::kSolve;
  const hipError_t e = qpk::launch(P, pl.threads, pl.m_in_lds, pl.lds, bt->B,
                                   static_cast<hipStream_t>(stream));
  return e == hipSuccess ? QPX_OK : QPX_ERR_HIP;
}

int qp_backward(qpx_ctx *ctx, const qp_batch *bt, const qp_opts *opts, const qp_out *sol,
                const float *dl_dx, const float *dl_dy, const float *dl_dz, qp_grads *grads,
                qp_out *relaxed, void *stream) {
  if (!ctx || !sol || !grads) return QPX_ERR_ARG;
  int rc = check_batch(bt);
  if (rc) return rc;
  qp_opts o;
  if (opts) o = *opts; else qp_default_opts(&o);
  if ((rc = check_opts(o))) return rc;
  if (!(o.kappa_relax > 0.f) || !(o.relax_tol > 0.f) || o.relax_max_iter < 0) return QPX_ERR_ARG;
  if (bt->B == 0) return QPX_OK;
  if (!dl_dx || !sol->x) return QPX_ERR_ARG;
  if (bt->p > 0 && !sol->y) return QPX_ERR_ARG;
  if (bt->m > 0 && (!sol->z || !sol->s)) return QPX_ERR_ARG;
  qpk::Plan pl;
  if ((rc = qpk::make_plan(bt->n, bt->m, bt->p, o, &pl))) return rc;
  if ((rc = set_device(ctx))) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lk(ctx->mu);
  if ((rc = ensure_ws(ctx, ws_bytes(pl, bt->B), st))) return rc;
  qpk::Params P;
  fill_common(P, bt, o, pl, ctx);
  P.x = sol->x; P.y = sol->y; P.z = sol->z; P.s = sol->s;
  P.gx = dl_dx; P.gy = bt->p ? dl_dy : nullptr; P.gz = bt->m ? dl_dz : nullptr;
  P.dQ = grads->dQ; P.dq = grads->dq; P.dA = grads->dA; P.db = grads->db;
  P.dG = grads->dG; P.dh = grads->dh;
  if (relaxed) {
    P.rx = relaxed->x; P.ry = relaxed->y; P.rz = relaxed->z; P.rs = relaxed->s;
    P.rstatus = relaxed->status; P.riters = relaxed->iters; P.res = relaxed->res;
    P.work = relaxed->work;
  }
  P.mode = qpk::kBackward;
  QPK_PHASES("backward", P, st, true);
  const hipError_t e = qpk::launch(P, pl.threads, pl.m_in_lds, pl.lds, bt->B, st);
  QPK_PHASES("backward", P, st, false);
  return e == hipSuccess ? QPX_OK : QPX_ERR_HIP;
}

const char *qp_status_string(int code) {
  switch (code) {
    case QPX_OK: return "ok";
    case QPX_PENDING: return "pending";
    case QPX_ERR_ARG: return "invalid argument";
    case QPX_ERR_OOM: return "out of memory";
    case QPX_ERR_HIP: return "HIP runtime error";
    case QPX_ERR_STATE: return "invalid state";
    case QPX_ERR_UNSUPPORTED: return "unsupported size";
    default: return "unknown return code";
  }
}

const char *qp_result_string(int32_t status) {
  static const char *outcome[4] = {"converged", "iteration limit reached", "non-finite value",
                                   "factorisation failed (non-positive pivot)"};
  static const char *stage[8] = {"", "scaling", "predictor", "centering", "corrector",
                                 "line search", "relax", "backward"};
  // every (outcome, stage) pair as one static string
  static char table[4][8][80];
  static std::once_flag once;
  std::call_once(once, [] {
    for (int o = 0; o < 4; ++o)
      for (int g = 0; g < 8; ++g) {
        if (g == 0) std::snprintf(table[o][g], sizeof(table[o][g]), "%s", outcome[o]);
        else std::snprintf(table[o][g], sizeof(table[o][g]), "%s (stage: %s)", outcome[o], stage[g]);
      }
  });
  const int o = status & 0xff, g = (status >> 8) & 0xff;
  if (status < 0 || o > 3 || g > 7 || (status >> 18) != 0) return "unknown per-QP status";
  return table[o][g];
}

}  // extern "C"
