// Internal interface between the host C-ABI (qp_api.cpp) and the HIP
// kernels (qp_kernel_impl.hpp, instantiated by qp_inst_*.hip and dispatched
// by qp_launch.hip).  Not installed; not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "../../include/qpx.h"

namespace qpk {

// Kernel modes.
enum Mode : int32_t {
  kSolve = 0,     // Algorithm 1 (or the standard IPM): init + Newton loop
  kBackward = 1,  // relax (Algorithm 2) + adjoint (Algorithm 3) + gradients
  kServe = 2,     // serving step: resume a resident QP for a few iterations
};

// Everything a kernel launch needs.  Problem pointers are batch bases;
// QP i's arrays start at i * (its size).  For serving, `desc` replaces the
// batch layout (one descriptor per slot).
struct Params {
  int32_t B, n, m, p;
  const float *Q, *q, *A, *b, *G, *h;
  // outputs of the solve / inputs of the backward
  float *x, *y, *z, *s;
  int32_t *status, *iters;
  float *res;
  double *work;
  // backward
  const float *gx, *gy, *gz;
  float *dQ, *dq, *dA, *db, *dG, *dh;
  float *rx, *ry, *rz, *rs;  // relaxed point (optional)
  int32_t *rstatus, *riters;
  // options
  int32_t form, max_iter, pc, kb, relax_max_iter, refine;
  int32_t asm_mode;  // H-block assembly: 0 FP32 VALU, 1 BF16x3 MFMA, 2 FP32 MFMA
  int32_t rmode;     // residual precision (qp_opts.fp64_residual)
  float tol, sigma, kappa_relax, relax_tol, delta_reg;
  float backoff;     // line-search back-off, resolved per form
  // factor storage in global memory (when it does not fit LDS)
  float *ws;
  int64_t ws_stride;  // floats per QP
  // serving
  const struct SlotDesc *desc;
  int32_t mode;
  long long *phase;  // [B][16] phase cycle counters (profiling builds only)
};

// One resident serving slot.  All pointers are device pointers into the
// server's arena; `state` holds x, y, z, s contiguously.
struct SlotDesc {
  int32_t n, m, p, kb;      // sizes; kb = cap on bordered inequality rows
  int32_t flags;            // bit0 = fresh (run the initialisation),
                            // bits 1-2 = H-block assembly mode (Params::asm_mode)
  int32_t budget;           // Newton iterations this step may take
  int32_t pad_[2];
  const float *Q, *q, *A, *b, *G, *h;
  float *state;             // x[n] y[p] z[m] s[m], then one word of sticky
                            // arithmetic state (assembly mode, FP64 residuals)
  float *ws;                // factor storage (global) or NULL
  float *out;               // copy of x y z s for the host (this launch's staging)
  int32_t *status, *iters;  // per slot
  float *res;
};

// Bytes of dynamic LDS a launch needs, and whether the factor matrix M
// lives in LDS.  Returns 0 if the configuration is unsupported.
size_t lds_bytes(int n, int m, int p, int kb, bool m_in_lds, int threads);
// Floats of global factor storage per QP when M is not in LDS.
int64_t ws_floats(int n, int m, int p, int kb);
// Whether the matrix-core assembly's LDS staging fits the per-QP layout.
bool mfma_stage_fits(int n, int m, int p, int kb, bool m_in_lds, int threads);
// Largest dynamic LDS per block the kernels may use on this device.
// LDS of a CU, the kernels' static LDS (context table, profiling counters;
// an upper bound) and the most dynamic LDS one QP may take.
constexpr size_t kCuLds = 160 * 1024;
constexpr size_t kStaticLds = 512;
size_t lds_limit();
// Allocation-free workspace (qp_noalloc.hip): resolve the current device's
// copy of the fixed scratch array (once per device), and look it up.
int noalloc_init(int device);
float *noalloc_scratch(int device);

// Launch the fused kernel for `P.mode` with `threads` per block.  Returns a
// hipError_t.
hipError_t launch(const Params &P, int threads, bool m_in_lds, size_t lds,
                  int grid, hipStream_t stream);

constexpr int kMaxN = 1024;  // bordered system dimension supported by the kernels
// (above 512 rows only with 512 threads per QP: 16 rows per lane in the solves)

// Launch configuration of one problem size: border cap, threads per QP,
// whether the factor fits LDS, dynamic LDS bytes, global factor floats.
struct Plan {
  int kb = 0;
  int threads = 256;
  bool m_in_lds = true;
  size_t lds = 0;
  int64_t ws_stride = 0;
  int amode = 0;  // resolved H-block assembly (Params::asm_mode)
};

inline int make_plan(int n, int m, int p, const qp_opts &o, Plan *pl) {
  int kb = o.kmax > 0 ? o.kmax : n;
  kb = std::min(kb, m);
  if (o.form != QPX_BOUNDED) kb = 0;  // standard and first condensed forms: no border
  if (kb < 0) kb = 0;
  if (n + kb + p > kMaxN) kb = kMaxN - n - p;
  if (kb < 0 || n + p > kMaxN) return QPX_ERR_UNSUPPORTED;
  if (m > 4096) return QPX_ERR_UNSUPPORTED;
  pl->kb = kb;
  const int N = n + kb + p;
  int T = o.block;
  if (T == 0) T = N <= 64 ? 128 : (N <= 256 ? 256 : 512);
  if (T != 128 && T != 256 && T != 512) return QPX_ERR_ARG;
  if (N > 512 && T != 512) return QPX_ERR_UNSUPPORTED;
  pl->threads = T;
  const size_t lim = qpk::lds_limit();
  const size_t with_m = qpk::lds_bytes(n, m, p, kb, true, T);
  // QPs resident per CU: LDS-limited, and at most the waves the register
  // allocation targets (three per SIMD up to 256 threads, four at 256
  // threads with more than 128 rows and the factor in global memory, two at
  // 512).  A
  // factor that fits LDS but halves (or worse) the residency of the
  // global-factor layout goes to global memory instead: at n = 100 the LDS
  // factor leaves one QP per CU, the global one three (15% faster).
  const size_t cu_lds = qpk::kCuLds;
  auto per_cu = [&](size_t bytes, bool global) {
    const int cu_waves = 4 * (T >= 512 ? 2 : (T == 256 && N > 128 && global ? 4 : 3));
    return std::min<size_t>(cu_lds / (bytes + qpk::kStaticLds), cu_waves / (T / 64));
  };
  const bool fits = with_m <= lim;
  const bool prefer_global =
      fits && per_cu(qpk::lds_bytes(n, m, p, kb, false, T), true) >= 2 * per_cu(with_m, false);
  if (fits && !prefer_global) {
    pl->m_in_lds = true;
    pl->lds = with_m;
    pl->ws_stride = 0;
  } else {
    pl->m_in_lds = false;
    // When the factor cannot fit LDS at all, the automatic cap borders
    // every row with v > 0 (up to m, within kMaxN), which keeps every
    // multiplier bounded also when more than n rows are active.  This costs
    // workspace, not LDS occupancy.  (A factor moved out of LDS only for
    // residency keeps the border of the LDS layout: same system.)
    if (!fits && o.kmax == 0 && o.form == QPX_BOUNDED) {
      const int kb2 = std::min(m, kMaxN - n - p);
      const int N2 = n + kb2 + p;
      const int T2 = o.block ? o.block : (N2 <= 256 ? 256 : 512);
      if (kb2 > kb && !(N2 > 512 && T2 != 512) &&
          qpk::lds_bytes(n, m, p, kb2, false, T2) <= lim) {
        kb = kb2;
        pl->kb = kb;
        T = T2;
        pl->threads = T;
      }
    }
    pl->lds = qpk::lds_bytes(n, m, p, kb, false, T);
    if (pl->lds > lim) return QPX_ERR_UNSUPPORTED;
    pl->ws_stride = qpk::ws_floats(n, m, p, kb);
  }
  const bool stage_fits = qpk::mfma_stage_fits(n, m, p, kb, pl->m_in_lds, T);
  int am = o.assembly;
  if (am == QPX_ASM_AUTO)
    am = (o.form == QPX_BOUNDED && n >= 96 && stage_fits) ? QPX_ASM_MFMA_FP32 : QPX_ASM_FP32;
  else if (am != QPX_ASM_FP32 && !stage_fits)
    return QPX_ERR_UNSUPPORTED;
  pl->amode = am == QPX_ASM_BF16X3 ? 1 : (am == QPX_ASM_MFMA_FP32 ? 2 : 0);
  return QPX_OK;
}


}  // namespace qpk

// Library context (opaque in the C-ABI).
struct qpx_ctx {
  int device = 0;
  float *ws = nullptr;     // global factor storage, grown on demand
  size_t ws_bytes = 0;
  hipStream_t ws_stream = nullptr;  // stream of the last call that used ws
  bool ws_used = false;
  std::mutex mu;           // guards ws growth
};


