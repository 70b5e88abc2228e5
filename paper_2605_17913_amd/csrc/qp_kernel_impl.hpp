// Kernel templates; included by the per-configuration instantiation units.
#pragma once
// Fused batched interior-point kernels for gfx950 (MI355X).
//
// One workgroup owns one QP for its whole solve: problem data is read from
// HBM (it stays L2/MALL resident across iterations), the iterate, residuals
// and directions live in LDS, and the bordered KKT factor lives in LDS when
// it fits (else in a per-QP global workspace).  No host synchronisation
// happens inside a solve; each QP exits its Newton loop on its own.
//
// Method (paper section 4): implicit complementarity with the softplus
// retraction b_kappa (eq. softplus, appendix C).  Each Newton step solves the
// reduced symmetric system of eq. implicit_partially_condensed
//
//     [ Q - G'G   G'      A' ] [dx]     [ r_t - G'(r_i + r_z - r_s) ]
//     [ G        -B(-v)   0  ] [dv] = - [ r_i - r_s - c r_kappa     ]
//     [ A         0       0  ] [dy]     [ r_e                       ]
//
// The paper only says the matrix is symmetric and admits LDL'; it is
// indefinite, so it is factored here by a sign-split elimination that is
// exact in exact arithmetic and needs no pivoting:
//   * rows with v_i <= 0 (D_i = b'(-v_i) >= 1/2) are eliminated: pivot
//     -D_i, which folds G_i' (E_i/D_i) G_i into the (1,1) block, with
//     E_i/D_i = z_i/s_i in (0, 1];
//   * rows with v_i > 0 are kept as a border with the change of variable
//     du_i = E_i dv_i, giving the diagonal -D_i/E_i = -s_i/z_i in (-1, 0);
//   * the equality rows A are kept as a border with a zero diagonal.
// The result is the quasi-definite matrix
//
//     M = [ H   C' ]    H = Q + G_I' diag(E/D) G_I  (positive definite),
//         [ C  -Dl ]    C = [G_B; A],  Dl = diag(s_B / z_B, 0_p) >= 0,
//
// factored as M = L diag(sg) L' with known signs sg = (+1 x n, -1 x k):
// a Cholesky whose trailing k pivots are negated.  Every multiplier is
// bounded (E, D in (0,1), E/D <= 1 on eliminated rows, D/E < 1 on border
// rows), which is the spectral bound the paper relies on.  When more than
// kb rows have v_i > 0, the kb rows with the largest v are bordered and the
// rest eliminated (their weight z/s is then > 1 but moderate).
//
// The standard (explicit) arm factors the normal matrix Q + G' diag(z/s) G
// bordered by A (eq. explicit_partially_condensed with dz eliminated) with
// the same signed Cholesky, and runs Mehrotra's predictor-corrector.
#include <hip/hip_runtime.h>
#include <float.h>
#include <stdint.h>

#include <type_traits>

#include "qp_internal.h"

namespace qpk {
namespace {

#define QPD __device__ __forceinline__
// Attribute of the solver's phases (residuals, partition, assembly,
// factorisation, solves, refinement, ...).  Small systems inline them into
// the kernel: the calls' saved registers and context copies would otherwise
// go through scratch memory.  Large systems keep them as separate functions,
// which bounds register pressure and compile time; the instantiation unit
// chooses by defining QPK_INLINE_PHASES.
#ifdef QPK_INLINE_PHASES
#define QPK_PHASE __device__ __forceinline__
#else
#define QPK_PHASE __device__ __noinline__
#endif

constexpr int kNB = 16;          // panel width of the blocked factorisation
constexpr float kBig = 3.0e38f;

// Explicit address spaces: LDS (3) and global (1).  Helpers that are not
// inlined keep 32-bit LDS addresses and emit ds_* / global_* instructions.
typedef __attribute__((address_space(3))) float lf;
typedef __attribute__((address_space(3))) int li;
typedef __attribute__((address_space(3))) double ldd;
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) f4v lf4;
typedef __attribute__((address_space(1))) float gf;
typedef __attribute__((address_space(1))) f4v gf4;
// LDS pointer type of a residual accumulator (FP32 or FP64).
template <class AT> struct LdsT;
template <> struct LdsT<float> { typedef __attribute__((address_space(3))) float type; };
template <> struct LdsT<double> { typedef __attribute__((address_space(3))) double type; };
template <class F> struct Vec4;
template <> struct Vec4<lf> { typedef lf4 type; };
template <> struct Vec4<gf> { typedef gf4 type; };
template <> struct Vec4<const lf> { typedef const lf4 type; };
template <> struct Vec4<const gf> { typedef const gf4 type; };
typedef float f2v __attribute__((ext_vector_type(2)));
template <class F> struct Vec2;
template <> struct Vec2<lf> { typedef const __attribute__((address_space(3))) f2v type; };
template <> struct Vec2<gf> { typedef const __attribute__((address_space(1))) f2v type; };

QPD bool finitef(float a) { return fabsf(a) <= FLT_MAX; }

QPD float readlane(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}


// Values that are the same in every lane.  Non-inlined helpers receive their
// arguments in VGPRs (or read them from the stack), which hides uniformity
// from the compiler; passing them through readfirstlane at entry puts loop
// bounds and base addresses back into SGPRs and keeps branches scalar.
QPD int rfl(int v) { return __builtin_amdgcn_readfirstlane(v); }
QPD float rflf(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }
template <class T>
QPD T *rflp(T *p) {
  if constexpr (sizeof(T *) == 4) {
    return (T *)(uintptr_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(uintptr_t)p);
  } else {
    const uint64_t v = (uint64_t)(uintptr_t)p;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return (T *)(uintptr_t)(((uint64_t)hi << 32) | lo);
  }
}

// Orders LDS / global accesses of one wavefront (lanes exchange data
// through memory without a workgroup barrier).
QPD void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Optional per-phase cycle counters for profiling builds (-DQPK_PHASE_TIMING):
// thread 0 accumulates clock64() deltas per phase in LDS; the kernel writes
// them to Params::phase.  Compiled out otherwise.
#ifdef QPK_PHASE_TIMING
#define QPK_PT(C, k)                                    \
  do {                                                  \
    __syncthreads();                                    \
    if (threadIdx.x == 0) {                             \
      const long long _t = clock64();                   \
      (C).pt[k] += _t - (C).pt[15];                     \
      (C).pt[15] = _t;                                  \
    }                                                   \
  } while (0)
#else
#define QPK_PT(C, k) ((void)0)
#endif
enum Phase { PH_INIT, PH_RESID, PH_PART, PH_ASM, PH_FACT, PH_RHS, PH_SOLVE, PH_REFINE,
             PH_RECOVER, PH_STEP, PH_BWD, PH_OUT, PH_N = 16 };

struct OpSum { template <class V> QPD static V f(V a, V b) { return a + b; } };
struct OpMax { QPD static float f(float a, float b) { return fmaxf(a, b); } };
struct OpMin { QPD static float f(float a, float b) { return fminf(a, b); } };

// One butterfly step: Op(v, value of lane ^ O) in every lane, on the VALU
// (DPP row rotations, gfx950's permlane swaps) instead of the LDS crossbar
// that shuffles use; V is float or double (two 32-bit halves).  Steps run
// in descending O: once the steps above O have run, lanes l and l ^ 2^k
// (2^k > O) hold equal values, so the rotation by O within a 16-lane row,
// which reaches lane (l - O) mod 16, reads the value of lane l ^ O (for
// O = 8 it is that lane); the swaps exchange whole rows (O = 16) or halves
// (O = 32) exactly.  With commutative operations the results are bitwise
// those of the shuffle butterfly.  All lanes of the wave must be active.
template <int O>
QPD int dpp_ror(int v) {
  static_assert(O == 8 || O == 4 || O == 2 || O == 1, "row rotation");
  return __builtin_amdgcn_update_dpp(0, v, 0x120 + O, 0xF, 0xF, false);  // row_ror:O
}
template <int O>
QPD void lane_swap(int v, int &a, int &b) {
  if constexpr (O == 32) {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    a = r[0]; b = r[1];
  } else {
    static_assert(O == 16, "row swap");
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    a = r[0]; b = r[1];
  }
}
template <int O, class Op, class V>
QPD V bfly(V v) {
  if constexpr (sizeof(V) == 4) {
    const int iv = __float_as_int(v);
    if constexpr (O >= 16) {
      int a, b;
      lane_swap<O>(iv, a, b);
      return Op::f(__int_as_float(a), __int_as_float(b));
    } else {
      return Op::f(v, __int_as_float(dpp_ror<O>(iv)));
    }
  } else {
    const long long w = __double_as_longlong(v);
    const int lo = (int)(unsigned)w, hi = (int)(unsigned)(w >> 32);
    auto join = [](int l, int h) {
      return __longlong_as_double((long long)(((unsigned long long)(unsigned)h << 32) |
                                              (unsigned)l));
    };
    if constexpr (O >= 16) {
      int al, bl, ah, bh;
      lane_swap<O>(lo, al, bl);
      lane_swap<O>(hi, ah, bh);
      return Op::f(join(al, ah), join(bl, bh));
    } else {
      return Op::f(v, join(dpp_ror<O>(lo), dpp_ror<O>(hi)));
    }
  }
}
// Op over the 16 lanes of each row, in every lane.
template <class Op, class V>
QPD V row_bfly(V v) {
  v = bfly<8, Op>(v);
  v = bfly<4, Op>(v);
  v = bfly<2, Op>(v);
  return bfly<1, Op>(v);
}
// Op over the wave, in every lane.
template <class Op, class V>
QPD V wave_bfly(V v) {
  v = bfly<32, Op>(v);
  v = bfly<16, Op>(v);
  return row_bfly<Op>(v);
}

// Reduce K values across the workgroup; every thread gets the results.
// `red` needs (T/64)*K floats.  Contains two barriers.
template <int T, class Op, int K>
QPD void block_reduce(float (&v)[K], lf *red) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    v[k] = wave_bfly<Op>(v[k]);
  }
  if constexpr (T > 64) {
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
      for (int k = 0; k < K; ++k) red[w * K + k] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
      float r = red[k];
#pragma unroll
      for (int i = 1; i < T / 64; ++i) r = Op::f(r, red[i * K + k]);
      v[k] = r;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Softplus retraction, cancellation-free (appendix C).
QPD float bk(float v, float kappa) {
  const float r = sqrtf(fmaf(v, v, 4.f * kappa));
  return v >= 0.f ? 0.5f * (v + r) : 2.f * kappa / (r - v);
}
// b_kappa'(v): (1 + v/r)/2 for v >= 0, 2 kappa / (r^2 - v r) for v < 0.
QPD float dbk(float v, float kappa, float r) {
  return v >= 0.f ? 0.5f * (1.f + v / r) : 2.f * kappa / (r * (r - v));
}

// ---------------------------------------------------------------------------
// Packed-blocked storage of the lower triangle of the bordered factor: row i
// holds columns 0 .. 16*floor(i/16)+15 (its lower part rounded up to a whole
// 16-column panel) plus 4 floats of padding, so every panel segment
// M[i][k0 .. k0+15] with k0 <= i is a 16-byte-aligned run and consecutive
// rows start on different LDS banks.  Element (i, j), j <= i, is at
// moff(i) + j.
__host__ __device__ inline int moff(int i) {
  const int q = i >> 4, rem = i & 15;
  return 20 * i + 16 * (8 * q * (q - 1) + q * rem);
}

// Lower-triangular tile t -> (ti, tj), tj <= ti, in row order.
QPD void tile_ij(int t, int &ti, int &tj) {
  int i = (int)((sqrtf(8.f * (float)t + 1.f) - 1.f) * 0.5f);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  ti = i;
  tj = t - i * (i + 1) / 2;
}

// ---------------------------------------------------------------------------
// Per-QP LDS layout (floats; ints share the float arena).  All blocks are
// 4-float aligned.
struct Layout {
  int n, m, p, kb, Nmax, ld;
  int x, y, z, s, v, q, h, b;
  int E, D, c;
  int rt, ri, re, rz, rs;
  int tGz, tAy;
  int t0, t1, u0, u1, dv0, dv1, dinv;
  int part, red;
  int w0, w1, rr, rd, dd;  // rhs copies / residual and last correction of
                           // the refinement; FP64 scratch
  int pan;             // (unused)
  int role, bidx, elist, iflag;
  int stg, stg_len;  // assembly staging: the span u0 .. end of dd, which
                     // holds nothing live while the matrix is assembled
  int M;      // offset of M if in LDS, else -1
  int total;  // floats
};

__host__ __device__ inline int al4(int a) { return (a + 3) & ~3; }


__host__ __device__ inline Layout make_layout(int n, int m, int p, int kb, bool m_lds, int T) {
  Layout L;
  L.n = n; L.m = m; L.p = p; L.kb = kb;
  L.Nmax = n + kb + p;
  L.ld = 0;  // unused: the factor uses the packed-blocked layout of moff()
  int o = 0;
  auto take = [&](int cnt) { int r = o; o += al4(cnt > 0 ? cnt : 1); return r; };
  L.x = take(n); L.y = take(p); L.z = take(m); L.s = take(m); L.v = take(m);
  L.q = take(n); L.h = take(m); L.b = take(p);
  L.E = take(m); L.D = take(m); L.c = take(m);
  L.rt = take(n); L.ri = take(m); L.re = take(p); L.rz = take(m); L.rs = take(m);
  L.tGz = take(n); L.tAy = take(n);
  const int tlen = max(max(m, p), L.Nmax);  // t0/t1 also hold refinement rhs copies
  L.t0 = take(tlen); L.t1 = take(tlen);
  L.u0 = take(L.Nmax); L.u1 = take(L.Nmax);
  L.dv0 = take(m); L.dv1 = take(m); L.dinv = take((L.Nmax + 15) & ~15);
  // partial sums (2 floats or 1 double per thread) and reduction scratch
  L.part = take(2 * T); L.red = take((T / 64) * 16);
  L.w0 = L.t0; L.w1 = L.t1; L.rr = take(L.Nmax); L.rd = take(L.Nmax);
  L.dd = take(2 * (2 * m + p + n + 8));
  L.pan = take(4);
  L.role = take(m); L.bidx = take(m); L.elist = take(m); L.iflag = take(16);
  L.stg = L.u0;
  L.stg_len = L.pan - L.u0;
  // M's storage ends with 16 floats past the last row: a zero row for the
  // triangular solves, in M's own address space
  if (m_lds) { L.M = o; o += al4(moff(L.Nmax) + kNB); } else { L.M = -1; }
  L.total = o;
  return L;
}

// ---------------------------------------------------------------------------
// Dense helpers on one workgroup of T threads.

// Columns jb + sub + 16q (q < 4) of row i of R (rows x cols, row stride
// ld), loaded from clamped in-bounds addresses without a branch, so that
// the loads of an unrolled row loop issue together; entries outside the
// matrix read as 0.  Needs rows >= 1 and cols >= 1.
template <class RF>
QPD void load_row4(const RF *R, int ld, int rows, int cols, int i, int jb, int sub,
                   float (&e)[4]) {
  const bool in = i < rows;
  const RF *Ri = R + (size_t)(in ? i : rows - 1) * ld;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int j = jb + sub + 16 * q;
    const float v = Ri[min(j, cols - 1)];
    e[q] = (in && j < cols) ? v : 0.f;
  }
}

// out[i] = sum_j R[i*ld + j] x[j] for i < rows.  16 lanes share a row
// (columns jb + sub + 16c, c < 4, in blocks of 64) and T/16 rows go at a
// time; the row loop is unrolled so that the loads of several rows are in
// flight before their arithmetic.
template <int T, int NV, class RF>
QPD void rowdot(const RF *R, int ld, int rows, int cols, const lf *const (&x)[NV],
                lf *const (&out)[NV]) {
  const int sub = threadIdx.x & 15, grp = threadIdx.x >> 4;
  for (int jb = 0; jb < cols; jb += 64) {
    float xv[NV][4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int j = jb + sub + 16 * c;
#pragma unroll
      for (int k = 0; k < NV; ++k) xv[k][c] = j < cols ? x[k][j] : 0.f;
    }
#pragma unroll 4
    for (int i0 = 0; i0 < rows; i0 += T / 16) {
      const int i = i0 + grp;
      float e[4] = {0.f, 0.f, 0.f, 0.f};
      if (i < rows) {
        const RF *Ri = R + (size_t)i * ld + jb + sub;
#pragma unroll
        for (int c = 0; c < 4; ++c)
          if (jb + sub + 16 * c < cols) e[c] = Ri[16 * c];
      }
      float acc[NV];
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        acc[k] = 0.f;
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[k] = fmaf(e[c], xv[k][c], acc[k]);
        acc[k] = row_bfly<OpSum>(acc[k]);
      }
      if (sub == 0 && i < rows) {
#pragma unroll
        for (int k = 0; k < NV; ++k) out[k][i] = jb ? out[k][i] + acc[k] : acc[k];
      }
    }
  }
}

// out[j] = sum_i R[i*ld + j] x[i] for j < cols.  The same lane layout as
// rowdot (16 lanes per row, 4 columns each, T/16 rows at a time, several
// rows' loads in flight); each lane sums its columns over its rows, then the
// row groups are combined by shuffles inside a wave and through `part`
// (2T floats) across waves.  Barriers inside; `x` must be visible to all
// threads on entry.
template <int T, int NV, class RF>
QPD void coldot(const RF *R, int ld, int rows, int cols, const lf *const (&x)[NV],
                lf *const (&out)[NV], lf *part) {
  static_assert(NV <= 2, "part holds two floats per thread");
  const int tid = threadIdx.x, sub = tid & 15, grp = tid >> 4, wid = tid >> 6;
  for (int jb = 0; jb < cols; jb += 64) {
    float c[NV][4];
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
      for (int q = 0; q < 4; ++q) c[k][q] = 0.f;
#pragma unroll 4
    for (int i0 = 0; i0 < rows; i0 += T / 16) {
      const int i = i0 + grp;
      float e[4] = {0.f, 0.f, 0.f, 0.f}, w[NV];
#pragma unroll
      for (int k = 0; k < NV; ++k) w[k] = 0.f;
      if (i < rows) {
        const RF *Ri = R + (size_t)i * ld + jb + sub;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (jb + sub + 16 * q < cols) e[q] = Ri[16 * q];
#pragma unroll
        for (int k = 0; k < NV; ++k) w[k] = x[k][i];
      }
#pragma unroll
      for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int q = 0; q < 4; ++q) c[k][q] = fmaf(e[q], w[k], c[k][q]);
    }
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        c[k][q] = bfly<32, OpSum>(bfly<16, OpSum>(c[k][q]));
      }
    if ((tid & 63) < 16) {
#pragma unroll
      for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int q = 0; q < 4; ++q) part[k * T + wid * 64 + 16 * q + sub] = c[k][q];
    }
    __syncthreads();
    if (tid < 64 && jb + tid < cols) {
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        float sum = 0.f;
#pragma unroll
        for (int w = 0; w < T / 64; ++w) sum += part[k * T + w * 64 + tid];
        out[k][jb + tid] = sum;
      }
    }
    __syncthreads();
  }
}

// One 16x16 tile of the rank-16 update on the matrix cores, by a whole wave:
// M[i][j] -= sum_c L[i][p0+c] sg_c L[j][p0+c] for i in block bi, j in block
// bj (16-row blocks), j <= i.  Lane l loads the 16-byte segment
// c = 4(l/16) .. 4(l/16)+3 of rows 16 bi + l%16 (A) and 16 bj + l%16 (B);
// instruction q multiplies component q, so the four v_mfma_f32_16x16x4_f32
// cover c = 0..15.  Register r of lane l holds row 4(l/16) + r, column l%16.
// Rows at or beyond N read row N-1 and their results are dropped.
template <class MF>
QPD void rank16_tile16(MF *M, int N, int npos, int p0, int bi, int bj) {
  typedef typename Vec4<const MF>::type CV4;
  const int lane = threadIdx.x & 63, g = lane >> 4, c16 = lane & 15;
  const int ia = min(16 * bi + c16, N - 1), jb = min(16 * bj + c16, N - 1);
  const f4v a = *reinterpret_cast<CV4 *>(M + moff(ia) + p0 + 4 * g);
  f4v b = *reinterpret_cast<CV4 *>(M + moff(jb) + p0 + 4 * g);
  const int c0 = p0 + 4 * g;
  b.x *= c0 + 0 < npos ? 1.f : -1.f;
  b.y *= c0 + 1 < npos ? 1.f : -1.f;
  b.z *= c0 + 2 < npos ? 1.f : -1.f;
  b.w *= c0 + 3 < npos ? 1.f : -1.f;
  f4v acc = {0.f, 0.f, 0.f, 0.f};
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b.z, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b.w, acc, 0, 0, 0);
  const int j = 16 * bj + c16;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = 16 * bi + 4 * g + r;
    if (i < N && j <= i) M[moff(i) + j] -= acc[r];
  }
}

// One row's 16-column panel segment M[i][k0 .. k0+15] into registers (zeros
// for rows at or beyond N), and back with exact zeros right of the diagonal
// (r = i - k0 is the row's position in the panel).
template <class MF>
QPD void panel_load(const MF *M, int N, int k0, int i, float (&R)[kNB]) {
  typedef typename Vec4<const MF>::type CV4;
  const bool in = i < N;
  const MF *row = M + moff(min(i, N - 1)) + k0;
#pragma unroll
  for (int c = 0; c < kNB; c += 4) {
    const f4v v4 = *reinterpret_cast<CV4 *>(row + c);
    R[c] = in ? v4.x : 0.f;
    R[c + 1] = in ? v4.y : 0.f;
    R[c + 2] = in ? v4.z : 0.f;
    R[c + 3] = in ? v4.w : 0.f;
  }
}
template <class MF>
QPD void panel_store(MF *M, int N, int k0, int i, const float (&R)[kNB], float &lmax) {
  typedef typename Vec4<MF>::type V4;
  if (i >= N) return;
  const int r = i - k0;
  MF *row = M + moff(i) + k0;
#pragma unroll
  for (int c = 0; c < kNB; c += 4) {
    f4v v4;
    v4.x = (c + 0 <= r) ? R[c + 0] : 0.f;
    v4.y = (c + 1 <= r) ? R[c + 1] : 0.f;
    v4.z = (c + 2 <= r) ? R[c + 2] : 0.f;
    v4.w = (c + 3 <= r) ? R[c + 3] : 0.f;
    *reinterpret_cast<V4 *>(row + c) = v4;
    // largest |L| written (a NaN counts as infinite)
    const float a = fmaxf(fmaxf(fabsf(v4.x), fabsf(v4.y)), fmaxf(fabsf(v4.z), fabsf(v4.w)));
    const bool nan = v4.x != v4.x || v4.y != v4.y || v4.z != v4.z || v4.w != v4.w;
    lmax = nan ? __int_as_float(0x7f800000) : fmaxf(lmax, a);
  }
}

// Factor the 16-column panel starting at k0 (rows k0..N-1) by one wave in
// registers (lane = row, readlane broadcasts); writes L back with exact
// zeros right of the diagonal.  Rows are taken 64 at a time: chunk 0 holds
// the diagonal block, and up to four more chunks are eliminated in the same
// sweep; any further chunks (more than 320 rows) replay the eliminations
// with the finished diagonal block, so registers stay bounded for any N.
// Returns true if a pivot failed.
//
// Dynamic regularisation (dyn): a pivot sg*a_jj that is not above
// kPivTol * pmax, with pmax the largest pivot accepted so far in its block
// (the H block, or the border from its first column on), is taken as
// numerically zero (or of the wrong sign through rounding) and replaced by
// kPivReg * pmax; nreg counts the replacements.  The factor is then that of
// M plus a small diagonal, and callers refine against the exact operator.
// This keeps a degenerate system (dependent border rows, e.g. more active
// rows plus equalities than unknowns) factorable in FP32.
constexpr float kPivTol = 1e-6f;
constexpr float kPivReg = 1e-5f;
constexpr float kGrowthMax = 1e2f;  // accepted max|L| / sqrt(largest pivot) with
                                    // replacements (a stable factor stays near 1)
// The panel's first sweep with G extra 64-row chunks in registers (rows
// k0 + lane + 64 (1 + g)); gact (uniform) counts those that hold rows of
// the system, and without any (gact = 0: chunks entirely past row N-1 would
// only carry zeros) a scalar branch per column skips their updates.  P0 holds chunk 0 (the diagonal
// block) on return and iv the signed pivot inverses, for the replay of any
// further chunks.  The multipliers of column jj are read from
// ps = a[.][jj] / L[jj][jj], which equals L[.][jj] sg_jj exactly (the sign
// is folded into the broadcast source instead of into every multiplier).
template <int G, class MF>
QPD bool panel_sweep(MF *M, int N, int npos, int k0, int kb, int gact, bool dyn, float &pmax,
                     float &pmaxh, int &nreg, float &lmax, float (&P0)[kNB], float (&iv)[kNB]) {
  const int lane = threadIdx.x & 63;
  float P[G > 0 ? G : 1][kNB];
  panel_load(M, N, k0, k0 + lane, P0);
#pragma unroll
  for (int g = 0; g < G; ++g) panel_load(M, N, k0, k0 + lane + 64 * (1 + g), P[g]);
  bool fail = false;
#pragma unroll
  for (int jj = 0; jj < kNB; ++jj) {
    iv[jj] = 0.f;
    if (jj < kb) {
      // row k0+jj is in lane jj of chunk 0
      const float sg = (k0 + jj) < npos ? 1.f : -1.f;
      // the border's pivots (its Schur complement, of order |C_j|^2 / |H|
      // plus the diagonal Dl, with the rows equilibrated: border_exponent)
      // are tested against the border's own largest pivot: at the first
      // border column the running maximum restarts (the H block's is kept
      // in pmaxh)
      if (k0 + jj == npos) {
        pmaxh = pmax;
        pmax = 0.f;
      }
      float tt = sg * readlane(P0[jj], jj);
      if (dyn && !(tt > kPivTol * pmax) && tt >= -FLT_MAX && pmax > 0.f) {
        tt = kPivReg * pmax;
        ++nreg;
      }
      const bool ok = tt > 0.f && tt <= FLT_MAX;
      if (ok) pmax = fmaxf(pmax, tt);
      fail |= !ok;
      // pivot sqrt(tt) and its signed inverse from one hardware reciprocal
      // square root (about 1 ulp): this chain is on the panel's critical path
      const float rs = ok ? __builtin_amdgcn_rsqf(tt) : 1.f;
      const float d = ok ? tt * rs : 1.f;
      const float inv = sg * rs;
      iv[jj] = inv;
      const float ps = P0[jj] * rs;  // L[k0+lane][k0+jj] sg below the diagonal
      P0[jj] = lane > jj ? ps * sg : (lane == jj ? d : P0[jj]);
      if constexpr (G <= 1) {
        // the multipliers first, into scalar registers, then the updates:
        // the broadcasts issue back to back instead of each waiting on the
        // last one's result
        float lc[kNB];
#pragma unroll
        for (int cc = jj + 1; cc < kNB; ++cc) lc[cc] = readlane(ps, cc);  // L[k0+cc][k0+jj] sg
#pragma unroll
        for (int cc = jj + 1; cc < kNB; ++cc) P0[cc] = fmaf(-P0[jj], lc[cc], P0[cc]);
        if (G == 1) {  // (zeros past row N-1: a branch on gact costs more)
          P[0][jj] *= inv;
#pragma unroll
          for (int cc = jj + 1; cc < kNB; ++cc) P[0][cc] = fmaf(-P[0][jj], lc[cc], P[0][cc]);
        }
      } else if (gact > 0) {
        // more chunks: one multiplier at a time (fewer scalar registers live)
#pragma unroll
        for (int g = 0; g < G; ++g) P[g][jj] *= inv;
#pragma unroll
        for (int cc = jj + 1; cc < kNB; ++cc) {
          const float lc = readlane(ps, cc);  // L[k0+cc][k0+jj] sg
          P0[cc] = fmaf(-P0[jj], lc, P0[cc]);
#pragma unroll
          for (int g = 0; g < G; ++g) P[g][cc] = fmaf(-P[g][jj], lc, P[g][cc]);
        }
      } else {
#pragma unroll
        for (int cc = jj + 1; cc < kNB; ++cc) P0[cc] = fmaf(-P0[jj], readlane(ps, cc), P0[cc]);
      }
    }
  }
  panel_store(M, N, k0, k0 + lane, P0, lmax);
  if (gact > 0) {
#pragma unroll
    for (int g = 0; g < G; ++g) panel_store(M, N, k0, k0 + lane + 64 * (1 + g), P[g], lmax);
  }
  return fail;
}

// The panel factorisation (see above).
template <int RPL, class MF>
QPD bool factor_panel(MF *M, int N, int npos, int k0, bool dyn, float &pmax, float &pmaxh,
                      int &nreg, float &lmax) {
  constexpr int GRP = RPL - 1 < 4 ? RPL - 1 : 4;
  const int lane = threadIdx.x & 63;
  const int kb = min(kNB, N - k0);
  float P0[kNB], iv[kNB];
  // extra chunks that hold rows of the system (uniform)
  const int gact = min(GRP, (N - k0 - 1) >> 6);
  const bool fail =
      panel_sweep<GRP>(M, N, npos, k0, kb, gact, dyn, pmax, pmaxh, nreg, lmax, P0, iv);
  // rows past the first 64 (1 + GRP): replay the eliminations with the
  // finished diagonal block, GRP chunks at a time
  float P[GRP > 0 ? GRP : 1][kNB];
#pragma unroll 1
  for (int t0 = 1 + GRP; t0 < RPL; t0 += GRP) {
    if (k0 + 64 * t0 >= N) break;
#pragma unroll
    for (int g = 0; g < GRP; ++g) panel_load(M, N, k0, k0 + lane + 64 * (t0 + g), P[g]);
#pragma unroll
    for (int jj = 0; jj < kNB; ++jj) {
      if (jj < kb) {
        const float sg = (k0 + jj) < npos ? 1.f : -1.f;
#pragma unroll
        for (int g = 0; g < GRP; ++g) P[g][jj] *= iv[jj];
#pragma unroll
        for (int cc = jj + 1; cc < kNB; ++cc) {
          const float lc = readlane(P0[jj], cc) * sg;
#pragma unroll
          for (int g = 0; g < GRP; ++g) P[g][cc] = fmaf(-P[g][jj], lc, P[g][cc]);
        }
      }
    }
#pragma unroll
    for (int g = 0; g < GRP; ++g) panel_store(M, N, k0, k0 + lane + 64 * (t0 + g), P[g], lmax);
  }
  return fail;
}

// Equilibration of the border for the pivot tests.  The regularisation
// test compares each border pivot with the largest border pivot accepted so
// far, so a border that mixes rows of very different norms (inequality rows
// of G and equality rows of A in different units) would have the small
// rows' pivots taken for numerical zeros.  Before the factorisation, border
// row i (i >= npos) is multiplied by s_i = 2^k_i and its diagonal entry by
// s_i^2, with k_i = floor((e_max - e_i) / 2), e_i the binary exponent of
// |C_i|^2 and e_max the largest one (rows within about a factor of two in
// norm of the largest keep s_i = 1); after it, row i of the factor is
// divided by s_i.  The scalings are powers of two and so exact: the result
// is bit for bit the factor of the unscaled matrix wherever the scaled
// tests decide as the unscaled ones would, and the factor with the scaled
// tests' replacements otherwise.  The assembly computes e_i while it copies
// the border rows and keeps it in the first float of row i's padding, the
// per-wave maxima of e in flag[8 ..] (at most 8 waves).
constexpr int kNoExp = -1000;
QPD int mpad(int i) { return moff(i) + 16 * ((i >> 4) + 1); }
template <int T>
QPD int border_emax(const li *flag) {
  int e = kNoExp;
#pragma unroll
  for (int w = 0; w < T / 64; ++w) e = max(e, flag[8 + w]);
  return e;
}
template <class MF>
QPD int border_shift(const MF *M, int i, int emax) {
  const int e = __float_as_int(M[mpad(i)]);
  return e == kNoExp ? 0 : min((emax - e) >> 1, 30);
}
// Exponent e_i of the squared norm ss (the same in all 16 lanes of row i's
// group) into row i's padding (if store), and the thread's running maximum.
template <class MF>
QPD void border_exponent(MF *M, int i, bool store, int sub, float ss, float &el) {
  ss = row_bfly<OpSum>(ss);
  int e = kNoExp;
  if (ss > 0.f && ss <= FLT_MAX) (void)frexpf(ss, &e);
  if (store) {
    if (sub == 0) M[mpad(i)] = __int_as_float(e);
    el = fmaxf(el, (float)e);
  }
}
// Per-wave maxima of the exponents into flag[8 ..]; read after a barrier.
template <int T>
QPD void border_exponents_done(float el, li *flag) {
  static_assert(T / 64 <= 8, "per-wave exponent slots");
  el = wave_bfly<OpMax>(el);
  if ((threadIdx.x & 63) == 0) flag[8 + (threadIdx.x >> 6)] = (int)el;
}
// Wave 0: f(i, k_i) for every border row i with k_i > 0, in row order (a
// lane per row reads the exponents; the rows to rescale, usually few, are
// then taken one at a time by the whole wave).
template <class MF, class F>
QPD void border_shifted_rows(const MF *M, int N, int npos, int emax, F &&f) {
  const int lane = threadIdx.x & 63, K = N - npos;
  for (int k0 = 0; k0 < K; k0 += 64) {
    const int k = k0 + lane;
    const int sh = k < K ? border_shift(M, npos + k, emax) : 0;
    unsigned long long b = __ballot(sh > 0);
    while (b) {
      const int l = __builtin_ctzll(b);
      b &= b - 1;
      f(npos + k0 + l, __builtin_amdgcn_readlane(sh, l));
    }
  }
}

// In-place M = L diag(sg) L' (lower triangle, packed-blocked layout),
// sg_j = +1 for j < npos, -1 otherwise.  Blocked right-looking with one
// panel of lookahead: after panel k is factored, all waves first apply it
// to the next panel's 16 columns; then wave 0 factors the next panel while
// the other waves apply panel k to the rest of the trailing matrix.  The
// updates run on the matrix cores in 16x16 tiles (rank16_tile16).  The
// strict upper part of each row's last 16-column segment is left at exact
// zeros.  Returns false (uniformly) if a pivot sg_j * a_jj is not a positive
// finite number.  With dyn, numerically zero pivots are regularised (see
// factor_panel; the tests see the border equilibrated, border_exponent) and
// flag[2] receives their count.  flag[0] is the failure flag, flag[4] the
// largest accepted pivot (float bits, the border's in equilibrated units);
// flag[1] and flag[3] are left alone, flag[8 ..] is scratch.  RPL = rows
// per lane, >= ceil(N / 64).
template <int T, int RPL, class MF>
QPK_PHASE bool signed_cholesky(MF *M, int N, int npos, li *flag, bool dyn) {
  M = rflp(M); N = rfl(N); npos = rfl(npos); flag = rflp(flag); dyn = rfl(dyn);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  // wave 0's running pivot scale and count of regularised pivots
  float pmax = 0.f, pmaxh = 0.f, lmax = 0.f;
  int nreg = 0;
  if (tid == 0) { flag[0] = 0; flag[2] = 0; }
  // with the pivot tests on, they see the border equilibrated: wave 0
  // scales the rows before its first panel (the other waves first read
  // them after the barrier that follows it) and takes the scaling back out
  // of the factor at the end (see border_exponent)
  const bool eq = dyn && N > npos;
  const int emax = eq ? border_emax<T>(flag) : 0;
  if (wid == 0) {
    if (eq) {
      border_shifted_rows(M, N, npos, emax, [&](int i, int sh) {
        MF *row = M + moff(i);
        const float s = ldexpf(1.f, sh);
        for (int j = lane; j < npos; j += 64) row[j] *= s;
        if (lane == 0) row[i] *= s * s;  // the border block is diagonal here
      });
      __threadfence_block();  // the panel's loads see the scaled rows
    }
    const bool fail = factor_panel<RPL>(M, N, npos, 0, dyn, pmax, pmaxh, nreg, lmax);
    if (fail && lane == 0) flag[0] = 1;
  }
  __syncthreads();
#pragma unroll 1
  for (int k0 = 0; k0 + kNB < N; k0 += kNB) {
    const int r0 = k0 + kNB, R = N - r0;
    // (1) apply panel k0 to the next panel's columns [r0, r0+16): 16x16
    // tiles on the matrix cores, one wave per tile
    {
      const int nbl = (R + 15) >> 4;
      for (int t = wid; t < nbl; t += T / 64) rank16_tile16(M, N, npos, k0, (r0 >> 4) + t, r0 >> 4);
    }
    __syncthreads();
    // (2) wave 0: factor the next panel; waves 1..: rest of the update
    if (wid == 0) {
      const bool fail = factor_panel<RPL>(M, N, npos, r0, dyn, pmax, pmaxh, nreg, lmax);
      if (fail && lane == 0) flag[0] = 1;
    } else {
      const int r1 = r0 + kNB, R1 = N - r1;
      if (R1 > 0) {
        const int nbl = (R1 + 15) >> 4;
        const int ntiles = nbl * (nbl + 1) / 2;
        for (int t = wid - 1; t < ntiles; t += T / 64 - 1) {
          int ti, tj;
          tile_ij(t, ti, tj);
          rank16_tile16(M, N, npos, k0, (r1 >> 4) + ti, (r1 >> 4) + tj);
        }
      }
    }
    __syncthreads();
  }
  if (wid == 0) {
    lmax = wave_bfly<OpMax>(lmax);
    // with regularised pivots, entries of L far beyond the scale sqrt(pmax)
    // of a stable factor mean the replaced pivots amplified rounding errors:
    // report a failure so the caller factors again with a uniform floor
    pmax = fmaxf(pmax, pmaxh);
    if (lane == 0 && nreg > 0 && !(lmax <= kGrowthMax * sqrtf(pmax))) flag[0] = 1;
    if (eq) {
      border_shifted_rows(M, N, npos, emax, [&](int i, int sh) {
        MF *row = M + moff(i);
        const float r = ldexpf(1.f, -sh);
        for (int j = lane; j <= i; j += 64) row[j] *= r;
      });
    }
  }
  if (tid == 0) {
    flag[2] = nreg;
    flag[4] = __float_as_int(pmax);  // largest accepted pivot (retry scale)
  }
  __syncthreads();
  return flag[0] == 0;
}

// dv[c] = dinv[c] for c < CW (CW a multiple of 4) as 16-byte loads; dinv
// is allocated in whole 16-entry blocks, and entries past the system's last
// row are never used.
template <int CW>
QPD void load_dinv(const lf *dinv, float (&dv)[CW]) {
#pragma unroll
  for (int c = 0; c < CW; c += 4) {
    const f4v v4 = *reinterpret_cast<const lf4 *>(dinv + c);
    dv[c] = v4.x; dv[c + 1] = v4.y; dv[c + 2] = v4.z; dv[c + 3] = v4.w;
  }
}

// o[t] = p[t] for t < RPL (p aligned to RPL floats) if `in`, else zeros, as
// one vector load for RPL <= 4 (16-byte loads above).
template <int RPL, class MF>
QPD void load_run(const MF *p, bool in, float (&o)[RPL]) {
  if constexpr (RPL == 1) {
    o[0] = in ? p[0] : 0.f;
  } else if constexpr (RPL == 2) {
    f2v v = {0.f, 0.f};
    if (in) v = *reinterpret_cast<const typename Vec2<MF>::type *>(p);
    o[0] = v.x; o[1] = v.y;
  } else {
    typedef typename Vec4<const MF>::type CV4;
#pragma unroll
    for (int t = 0; t < RPL; t += 4) {
      f4v v = {0.f, 0.f, 0.f, 0.f};
      if (in) v = *reinterpret_cast<CV4 *>(p + t);
      o[t] = v.x; o[t + 1] = v.y; o[t + 2] = v.z; o[t + 3] = v.w;
    }
  }
}

// Solve (L diag(sg) L') u = r in place for one right-hand side held in
// `r` (length N), by a single wave with the vector in registers (lane owns
// rows RPL*lane + t).  The forward sweep walks rows of L, the backward sweep
// reads L[j][i] from row j; dinv[j] = 1 / L[j][j].  Each 16-column block of L
// is loaded into registers in bursts of CW columns (all 16, or two halves
// of 8 when RPL = 16 to bound registers), then its dependent steps run
// register-only.
template <int RPL, class MF>
QPD void signed_solve_wave(const MF *M, int N, int npos, const lf *dinv, lf *r, const MF *zrow) {
  typedef typename Vec4<const MF>::type CV4;
  static_assert(kNB % RPL == 0, "row slot must be static within a block");
  constexpr int CW = RPL > 8 ? 8 : kNB;
  const int lane = threadIdx.x & 63;
  // lane l owns rows RPL*l + t, so row j sits in lane j/RPL, slot j%RPL.
  // The factor holds exact zeros right of the diagonal inside every row's
  // padded 16-column segment; rows that must not be touched in a block read
  // the zero row `zrow` (16 zeros stored after M's last row, so both
  // pointers are in M's address space) instead, so no per-step masking is
  // needed.  The
  // diagonal entry is applied by overwriting the owner's value after the FMA.
  float a[RPL];
#pragma unroll
  for (int t = 0; t < RPL; ++t) {
    const int i = RPL * lane + t;
    a[t] = i < N ? r[i] : 0.f;
  }
  // forward sweep L w = r: w_j = a_j / L[j][j], then a_i -= L[i][j] w_j, i > j
#pragma unroll 1
  for (int j0 = 0; j0 < N; j0 += kNB) {
#pragma unroll
    for (int h = 0; h < kNB; h += CW) {
      float Lc[RPL][CW], dv[CW];
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int i = RPL * lane + t;
        const bool in = i >= j0 && i < N;
        // rows below the block: L[i][j0..j0+15]; rows in the block: their
        // lower part with zeros right of the diagonal; finished rows: zeros
        const MF *row = in ? M + moff(i) + j0 + h : zrow + h;
#pragma unroll
        for (int c = 0; c < CW; c += 4) {
          const f4v v4 = *reinterpret_cast<CV4 *>(row + c);
          Lc[t][c] = v4.x; Lc[t][c + 1] = v4.y; Lc[t][c + 2] = v4.z; Lc[t][c + 3] = v4.w;
        }
      }
      load_dinv<CW>(dinv + j0 + h, dv);
#pragma unroll
      for (int c = 0; c < CW; ++c) {
        const int j = j0 + h + c;
        if (j < N) {
          const float wj = readlane(a[(h + c) % RPL], j / RPL) * dv[c];
#pragma unroll
          for (int t = 0; t < RPL; ++t) a[t] = fmaf(-Lc[t][c], wj, a[t]);
          if (lane == j / RPL) a[(h + c) % RPL] = wj;
        }
      }
    }
  }
  // sign: w <- sg w
#pragma unroll
  for (int t = 0; t < RPL; ++t) {
    const int i = RPL * lane + t;
    if (i >= npos) a[t] = -a[t];
  }
  // backward sweep L' u = w: u_j = a_j / L[j][j], then a_i -= L[j][i] u_j, i < j
#pragma unroll 1
  for (int b0 = ((N - 1) / kNB) * kNB; b0 >= 0; b0 -= kNB) {
#pragma unroll
    for (int h = kNB - CW; h >= 0; h -= CW) {
      float Lr[RPL][CW], dv[CW];
      // rows b0 .. b0+15 are one block: row b0+c starts c * rstride floats
      // after row b0 (the last rows, past N-1, read row N-1)
      const int rstride = 20 + 16 * (b0 >> 4);
      const MF *brow = M + moff(b0) + RPL * lane;
      // rows above the block read row j; rows in the block read row j's
      // zero padding right of its diagonal; rows below read zeros.  A lane's
      // RPL rows are all above the block or all at or below it.
      const bool above = RPL * lane < b0 + kNB;
#pragma unroll
      for (int c = 0; c < CW; ++c) {
        float run[RPL];
        load_run<RPL>(brow + min(h + c, N - 1 - b0) * rstride, above, run);
#pragma unroll
        for (int t = 0; t < RPL; ++t) Lr[t][c] = run[t];
      }
      load_dinv<CW>(dinv + b0 + h, dv);
#pragma unroll
      for (int c = CW - 1; c >= 0; --c) {
        const int j = b0 + h + c;
        if (j < N) {
          const float uj = readlane(a[(h + c) % RPL], j / RPL) * dv[c];
#pragma unroll
          for (int t = 0; t < RPL; ++t) a[t] = fmaf(-Lr[t][c], uj, a[t]);
          if (lane == j / RPL) a[(h + c) % RPL] = uj;
        }
      }
    }
  }
#pragma unroll
  for (int t = 0; t < RPL; ++t) {
    const int i = RPL * lane + t;
    if (i < N) r[i] = a[t];
  }
}

// out[j] (+)= sum_i R[i*ld + j] x[i], accumulated in AT (FP32 or FP64);
// barriers inside.
template <int T, class AT, class RF, class XF>
QPD float coldot_d(const RF *R, int ld, int rows, int cols, const XF *x,
                   typename LdsT<AT>::type *out, bool add, typename LdsT<AT>::type *part) {
  float mx = 0.f;  // largest |column sum| this thread produced
  const int cw = cols <= 64 ? 64 : (cols <= 128 ? (T >= 128 ? 128 : 64) : (T >= 256 ? 256 : T));
  const int groups = T / cw;
  const int g = threadIdx.x / cw, jl = threadIdx.x % cw;
  for (int jb = 0; jb < cols; jb += cw) {
    const int j = jb + jl;
    AT acc = 0;
    if (j < cols) {
      // independent loads first (several in flight), then the accumulation chain
#pragma unroll 8
      for (int i = g; i < rows; i += groups) acc = fma((AT)R[(size_t)i * ld + j], (AT)x[i], acc);
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    if (g == 0 && j < cols) {
      AT s = 0;
      for (int gg = 0; gg < groups; ++gg) s += part[gg * cw + jl];
      out[j] = add ? out[j] + s : s;
      mx = fmaxf(mx, fabsf((float)s));
    }
    __syncthreads();
  }
  return mx;
}

// The products the residuals need, in one pass over Q, G and A (each n
// columns wide), accumulated in AT (FP32, or FP64 for the residuals of the
// FP64 policy and of escalated refinements): gx = G x and ax = A x (row dots) and
// rt = Q'x + G'z + A'y (column sums).  16 lanes share a row (columns
// jb + sub + 16k, k < 4, in blocks of 64), T/16 rows at a time, with the
// loads of several rows in flight before their arithmetic, so each input
// element is read once.  The column sums of each matrix are reduced across
// row groups (shuffles inside a wave, then `part`, T values, across
// waves); their largest magnitudes, which scale the residuals, come back in
// mq, mg, ma (per-thread partial maxima).  Without gcols, G contributes
// its row dots only (z is not read).  No LDS pointer is tested against
// NULL: LDS address 0 is a valid address.  Barriers inside.
template <int T, class AT>
QPD void kkt_matvecs(const gf *Q, const gf *G, const gf *A, int n, int m, int p, const lf *x,
                     const lf *z, bool gcols, const lf *y, typename LdsT<AT>::type *gx,
                     typename LdsT<AT>::type *ax, typename LdsT<AT>::type *rt,
                     typename LdsT<AT>::type *part, float &mq, float &mg, float &ma) {
  typedef typename LdsT<AT>::type la;
  constexpr int RG = T / 16;
  const int tid = threadIdx.x, sub = tid & 15, grp = tid >> 4, wid = tid >> 6;
  mq = mg = ma = 0.f;
  for (int jb = 0; jb < n; jb += 64) {
    AT xv[4], cq[4], cg[4], ca[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int j = jb + sub + 16 * k;
      xv[k] = j < n ? (AT)x[j] : (AT)0;
      cq[k] = cg[k] = ca[k] = 0;
    }
    // rows of R weighted by w (if cols) into c; with dots, also the row dots
    // with x into out
    auto sweep = [&](const gf *R, int rows, const lf *w, bool cols, la *out, bool dots,
                     AT(&c)[4]) {
#pragma unroll 4
      for (int i0 = 0; i0 < rows; i0 += RG) {
        const int i = i0 + grp;
        float e[4] = {0.f, 0.f, 0.f, 0.f};
        AT wi = 0;
        if (i < rows) {
          const gf *Ri = R + (size_t)i * n + jb + sub;
#pragma unroll
          for (int k = 0; k < 4; ++k)
            if (jb + sub + 16 * k < n) e[k] = Ri[16 * k];
          if (cols) wi = (AT)w[i];
        }
        AT d = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          c[k] = fma((AT)e[k], wi, c[k]);
          if (dots) d = fma((AT)e[k], xv[k], d);
        }
        if (dots) {
          d = row_bfly<OpSum>(d);
          if (sub == 0 && i < rows) out[i] = jb ? out[i] + d : d;
        }
      }
    };
    sweep(Q, n, x, true, gx, false, cq);
    if (m) sweep(G, m, z, gcols, gx, true, cg);
    if (p) sweep(A, p, y, true, ax, true, ca);
    // column sums across the row groups, one matrix at a time
    auto reduce = [&](AT(&c)[4], bool first, float &mx) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        c[k] = bfly<32, OpSum>(bfly<16, OpSum>(c[k]));
      }
      if ((tid & 63) < 16) {
#pragma unroll
        for (int k = 0; k < 4; ++k) part[wid * 64 + 16 * k + sub] = c[k];
      }
      __syncthreads();
      if (tid < 64 && jb + tid < n) {
        AT sum = 0;
#pragma unroll
        for (int w = 0; w < T / 64; ++w) sum += part[w * 64 + tid];
        rt[jb + tid] = first ? sum : rt[jb + tid] + sum;
        mx = fmaxf(mx, fabsf((float)sum));
      }
      __syncthreads();
    };
    reduce(cq, true, mq);
    if (m && gcols) reduce(cg, false, mg);
    if (p) reduce(ca, false, ma);
  }
}

// ---------------------------------------------------------------------------
// The per-QP context: LDS views plus this QP's global problem data.
//
// The addresses of the views live in a small table in LDS (one per
// workgroup, written once per QP), not in the context object: each use
// reads its entry back (a broadcast LDS load, made uniform), so no address
// stays live in registers from one phase to the next.  Kept live, the
// fifty-odd addresses overflow the scalar register file and are spilled and
// reloaded one by one at every phase entry.  Global addresses take two
// words.
enum CtxSlot {
  CS_X, CS_Y, CS_Z, CS_S, CS_V, CS_Q, CS_H, CS_B, CS_E, CS_D, CS_C,
  CS_RT, CS_RI, CS_RE, CS_RZ, CS_RS, CS_TGZ, CS_TAY,
  CS_T0, CS_T1, CS_U0, CS_U1, CS_DV0, CS_DV1, CS_DINV, CS_PART, CS_RED,
  CS_W0, CS_W1, CS_RR, CS_RD, CS_PAN, CS_DD, CS_ROLE, CS_BIDX, CS_ELIST, CS_IFLAG, CS_STG,
  CS_M = 40, CS_MZ = 42, CS_GQ = 44, CS_GQV = 46, CS_GA = 48, CS_GB = 50, CS_GG = 52,
  CS_GH = 54, CS_N = 56
};
static __shared__ unsigned qpk_ctab[CS_N];
static_assert(CS_N * 4 + 16 * 8 <= kStaticLds, "static LDS bound of the launch planning");

// A context address: reads entry K of the table (PT carries the address
// space, 32-bit LDS or 64-bit global addresses).
template <class PT, int K>
struct CtxRef {
  QPD PT *get() const {
    if constexpr (sizeof(PT *) == 4) {
      return (PT *)(uintptr_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)qpk_ctab[K]);
    } else {
      const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)qpk_ctab[K]);
      const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)qpk_ctab[K + 1]);
      return (PT *)(uintptr_t)(((uint64_t)hi << 32) | lo);
    }
  }
  QPD operator PT *() const { return get(); }
  // by one thread; a barrier must follow before any use
  QPD void set(PT *a) const {
    const uint64_t v = (uint64_t)(uintptr_t)a;
    qpk_ctab[K] = (uint32_t)v;
    if constexpr (sizeof(PT *) == 8) qpk_ctab[K + 1] = (uint32_t)(v >> 32);
  }
};

template <class MF>
struct Ctx {
  typedef MF MT;
  int n, m, p, kb;
  CtxRef<const gf, CS_GQ> Q;
  CtxRef<const gf, CS_GQV> q_g;
  CtxRef<const gf, CS_GA> A;
  CtxRef<const gf, CS_GB> b_g;
  CtxRef<const gf, CS_GG> G;
  CtxRef<const gf, CS_GH> h_g;
  CtxRef<MF, CS_M> M;    // factor storage (LDS or global)
  CtxRef<lf, CS_X> x; CtxRef<lf, CS_Y> y; CtxRef<lf, CS_Z> z; CtxRef<lf, CS_S> s;
  CtxRef<lf, CS_V> v; CtxRef<lf, CS_Q> q; CtxRef<lf, CS_H> h; CtxRef<lf, CS_B> b;
  CtxRef<lf, CS_E> E; CtxRef<lf, CS_D> D; CtxRef<lf, CS_C> c;
  CtxRef<lf, CS_RT> rt; CtxRef<lf, CS_RI> ri; CtxRef<lf, CS_RE> re; CtxRef<lf, CS_RZ> rz;
  CtxRef<lf, CS_RS> rs; CtxRef<lf, CS_TGZ> tGz; CtxRef<lf, CS_TAY> tAy;
  CtxRef<lf, CS_T0> t0; CtxRef<lf, CS_T1> t1; CtxRef<lf, CS_U0> u0; CtxRef<lf, CS_U1> u1;
  CtxRef<lf, CS_DV0> dv0; CtxRef<lf, CS_DV1> dv1; CtxRef<lf, CS_DINV> dinv;
  CtxRef<lf, CS_PART> part; CtxRef<lf, CS_RED> red;
  CtxRef<lf, CS_W0> w0; CtxRef<lf, CS_W1> w1; CtxRef<lf, CS_RR> rr; CtxRef<lf, CS_RD> rd;
  CtxRef<lf, CS_PAN> pan;
  CtxRef<MF, CS_MZ> mz;  // 16 zeros after M's last row (same address space as M)
  CtxRef<ldd, CS_DD> dd;
  CtxRef<li, CS_ROLE> role; CtxRef<li, CS_BIDX> bidx; CtxRef<li, CS_ELIST> elist;
  CtxRef<li, CS_IFLAG> iflag;
  CtxRef<lf, CS_STG> stg;  // matrix-core assembly staging (aliases u0 .. dd)
  int amode;  // H-block assembly: 0 FP32 VALU, 1 BF16x3 MFMA, 2 FP32 MFMA
  int dyn;    // bounded form: regularise degenerate factorisations (R13)
  int rmode;  // residual precision: 0 FP32 first (FP64 refinement after a
              // stall), 1 FP64 residuals everywhere, 2 FP32 only
  float bo;   // line-search back-off factor (1 = none)
  __attribute__((address_space(3))) long long *pt;
};

// Sizes and scalar settings of the context, and (thread 0) the address
// table; the caller's next barrier publishes the table.
template <class MF>
QPD void init_ctx(Ctx<MF> &C, lf *sm, const Layout &L, MF *Mptr, const gf *Qg, const gf *qg,
                  const gf *Ag, const gf *bg, const gf *Gg, const gf *hg) {
  C.n = L.n; C.m = L.m; C.p = L.p; C.kb = L.kb;
  if (threadIdx.x == 0) {
    C.Q.set(Qg); C.q_g.set(qg); C.A.set(Ag); C.b_g.set(bg); C.G.set(Gg); C.h_g.set(hg);
    C.M.set(Mptr);
    C.x.set(sm + L.x); C.y.set(sm + L.y); C.z.set(sm + L.z); C.s.set(sm + L.s);
    C.v.set(sm + L.v); C.q.set(sm + L.q); C.h.set(sm + L.h); C.b.set(sm + L.b);
    C.E.set(sm + L.E); C.D.set(sm + L.D); C.c.set(sm + L.c);
    C.rt.set(sm + L.rt); C.ri.set(sm + L.ri); C.re.set(sm + L.re); C.rz.set(sm + L.rz);
    C.rs.set(sm + L.rs); C.tGz.set(sm + L.tGz); C.tAy.set(sm + L.tAy);
    C.t0.set(sm + L.t0); C.t1.set(sm + L.t1); C.u0.set(sm + L.u0); C.u1.set(sm + L.u1);
    C.dv0.set(sm + L.dv0); C.dv1.set(sm + L.dv1); C.dinv.set(sm + L.dinv);
    C.part.set(sm + L.part); C.red.set(sm + L.red);
    C.w0.set(sm + L.w0); C.w1.set(sm + L.w1); C.rr.set(sm + L.rr); C.rd.set(sm + L.rd);
    C.pan.set(sm + L.pan);
    C.mz.set(Mptr + moff(L.Nmax));
    C.dd.set(reinterpret_cast<ldd *>(sm + L.dd));
    C.role.set(reinterpret_cast<li *>(sm + L.role));
    C.bidx.set(reinterpret_cast<li *>(sm + L.bidx));
    C.elist.set(reinterpret_cast<li *>(sm + L.elist));
    C.iflag.set(reinterpret_cast<li *>(sm + L.iflag));
    C.stg.set(sm + L.stg);
  }
  C.amode = 0;
  C.dyn = 1;
  C.rmode = 0;
  C.bo = 1.f;
  C.pt = nullptr;  // set by profiling builds
}


// Uniform copy of a context (see rfl): the sizes and settings; the
// addresses are read from the table where they are used.
template <class MF>
QPD Ctx<MF> uctx(const Ctx<MF> &I) {
  Ctx<MF> C;
  C.n = rfl(I.n); C.m = rfl(I.m); C.p = rfl(I.p); C.kb = rfl(I.kb);
  C.amode = rfl(I.amode); C.dyn = rfl(I.dyn); C.rmode = rfl(I.rmode); C.bo = rflf(I.bo);
  C.pt = rflp(I.pt);
  return C;
}

// Residuals at (x, y, z, s) and, for the bounded form, (v, kappa).
// Returns the scaled residual measure (uniform); `bad` = a non-finite value
// was seen.  Complementarity: max(z s) in the solve; in the relaxation
// (kr > 0) |kappa - kr| / kr for the implicit forms, whose retraction keeps
// every z_i s_i equal to kappa (per-row products differ from it only by
// rounding, about 1e-7 relative in FP32), and max|z s - kr| / kr for the
// standard form.  The matrix-vector products are accumulated in AT: FP32 by
// default, FP64 under the FP64 residual policy (the FP32 iterate is exact in
// FP64, so that residual is limited only by the iterate's rounding).
template <int T, class AT, class CT>
QPK_PHASE float residuals(CT &Cin_, bool bounded, float kappa, float kr, bool *bad) {
  CT C = uctx(Cin_);
  bounded = rfl(bounded); kappa = rflf(kappa); kr = rflf(kr);
  typedef typename LdsT<AT>::type la;
  const int n = C.n, m = C.m, p = C.p, tid = threadIdx.x;
  // one accumulator for Qx + G'z + A'y; the pieces' norms are taken as they
  // are produced
  la *gxd = reinterpret_cast<la *>(C.dd.get()), *axd = gxd + m, *rtd = gxd + m + p;
  la *pd = reinterpret_cast<la *>(C.part.get());
  enum { RT, QX, QQ, GZ, AY, RI, GX, SS, HH, RE, AX, BB, RZS, ZZ, CC, NF, NK };
  float mx[NK];
#pragma unroll
  for (int k = 0; k < NK; ++k) mx[k] = 0.f;
  kkt_matvecs<T, AT>(C.Q, C.G, C.A, n, m, p, C.x, C.z, true, C.y, gxd, axd, rtd, pd, mx[QX],
                     mx[GZ], mx[AY]);
  const bool man = bounded && kr > 0.f;  // relaxation of an implicit form
  for (int i = tid; i < n; i += T) {
    const float r = (float)(rtd[i] + (AT)C.q[i]);
    C.rt[i] = r;
    mx[RT] = fmaxf(mx[RT], fabsf(r));
    mx[QQ] = fmaxf(mx[QQ], fabsf(C.q[i]));
    if (!finitef(r)) mx[NF] = 1.f;
  }
  for (int i = tid; i < m; i += T) {
    const AT gx = gxd[i];
    const float si = C.s[i], zi = C.z[i];
    const float r = (float)(gx + (AT)si - (AT)C.h[i]);
    C.ri[i] = r;
    mx[RI] = fmaxf(mx[RI], fabsf(r));
    mx[GX] = fmaxf(mx[GX], fabsf((float)gx));
    mx[SS] = fmaxf(mx[SS], fabsf(si));
    mx[HH] = fmaxf(mx[HH], fabsf(C.h[i]));
    mx[ZZ] = fmaxf(mx[ZZ], fabsf(zi));
    float rz = 0.f, rs = 0.f;
    if (bounded) {
      const float vi = C.v[i];
      rz = zi - bk(vi, kappa);
      rs = si - bk(-vi, kappa);
      C.rz[i] = rz;
      C.rs[i] = rs;
    }
    mx[RZS] = fmaxf(mx[RZS], fmaxf(fabsf(rz), fabsf(rs)));
    const float zs = zi * si;
    if (!man) mx[CC] = fmaxf(mx[CC], kr > 0.f ? fabsf(zs - kr) / kr : zs);
    if (!finitef(r) || !finitef(zs) || !finitef(rz) || !finitef(rs)) mx[NF] = 1.f;
  }
  for (int i = tid; i < p; i += T) {
    const AT ax = axd[i];
    const float r = (float)(ax - (AT)C.b[i]);
    C.re[i] = r;
    mx[RE] = fmaxf(mx[RE], fabsf(r));
    mx[AX] = fmaxf(mx[AX], fabsf((float)ax));
    mx[BB] = fmaxf(mx[BB], fabsf(C.b[i]));
    if (!finitef(r)) mx[NF] = 1.f;
  }
  block_reduce<T, OpMax, NK>(mx, C.red);
  const float rt_s = mx[RT] / (1.f + fmaxf(fmaxf(mx[QX], mx[QQ]), fmaxf(mx[GZ], mx[AY])));
  const float ri_s = m ? mx[RI] / (1.f + fmaxf(mx[GX], fmaxf(mx[SS], mx[HH]))) : 0.f;
  const float re_s = p ? mx[RE] / (1.f + fmaxf(mx[AX], mx[BB])) : 0.f;
  const float rzs = m ? mx[RZS] / (1.f + fmaxf(mx[ZZ], mx[SS])) : 0.f;
  const float cc = m ? (man ? fabsf(kappa - kr) / kr : mx[CC]) : 0.f;
  *bad = mx[NF] != 0.f;
  return fmaxf(fmaxf(rt_s, ri_s), fmaxf(fmaxf(re_s, rzs), cc));
}

// Workgroup-wide exclusive compaction of rows with flag set, in row order.
// Writes the compacted indices to out[] and returns the count (uniform).
template <int T>
QPD int compact_rows(const li *flag, int m, li *out, lf *red) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int base = 0;
  for (int i0 = 0; i0 < m; i0 += T) {
    const int i = i0 + tid;
    const bool f = i < m && flag[i];
    const unsigned long long bal = __ballot(f);
    const int pre = __popcll(bal & ((1ull << lane) - 1ull));
    const int wcnt = __popcll(bal);
    li *wsum = reinterpret_cast<li *>(red);
    if (lane == 0) wsum[w] = wcnt;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < T / 64; ++k) {
      const int c = wsum[k];
      off += k < w ? c : 0;
      tot += c;
    }
    if (f) out[base + off + pre] = i;
    base += tot;
    __syncthreads();
  }
  return base;
}

// Bounded form: retraction derivatives and the sign split.  Returns the
// number of bordered rows nb; fills E, D, c, role (border index or -1),
// bidx (border rows), elist (eliminated rows) and iflag[1] = #eliminated.
template <int T, class CT>
QPK_PHASE int partition_bounded(CT &Cin_, float kappa) {
  CT C = uctx(Cin_);
  kappa = rflf(kappa);
  const int m = C.m, kb = C.kb, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  constexpr int NW = T / 64;
  li *ws = reinterpret_cast<li *>(C.red.get());  // per-wave counts [2][NW]
  const unsigned long long below = (1ull << lane) - 1ull;
  // One sweep: retraction derivatives, and the border / eliminated lists in
  // row order from wave ballots (the common case: at most kb rows with v > 0)
  int nb = 0, ne = 0;
  for (int i0 = 0; i0 < m; i0 += T) {
    const int i = i0 + tid;
    const bool valid = i < m;
    bool f = false;
    if (valid) {
      const float vi = C.v[i];
      const float r = sqrtf(fmaf(vi, vi, 4.f * kappa));
      C.E[i] = dbk(vi, kappa, r);
      C.D[i] = dbk(-vi, kappa, r);
      C.c[i] = 1.f / r;
      f = vi > 0.f;
    }
    const unsigned long long bb = __ballot(valid && f), be = __ballot(valid && !f);
    if (lane == 0) {
      ws[w] = __popcll(bb);
      ws[NW + w] = __popcll(be);
    }
    __syncthreads();
    int ob = 0, oe = 0, tb = 0, te = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      const int cb = ws[k], ce = ws[NW + k];
      ob += k < w ? cb : 0;
      oe += k < w ? ce : 0;
      tb += cb;
      te += ce;
    }
    if (valid) {
      if (f) {
        const int k = nb + ob + __popcll(bb & below);
        if (k < kb) C.bidx[k] = i;
        C.role[i] = k;
      } else {
        C.elist[ne + oe + __popcll(be & below)] = i;
        C.role[i] = -1;
      }
    }
    nb += tb;
    ne += te;
    __syncthreads();
  }
  if (nb > kb) {
    // more candidates than border slots: keep the kb largest v (ties by row
    // index) and eliminate the rest.  The rank of row i counts the rows
    // ahead of it; v is read four rows per 16-byte broadcast load, several
    // loads in flight, and the padding past row m is masked.
    li *cand = C.role;
    const lf4 *v4 = reinterpret_cast<const lf4 *>(C.v.get());
    const int m4 = (m + 3) >> 2;
    for (int i = tid; i < m; i += T) {
      int f = 0;
      const float vi = C.v[i];
      if (vi > 0.f) {
        int rank = 0;
        auto ahead = [&](float vj, int j) {
          return (int)(j < m && ((vj > vi) || (vj == vi && j < i)));
        };
#pragma unroll 4
        for (int q = 0; q < m4; ++q) {
          const f4v w4 = v4[q];
          rank += ahead(w4.x, 4 * q) + ahead(w4.y, 4 * q + 1) + ahead(w4.z, 4 * q + 2) +
                  ahead(w4.w, 4 * q + 3);
        }
        f = rank < kb;
      }
      cand[i] = f;
    }
    __syncthreads();
    nb = compact_rows<T>(cand, m, C.bidx, C.red);
    for (int i = tid; i < m; i += T) cand[i] = !cand[i];
    __syncthreads();
    ne = compact_rows<T>(cand, m, C.elist, C.red);
    for (int i = tid; i < m; i += T) C.role[i] = -1;
    __syncthreads();
    for (int k = tid; k < nb; k += T) C.role[C.bidx[k]] = k;
  }
  if (tid == 0) C.iflag[1] = ne;
  __syncthreads();
  return nb;
}

// ---------------------------------------------------------------------------
// H-block assembly on the matrix cores (used for large n).
//
// H = Q + Y'Y with Y = diag(sqrt(w)) G_I (rows of G in elist).  Y is staged
// through LDS 16 rows at a time, column-major: column c of the chunk is a
// record of kStgRec floats, so the MFMA fragment of a lane (4 consecutive
// rows of one column) is a single 8- or 16-byte load, and the A operand of a
// tile (Y_i') and its B operand (Y_j) come from the same records.  Each wave
// owns up to kAsmTiles 16x16 tiles of the lower triangle per pass and
// accumulates them over all chunks in FP32.
//   amode 1 (BF16x3): y = hi + lo with hi = bf16(y), lo = bf16(y - hi);
//     Y_i'Y_j ~ hi_i'hi_j + lo_i'hi_j + hi_i'lo_j on gfx950's 16x16x32 bf16
//     matrix cores with FP32 accumulation: per 16-row chunk one instruction
//     takes K = 32 as [hi; lo]_i against [hi; hi]_j (the first two terms),
//     a second [hi; 0]_i against [lo; 0]_j.  The dropped lo'lo term and the
//     rounding of lo leave a relative error of about 2^-16 per product; the
//     Newton and adjoint solves refine against the exact operator to
//     recover FP32 accuracy.
//   amode 2: FP32 inputs on the 16x16x4 FP32 MFMA.
// Record layout: amode 1: hi of rows 0..15 as 16 bf16 (floats 0..7), lo as
// 16 bf16 (floats 8..15); amode 2: rows 0..15 as floats 0..15.  Floats
// 16..19 pad the record to 80 bytes, which spreads the 16 columns a
// fragment load touches over the LDS banks.
constexpr int kStgRec = 20;
constexpr int kAsmTiles = 9;
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) unsigned lu;

QPD unsigned bf16_pair(float a, float b) {
  return (unsigned)__builtin_bit_cast(unsigned short, (__bf16)a) |
         ((unsigned)__builtin_bit_cast(unsigned short, (__bf16)b) << 16);
}

// LDS floats the matrix-core assembly stages for n columns.
__host__ __device__ inline int stage_floats(int n) { return ((n + 15) & ~15) * kStgRec; }

template <int T, class CT>
QPD void assemble_h_mfma(CT &C, int ne, const lf *wts) {
  constexpr int W = T / 64;
  const int n = C.n, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int n16 = (n + 15) & ~15, nt = n16 >> 4;
  const int ntl = nt * (nt + 1) / 2;
  const int passes = (ntl + W * kAsmTiles - 1) / (W * kAsmTiles);
  const int tpw = (ntl + passes * W - 1) / (passes * W);
  const bool bf = C.amode == 1;
  const int g = lane >> 4, c16 = lane & 15;
  lf *stg = C.stg;
  auto *M = C.M.get();
  for (int pass = 0; pass < passes; ++pass) {
    int ti[kAsmTiles], tj[kAsmTiles];
    bool val[kAsmTiles];
    f4v acc[kAsmTiles];
#pragma unroll
    for (int j = 0; j < kAsmTiles; ++j) {
      const int t = (pass * W + wid) * tpw + j;
      val[j] = j < tpw && t < ntl;
      ti[j] = tj[j] = 0;
      if (val[j]) tile_ij(t, ti[j], tj[j]);
      acc[j] = f4v{0.f, 0.f, 0.f, 0.f};
    }
    for (int k0 = 0; k0 < ne; k0 += 16) {
      __syncthreads();  // the previous chunk has been consumed
      // stage rows k0 .. k0+15 of Y; item e covers rows 2kp, 2kp+1 of column c
      for (int e = tid; e < 8 * n16; e += T) {
        const int kp = e / n16, c = e - kp * n16;
        float y0 = 0.f, y1 = 0.f;
        const int k = k0 + 2 * kp;
        if (c < n) {
          if (k < ne) {
            const int r = C.elist[k];
            y0 = sqrtf(wts[r]) * C.G[(size_t)r * n + c];
          }
          if (k + 1 < ne) {
            const int r = C.elist[k + 1];
            y1 = sqrtf(wts[r]) * C.G[(size_t)r * n + c];
          }
        }
        lf *rec = stg + c * kStgRec;
        if (bf) {
          const float h0 = (float)(__bf16)y0, h1 = (float)(__bf16)y1;
          reinterpret_cast<lu *>(rec)[kp] = bf16_pair(y0, y1);
          reinterpret_cast<lu *>(rec)[8 + kp] = bf16_pair(y0 - h0, y1 - h1);
        } else {
          rec[2 * kp] = y0;
          rec[2 * kp + 1] = y1;
        }
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < kAsmTiles; ++j) {
        if (!val[j]) continue;
        const lf *ra = stg + (16 * ti[j] + c16) * kStgRec;
        const lf *rb = stg + (16 * tj[j] + c16) * kStgRec;
        if (bf) {
          // lane group g holds K = 8g .. 8g+7 of its row (A) or column (B);
          // a record's 16-byte quarters are hi rows 0-7, hi 8-15, lo 0-7,
          // lo 8-15
          const lf4 *RA = reinterpret_cast<const lf4 *>(ra);
          const lf4 *RB = reinterpret_cast<const lf4 *>(rb);
          const f4v zero = {0.f, 0.f, 0.f, 0.f};
          const f4v a1 = RA[g], b1 = RB[g & 1];
          const f4v a2 = g < 2 ? RA[g] : zero, b2 = g < 2 ? RB[2 + g] : zero;
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8v, a1),
                                                          __builtin_bit_cast(bf8v, b1), acc[j],
                                                          0, 0, 0);
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8v, a2),
                                                          __builtin_bit_cast(bf8v, b2), acc[j],
                                                          0, 0, 0);
        } else {
          const f4v a = *reinterpret_cast<const lf4 *>(ra + 4 * g);
          const f4v b = *reinterpret_cast<const lf4 *>(rb + 4 * g);
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, acc[j], 0, 0, 0);
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, acc[j], 0, 0, 0);
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b.z, acc[j], 0, 0, 0);
          acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b.w, acc[j], 0, 0, 0);
        }
      }
    }
    // result layout: register r of lane l is row 4(l/16) + r, column l%16
#pragma unroll
    for (int j = 0; j < kAsmTiles; ++j) {
      if (!val[j]) continue;
      const int col = 16 * tj[j] + c16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * ti[j] + 4 * g + r;
        if (row < n && col <= row) M[moff(row) + col] = C.Q[(size_t)row * n + col] + acc[j][r];
      }
    }
  }
}

// Assemble M = [[H, C'], [C, -Dl]] (lower triangle) for N = n + nb + p.
// H = Q + sum_{r in elist} w_r g_r g_r' with w = weights (E/D bounded,
// z/s standard); border rows = G[bidx] then A; Dl = dl (per border row) and
// delta on the diagonal of the border block.
template <int T, class CT>
QPK_PHASE void assemble(CT &Cin_, int nb, int ne, const lf *wts, bool bounded, float delta) {
  CT C = uctx(Cin_);
  nb = rfl(nb); ne = rfl(ne); wts = rflp(wts); bounded = rfl(bounded); delta = rflf(delta);
  const int n = C.n, p = C.p, tid = threadIdx.x;
  auto *M = C.M.get();
  if (C.amode != 0) {
    assemble_h_mfma<T>(C, ne, wts);
  } else {
  // H block in 4x4 tiles.  Rows of G_I are staged through LDS in chunks
  // (coalesced cooperative loads), then each tile thread reads its 4 + 4
  // entries per row as 16-byte LDS loads.  The staging area is the (not yet
  // written) border part of M when M is in LDS, else the `part` buffer.
  const int ldg = al4(n);
  lf *stage = C.part;
  int cap = 2 * T;
  if constexpr (std::is_same<typename CT::MT, lf>::value) {
    const int N = n + nb + p;
    const int room = moff(N) - moff(n);
    if (room > cap) { stage = (lf *)C.M + moff(n); cap = room; }
  }
  const int R = max(1, cap / ldg);
  const int nt = (n + 3) >> 2;
  const int ntiles = nt * (nt + 1) / 2;
  // tile threads are split into `groups` that take every groups-th staged
  // row; group 0 writes Q + its sum, the others add theirs in a fixed order
  const int groups = ntiles <= T ? min(4, T / ntiles) : 1;
  for (int tb = 0; tb < ntiles; tb += T) {
    const int t = tb + (tid % (groups > 1 ? ntiles : T));
    const int g = groups > 1 ? tid / ntiles : 0;
    const bool act = t < ntiles && g < groups;
    int i0 = 0, j0 = 0;
    if (act) {
      int ti = (int)((sqrtf(8.f * (float)t + 1.f) - 1.f) * 0.5f);
      while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
      while (ti * (ti + 1) / 2 > t) --ti;
      const int tj = t - ti * (ti + 1) / 2;
      i0 = 4 * ti;
      j0 = 4 * tj;
    }
    float acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int bq = 0; bq < 4; ++bq) {
        const int i = min(i0 + a, n - 1), j = min(j0 + bq, n - 1);
        acc[a][bq] = (act && g == 0) ? C.Q[(size_t)i * n + j] : 0.f;
      }
    for (int k0 = 0; k0 < ne; k0 += R) {
      const int kr = min(R, ne - k0);
      __syncthreads();  // the previous chunk has been consumed
      // 16 lanes per staged row (4 columns each, blocks of 64), T/16 rows at
      // a time: the loads of four row batches first, then the stores
      for (int jb = 0; jb < ldg; jb += 64) {
        for (int r0 = 0; r0 < kr; r0 += 4 * (T / 16)) {
          float e[4][4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int r = min(r0 + u * (T / 16) + (tid >> 4), kr - 1);
            load_row4(C.G + (size_t)C.elist[k0 + r] * n, n, 1, n, 0, jb, tid & 15, e[u]);
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int r = r0 + u * (T / 16) + (tid >> 4);
            if (r < kr) {
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const int j = jb + (tid & 15) + 16 * q;
                if (j < ldg) stage[r * ldg + j] = e[u][q];
              }
            }
          }
        }
      }
      __syncthreads();
      if (act) {
#pragma unroll 2
        for (int r = g; r < kr; r += groups) {
          const float w = wts[C.elist[k0 + r]];
          const f4v gi = *reinterpret_cast<const lf4 *>(stage + r * ldg + i0);
          const f4v gj = *reinterpret_cast<const lf4 *>(stage + r * ldg + j0) * w;
          const float gia[4] = {gi.x, gi.y, gi.z, gi.w};
          const float gja[4] = {gj.x, gj.y, gj.z, gj.w};
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int bq = 0; bq < 4; ++bq) acc[a][bq] = fmaf(gia[a], gja[bq], acc[a][bq]);
        }
      }
    }
    for (int gg = 0; gg < groups; ++gg) {
      __syncthreads();  // staging area (may alias M's border rows) / previous group
      if (act && g == gg) {
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const int i = i0 + a;
          if (i < n) {
#pragma unroll
            for (int bq = 0; bq < 4; ++bq) {
              const int j = j0 + bq;
              if (j <= i) {
                if (gg == 0) M[moff(i) + j] = acc[a][bq];
                else M[moff(i) + j] += acc[a][bq];
              }
            }
          }
        }
      }
    }
  }
  }
  __syncthreads();
  // border rows: [C | -Dl (lower part)].  C = [G_B; A] copied by 16 lanes
  // per row, which also take each row's squared norm for the border
  // equilibration of the factorisation (border_exponent); then the lower
  // triangle of the diagonal block.
  const int K = nb + p;
  {
    constexpr int NG = T / 16;
    const int sub = tid & 15, grp = tid >> 4;
    float el = (float)kNoExp;
    for (int k0 = 0; k0 < K; k0 += NG) {
      // groups past the last row repeat it (the row reduction needs all 16
      // lanes) and store nothing
      const int k = k0 + grp, kc = min(k, K - 1);
      const gf *src = kc < nb ? C.G.get() + (size_t)C.bidx[kc] * n : C.A.get() + (size_t)(kc - nb) * n;
      auto *row = M + moff(n + kc);
      float ss = 0.f;
      for (int j = sub; j < n; j += 16) {
        const float v = src[j];
        if (k < K) row[j] = v;
        ss = fmaf(v, v, ss);
      }
      border_exponent(M, n + kc, k < K, sub, ss, el);
    }
    border_exponents_done<T>(el, C.iflag);
  }
  for (int e = tid; e < K * K; e += T) {
    const int k = e / K, l = e - k * K;
    if (l > k) continue;
    float val = 0.f;
    if (l == k) {
      float dl = 0.f;
      if (k < nb && bounded) {
        const int r = C.bidx[k];
        dl = C.D[r] / C.E[r];
      }
      val = -(dl + delta);
    }
    M[moff(n + k) + n + l] = val;
  }
  __syncthreads();
}

// dinv[j] = 1 / L[j][j]
template <int T, class CT>
QPD void make_dinv(CT &C, int N) {
  for (int j = threadIdx.x; j < N; j += T) C.dinv[j] = 1.f / C.M[moff(j) + j];
  __syncthreads();
}

// Solve for both right-hand sides u0 and u1 (wave 0 and wave 1 in parallel
// when the workgroup has two waves).
template <int T, int RPL, class CT>
QPK_PHASE void solve2(CT &Cin_, int N, bool both) {
  CT C = uctx(Cin_);
  N = rfl(N); both = rfl(both);
  const int wid = threadIdx.x >> 6;
  if constexpr (T >= 128) {
    if (wid == 0) signed_solve_wave<RPL>(C.M.get(), N, C.n, C.dinv, C.u0, C.mz.get());
    else if (wid == 1 && both) signed_solve_wave<RPL>(C.M.get(), N, C.n, C.dinv, C.u1, C.mz.get());
  } else {
    signed_solve_wave<RPL>(C.M.get(), N, C.n, C.dinv, C.u0, C.mz.get());
    if (both) signed_solve_wave<RPL>(C.M.get(), N, C.n, C.dinv, C.u1, C.mz.get());
  }
  __syncthreads();
}


// Iterative refinement of a solution u of the augmented system
//   [[H, C'], [C, -Dl]] u = w,  H = Q + G_I' diag(wts_I) G_I,  C = [G_B; A],
// wts = E/D (bounded form) or E (standard form / initialisation, where E
// holds z/s or 1),
// Dl = D/E on bounded border rows and 0 on equality rows, against the
// operator WITHOUT any regularisation, with the residual w - K u
// accumulated in AT (FP32, or FP64 once a QP's FP32 refinement stalled)
// from the original Q, G, A.  Each step solves for the correction with the
// existing factor (one wave) and adds it.  A step whose residual is not
// smaller than the previous one is taken back and ends the refinement.
// Returns the contraction of the first correction (residual max-norm after
// it over the one before; 0 after a single step, kBig for a non-finite
// residual): above 1/2 the factor is too coarse a preconditioner in this
// arithmetic.
constexpr float kRefineSlow = 0.5f;

// out = w - K u (sub) or K u, for the augmented operator of refine (below),
// accumulated in AT from the original Q, G, A and rounded to FP32.
// Barriers inside; u must be visible to all threads on entry.
template <int T, class AT, class CT>
QPD void kkt_apply(CT &C, int nb, bool bounded, const lf *w, const lf *u, lf *out, bool sub) {
  typedef typename LdsT<AT>::type la;
  const int n = C.n, m = C.m, p = C.p, tid = threadIdx.x;
  la *gx = reinterpret_cast<la *>(C.dd.get()), *ax = gx + m, *phi = gx + m + p, *kx = gx + 2 * m + p;
  la *pd = reinterpret_cast<la *>(C.part.get());
  // G u, A u and Q'u_x + A'u_y in one pass; then G' phi, which needs G u
  float unused[3];
  kkt_matvecs<T, AT>(C.Q, C.G, C.A, n, m, p, u, u, false, u + n + nb, gx, ax, kx, pd, unused[0],
                     unused[1], unused[2]);
  for (int i = tid; i < m; i += T) {
    const int k = C.role[i];
    const AT wi = bounded ? (AT)C.E[i] / (AT)C.D[i] : (AT)C.E[i];
    phi[i] = k >= 0 ? (AT)u[n + k] : wi * gx[i];
  }
  __syncthreads();
  if (m) coldot_d<T, AT>(C.G.get(), n, m, n, phi, kx, true, pd);
  const AT sg = sub ? (AT)-1 : (AT)1;
  for (int j = tid; j < n; j += T) out[j] = (float)((sub ? (AT)w[j] : (AT)0) + sg * kx[j]);
  for (int k = tid; k < nb; k += T) {
    const int i = C.bidx[k];
    const AT dl = bounded ? (AT)C.D[i] / (AT)C.E[i] : (AT)0;
    out[n + k] = (float)((sub ? (AT)w[n + k] : (AT)0) + sg * (gx[i] - dl * (AT)u[n + k]));
  }
  for (int a = tid; a < p; a += T)
    out[n + nb + a] = (float)((sub ? (AT)w[n + nb + a] : (AT)0) + sg * ax[a]);
  __syncthreads();
}

// Largest |r_j| over j < N (kBig if any entry is not finite); uniform.
template <int T>
QPD float maxnorm(const lf *r, int N, lf *red) {
  float mx[2] = {0.f, 0.f};
  for (int j = threadIdx.x; j < N; j += T) {
    const float a = fabsf(r[j]);
    mx[0] = fmaxf(mx[0], a);
    if (!(a <= FLT_MAX)) mx[1] = 1.f;
  }
  block_reduce<T, OpMax, 2>(mx, red);
  return mx[1] != 0.f ? kBig : mx[0];
}

// Iterative refinement of a solution u of the augmented system
//   [[H, C'], [C, -Dl]] u = w,  H = Q + G_I' diag(wts_I) G_I,  C = [G_B; A],
// wts = E/D (bounded form) or E (standard form / initialisation, where E
// holds z/s or 1),
// Dl = D/E on bounded border rows and 0 on equality rows, against the
// operator WITHOUT any regularisation, with the residual w - K u
// accumulated in AT (FP32, or FP64 once a QP's FP32 refinement stalled)
// from the original Q, G, A.  Each step solves for the correction with the
// existing factor (one wave) and adds it; the residual after each
// correction is checked, and a correction that did not make it smaller is
// taken back and ends the refinement.  Returns the contraction of the first
// correction (residual max-norm after it over the one before; kBig for a
// non-finite residual): above 1/2 the factor is too coarse a
// preconditioner in this arithmetic.  iflag[7] receives the residual
// max-norm of the returned u (float bits).
template <int T, int RPL, class AT, class CT>
QPK_PHASE float refine(CT &Cin_, int nb, bool bounded, const lf *w, lf *u, int steps) {
  CT C = uctx(Cin_);
  nb = rfl(nb); bounded = rfl(bounded); w = rflp(w); u = rflp(u); steps = rfl(steps);
  const int n = C.n, p = C.p, tid = threadIdx.x, N = n + nb + p;
  lf *r = C.rr;
  float prev = 0.f, first = 0.f, cur = 0.f;
  for (int it = 0; it <= steps; ++it) {
    kkt_apply<T, AT>(C, nb, bounded, w, u, r, true);
    const float nrm = maxnorm<T>(r, N, C.red);
    cur = nrm;
    if (it > 0) {
      if (it == 1) first = prev > 0.f ? nrm / prev : 0.f;
      if (!(nrm < prev)) {
        // the last correction did not help: take it back and stop
        for (int j = tid; j < N; j += T) u[j] -= C.rd[j];
        cur = prev;
        __syncthreads();
        break;
      }
    } else if (nrm == 0.f) {
      break;  // exact already
    }
    if (it == steps) break;
    prev = nrm;
    if (threadIdx.x < 64) signed_solve_wave<RPL>(C.M.get(), N, n, C.dinv, r, C.mz.get());
    __syncthreads();
    for (int j = tid; j < N; j += T) {
      C.rd[j] = r[j];
      u[j] += r[j];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) C.iflag[7] = __float_as_int(cur);
  __syncthreads();
  return first;
}

// Residual precision of the refinement (qp_opts.fp64_residual): refine in
// FP32; under the automatic policy a QP whose FP32 refinement contracts by
// less than kRefineSlow per step continues in FP64 residuals, and keeps
// them for the rest of its solve (iflag[5]).  Returns the contraction of
// the arithmetic that ran last.
template <int T, int RPL, class CT>
QPD float refine_policy(CT &C, int nb, bool bounded, const lf *w, lf *u, int steps) {
  float q;
  if (C.rmode == 1 || C.iflag[5]) {
    q = refine<T, RPL, double>(C, nb, bounded, w, u, steps);
  } else {
    q = refine<T, RPL, float>(C, nb, bounded, w, u, steps);
    if (C.rmode == 0 && !(q <= kRefineSlow)) {
      __syncthreads();
      if (threadIdx.x == 0) C.iflag[5] = 1;
      __syncthreads();
      q = refine<T, RPL, double>(C, nb, bounded, w, u, steps);
    }
  }
  return q;
}

// Refinement steps of a solve with a factor of the exact operator (neither
// regularised nor assembled from split products): at least `min_steps`
// where the answer needs it (the adjoint solve, the equality-only solve; an
// FP32 factor's backward error grows with the system size, so FP32
// residuals still improve these).
QPD int plain_refine_steps(int rmode, int user_steps, int min_steps) {
  (void)rmode;
  return max(user_steps, min_steps);
}


// Add -delta to the diagonal of the border block, with delta = rel * (largest
// squared border-row norm) / (largest diagonal of H), and at least floor_abs:
// a Tikhonov floor on the Schur complement Dl + C H^-1 C'.
template <int T, class CT>
QPK_PHASE void border_delta(CT &Cin_, int nb, float rel, float floor_abs) {
  CT C = uctx(Cin_);
  nb = rfl(nb); rel = rflf(rel); floor_abs = rflf(floor_abs);
  const int n = C.n, K = nb + C.p, tid = threadIdx.x;
  float mx[2] = {0.f, 0.f};
  for (int j = tid; j < n; j += T) mx[0] = fmaxf(mx[0], C.M[moff(j) + j]);
  for (int k = tid; k < K; k += T) {
    float ss = 0.f;
    for (int j = 0; j < n; ++j) {
      const float c = C.M[moff(n + k) + j];
      ss = fmaf(c, c, ss);
    }
    mx[1] = fmaxf(mx[1], ss);
  }
  block_reduce<T, OpMax, 2>(mx, C.red);
  const float delta = fmaxf(fmaxf(rel * mx[1] / fmaxf(mx[0], 1e-30f), floor_abs), 1e-30f);
  for (int k = tid; k < K; k += T) C.M[moff(n + k) + n + k] -= delta;
  __syncthreads();
}

// True (uniformly) if a[0..N) or, with two, b[0..N) holds a
// non-finite value.
template <int T>
QPD bool any_nonfinite(const lf *a, const lf *b, bool two, int N, lf *red) {
  float f[1] = {0.f};
  for (int j = threadIdx.x; j < N; j += T) {
    if (!finitef(a[j]) || (two && !finitef(b[j]))) f[0] = 1.f;
  }
  block_reduce<T, OpMax, 1>(f, red);
  return f[0] != 0.f;
}

// Assemble and factor the bounded-form matrix.  On a pivot breakdown the
// matrix is rebuilt with a border floor and factored again; *regularised
// tells the caller to refine against the unregularised operator.
constexpr float kRetryReg = 1e-4f;
template <int T, int RPL, class CT>
QPD bool factor_bounded(CT &C, int nb, int ne, const lf *wts, float delta_rel, bool *regularised,
                        bool floor = false) {
  const int N = C.n + nb + C.p;
  assemble<T>(C, nb, ne, wts, true, 0.f);
  if (floor) {
    // asked for by a caller whose solve came out non-finite: floor the
    // border at the scale of the previous factorisation's pivots
    border_delta<T>(C, nb, fmaxf(delta_rel, 1e-6f), kRetryReg * __int_as_float(C.iflag[4]));
  } else if (delta_rel > 0.f) {
    border_delta<T>(C, nb, delta_rel, 0.f);
  }
  QPK_PT(C, PH_ASM);
  bool ok = signed_cholesky<T, RPL>(C.M.get(), N, C.n, C.iflag, C.dyn != 0);
  QPK_PT(C, PH_FACT);
  *regularised = delta_rel > 0.f || floor || C.iflag[2] > 0;
  if (!ok && C.dyn) {
    // the floor is at least kRetryReg times the largest pivot the failed
    // attempt accepted, i.e. scaled like the Schur complement's entries
    const float pmax = __int_as_float(C.iflag[4]);
    assemble<T>(C, nb, ne, wts, true, 0.f);
    border_delta<T>(C, nb, fmaxf(delta_rel, 1e-6f), kRetryReg * pmax);
    ok = signed_cholesky<T, RPL>(C.M.get(), N, C.n, C.iflag, true);
    *regularised = true;
  }
  return ok;
}

// Bounded-form right-hand sides of the augmented system for two columns:
//   column 0: rho = (r_t - G'(r_i + r_z - r_s), r_i - r_s - c (kappa - kt0), r_e)
//   column 1: rho = (0, c, 0)   (derivative with respect to kappa_target)
// or, for the adjoint (mode adj): column 0 rho = (gx, E gz, gy), no column 1.
// With psi_i = rho2_i / D_i on eliminated rows and rho2_i on border rows:
//   u = [ -rho1 - G' psi ;  -rho2_B ;  -rho3 ].
// rho2 of each column is left in dv0 / dv1 for the recovery.
template <int T, class CT>
QPK_PHASE void rhs_bounded(CT &Cin_, int nb, float kappa, const gf *gx, const gf *gz,
                     const gf *gy, bool adj) {
  CT C = uctx(Cin_);
  nb = rfl(nb); kappa = rflf(kappa); adj = rfl(adj);
  gx = rflp(gx); gz = rflp(gz); gy = rflp(gy);
  const int n = C.n, m = C.m, p = C.p, tid = threadIdx.x;
  // phi0 = -(r_i + r_z - r_s) + psi0 would give u_x = -r_t - G' phi0;
  // we compute w0 = (r_i + r_z - r_s) - psi0 so u_x = -r_t + G' w0, and
  // w1 = -psi1 so u_x1 = G' w1.
  for (int i = tid; i < m; i += T) {
    const bool border = C.role[i] >= 0;
    float r2a, w0, w1 = 0.f;
    if (!adj) {
      r2a = C.ri[i] - C.rs[i] - C.c[i] * kappa;
      const float psi0 = border ? r2a : r2a / C.D[i];
      w0 = (C.ri[i] + C.rz[i] - C.rs[i]) - psi0;
      const float r2b = C.c[i];
      const float psi1 = border ? r2b : r2b / C.D[i];
      w1 = -psi1;
      C.dv1[i] = r2b;
    } else {
      r2a = gz ? C.E[i] * gz[i] : 0.f;
      const float psi0 = border ? r2a : r2a / C.D[i];
      w0 = -psi0;
    }
    C.dv0[i] = r2a;
    C.t0[i] = w0;
    C.t1[i] = w1;
  }
  __syncthreads();
  if (m) {
    if (!adj) {
      const lf *xv[2] = {C.t0, C.t1};
      lf *o[2] = {C.tGz, C.tAy};
      coldot<T, 2>(C.G.get(), n, m, n, xv, o, C.part);
    } else {
      const lf *xv[1] = {C.t0};
      lf *o[1] = {C.tGz};
      coldot<T, 1>(C.G.get(), n, m, n, xv, o, C.part);
    }
  }
  for (int i = tid; i < n; i += T) {
    const float g0 = m ? C.tGz[i] : 0.f;
    if (!adj) {
      C.u0[i] = -C.rt[i] + g0;
      C.u1[i] = m ? C.tAy[i] : 0.f;
    } else {
      C.u0[i] = -gx[i] + g0;
    }
  }
  for (int k = tid; k < nb; k += T) {
    const int r = C.bidx[k];
    C.u0[n + k] = -C.dv0[r];
    if (!adj) C.u1[n + k] = -C.dv1[r];
  }
  for (int k = tid; k < p; k += T) {
    C.u0[n + nb + k] = adj ? (gy ? -gy[k] : 0.f) : -C.re[k];
    if (!adj) C.u1[n + nb + k] = 0.f;
  }
  __syncthreads();
}

// Recover dv for the solved columns: eliminated rows dv = (G dx + rho2)/D,
// border rows dv = du / E.  rho2 is read from dv0 / dv1 and overwritten.
template <int T, class CT>
QPK_PHASE void recover_bounded(CT &Cin_, int nb, bool both) {
  CT C = uctx(Cin_);
  nb = rfl(nb); both = rfl(both);
  const int n = C.n, m = C.m, tid = threadIdx.x;
  if (!m) return;
  if (both) {
    const lf *xv[2] = {C.u0, C.u1};
    lf *o[2] = {C.t0, C.t1};
    rowdot<T, 2>(C.G.get(), n, m, n, xv, o);
  } else {
    const lf *xv[1] = {C.u0};
    lf *o[1] = {C.t0};
    rowdot<T, 1>(C.G.get(), n, m, n, xv, o);
  }
  __syncthreads();
  for (int i = tid; i < m; i += T) {
    const int k = C.role[i];
    if (k >= 0) {
      const float ie = 1.f / C.E[i];
      C.dv0[i] = C.u0[n + k] * ie;
      if (both) C.dv1[i] = C.u1[n + k] * ie;
    } else {
      const float id = 1.f / C.D[i];
      C.dv0[i] = (C.t0[i] + C.dv0[i]) * id;
      if (both) C.dv1[i] = (C.t1[i] + C.dv1[i]) * id;
    }
  }
  __syncthreads();
}

// Ratio test of eq. linesearch over (s, ds), (z, dz); returns the min of the
// ratios (uninclusive of the cap 1).
QPD float ratio(float s, float ds) { return ds < 0.f ? -s / ds : kBig; }

constexpr int ST_CONV = 0, ST_MAXIT = 1, ST_NONFIN = 2, ST_FACT = 3;
constexpr int SG_NONE = 0, SG_SCAL = 1, SG_PRED = 2, SG_CENT = 3, SG_CORR = 4, SG_LS = 5,
              SG_RELAX = 6, SG_BWD = 7;

QPD int mkstatus(int st, int stage) { return st | (stage << 8); }

// Precision events of a QP's run, reported in status bits 16-17: FP64
// refinement residuals were needed; the split-product assembly fell back to
// FP32.
template <class CT>
QPD int precision_bits(const CT &C, int amode0) {
  return (C.iflag[5] ? 1 << 16 : 0) | (amode0 == 1 && C.iflag[3] != 1 ? 1 << 17 : 0);
}

// ---------------------------------------------------------------------------
// Initialisation (CVXOPT convention): solve [[Q+G'G, A'], [A, 0]] [x; y] =
// [-q + G'h; b], zt = Gx - h, s = -zt, z = zt, each shifted positive.
template <int T, int RPL, class CT>
QPK_PHASE bool initialize(CT &Cin_, double &work, bool dyn) {
  CT C = uctx(Cin_);
  dyn = rfl(dyn);
  const int n = C.n, m = C.m, p = C.p, tid = threadIdx.x;
  for (int i = tid; i < m; i += T) C.E[i] = 1.f;  // unit weights
  for (int i = tid; i < m; i += T) C.role[i] = 1;
  __syncthreads();
  const int ne = compact_rows<T>(C.role, m, C.elist, C.red);
  assemble<T>(C, 0, ne, C.E, false, 0.f);
  const int N = n + p;
  const bool ok = signed_cholesky<T, RPL>(C.M.get(), N, n, C.iflag, dyn);
  make_dinv<T>(C, N);
  if (m) {
    const lf *hv[1] = {C.h};
    lf *o[1] = {C.tGz};
    coldot<T, 1>(C.G.get(), n, m, n, hv, o, C.part);
  }
  for (int i = tid; i < n; i += T) C.u0[i] = C.w0[i] = -C.q[i] + (m ? C.tGz[i] : 0.f);
  for (int k = tid; k < p; k += T) C.u0[n + k] = C.w0[n + k] = C.b[k];
  for (int i = tid; i < m; i += T) C.role[i] = -1;
  __syncthreads();
  solve2<T, RPL>(C, N, false);
  // without inequalities this solve is the answer
  const int nref0 = m == 0 ? plain_refine_steps(C.rmode, 0, 2) : 0;
  if (nref0) refine_policy<T, RPL>(C, 0, false, C.w0, C.u0, nref0);
  for (int i = tid; i < n; i += T) C.x[i] = C.u0[i];
  for (int k = tid; k < p; k += T) C.y[k] = C.u0[n + k];
  __syncthreads();
  if (m) {
    const lf *xv[1] = {C.x};
    lf *o[1] = {C.t0};
    rowdot<T, 1>(C.G.get(), n, m, n, xv, o);
    __syncthreads();
    float mx[2] = {-kBig, -kBig};
    for (int i = tid; i < m; i += T) {
      const float zt = C.t0[i] - C.h[i];
      C.s[i] = -zt;
      C.z[i] = zt;
      mx[0] = fmaxf(mx[0], zt);    // max(-s)
      mx[1] = fmaxf(mx[1], -zt);   // max(-z)
    }
    block_reduce<T, OpMax, 2>(mx, C.red);
    for (int i = tid; i < m; i += T) {
      if (mx[0] >= 0.f) C.s[i] += 1.f + mx[0];
      if (mx[1] >= 0.f) C.z[i] += 1.f + mx[1];
    }
  }
  __syncthreads();
  const double dn = n, dm = m, dN = N;
  work += dm * dn * (dn + 1.0) + dN * dN * dN / 3.0 + 2.0 * dN * dN + 4.0 * dm * dn;
  work += nref0 * (2.0 * dN * dN + 2.0 * dn * dn);  // refinement steps
  return ok;
}

// One Newton iteration of the bounded (implicit) form.  Mode of the target:
// kt_mode 0 = predictor-corrector, 1 = fixed sigma, 2 = relax (kt = kr).
// Returns a status code (ST_CONV meaning "keep going"), with the stage in
// *stage on failure.  Updates x, y, v, kappa, z, s.
template <int T, int RPL, class CT>
QPK_PHASE int newton_bounded(CT &Cin_, float &kappa, int kt_mode, float sigma, float kr,
                       float delta_reg, int refine_steps, double &work, int *stage) {
  CT C = uctx(Cin_);
  kappa = rflf(kappa); kt_mode = rfl(kt_mode); sigma = rflf(sigma); kr = rflf(kr);
  delta_reg = rflf(delta_reg); refine_steps = rfl(refine_steps);
  const int n = C.n, m = C.m, p = C.p, tid = threadIdx.x;
  C.amode = rfl(C.iflag[3]);  // this QP's assembly arithmetic (may have fallen back)
  const int nb = partition_bounded<T>(C, kappa);
  const int ne = C.iflag[1];
  QPK_PT(C, PH_PART);
  const int N = n + nb + p;
  const double dn = n, dm = m, dp = p, dN = N;
  work += 2.0 * dn * dn + 4.0 * dm * dn + 4.0 * dp * dn;            // residuals
  // Factor, solve and refine.  With split-product (BF16x3) assembly, a
  // refinement that contracts by less than kRefineSlow per step means the
  // assembly error is too large for this system's conditioning: the QP
  // switches to FP32 matrix-core assembly and the step is redone.
  // at most one switch of the assembly arithmetic and one floored redo
  bool ok = false, floor = false;
  for (int attempt = 0; attempt < 3; ++attempt) {
    // weights E/D for eliminated rows (in t1 until the right-hand sides)
    for (int i = tid; i < m; i += T) C.t1[i] = C.E[i] / C.D[i];
    __syncthreads();
    bool reg = false;
    ok = factor_bounded<T, RPL>(C, nb, ne, C.t1, delta_reg, &reg, floor);
    work += (double)ne * dn * (dn + 1.0) + dN * dN * dN / 3.0;      // assembly + factor
    work += 2.0 * (2.0 * dN * dN + 4.0 * dm * dn);                  // two solves
    if (!ok) break;
    make_dinv<T>(C, N);
    rhs_bounded<T>(C, nb, kappa, nullptr, nullptr, nullptr, false);
    QPK_PT(C, PH_RHS);
    const int nref = (reg || C.amode == 1) ? max(refine_steps, 2)
                                           : plain_refine_steps(C.rmode, refine_steps, 0);
    if (nref) {
      for (int j = tid; j < N; j += T) { C.w0[j] = C.u0[j]; C.w1[j] = C.u1[j]; }
      __syncthreads();
    }
    solve2<T, RPL>(C, N, true);
    QPK_PT(C, PH_SOLVE);
    if (nref) {
      const float q0 = refine_policy<T, RPL>(C, nb, true, C.w0, C.u0, nref);
      const float q1 = refine_policy<T, RPL>(C, nb, true, C.w1, C.u1, nref);
      work += 2.0 * nref * (2.0 * dN * dN + 4.0 * dm * dn + 2.0 * dn * dn + 4.0 * dp * dn);
      if (C.amode == 1 && !(fmaxf(q0, q1) <= kRefineSlow)) {
        C.amode = 2;
        if (tid == 0) C.iflag[3] = 2;
        __syncthreads();
        continue;
      }
    }
    // a factor that passed its checks can still give a non-finite solution
    // when it is nearly singular: redo the step once with a border floor
    if (C.dyn && !floor && any_nonfinite<T>(C.u0, C.u1, true, N, C.red)) {
      floor = true;
      continue;
    }
    break;
  }
  if (!ok) { *stage = SG_PRED; return ST_FACT; }
  QPK_PT(C, PH_REFINE);
  recover_bounded<T>(C, nb, true);
  QPK_PT(C, PH_RECOVER);
  // predictor step length (kappa_target = 0) and kappa_aff
  float kt;
  if (kt_mode == 0) {
    float mn[2] = {1.f, 0.f};
    for (int i = tid; i < m; i += T) {
      const float dv = C.dv0[i];
      const float dz = -C.rz[i] + C.E[i] * dv - C.c[i] * kappa;
      const float ds = -C.rs[i] - C.D[i] * dv - C.c[i] * kappa;
      mn[0] = fminf(mn[0], fminf(ratio(C.s[i], ds), ratio(C.z[i], dz)));
      if (!finitef(dz) || !finitef(ds)) mn[1] = -1.f;
    }
    block_reduce<T, OpMin, 2>(mn, C.red);
    if (mn[1] < 0.f) { *stage = SG_PRED; return ST_NONFIN; }
    const float aa = mn[0];
    float sm[1] = {0.f};
    for (int i = tid; i < m; i += T) {
      const float dv = C.dv0[i];
      const float dz = -C.rz[i] + C.E[i] * dv - C.c[i] * kappa;
      const float ds = -C.rs[i] - C.D[i] * dv - C.c[i] * kappa;
      sm[0] += (C.s[i] + aa * ds) * (C.z[i] + aa * dz);
    }
    block_reduce<T, OpSum, 1>(sm, C.red);
    const float kaff = sm[0] / (float)m;
    const float ratio_k = kaff / kappa;
    const float sg = ratio_k * ratio_k * ratio_k;
    kt = sg * kappa;
    if (!finitef(kt)) { *stage = SG_CENT; return ST_NONFIN; }
    kt = fmaxf(kt, 1e-12f);  // keep the central-path parameter positive
  } else if (kt_mode == 1) {
    kt = sigma * kappa;
  } else {
    kt = kr;
  }
  // combined direction and its step length
  const float dk = kt - kappa;
  float mn[2] = {1.f, 0.f};
  for (int i = tid; i < m; i += T) {
    const float dv = fmaf(kt, C.dv1[i], C.dv0[i]);
    const float dz = -C.rz[i] + C.E[i] * dv + C.c[i] * dk;
    const float ds = -C.rs[i] - C.D[i] * dv + C.c[i] * dk;
    mn[0] = fminf(mn[0], fminf(ratio(C.s[i], ds), ratio(C.z[i], dz)));
    if (!finitef(dz) || !finitef(ds)) mn[1] = -1.f;
  }
  block_reduce<T, OpMin, 2>(mn, C.red);
  if (mn[1] < 0.f) { *stage = kt_mode == 2 ? SG_RELAX : SG_CORR; return ST_NONFIN; }
  const float alpha = fminf(1.f, C.bo * mn[0]);
  if (!(alpha > 0.f)) { *stage = SG_LS; return ST_NONFIN; }
  // step on (x, y, v, kappa), then retract z, s
  for (int i = tid; i < n; i += T) C.x[i] += alpha * fmaf(kt, C.u1[i], C.u0[i]);
  for (int k = tid; k < p; k += T) C.y[k] += alpha * fmaf(kt, C.u1[n + nb + k], C.u0[n + nb + k]);
  // kappa + alpha (kt - kappa) lies between kt and kappa, but with alpha = 1
  // and kt below kappa's rounding unit the sum rounds to exactly zero: z of
  // every inactive row would then be 0 and the next centering would divide
  // by kappa = 0.  Held at the bound the step cannot cross.
  const float knew = fmaxf(kappa + alpha * dk, fminf(kt, kappa));
  for (int i = tid; i < m; i += T) {
    const float vn = C.v[i] + alpha * fmaf(kt, C.dv1[i], C.dv0[i]);
    C.v[i] = vn;
    C.z[i] = bk(vn, knew);
    C.s[i] = bk(-vn, knew);
  }
  kappa = knew;
  __syncthreads();
  QPK_PT(C, PH_STEP);
  return ST_CONV;
}

// One Mehrotra predictor-corrector iteration of the standard form.
template <int T, int RPL, class CT>
QPK_PHASE int newton_standard(CT &Cin_, float mu, int kt_mode, float kr, float delta_reg, double &work,
                        int *stage) {
  CT C = uctx(Cin_);
  mu = rflf(mu); kt_mode = rfl(kt_mode); kr = rflf(kr); delta_reg = rflf(delta_reg);
  const int n = C.n, m = C.m, p = C.p, tid = threadIdx.x;
  float bad[1] = {0.f};
  for (int i = tid; i < m; i += T) {
    const float w = C.z[i] / C.s[i];
    C.t1[i] = w;
    C.role[i] = 1;
    if (!finitef(w)) bad[0] = 1.f;
  }
  block_reduce<T, OpMax, 1>(bad, C.red);
  if (bad[0] != 0.f) { *stage = SG_SCAL; return ST_NONFIN; }
  const int ne = compact_rows<T>(C.role, m, C.elist, C.red);
  // the weights t1 must survive: copy to E (unused in the standard form)
  for (int i = tid; i < m; i += T) C.E[i] = C.t1[i];
  __syncthreads();
  const int N = n + p;
  assemble<T>(C, 0, ne, C.E, false, delta_reg);
  const bool ok = signed_cholesky<T, RPL>(C.M.get(), N, n, C.iflag, false);
  const double dn = n, dm = m, dp = p, dN = N;
  work += 2.0 * dn * dn + 4.0 * dm * dn + 4.0 * dp * dn;
  work += dm * dn * (dn + 1.0) + dN * dN * dN / 3.0;
  work += 2.0 * (2.0 * dN * dN + 4.0 * dm * dn);
  if (!ok) { *stage = SG_PRED; return ST_FACT; }
  make_dinv<T>(C, N);
  // rhs for a given r_c / s =: q_i;  u_x = -r_t - G'(w r_i - q), u_y = -r_e
  // then dz = w (r_i + G dx) - q, ds = -r_i - G dx
  auto rhs_and_solve = [&](const lf *qv) {
    for (int i = tid; i < m; i += T) C.t0[i] = C.E[i] * C.ri[i] - qv[i];
    __syncthreads();
    {
      const lf *xv[1] = {C.t0};
      lf *o[1] = {C.tGz};
      if (m) coldot<T, 1>(C.G.get(), n, m, n, xv, o, C.part);
    }
    for (int i = tid; i < n; i += T) C.u0[i] = -C.rt[i] - (m ? C.tGz[i] : 0.f);
    for (int k = tid; k < p; k += T) C.u0[n + k] = -C.re[k];
    __syncthreads();
    solve2<T, RPL>(C, N, false);
    const lf *xv[1] = {C.u0};
    lf *o[1] = {C.t0};
    if (m) rowdot<T, 1>(C.G.get(), n, m, n, xv, o);
    __syncthreads();
  };
  float sgm;
  if (kt_mode == 2) {
    // relax: r_c = z s - kr  =>  q = z - kr / s
    for (int i = tid; i < m; i += T) C.dv1[i] = C.z[i] - kr / C.s[i];
    __syncthreads();
    rhs_and_solve(C.dv1);
  } else {
    // affine predictor: q = z
    rhs_and_solve(C.z);
    float mn[2] = {1.f, 0.f};
    for (int i = tid; i < m; i += T) {
      const float gdx = C.t0[i];
      const float dz = C.E[i] * (C.ri[i] + gdx) - C.z[i];
      const float ds = -C.ri[i] - gdx;
      C.dv0[i] = dz;
      C.dv1[i] = ds;
      mn[0] = fminf(mn[0], fminf(ratio(C.s[i], ds), ratio(C.z[i], dz)));
      if (!finitef(dz) || !finitef(ds)) mn[1] = -1.f;
    }
    block_reduce<T, OpMin, 2>(mn, C.red);
    if (mn[1] < 0.f) { *stage = SG_PRED; return ST_NONFIN; }
    const float aa = mn[0];
    float sm[1] = {0.f};
    for (int i = tid; i < m; i += T)
      sm[0] += (C.s[i] + aa * C.dv1[i]) * (C.z[i] + aa * C.dv0[i]);
    block_reduce<T, OpSum, 1>(sm, C.red);
    const float muaff = sm[0] / (float)m;
    const float rr = muaff / mu;
    sgm = rr * rr * rr;
    if (!finitef(sgm) || !finitef(mu)) { *stage = SG_CENT; return ST_NONFIN; }
    // corrector: r_c = z s + ds_a dz_a - sigma mu  =>  q = z + (ds_a dz_a - sigma mu)/s
    for (int i = tid; i < m; i += T)
      C.dv1[i] = C.z[i] + (C.dv1[i] * C.dv0[i] - sgm * mu) / C.s[i];
    __syncthreads();
    rhs_and_solve(C.dv1);
    if (kt_mode == 1) { /* fixed sigma is not used by the standard arm */ }
  }
  float mn[2] = {kBig, 0.f};
  for (int i = tid; i < m; i += T) {
    const float gdx = C.t0[i];
    const float dz = C.E[i] * (C.ri[i] + gdx) - C.dv1[i];
    const float ds = -C.ri[i] - gdx;
    C.dv0[i] = dz;
    C.dv1[i] = ds;
    mn[0] = fminf(mn[0], fminf(ratio(C.s[i], ds), ratio(C.z[i], dz)));
    if (!finitef(dz) || !finitef(ds)) mn[1] = -1.f;
  }
  block_reduce<T, OpMin, 2>(mn, C.red);
  if (mn[1] < 0.f) { *stage = kt_mode == 2 ? SG_RELAX : SG_CORR; return ST_NONFIN; }
  const float alpha = fminf(1.f, C.bo * mn[0]);
  if (!(alpha > 0.f) || !finitef(alpha)) { *stage = SG_LS; return ST_NONFIN; }
  for (int i = tid; i < n; i += T) C.x[i] += alpha * C.u0[i];
  for (int k = tid; k < p; k += T) C.y[k] += alpha * C.u0[n + k];
  for (int i = tid; i < m; i += T) {
    C.z[i] += alpha * C.dv0[i];
    C.s[i] += alpha * C.dv1[i];
  }
  __syncthreads();
  return ST_CONV;
}

// Without inequalities (m = 0) the refined KKT solve of the initialisation
// is the answer, and its accuracy is that of a direct solve: the backward
// error max(|r_t| / (1 + | |Q||x| + |q| + |A'||y| |), |r_e| / (1 + | |A||x|
// + |b| |)) (infinity norms) measures it.  The scaled residual of the
// general test divides by the largest term instead, which for a solution
// with heavy cancellation (|Q||x| >> |Qx|) lies below what any float32
// vector attains.  Uses r_t, r_e from residuals(); uniform result.
template <int T, class CT>
QPD float direct_backward_error(CT &C) {
  const int n = C.n, p = C.p, tid = threadIdx.x;
  float mx[4] = {0.f, 0.f, 0.f, 0.f};  // |r_t|, its scale, |r_e|, its scale
  for (int j = tid; j < n; j += T) {
    float a = fabsf(C.q[j]);
    for (int i = 0; i < n; ++i) a = fmaf(fabsf(C.Q[(size_t)i * n + j]), fabsf(C.x[i]), a);
    for (int k = 0; k < p; ++k) a = fmaf(fabsf(C.A[(size_t)k * n + j]), fabsf(C.y[k]), a);
    mx[0] = fmaxf(mx[0], fabsf(C.rt[j]));
    mx[1] = fmaxf(mx[1], a);
  }
  for (int k = tid; k < p; k += T) {
    float a = fabsf(C.b[k]);
    for (int j = 0; j < n; ++j) a = fmaf(fabsf(C.A[(size_t)k * n + j]), fabsf(C.x[j]), a);
    mx[2] = fmaxf(mx[2], fabsf(C.re[k]));
    mx[3] = fmaxf(mx[3], a);
  }
  block_reduce<T, OpMax, 4>(mx, C.red);
  return fmaxf(mx[0] / (1.f + mx[1]), p ? mx[2] / (1.f + mx[3]) : 0.f);
}

// Newton loop shared by the solve, the relaxation and the serving step.
// Returns the final status; iters counts Newton steps taken.
template <int T, int RPL, class CT>
QPD int newton_loop(CT &C, bool bounded, int max_iter, float tol, int kt_mode, float sigma,
                    float kr, float delta_reg, int refine_steps, double &work, int &iters,
                    float &res) {
  const int m = C.m, tid = threadIdx.x;
  int status = ST_MAXIT;
  int stage = SG_NONE;
  for (int it = 0;; ++it) {
    // manifold coordinates v = z - s, kappa = s'z / m
    float sm[1] = {0.f};
    for (int i = tid; i < m; i += T) {
      sm[0] += C.s[i] * C.z[i];
      if (bounded) C.v[i] = C.z[i] - C.s[i];
    }
    block_reduce<T, OpSum, 1>(sm, C.red);
    float kappa = m ? sm[0] / (float)m : 0.f;
    bool bad = false;
    // FP64 residuals under the FP64 policy, and for a QP whose refinement
    // has already needed FP64 (FP32 cannot resolve its residuals either)
    const bool r64 = C.rmode == 1 || (C.rmode == 0 && C.iflag[5] != 0);
    res = r64 ? residuals<T, double>(C, bounded, kappa, kt_mode == 2 ? kr : 0.f, &bad)
              : residuals<T, float>(C, bounded, kappa, kt_mode == 2 ? kr : 0.f, &bad);
    QPK_PT(C, PH_RESID);
    if (bad || !finitef(res)) {
      status = ST_NONFIN;
      stage = kt_mode == 2 ? SG_RELAX : (it == 0 ? SG_NONE : SG_LS);
      iters = it;
      break;
    }
    if (res < tol) { status = ST_CONV; iters = it; break; }
    if (m == 0) {
      res = direct_backward_error<T>(C);
      status = res < tol ? ST_CONV : ST_MAXIT;
      iters = it;
      break;
    }
    if (it >= max_iter) {
      // an iteration limit inside Algorithm 2 is reported at the relax stage
      status = ST_MAXIT;
      if (kt_mode == 2) stage = SG_RELAX;
      iters = it;
      break;
    }
    int st;
    if (bounded)
      st = newton_bounded<T, RPL>(C, kappa, kt_mode, sigma, kr, delta_reg, refine_steps, work, &stage);
    else st = newton_standard<T, RPL>(C, kappa, kt_mode, kr, delta_reg, work, &stage);
    if (st != ST_CONV) {
      status = st;
      // a failure inside the relaxation (Algorithm 2) is attributed to it as
      // a whole, whichever sub-step produced it
      if (kt_mode == 2) stage = SG_RELAX;
      iters = it + 1;
      break;
    }
  }
  return mkstatus(status, stage);
}

// Load this QP's small vectors into LDS.
template <int T, class CT>
QPD void load_vectors(CT &C) {
  const int tid = threadIdx.x;
  for (int i = tid; i < C.n; i += T) C.q[i] = C.q_g[i];
  for (int i = tid; i < C.m; i += T) C.h[i] = C.h_g[i];
  for (int i = tid; i < C.p; i += T) C.b[i] = C.b_g[i];
  if (tid < kNB) C.mz[tid] = 0.f;
  __syncthreads();
}

// Factor at the current (relaxed) point and solve the adjoint system for
// the upstream gradient; returns dx in u0[0:n], dy in u0[n+nb:], dz in dv0.
// Returns kAdjOk, kAdjFactorFail, or kAdjInaccurate when the refinement of
// the adjoint solve stalled (contraction above 1/2 in the last arithmetic
// it used) with a residual above kAdjResTol of the right-hand side: the
// factor is too coarse a preconditioner for this system and the gradient
// is not reliable.
constexpr int kAdjOk = 0, kAdjFactorFail = 1, kAdjInaccurate = 2;
constexpr float kAdjResTol = 1e-5f;
template <int T, int RPL, class CT>
QPK_PHASE int adjoint(CT &Cin_, bool bounded, const gf *gx, const gf *gy, const gf *gz,
                 float delta_reg, int refine_steps, double &work) {
  CT C = uctx(Cin_);
  bounded = rfl(bounded); gx = rflp(gx); gy = rflp(gy); gz = rflp(gz);
  delta_reg = rflf(delta_reg); refine_steps = rfl(refine_steps);
  const int n = C.n, m = C.m, p = C.p, tid = threadIdx.x;
  float sm[1] = {0.f};
  for (int i = tid; i < m; i += T) {
    sm[0] += C.s[i] * C.z[i];
    if (bounded) C.v[i] = C.z[i] - C.s[i];
  }
  block_reduce<T, OpSum, 1>(sm, C.red);
  const float kappa = m ? sm[0] / (float)m : 0.f;
  int nb = 0, ne = 0;
  if (bounded && m) {
    nb = partition_bounded<T>(C, kappa);
    ne = C.iflag[1];
    for (int i = tid; i < m; i += T) C.t1[i] = C.E[i] / C.D[i];
  } else {
    for (int i = tid; i < m; i += T) {
      C.t1[i] = C.z[i] / C.s[i];
      C.role[i] = 1;
    }
    __syncthreads();
    ne = compact_rows<T>(C.role, m, C.elist, C.red);
    for (int i = tid; i < m; i += T) C.role[i] = -1;
  }
  __syncthreads();
  // keep the weights: E holds E (bounded) or z/s (standard)
  if (!bounded)
    for (int i = tid; i < m; i += T) C.E[i] = C.t1[i];
  __syncthreads();
  const int N = n + nb + p;
  const double dn = n, dN = N;
  const double wfac = (double)ne * dn * (dn + 1.0) + dN * dN * dN / 3.0 + 2.0 * dN * dN + 8.0 * m * dn;
  const double wstep = 2.0 * dN * dN + 2.0 * dn * dn + 8.0 * m * dn + 4.0 * p * dn;
  bool ok = false, inaccurate = false;
  if (bounded) {
    C.amode = rfl(C.iflag[3]);
    // as in newton_bounded: fall back from split-product assembly when the
    // refinement does not contract, and floor the border when the solve is
    // not finite
    bool floor = false;
    for (int attempt = 0; attempt < 3; ++attempt) {
      if (attempt) {
        for (int i = tid; i < m; i += T) C.t1[i] = C.E[i] / C.D[i];
        __syncthreads();
      }
      bool reg = false;
      ok = factor_bounded<T, RPL>(C, nb, ne, C.t1, delta_reg, &reg, floor);
      // the adjoint solve gives the gradient directly: a regularised or
      // split-product factor is always refined against the exact operator
      const int nref = (reg || C.amode == 1) ? max(refine_steps, 2)
                                             : plain_refine_steps(C.rmode, refine_steps, 2);
      work += wfac + nref * wstep;
      if (!ok) break;
      make_dinv<T>(C, N);
      rhs_bounded<T>(C, nb, kappa, gx, gz, gy, true);
      for (int j = tid; j < N; j += T) C.w0[j] = C.u0[j];
      __syncthreads();
      const float wn = maxnorm<T>(C.w0, N, C.red);
      solve2<T, RPL>(C, N, false);
      const float q = nref ? refine_policy<T, RPL>(C, nb, true, C.w0, C.u0, nref) : 0.f;
      inaccurate = nref && !(q <= kRefineSlow) &&
                   !(__int_as_float(C.iflag[7]) <= kAdjResTol * wn);
      if (C.amode == 1 && !(q <= kRefineSlow)) {
        C.amode = 2;
        if (tid == 0) C.iflag[3] = 2;
        __syncthreads();
        continue;
      }
      if (C.dyn && !floor && any_nonfinite<T>(C.u0, C.u0, false, N, C.red)) {
        floor = true;
        continue;
      }
      break;
    }
    if (!ok) return kAdjFactorFail;
    recover_bounded<T>(C, nb, false);
    // dz = E (dv + gz)
    for (int i = tid; i < m; i += T) C.dv0[i] = C.E[i] * (C.dv0[i] + (gz ? gz[i] : 0.f));
  } else {
    assemble<T>(C, nb, ne, C.t1, false, 0.f);
    ok = signed_cholesky<T, RPL>(C.M.get(), N, n, C.iflag, false);
    const int nref = plain_refine_steps(C.rmode, refine_steps, 2);
    work += wfac + nref * wstep;
    if (!ok) return kAdjFactorFail;
    make_dinv<T>(C, N);
    // standard: [H A'; A 0][a; c] = [-gx - G' W gz; -gy], dz = W (G a + gz)
    for (int i = tid; i < m; i += T) C.t0[i] = gz ? C.E[i] * gz[i] : 0.f;
    __syncthreads();
    if (m) {
      const lf *xv[1] = {C.t0};
      lf *o[1] = {C.tGz};
      coldot<T, 1>(C.G.get(), n, m, n, xv, o, C.part);
    }
    for (int i = tid; i < n; i += T) C.u0[i] = C.w0[i] = -gx[i] - (m ? C.tGz[i] : 0.f);
    for (int k = tid; k < p; k += T) C.u0[n + k] = C.w0[n + k] = gy ? -gy[k] : 0.f;
    __syncthreads();
    const float wn = maxnorm<T>(C.w0, N, C.red);
    solve2<T, RPL>(C, N, false);
    if (nref) {
      const float q = refine_policy<T, RPL>(C, 0, false, C.w0, C.u0, nref);
      inaccurate = !(q <= kRefineSlow) && !(__int_as_float(C.iflag[7]) <= kAdjResTol * wn);
    }
    if (m) {
      const lf *xv[1] = {C.u0};
      lf *o[1] = {C.t0};
      rowdot<T, 1>(C.G.get(), n, m, n, xv, o);
    }
    __syncthreads();
    for (int i = tid; i < m; i += T) C.dv0[i] = C.E[i] * (C.t0[i] + (gz ? gz[i] : 0.f));
  }
  // move dy next to dx: u0[n : n+p] = dy
  __syncthreads();
  if (nb) {
    float tmp[4];
    for (int k0 = 0; k0 < p; k0 += 4 * T) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = k0 + tid + u * T;
        tmp[u] = k < p ? C.u0[n + nb + k] : 0.f;
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = k0 + tid + u * T;
        if (k < p) C.u0[n + k] = tmp[u];
      }
      __syncthreads();
    }
  }
  return inaccurate ? kAdjInaccurate : kAdjOk;
}

// Write the parameter gradients of Algorithm 3 with coalesced stores.
template <int T, class CT>
QPK_PHASE void write_grads(CT &Cin_, const Params &P, size_t qi) {
  CT C = uctx(Cin_);
  const int n = C.n, m = C.m, p = C.p, tid = threadIdx.x;
  const lf *dx = C.u0, *dy = C.u0 + n, *dz = C.dv0;
  if (P.dQ) {
    gf *o = (gf *)P.dQ + qi * (size_t)n * n;
    for (int e = tid; e < n * n; e += T) {
      const int i = e / n, j = e % n;
      o[e] = 0.5f * (dx[i] * C.x[j] + C.x[i] * dx[j]);
    }
  }
  if (P.dq) {
    gf *o = (gf *)P.dq + qi * (size_t)n;
    for (int i = tid; i < n; i += T) o[i] = dx[i];
  }
  if (P.dA && p) {
    gf *o = (gf *)P.dA + qi * (size_t)p * n;
    for (int e = tid; e < p * n; e += T) {
      const int i = e / n, j = e % n;
      o[e] = dy[i] * C.x[j] + C.y[i] * dx[j];
    }
  }
  if (P.db && p) {
    gf *o = (gf *)P.db + qi * (size_t)p;
    for (int i = tid; i < p; i += T) o[i] = -dy[i];
  }
  if (P.dG && m) {
    gf *o = (gf *)P.dG + qi * (size_t)m * n;
    for (int e = tid; e < m * n; e += T) {
      const int i = e / n, j = e % n;
      o[e] = dz[i] * C.x[j] + C.z[i] * dx[j];
    }
  }
  if (P.dh && m) {
    gf *o = (gf *)P.dh + qi * (size_t)m;
    for (int i = tid; i < m; i += T) o[i] = -dz[i];
  }
}

// ---------------------------------------------------------------------------
template <int T, int RPL, bool MLDS, int MODE>
QPD void qp_body(const Params &P) {
  extern __shared__ __attribute__((aligned(16))) float smem[];
  typedef typename std::conditional<MLDS, lf, gf>::type MF;
  const size_t qi = blockIdx.x;
  // sizes and data pointers: from the batch (solve / backward) or from this
  // block's slot descriptor (serving step)
  int n, m, p, kb;
  const float *Qp, *qp, *Ap, *bp, *Gp, *hp;
  float *wsp;
  if constexpr (MODE == kServe) {
    const SlotDesc &d = P.desc[qi];
    n = d.n; m = d.m; p = d.p; kb = d.kb;
    Qp = d.Q; qp = d.q; Ap = d.A; bp = d.b; Gp = d.G; hp = d.h;
    wsp = d.ws;
  } else {
    n = P.n; m = P.m; p = P.p; kb = P.kb;
    Qp = P.Q + qi * (size_t)n * n;
    qp = P.q + qi * (size_t)n;
    Ap = p ? P.A + qi * (size_t)p * n : nullptr;
    bp = p ? P.b + qi * (size_t)p : nullptr;
    Gp = m ? P.G + qi * (size_t)m * n : nullptr;
    hp = m ? P.h + qi * (size_t)m : nullptr;
    wsp = MLDS ? nullptr : P.ws + (size_t)qi * P.ws_stride;
  }
  const Layout L = make_layout(n, m, p, kb, MLDS, T);
  lf *sm = (lf *)smem;
  MF *Mp;
  if constexpr (MLDS) Mp = sm + L.M;
  else Mp = (gf *)wsp;
  Ctx<MF> C;
  init_ctx(C, sm, L, Mp, (const gf *)Qp, (const gf *)qp, (const gf *)Ap, (const gf *)bp,
           (const gf *)Gp, (const gf *)hp);
  __syncthreads();  // the context table
  if constexpr (MODE == kServe) C.amode = (P.desc[qi].flags >> 1) & 3;
  else C.amode = P.asm_mode;
  const int amode0 = C.amode;
  const int refine = P.refine;
  const int tid = threadIdx.x;
  // per-QP assembly mode for the Newton steps (a BF16x3 QP may fall back)
  if (tid == 0) C.iflag[3] = C.amode;
  // implicit complementarity (bounded form 0, or the first partially
  // condensed form 2 as a negative control: no border rows, no
  // regularisation); form 1 is the standard explicit IPM
  const bool bounded = P.form != 1;
  C.dyn = P.form == 0;
  C.rmode = P.rmode;
  C.bo = P.backoff;
  if (tid == 0) {
    C.iflag[5] = 0;  // refinement residuals start in FP32
  }
#ifdef QPK_PHASE_TIMING
  __shared__ long long pt_acc[PH_N];
  C.pt = (__attribute__((address_space(3))) long long *)pt_acc;
  if (tid < PH_N) C.pt[tid] = 0;
  __syncthreads();
  if (tid == 0) C.pt[15] = clock64();
#endif
  load_vectors<T>(C);
  double work = 0.0;
  int iters = 0;
  float res = 0.f;
  int status;
  if constexpr (MODE == kServe) {
    // resume one resident QP for at most d.budget Newton iterations; the
    // iterate (x, y, z, s) and the QP's arithmetic state (its assembly
    // arithmetic after any fallback, FP64 refinement residuals) persist in
    // the slot's state between steps, so the split into steps does not
    // change what is computed
    const SlotDesc &d = P.desc[qi];
    gf *st = (gf *)d.state;
    const int sticky = n + p + 2 * m;
    bool ok = true;
    if (d.flags & 1) {
      ok = initialize<T, RPL>(C, work, C.dyn != 0);
    } else {
      for (int i = tid; i < n; i += T) C.x[i] = st[i];
      for (int k = tid; k < p; k += T) C.y[k] = st[n + k];
      for (int i = tid; i < m; i += T) {
        C.z[i] = st[n + p + i];
        C.s[i] = st[n + p + m + i];
      }
      if (tid == 0) {
        const int f = __float_as_int(st[sticky]);
        C.iflag[3] = f & 3;
        C.iflag[5] = (f >> 2) & 1;
      }
      __syncthreads();
    }
    if (!ok) {
      status = mkstatus(ST_FACT, SG_PRED);
    } else {
      status = newton_loop<T, RPL>(C, bounded, d.budget, P.tol, P.pc ? 0 : 1, P.sigma, 0.f,
                                   P.delta_reg, refine, work, iters, res);
    }
    for (int i = tid; i < n; i += T) st[i] = C.x[i];
    for (int k = tid; k < p; k += T) st[n + k] = C.y[k];
    for (int i = tid; i < m; i += T) {
      st[n + p + i] = C.z[i];
      st[n + p + m + i] = C.s[i];
    }
    gf *out = (gf *)d.out;
    for (int i = tid; i < n; i += T) out[i] = C.x[i];
    for (int k = tid; k < p; k += T) out[n + k] = C.y[k];
    for (int i = tid; i < m; i += T) {
      out[n + p + i] = C.z[i];
      out[n + p + m + i] = C.s[i];
    }
    __syncthreads();
    if (tid == 0) st[sticky] = __int_as_float((C.iflag[3] & 3) | ((C.iflag[5] & 1) << 2));
    if (tid == 0) {
      *d.status = status | precision_bits(C, amode0);
      *d.iters = iters;
      *d.res = res;
    }
  } else if constexpr (MODE == kSolve) {
    const bool ok = initialize<T, RPL>(C, work, C.dyn != 0);
    QPK_PT(C, PH_INIT);
    if (!ok) {
      status = mkstatus(ST_FACT, SG_PRED);
      res = __int_as_float(0x7fc00000);
    } else {
      status = newton_loop<T, RPL>(C, bounded, P.max_iter, P.tol, P.pc ? 0 : 1, P.sigma, 0.f,
                                   P.delta_reg, refine, work, iters, res);
    }
    gf *xo = (gf *)P.x + qi * (size_t)n;
    for (int i = tid; i < n; i += T) xo[i] = C.x[i];
    if (p && P.y) for (int k = tid; k < p; k += T) ((gf *)P.y)[qi * p + k] = C.y[k];
    if (m && P.z) for (int i = tid; i < m; i += T) ((gf *)P.z)[qi * m + i] = C.z[i];
    if (m && P.s) for (int i = tid; i < m; i += T) ((gf *)P.s)[qi * m + i] = C.s[i];
    __syncthreads();
    if (tid == 0) {
      P.status[qi] = status | precision_bits(C, amode0);
      if (P.iters) P.iters[qi] = iters;
      if (P.res) P.res[qi] = res;
      if (P.work) P.work[qi] = work;
    }
  } else {
    // backward: warm start from the solution
    const gf *xs = (const gf *)P.x, *ys = (const gf *)P.y, *zs = (const gf *)P.z,
             *ss = (const gf *)P.s;
    for (int i = tid; i < n; i += T) C.x[i] = xs[qi * n + i];
    for (int k = tid; k < p; k += T) C.y[k] = ys[qi * p + k];
    for (int i = tid; i < m; i += T) {
      C.z[i] = zs[qi * m + i];
      C.s[i] = ss[qi * m + i];
    }
    __syncthreads();
    // On QPs with at least three inequality rows per variable the
    // relaxation refines its steps: H then sums that many rank-one terms in
    // FP32, and the relaxed multipliers, to which the gradients are
    // sensitive, drift by about 1e-5 relative (n = 56, m = 896, p = 28:
    // gradient entries off by up to 0.8% without; with one refinement step
    // per relaxation step every entry is within 0.4% of its 1e-3 bound;
    // n = 200, m = 800 missed the bound by 2.6x without).  At m = 2n (the
    // benchmark shapes) it would cost 44% of the backward pass for no
    // measurable gain.
    const int refine_relax = bounded && m >= 3 * n ? max(refine, 1) : refine;
    status = newton_loop<T, RPL>(C, bounded, P.relax_max_iter, P.relax_tol, 2, 0.f, P.kappa_relax,
                                 P.delta_reg, refine_relax, work, iters, res);
    // without inequalities there is nothing to relax: the relaxed point is
    // the solution (whose own status reports its accuracy)
    if (m == 0 && (status & 0xff) == ST_MAXIT) status = mkstatus(ST_CONV, SG_NONE);
    const gf *gx = (const gf *)P.gx + qi * (size_t)n;
    const gf *gy = P.gy ? (const gf *)P.gy + qi * (size_t)p : nullptr;
    const gf *gz = P.gz ? (const gf *)P.gz + qi * (size_t)m : nullptr;
    const int adj = adjoint<T, RPL>(C, bounded, gx, gy, gz, P.delta_reg, refine, work);
    QPK_PT(C, PH_BWD);
    // Algorithm 2 hands the factorisation at the relaxed point to the
    // gradient computation, so a breakdown there counts as a relax failure;
    // an adjoint solve whose refinement stalled is reported at the backward
    // stage (the gradients are written but not reliable)
    if (adj == kAdjFactorFail) status = mkstatus(ST_FACT, SG_RELAX);
    else if (adj == kAdjInaccurate && (status & 0xff) == ST_CONV) status = mkstatus(ST_MAXIT, SG_BWD);
    __syncthreads();
    write_grads<T>(C, P, qi);
    if (P.rx) for (int i = tid; i < n; i += T) ((gf *)P.rx)[qi * n + i] = C.x[i];
    if (P.ry && p) for (int k = tid; k < p; k += T) ((gf *)P.ry)[qi * p + k] = C.y[k];
    if (P.rz && m) for (int i = tid; i < m; i += T) ((gf *)P.rz)[qi * m + i] = C.z[i];
    if (P.rs && m) for (int i = tid; i < m; i += T) ((gf *)P.rs)[qi * m + i] = C.s[i];
    __syncthreads();
    if (tid == 0) {
      if (P.rstatus) P.rstatus[qi] = status | precision_bits(C, amode0);
      if (P.riters) P.riters[qi] = iters;
      if (P.res) P.res[qi] = res;
      if (P.work) P.work[qi] = work;
    }
  }
#ifdef QPK_PHASE_TIMING
  QPK_PT(C, PH_OUT);
  if (P.phase && tid < PH_N - 1) P.phase[qi * PH_N + tid] = C.pt[tid];
#endif
}

// Waves per SIMD the register allocation targets: 3 (168 VGPRs) up to 256
// threads per QP, 2 (256 VGPRs) at 512, and 4 (128 VGPRs) for 256 threads
// with 4 rows per lane and the factor in global memory in the solve and
// serving kernels: their systems (129 to 256 rows) leave a small LDS
// footprint, so four QPs fit a CU (n = 100: solve 13.6 -> 12.5 ms; the
// backward kernel at four waves spilled into a 25% slower launch and keeps
// three).  At 128 threads, 4 waves spilled about twice as much and ran 24%
// slower on n = 10 and n = 20; kernels with the factor in LDS are held to
// three QPs per CU or fewer by LDS.
#define QPK_MIN_WAVES(T, RPL, MLDS) \
  ((T) >= 512 ? 2 : ((T) == 256 && (RPL) == 4 && !(MLDS) ? 4 : 3))
#define QPK_MIN_WAVES_BWD(T) ((T) >= 512 ? 2 : 3)

// One workgroup per QP: Algorithm 1 (or the standard IPM) end to end.
template <int T, int RPL, bool MLDS>
__global__ void __launch_bounds__(T, QPK_MIN_WAVES(T, RPL, MLDS)) qp_solve_kernel(Params P) {
  qp_body<T, RPL, MLDS, kSolve>(P);
}

// One workgroup per QP: relax (Algorithm 2), adjoint solve and parameter
// gradients (Algorithm 3).
template <int T, int RPL, bool MLDS>
__global__ void __launch_bounds__(T, QPK_MIN_WAVES_BWD(T)) qp_backward_kernel(Params P) {
  qp_body<T, RPL, MLDS, kBackward>(P);
}

// One workgroup per resident serving slot: resume its Newton loop.
template <int T, int RPL, bool MLDS>
__global__ void __launch_bounds__(T, QPK_MIN_WAVES(T, RPL, MLDS)) qp_serve_kernel(Params P) {
  qp_body<T, RPL, MLDS, kServe>(P);
}

template <class K>
hipError_t launch_k(K k, const Params &P, int T, size_t lds, int grid, hipStream_t st) {
  (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k, dim3(grid), dim3(T), lds, st, P);
  return hipGetLastError();
}

}  // namespace

template <int T, int RPL>
hipError_t launch_t(const Params &P, bool m_in_lds, size_t lds, int grid, hipStream_t st) {
  if (P.mode == kSolve) {
    if (m_in_lds) return launch_k(qp_solve_kernel<T, RPL, true>, P, T, lds, grid, st);
    return launch_k(qp_solve_kernel<T, RPL, false>, P, T, lds, grid, st);
  }
  if (P.mode == kServe) {
    if (m_in_lds) return launch_k(qp_serve_kernel<T, RPL, true>, P, T, lds, grid, st);
    return launch_k(qp_serve_kernel<T, RPL, false>, P, T, lds, grid, st);
  }
  if (m_in_lds) return launch_k(qp_backward_kernel<T, RPL, true>, P, T, lds, grid, st);
  return launch_k(qp_backward_kernel<T, RPL, false>, P, T, lds, grid, st);
}

}  // namespace qpk
