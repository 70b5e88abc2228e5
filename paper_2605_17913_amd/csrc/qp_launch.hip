// Non-template entry points of the kernel layer: LDS sizing and dispatch to
// the instantiated (threads, rows-per-lane) configurations.
#include "qp_kernel_impl.hpp"

namespace qpk {

size_t lds_bytes(int n, int m, int p, int kb, bool m_in_lds, int threads) {
  return (size_t)make_layout(n, m, p, kb, m_in_lds, threads).total * sizeof(float);
}

int64_t ws_floats(int n, int m, int p, int kb) {
  const Layout L = make_layout(n, m, p, kb, false, 128);
  return (int64_t)al4(moff(L.Nmax) + kNB);
}

size_t lds_limit() { return kCuLds - kStaticLds; }

bool mfma_stage_fits(int n, int m, int p, int kb, bool m_in_lds, int threads) {
  const Layout L = make_layout(n, m, p, kb, m_in_lds, threads);
  return stage_floats(n) <= L.stg_len;
}

#define QPK_EXTERN(TT, RR) \
  extern template hipError_t launch_t<TT, RR>(const Params &, bool, size_t, int, hipStream_t);
QPK_EXTERN(128, 1) QPK_EXTERN(128, 2) QPK_EXTERN(128, 4) QPK_EXTERN(128, 8)
QPK_EXTERN(256, 1) QPK_EXTERN(256, 2) QPK_EXTERN(256, 4) QPK_EXTERN(256, 8)
QPK_EXTERN(512, 1) QPK_EXTERN(512, 2) QPK_EXTERN(512, 4) QPK_EXTERN(512, 8)
QPK_EXTERN(512, 16)
#undef QPK_EXTERN

hipError_t launch(const Params &P, int threads, bool m_in_lds, size_t lds, int grid,
                  hipStream_t stream) {
  const int Nmax = P.n + P.kb + P.p;
  const int rpl = (Nmax + 63) / 64;
#define QPK_DISPATCH(TT)                                                  \
  if (threads == TT) {                                                    \
    if (rpl <= 1) return launch_t<TT, 1>(P, m_in_lds, lds, grid, stream); \
    if (rpl <= 2) return launch_t<TT, 2>(P, m_in_lds, lds, grid, stream); \
    if (rpl <= 4) return launch_t<TT, 4>(P, m_in_lds, lds, grid, stream); \
    if (rpl <= 8) return launch_t<TT, 8>(P, m_in_lds, lds, grid, stream); \
    if (rpl <= 16 && TT == 512)                                           \
      return launch_t<512, 16>(P, m_in_lds, lds, grid, stream);           \
    return hipErrorInvalidValue;                                          \
  }
  QPK_DISPATCH(128)
  QPK_DISPATCH(256)
  QPK_DISPATCH(512)
#undef QPK_DISPATCH
  return hipErrorInvalidValue;
}

}  // namespace qpk
