// Instantiation of the fused kernel for 256 threads per QP and up to 256 rows of
// the bordered KKT system.
// phases inlined into the kernels: measured on the differentiation workload
// (n = 100, factor in global memory), the solve kernel takes 14.8 instead of
// 16.5 ms and the backward kernel 4.18 instead of 4.41 ms (scratch per lane
// 504 instead of 1244 bytes); at 512 threads and 16 rows per lane inlining
// was 22% slower (n = 256), so that instantiation keeps separate phases
#define QPK_INLINE_PHASES
#include "qp_kernel_impl.hpp"

namespace qpk {
template hipError_t launch_t<256, 4>(const Params &, bool, size_t, int, hipStream_t);
}  // namespace qpk
