// Instantiation of the fused kernel for 512 threads per QP and up to 64 rows of
// the bordered KKT system.
// small systems: phases inlined into the kernels
#define QPK_INLINE_PHASES
#include "qp_kernel_impl.hpp"

namespace qpk {
template hipError_t launch_t<512, 1>(const Params &, bool, size_t, int, hipStream_t);
}  // namespace qpk
