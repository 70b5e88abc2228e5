// Instantiation of the fused kernel for 512 threads per QP and up to 1024 rows of
// the bordered KKT system.
#include "qp_kernel_impl.hpp"

namespace qpk {
template hipError_t launch_t<512, 16>(const Params &, bool, size_t, int, hipStream_t);
}  // namespace qpk
