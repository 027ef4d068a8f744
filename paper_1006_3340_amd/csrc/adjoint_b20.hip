// adjoint_b20.hip -- adjoint kernel for the 20-slot register bucket.
#define LLL_BUCKET_TU
#include "adjoint_kernel.hpp"

namespace lll {
namespace adj {
template hipError_t launch_adjoint_bucket<20>(const PathArgs<float> &, const AdjArgs &, hipStream_t);
template hipError_t launch_vjp_bucket<20>(const PathArgs<float> &, const AdjArgs &, const VjpArgs &,
                                           hipStream_t);
}  // namespace adj
}  // namespace lll
