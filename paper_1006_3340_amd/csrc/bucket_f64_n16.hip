// bucket_f64_n16.hip -- path kernel instantiations for double state, 16 rate slots.
#define LLL_BUCKET_TU
#include "path_kernel.hpp"

namespace lll {
namespace detail {
LLL_BUCKET_DECL(, double, 16)
}  // namespace detail
}  // namespace lll
