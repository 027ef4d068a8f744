// bucket_f64_n8.hip -- path kernel instantiations for double state, 8 rate slots.
#define LLL_BUCKET_TU
#include "path_kernel.hpp"

namespace lll {
namespace detail {
LLL_BUCKET_DECL(, double, 8)
}  // namespace detail
}  // namespace lll
