// bucket_f32_n24.hip -- path kernel instantiations for float state, 24 rate slots.
#define LLL_BUCKET_TU
#include "path_kernel.hpp"

namespace lll {
namespace detail {
LLL_BUCKET_DECL(, float, 24)
}  // namespace detail
}  // namespace lll
