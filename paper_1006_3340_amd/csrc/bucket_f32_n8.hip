// bucket_f32_n8.hip -- path kernel instantiations for float state, 8 rate slots.
#define LLL_BUCKET_TU
#include "path_kernel.hpp"

namespace lll {
namespace detail {
LLL_BUCKET_DECL(, float, 8)
}  // namespace detail
}  // namespace lll
