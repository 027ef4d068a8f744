// bucket_f32_n16.hip -- path kernel instantiations for float state, 16 rate slots.
#define LLL_BUCKET_TU
#include "path_kernel.hpp"

namespace lll {
namespace detail {
LLL_BUCKET_DECL(, float, 16)
}  // namespace detail
}  // namespace lll
