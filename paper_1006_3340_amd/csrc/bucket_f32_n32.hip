// bucket_f32_n32.hip -- path kernel instantiations for float state, 32 rate slots.
#define LLL_BUCKET_TU
#include "path_kernel.hpp"

namespace lll {
namespace detail {
LLL_BUCKET_DECL(, float, 32)
}  // namespace detail
}  // namespace lll
