// bucket_f32_n40.hip -- path kernel instantiations for float state, 40 rate slots.
#define LLL_BUCKET_TU
#include "path_kernel.hpp"

namespace lll {
namespace detail {
LLL_BUCKET_DECL(, float, 40)
}  // namespace detail
}  // namespace lll
