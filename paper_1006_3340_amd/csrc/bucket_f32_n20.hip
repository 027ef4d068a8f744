// bucket_f32_n20.hip -- path kernel instantiations for float state, 20 rate slots.
#define LLL_BUCKET_TU
#include "path_kernel.hpp"

namespace lll {
namespace detail {
LLL_BUCKET_DECL(, float, 20)
}  // namespace detail
}  // namespace lll
