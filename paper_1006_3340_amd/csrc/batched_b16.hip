// batched_b16.hip -- persistent batched kernels of the 16-slot register bucket.
#define LLL_BUCKET_TU
#define LLL_BATCH_BUCKET_TU
#include "batched_kernel.hpp"

namespace lll {
namespace batch {
LLL_BATCH_BUCKET_DECL(, 16)
}  // namespace batch
}  // namespace lll
