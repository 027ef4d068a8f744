// Host-only stand-ins for the library's kernel launchers, so that the C ABI's
// host code (abi.hip, noalloc.hip) links into a sanitizer build without device
// code (tests/test_abi_sanitizers.py).  Every launcher reports that it is not
// available; allocation-free helpers do nothing.  Only the validation and
// error paths that run before any launch are exercised through them.
#include <hip/hip_runtime.h>

#include "lll.h"
#include "lll_internal.hpp"

namespace lll {
int bucket_for(int n, bool slots20) { return n <= 8 ? 8 : n <= 16 ? 16 : (slots20 && n <= 20) ? 20 : n <= 24 ? 24 : n <= 32 ? 32 : n <= 40 ? 40 : 64; }
hipError_t greeks_alloc(lll_plan &) { return hipErrorNotSupported; }
void greeks_free(lll_plan &) {}
void mlp_plan_free(lll_plan &) {}
void picard_mp_free(lll_plan &) {}
hipError_t picard_mp_alloc(lll_plan &) { return hipErrorNotSupported; }
size_t batch_args_bytes() { return 256; }
size_t batch_item_bytes() { return 16; }
int64_t exact_table_entries(int, int) { return 0; }
int64_t exact_state_entries(int, int64_t) { return 0; }
hipError_t launch_drift(const lll_plan &, int, const double *, int64_t, double *, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_exact(const lll_plan &, int64_t, int64_t, uint64_t, double *, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_paths(const lll_plan &, int, int64_t, int64_t, uint64_t, double *, hipStream_t) { return hipErrorNotSupported; }
hipError_t batch_prepare(lll_batch &, int64_t, uint64_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_greeks(const lll_plan &, int64_t, uint64_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_philox(const uint32_t *, const uint32_t *, int64_t, uint32_t *, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_sampler_math(int, const double *, int64_t, double *, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_reduce(const lll_plan &, int64_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_batched(const lll_batch &, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_picard_mp(const lll_plan &, int64_t, int64_t, uint64_t, double *, hipStream_t) { return hipErrorNotSupported; }
hipError_t measure_fma_peak(hipStream_t, double *) { return hipErrorNotSupported; }
hipError_t measure_mix_peak(hipStream_t, double *) { return hipErrorNotSupported; }
hipError_t measure_mfma_peak(hipStream_t, double *) { return hipErrorNotSupported; }
hipError_t launch_greeks_vjp(const lll_plan &, int64_t, uint64_t, const double *, const double *, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_increments(const lll_plan &, int, int64_t, int64_t, uint64_t, double *, double *, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_precompute(const lll_plan &, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_set_inputs(const lll_plan &, const double *, const double *, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_first_order_tables(const lll_plan &, hipStream_t) { return hipErrorNotSupported; }
}  // namespace lll

extern "C" int lll_plan_execute_mlp(lll_plan *, const lll_mlp *, int, int64_t, uint64_t, int, double *, void *) {
    return LLL_EUNSUPPORTED;
}
