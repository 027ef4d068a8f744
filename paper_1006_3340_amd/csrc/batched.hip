// batched.hip -- many independent term structures in one persistent launch.
//
// Work items are (structure, block of 256 paths), sorted by decreasing cost
// (N^2 s per path) on the host.  A grid sized to the resident capacity of the
// GPU pulls items from an atomic counter until none are left, so long tenors
// start first and the tail is filled by short ones.  Every structure uses the
// 40-slot register bucket (its rates occupy the top N slots) and its own
// precompute tables, addressed through a per-structure argument block.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "lll_device.hpp"
#include "lll_internal.hpp"
#define LLL_BUCKET_TU
#include "path_kernel.hpp"

namespace lll {
namespace {

using detail::cptr;
using detail::PathArgs;

constexpr int kBatchSlots = 40;

struct BatchItem {
    int32_t s;      // structure
    int32_t pad;
    int64_t first;  // first path of the block
};

__global__ void zero_counter_kernel(int *counter) { *counter = 0; }

// Copy of a trivially copyable struct read word by word through the constant
// address space (uniform address: scalar loads).
template <typename T>
__device__ __forceinline__ T load_uniform(cptr<T> p) {
    static_assert(sizeof(T) % 4 == 0, "word-sized struct");
    T v;
    const cptr<uint32_t> w = (cptr<uint32_t>)(p);
    uint32_t *d = reinterpret_cast<uint32_t *>(&v);
#pragma unroll
    for (int i = 0; i < static_cast<int>(sizeof(T) / 4); ++i) d[i] = w[i];
    return v;
}

template <int SCHEME>
__global__ void __launch_bounds__(kBlock) batched_kernel(cptr<PathArgs<float>> args,
                                                         cptr<BatchItem> items, int n_items,
                                                         int *__restrict__ counter) {
    // The block shares one item (its four wavefronts then stream the same
    // step tables through the CU's scalar cache).  With the state in LDS the
    // item index travels through the first word of that array, which no
    // simulation touches between the two barriers (so the block's LDS stays
    // at 40 KiB: four blocks per CU).
    int *slot;
    if constexpr (detail::kStateInLds<float, kBatchSlots, SCHEME>) {
        slot = reinterpret_cast<int *>(detail::state_lds<float, kBatchSlots>());
    } else {
        __shared__ int s_item;
        slot = &s_item;
    }
    for (;;) {
        if (threadIdx.x == 0) *slot = atomicAdd(counter, 1);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(*slot);
        __syncthreads();
        if (item >= n_items) return;  // same value in every lane of the block
        const BatchItem it = load_uniform<BatchItem>(items + item);
        const PathArgs<float> a = load_uniform<PathArgs<float>>(args + it.s);
        const int64_t gid = it.first + threadIdx.x;
        const int64_t wave_first = gid - (threadIdx.x % kWave);
        if (wave_first < a.n_paths) detail::simulate<float, kBatchSlots, SCHEME, true, detail::kAnyProduct>(a, gid);
    }
}

template <int SCHEME>
hipError_t launch_batched_t(const lll_batch &b, hipStream_t st) {
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batched_kernel<SCHEME>, kBlock, 0);
    if (e != hipSuccess) return e;
    const int grid = std::max(1, std::min(cus * std::max(per_cu, 1), b.n_items));
    hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(1), 0, st, b.counter);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(batched_kernel<SCHEME>, dim3(grid), dim3(kBlock), 0, st,
                       detail::as_const(static_cast<const PathArgs<float> *>(b.args)),
                       detail::as_const(static_cast<const BatchItem *>(b.items)), b.n_items,
                       b.counter);
    return hipGetLastError();
}

}  // namespace

size_t batch_item_bytes() { return sizeof(BatchItem); }
size_t batch_args_bytes() { return sizeof(PathArgs<float>); }

// Host side: argument blocks of every structure for this pass and the item list.
hipError_t batch_prepare(lll_batch &b, int64_t n_paths_each, uint64_t seed, hipStream_t st) {
    std::vector<PathArgs<float>> args(b.plans.size());
    for (size_t i = 0; i < b.plans.size(); ++i)
        args[i] = detail::make_args<float>(*b.plans[i], seed, n_paths_each, 0, nullptr);
    std::vector<BatchItem> items;
    const int64_t blocks = (n_paths_each + kBlock - 1) / kBlock;
    for (size_t i = 0; i < b.plans.size(); ++i)
        for (int64_t j = 0; j < blocks; ++j) items.push_back({static_cast<int32_t>(i), 0, j * kBlock});
    std::stable_sort(items.begin(), items.end(), [&](const BatchItem &x, const BatchItem &y) {
        const lll_plan &px = *b.plans[x.s], &py = *b.plans[y.s];
        const int64_t cx = (int64_t)px.N * px.N * px.s, cy = (int64_t)py.N * py.N * py.s;
        return cx > cy;
    });
    b.n_items = static_cast<int>(items.size());
    hipError_t e = hipMemcpyAsync(b.args, args.data(), args.size() * sizeof(PathArgs<float>),
                                  hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b.items, items.data(), items.size() * sizeof(BatchItem),
                           hipMemcpyHostToDevice, st);
    // the host vectors die at return: make the copies complete first
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
}

hipError_t launch_batched(const lll_batch &b, int scheme, hipStream_t st) {
    switch (scheme) {
        case kFull: return launch_batched_t<kFull>(b, st);
        case kPicard: return launch_batched_t<kPicard>(b, st);
        default: return launch_batched_t<kFrozen>(b, st);
    }
}

}  // namespace lll
