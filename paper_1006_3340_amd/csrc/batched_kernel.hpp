// batched_kernel.hpp -- the persistent kernel of one register bucket.
//
// Work items are (structure, block of 256 paths) of the structures whose rates
// fit the bucket NMAX; a grid sized to the kernel's resident capacity pulls
// items from a device counter until none are left.  Each structure keeps its
// own precompute tables (laid out for its bucket) behind a per-structure
// argument block.  Instantiated per bucket in batched_b*.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

#include "lll_device.hpp"
#include "lll_internal.hpp"
#include "path_kernel.hpp"

namespace lll {
namespace batch {

using detail::cptr;
using detail::PathArgs;

struct BatchItem {
    int32_t s;      // structure
    int32_t pad;
    int64_t first;  // first path of the block
};

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

template <int NMAX, int SCHEME>
__global__ void __launch_bounds__(kBlock) batched_kernel(cptr<PathArgs<float>> args,
                                                         cptr<BatchItem> items, int n_items,
                                                         int *__restrict__ counter) {
    // The block shares one item (its four wavefronts then stream the same
    // step tables through the CU's scalar cache).  With the state in LDS the
    // item index travels through the first word of that array, which no
    // simulation touches between the two barriers (so the block's LDS stays
    // at the state's size).
    int *slot;
    if constexpr (detail::kStateInLds<float, NMAX, SCHEME>) {
        slot = reinterpret_cast<int *>(detail::state_lds<float, NMAX>());
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
        if (wave_first < a.n_paths)
            detail::simulate<float, NMAX, SCHEME, true, detail::kAnyProduct>(a, gid);
    }
}

namespace {
__global__ void zero_counter_kernel(int *counter) { *counter = 0; }
}  // namespace

template <int NMAX, int SCHEME>
hipError_t launch_bucket_t(cptr<PathArgs<float>> args, cptr<BatchItem> items, int n_items,
                           int *counter, hipStream_t st) {
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batched_kernel<NMAX, SCHEME>,
                                                         kBlock, 0);
    if (e != hipSuccess) return e;
    const int grid = std::max(1, std::min(cus * std::max(per_cu, 1), n_items));
    hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(1), 0, st, counter);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((batched_kernel<NMAX, SCHEME>), dim3(grid), dim3(kBlock), 0, st, args,
                       items, n_items, counter);
    return hipGetLastError();
}

// The persistent launch of one bucket: items[0 .. n_items) all belong to
// structures of this bucket.
template <int NMAX>
hipError_t launch_bucket(int scheme, cptr<PathArgs<float>> args, cptr<BatchItem> items,
                         int n_items, int *counter, hipStream_t st) {
    switch (scheme) {
        case kFull: return launch_bucket_t<NMAX, kFull>(args, items, n_items, counter, st);
        case kPicard: return launch_bucket_t<NMAX, kPicard>(args, items, n_items, counter, st);
        default: return launch_bucket_t<NMAX, kFrozen>(args, items, n_items, counter, st);
    }
}

#define LLL_BATCH_BUCKET_DECL(EXT, NMAX)                                                          \
    EXT template hipError_t launch_bucket<NMAX>(int, cptr<PathArgs<float>>, cptr<BatchItem>, int, \
                                                int *, hipStream_t);
#ifndef LLL_BATCH_BUCKET_TU
LLL_BATCH_BUCKET_DECL(extern, 8)
LLL_BATCH_BUCKET_DECL(extern, 16)
LLL_BATCH_BUCKET_DECL(extern, 24)
LLL_BATCH_BUCKET_DECL(extern, 32)
LLL_BATCH_BUCKET_DECL(extern, 40)
#endif

}  // namespace batch
}  // namespace lll
