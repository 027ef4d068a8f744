// batched.hip -- many independent term structures, one persistent launch per
// register bucket.
//
// Every structure is planned in the smallest bucket that holds its rates (8,
// 16, 24, 32 or 40 slots), so its path kernel runs at that bucket's register
// and LDS footprint.  Work items are (structure, block of 256 paths), grouped
// by bucket and sorted by decreasing cost (N^2 s per path) inside each group;
// each bucket's persistent kernel pulls its items from its own device counter.
// The buckets' launches run concurrently on the batch's side streams (forked
// from and joined back into the caller's stream), so a bucket that runs out
// of items leaves its compute units to the others instead of idling them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "batched_kernel.hpp"
#include "lll_internal.hpp"

namespace lll {

using batch::BatchItem;
using detail::PathArgs;

namespace {

constexpr int kBuckets[kBatchBuckets] = {40, 32, 24, 16, 8};

int bucket_index(int nmax) {
    for (int b = 0; b < kBatchBuckets; ++b)
        if (kBuckets[b] == nmax) return b;
    return -1;
}

hipError_t launch_one(int nmax, int scheme, detail::cptr<PathArgs<float>> args,
                      detail::cptr<BatchItem> items, int n, int *counter, hipStream_t st) {
    switch (nmax) {
        case 8: return batch::launch_bucket<8>(scheme, args, items, n, counter, st);
        case 16: return batch::launch_bucket<16>(scheme, args, items, n, counter, st);
        case 24: return batch::launch_bucket<24>(scheme, args, items, n, counter, st);
        case 32: return batch::launch_bucket<32>(scheme, args, items, n, counter, st);
        case 40: return batch::launch_bucket<40>(scheme, args, items, n, counter, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

size_t batch_item_bytes() { return sizeof(BatchItem); }
size_t batch_args_bytes() { return sizeof(PathArgs<float>); }

// Host side: argument blocks of every structure for this pass and the item
// list, grouped by bucket (largest first) and by decreasing cost inside a bucket.
hipError_t batch_prepare(lll_batch &b, int64_t n_paths_each, uint64_t seed, hipStream_t st) {
    std::vector<PathArgs<float>> args(b.plans.size());
    for (size_t i = 0; i < b.plans.size(); ++i)
        args[i] = detail::make_args<float>(*b.plans[i], seed, n_paths_each, 0, nullptr);
    std::vector<BatchItem> items;
    const int64_t blocks = (n_paths_each + kBlock - 1) / kBlock;
    for (size_t i = 0; i < b.plans.size(); ++i)
        for (int64_t j = 0; j < blocks; ++j) items.push_back({static_cast<int32_t>(i), 0, j * kBlock});
    auto bucket_of = [&](const BatchItem &x) { return bucket_index(b.plans[x.s]->nmax); };
    std::stable_sort(items.begin(), items.end(), [&](const BatchItem &x, const BatchItem &y) {
        const int bx = bucket_of(x), by = bucket_of(y);
        if (bx != by) return bx < by;
        const lll_plan &px = *b.plans[x.s], &py = *b.plans[y.s];
        const int64_t cx = (int64_t)px.N * px.N * px.s, cy = (int64_t)py.N * py.N * py.s;
        return cx > cy;
    });
    for (int k = 0; k < kBatchBuckets; ++k) b.bucket_begin[k] = b.bucket_end[k] = 0;
    for (size_t i = 0; i < items.size(); ++i) {
        const int k = bucket_of(items[i]);
        if (k < 0) return hipErrorInvalidValue;
        if (b.bucket_end[k] == 0) b.bucket_begin[k] = static_cast<int>(i);
        b.bucket_end[k] = static_cast<int>(i) + 1;
    }
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

// One persistent launch per bucket present: the largest on the caller's
// stream, the others on side streams that wait for the caller's stream and
// that the caller's stream waits for in turn.
hipError_t launch_batched(const lll_batch &b, int scheme, hipStream_t st) {
    const auto args = detail::as_const(static_cast<const PathArgs<float> *>(b.args));
    const auto *items = static_cast<const BatchItem *>(b.items);
    hipError_t e = hipEventRecord(b.fork, st);
    bool first = true;
    for (int k = 0; k < kBatchBuckets && e == hipSuccess; ++k) {
        const int n = b.bucket_end[k] - b.bucket_begin[k];
        if (n <= 0) continue;
        hipStream_t s = first ? st : b.side[k];
        if (!first) e = hipStreamWaitEvent(s, b.fork, 0);
        if (e == hipSuccess)
            e = launch_one(kBuckets[k], scheme, args, detail::as_const(items + b.bucket_begin[k]), n,
                           b.counter + 64 * k, s);
        if (e == hipSuccess && !first) e = hipEventRecord(b.join[k], s);
        if (e == hipSuccess && !first) e = hipStreamWaitEvent(st, b.join[k], 0);
        first = false;
    }
    return e;
}

}  // namespace lll
