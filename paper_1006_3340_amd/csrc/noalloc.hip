// noalloc.hip -- one pricing pass with no device allocation.
//
// lll_price_caplets_static is lll_price_caplets (plan, FP64 precompute, path
// kernel, fixed-order reduction, results) with every device buffer of the
// pass -- the copied inputs, the precompute tables, the per-wavefront payoff
// partials and the reduction rows -- carved out of one file-scope device
// array instead of hipMalloc'd plan storage.  The kernels and launches are the
// plan path's own, so the prices are the same numbers bit for bit.
//
// The array lives in the code object: each GPU the library runs on holds its
// own copy (LLL_STATIC_WORKSPACE_BYTES) from the first use until the process
// ends.  Host code never passes the array's name to a kernel or copy (on the
// host that name is only a stand-in for the symbol): its device address is
// looked up once per device with hipGetSymbolAddress, with that device
// current, and kept in `g_scratch_dev`.
//
// Every buffer carved from the array is written by this pass before it is
// read (the path kernel writes every wavefront's row of every caplet, the
// reduction every chunk row), so nothing depends on what the previous call
// left there and nothing needs clearing.  Calls that overlap on one GPU (from
// two threads, or on two streams without ordering) share the array and race.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "lll.h"
#include "lll_internal.hpp"

namespace lll {
namespace {

constexpr size_t kScratchBytes = LLL_STATIC_WORKSPACE_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`, looked up on the
// first call on that device.
int scratch_for_current_device(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(LLL_EUNSUPPORTED, "device %d beyond the %d the static workspace tracks", dev,
                    kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(static workspace)");
        if (!ptr) return fail(LLL_EHIP, "static workspace has no device address");
        g_scratch_dev[dev] = ptr;
    }
    *out = g_scratch_dev[dev];
    return LLL_OK;
}

// Lays the plan's device buffers out from `base` (256-byte aligned pieces);
// with base == nullptr only counts.  Returns the bytes used.
size_t carve(lll_plan &p, unsigned char *base, int64_t n_paths, bool first_order) {
    const size_t esz = p.precision == LLL_FP64 ? sizeof(double) : sizeof(float);
    const size_t N = p.N, K = p.K, NM = p.nmax, S = p.S, Q = kQSize;
    const size_t nstat = 3 * S + 2;
    const size_t waves = (size_t)((n_paths + kWaveSize - 1) / kWaveSize);
    const size_t chunks = (waves + 255) / 256;
    size_t at = 0;
    auto take = [&](size_t bytes) -> unsigned char * {
        unsigned char *ptr = base ? base + at : nullptr;
        at += (bytes + 255) & ~size_t(255);
        return ptr;
    };
    auto D = [&](double **ptr, size_t n) { *ptr = reinterpret_cast<double *>(take(n * 8)); };
    auto R = [&](void **ptr, size_t n) { *ptr = take(n * esz); };
    DeviceTables &d = p.d;
    D(&d.tenor, N); D(&d.delta, N); D(&d.L0, N); D(&d.vol, K * N); D(&d.strikes, N * S);
    D(&d.x, Q); D(&d.w, Q); D(&d.kappa, K * N); D(&d.E, K * N * Q); D(&d.b0, K * N);
    D(&d.steps, 4 * N); D(&d.lam_pm, 4);
    R(&d.ew, K * Q * NM * 2); R(&d.lam, K * NM); R(&d.drift0, K * NM); R(&d.frozen, K * NM);
    R(&d.dt, K); R(&d.cinv, NM);
    if (first_order) R(&d.k2, K * NM * NM);
    D(&d.L0s, NM); D(&d.deltas, NM);
    D(&d.partials, waves * N * nstat);
    D(&d.chunks, chunks * N * nstat);
    D(&d.sums, N * nstat);
    D(&d.results, 3 * N * S + 2 * N);
    return at;
}

}  // namespace
}  // namespace lll

extern "C" int lll_price_caplets_static(const lll_term_structure *ts, int64_t n_paths,
                                        int scheme, uint64_t seed, int precision,
                                        double *price_host, double *stderr_host,
                                        double *mart_resid_host, void *stream) {
    using namespace lll;
    int rc = validate(ts);
    if (rc != LLL_OK) return rc;
    if (precision != LLL_FP32 && precision != LLL_FP64)
        return fail(LLL_EINVAL, "unknown precision %d", precision);
    if (scheme < LLL_FULL || scheme > LLL_SECOND_ORDER)
        return fail(scheme == LLL_PICARD_MP || scheme == LLL_EXACT || scheme == LLL_MLP_DRIFT
                        ? LLL_EUNSUPPORTED
                        : LLL_EINVAL,
                    "scheme %d: the static workspace runs FULL, PICARD, FROZEN, FIRST_ORDER and "
                    "SECOND_ORDER",
                    scheme);
    if (ts->n_rates > LLL_N_MAX)
        return fail(LLL_EUNSUPPORTED, "N=%d > %d rates runs only as LLL_PICARD_MP", ts->n_rates,
                    LLL_N_MAX);
    if (precision == LLL_FP64 && ts->n_rates > LLL_N_MAX_FP64)
        return fail(LLL_EUNSUPPORTED, "FP64 path kernel handles N <= %d", LLL_N_MAX_FP64);
    if (n_paths < 1 || n_paths > ((int64_t)1 << 36))
        return fail(LLL_EINVAL, "n_paths=%lld outside 1..2^36", (long long)n_paths);

    lll_plan p;  // host header only: its input vectors stay empty
    fill_plan_header(p, ts, precision, n_paths, 0);
    const size_t need = carve(p, nullptr, n_paths, scheme == LLL_FIRST_ORDER);
    if (need > kScratchBytes)
        return fail(LLL_EINVAL,
                    "this pass needs %zu bytes of device workspace (N=%d, %d steps, %lld paths); "
                    "the static workspace holds %zu",
                    need, p.N, p.K, (long long)n_paths, kScratchBytes);

    void *base = nullptr;
    rc = scratch_for_current_device(&base);
    if (rc != LLL_OK) return rc;
    carve(p, static_cast<unsigned char *>(base), n_paths, scheme == LLL_FIRST_ORDER);

    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const size_t N = p.N, S = p.S, K = p.K;
    hipError_t e = hipSuccess;
    auto H2D = [&](double *dst, const double *src, size_t n) {
        if (e == hipSuccess) e = hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyHostToDevice, st);
    };
    H2D(p.d.tenor, ts->tenor, N);
    H2D(p.d.delta, ts->delta, N);
    H2D(p.d.L0, ts->L0, N);
    H2D(p.d.vol, ts->vol, K * N);
    H2D(p.d.strikes, ts->strikes, N * S);
    if (e != hipSuccess) return hip_fail(e, "copying inputs to the static workspace");
    e = launch_precompute(p, st);
    if (e == hipSuccess && scheme == LLL_FIRST_ORDER) e = launch_first_order_tables(p, st);
    if (e != hipSuccess) return hip_fail(e, "precompute launch");
    e = launch_paths(p, scheme, n_paths, 0, seed, nullptr, st);
    if (e != hipSuccess) return hip_fail(e, "path kernel launch");
    e = launch_reduce(p, n_paths, st);
    if (e != hipSuccess) return hip_fail(e, "reduction launch");

    double res[3 * LLL_N_MAX * LLL_S_MAX + 2 * LLL_N_MAX];
    const size_t nres = 3 * N * S + 2 * N;
    e = hipMemcpyAsync(res, p.d.results, nres * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "reading results");
    const double *price = res, *se = res + N * S, *mart = res + 3 * N * S;
    if (price_host) std::memcpy(price_host, price, N * S * sizeof(double));
    if (stderr_host) std::memcpy(stderr_host, se, N * S * sizeof(double));
    if (mart_resid_host) std::memcpy(mart_resid_host, mart, N * sizeof(double));
    for (size_t i = 0; i < 2 * N * S; ++i)
        if (!std::isfinite(res[i])) return fail(LLL_ENUMERIC, "non-finite caplet price or standard error");
    return LLL_OK;
}
