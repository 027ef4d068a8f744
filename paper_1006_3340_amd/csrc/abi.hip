// abi.hip -- the extern "C" boundary: validation, plan lifetime, launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lll.h"
#include "lll_internal.hpp"

namespace lll {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(LLL_EHIP, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace lll

namespace {

using lll::fail;
using lll::g_last_error;
using lll::hip_fail;

bool finite_all(const double *a, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

}  // namespace

namespace lll {

// Input checks of paper Section 2: (LR2) positive forwards and a strictly
// increasing tenor with matching accrual fractions; (LR1) bounded vols with
// exponential moments -- for the NIG driver the drift integral is finite iff
// the live vols satisfy Lambda_+ < alpha - beta and Lambda_- < alpha + beta.
int validate(const lll_term_structure *ts) {
    if (!ts) return fail(LLL_EINVAL, "term structure is NULL");
    const int N = ts->n_rates, s = ts->steps_per_period, S = ts->n_strikes;
    if (N < 1 || N > LLL_N_MAX_MP)
        return fail(LLL_EINVAL, "n_rates=%d outside 1..%d", N, LLL_N_MAX_MP);
    if (s < 1 || s > 100000) return fail(LLL_EINVAL, "steps_per_period=%d must be >= 1", s);
    if ((int64_t)N * s > (int64_t)1 << 24) return fail(LLL_EINVAL, "too many Euler steps");
    if (S < 1 || S > LLL_S_MAX) return fail(LLL_EINVAL, "n_strikes=%d outside 1..%d", S, LLL_S_MAX);
    if (!ts->tenor || !ts->delta || !ts->L0 || !ts->vol || !ts->strikes)
        return fail(LLL_EINVAL, "NULL input array");
    if (ts->driver != LLL_DRIVER_NIG && ts->driver != LLL_DRIVER_BROWNIAN)
        return fail(LLL_EINVAL, "unknown driver %d", ts->driver);
    if (ts->product != LLL_CAPLETS && ts->product != LLL_SWAPTIONS)
        return fail(LLL_EINVAL, "unknown product %d", ts->product);
    if (!finite_all(ts->tenor, N) || !finite_all(ts->delta, N) || !finite_all(ts->L0, N) ||
        !finite_all(ts->vol, (size_t)N * s * N) || !finite_all(ts->strikes, (size_t)N * S) ||
        !std::isfinite(ts->B0_T1))
        return fail(LLL_EINVAL, "non-finite input value");
    double prev = 0.0;
    for (int r = 0; r < N; ++r) {
        if (!(ts->tenor[r] > prev)) return fail(LLL_EINVAL, "tenor not strictly increasing at %d", r);
        if (!(ts->delta[r] > 0.0)) return fail(LLL_EINVAL, "delta[%d] <= 0", r);
        if (!(ts->L0[r] > 0.0)) return fail(LLL_EINVAL, "L0[%d] <= 0", r);
        prev = ts->tenor[r];
    }
    for (int r = 0; r + 1 < N; ++r) {
        const double gap = ts->tenor[r + 1] - ts->tenor[r];
        if (std::fabs(gap - ts->delta[r]) > 1e-9 * std::fmax(1.0, gap))
            return fail(LLL_EINVAL, "delta[%d]=%g does not match tenor gap %g", r, ts->delta[r], gap);
    }
    if (ts->B0_T1 > 1.0) return fail(LLL_EINVAL, "B0_T1=%g > 1", ts->B0_T1);
    if (ts->driver == LLL_DRIVER_NIG) {
        if (!(ts->alpha > std::fabs(ts->beta)) || !std::isfinite(ts->alpha))
            return fail(LLL_EINVAL, "NIG needs alpha > |beta| (alpha=%g beta=%g)", ts->alpha, ts->beta);
        if (!(ts->delta_nig > 0.0) || !std::isfinite(ts->delta_nig))
            return fail(LLL_EINVAL, "NIG delta must be > 0");
        double lp = 0.0, lm = 0.0;
        for (int k = 0; k < N * s; ++k) {
            double sp = 0.0, sm = 0.0;
            for (int r = k / s; r < N; ++r) {
                const double v = ts->vol[(size_t)k * N + r];
                sp += std::fmax(v, 0.0);
                sm += std::fmax(-v, 0.0);
            }
            lp = std::fmax(lp, sp);
            lm = std::fmax(lm, sm);
        }
        if (!(lp < ts->alpha - ts->beta) || !(lm < ts->alpha + ts->beta))
            return fail(LLL_EMOMENT,
                        "exponential moments fail: Lambda+=%g vs alpha-beta=%g, Lambda-=%g vs "
                        "alpha+beta=%g",
                        lp, ts->alpha - ts->beta, lm, ts->alpha + ts->beta);
    } else {
        if (!(ts->c >= 0.0) || !std::isfinite(ts->c)) return fail(LLL_EINVAL, "Brownian c < 0");
    }
    return LLL_OK;
}

// Scalar fields of a plan (sizes, bucket, driver, B(0, T_1)); the host copies
// of the input arrays and the device buffers are set by the caller.
void fill_plan_header(lll_plan &p, const lll_term_structure *ts, int precision, int64_t max_paths,
                      int nmax) {
    p.N = ts->n_rates;
    p.s = ts->steps_per_period;
    p.S = ts->n_strikes;
    p.K = p.N * p.s;
    p.driver = ts->driver;
    p.precision = precision;
    p.nmax = nmax > 0 ? nmax : bucket_for(p.N, precision == LLL_FP32);
    p.off = p.nmax - p.N;
    p.struct_id = ts->struct_id;
    p.product = ts->product;
    p.B0_T1 = ts->B0_T1 > 0.0 ? ts->B0_T1 : 1.0 / (1.0 + ts->tenor[0] * ts->L0[0]);
    p.alpha = ts->alpha;
    p.beta = ts->beta;
    p.delta_nig = ts->delta_nig;
    p.c = ts->c;
    p.max_paths = max_paths;
    p.max_waves = (max_paths + kWaveSize - 1) / kWaveSize;
    p.max_chunks = (p.max_waves + 255) / 256;
    (void)hipGetDevice(&p.device);
}

}  // namespace lll

namespace {

using lll::validate;

template <typename T>
hipError_t dalloc(T **p, size_t n) {
    return hipMalloc(reinterpret_cast<void **>(p), n * sizeof(T) + 16);
}

void free_tables(lll::DeviceTables &d) {
    void *ptrs[] = {d.tenor, d.delta, d.L0, d.vol, d.strikes, d.x, d.w, d.kappa, d.E, d.b0,
                    d.steps, d.lam_pm, d.vol_base, d.ew, d.lam, d.drift0, d.frozen, d.dt, d.cinv, d.k2, d.kex, d.xex, d.L0s,
                    d.deltas, d.partials, d.chunks, d.sums, d.results};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    d = lll::DeviceTables{};
}

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Status of a pass whose results are not finite: the precompute's flags of
// inputs set from device memory (non-finite or non-positive values, the
// moment condition of (LR1)) or else non-finite payoffs.
int nonfinite_status(lll_plan *plan, hipStream_t st) {
    double flags[4] = {0, 0, 0, 0};
    hipError_t e = hipMemcpyAsync(flags, plan->d.lam_pm, sizeof flags, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "reading input status");
    if (flags[3] != 0.0)
        return fail(LLL_EINVAL, "device inputs: a forward is not positive or a vol is not finite");
    if (flags[2] != 0.0)
        return fail(LLL_EMOMENT,
                    "device inputs: exponential moments fail (Lambda+=%g vs alpha-beta=%g, "
                    "Lambda-=%g vs alpha+beta=%g)",
                    flags[0], plan->alpha - plan->beta, flags[1], plan->alpha + plan->beta);
    return fail(LLL_ENUMERIC, "non-finite caplet price or standard error");
}

}  // namespace

extern "C" {

const char *lll_version(void) { return "lll-mi355x 0.1 (gfx950)"; }

const char *lll_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

namespace {

// Plan creation with an explicit register bucket (0 = smallest that fits N).
int create_plan(const lll_term_structure *ts, int precision, int64_t max_paths, int nmax,
                lll_plan **plan_out) {
    if (!plan_out) return fail(LLL_EINVAL, "plan_out is NULL");
    *plan_out = nullptr;
    int rc = validate(ts);
    if (rc != LLL_OK) return rc;
    if (precision != LLL_FP32 && precision != LLL_FP64)
        return fail(LLL_EINVAL, "unknown precision %d", precision);
    if (max_paths < 1 || max_paths > ((int64_t)1 << 36))
        return fail(LLL_EINVAL, "max_paths=%lld outside 1..2^36", (long long)max_paths);
    if (precision == LLL_FP64 && ts->n_rates > LLL_N_MAX_FP64)
        return fail(LLL_EUNSUPPORTED, "FP64 path kernel handles N <= %d", LLL_N_MAX_FP64);

    lll_plan *p = new (std::nothrow) lll_plan();
    if (!p) return fail(LLL_ENOMEM, "host allocation failed");
    lll::fill_plan_header(*p, ts, precision, max_paths, nmax);
    p->tenor.assign(ts->tenor, ts->tenor + p->N);
    p->delta.assign(ts->delta, ts->delta + p->N);
    p->L0.assign(ts->L0, ts->L0 + p->N);
    p->vol.assign(ts->vol, ts->vol + (size_t)p->K * p->N);
    p->strikes.assign(ts->strikes, ts->strikes + (size_t)p->N * p->S);

    const size_t esz = precision == LLL_FP64 ? sizeof(double) : sizeof(float);
    const size_t N = p->N, K = p->K, NM = p->nmax, S = p->S;
    const size_t nstat = 3 * S + 2;
    lll::DeviceTables &d = p->d;
    hipError_t e = hipSuccess;
    auto A = [&](auto **ptr, size_t n) {
        if (e == hipSuccess) e = dalloc(ptr, n);
    };
    A(&d.tenor, N); A(&d.delta, N); A(&d.L0, N); A(&d.vol, K * N); A(&d.strikes, N * S);
    A(&d.x, lll::kQSize); A(&d.w, lll::kQSize); A(&d.kappa, K * N); A(&d.E, K * N * lll::kQSize);
    A(&d.b0, K * N); A(&d.steps, 4 * N); A(&d.lam_pm, 4);
    auto AB = [&](void **ptr, size_t n) {
        if (e == hipSuccess) e = hipMalloc(ptr, n * esz + 16);
    };
    AB(&d.ew, K * lll::kQSize * NM * 2); AB(&d.lam, K * NM); AB(&d.drift0, K * NM);
    AB(&d.frozen, K * NM); AB(&d.dt, K); AB(&d.cinv, NM);
    A(&d.L0s, NM); A(&d.deltas, NM);
    A(&d.partials, (size_t)p->max_waves * N * nstat);
    A(&d.chunks, (size_t)p->max_chunks * N * nstat);
    A(&d.sums, N * nstat);
    A(&d.results, 3 * N * S + 2 * N);
    if (e != hipSuccess) {
        free_tables(d);
        delete p;
        return fail(e == hipErrorOutOfMemory ? LLL_ENOMEM : LLL_EHIP, "device allocation: %s",
                    hipGetErrorString(e));
    }
    auto H2D = [&](double *dst, const std::vector<double> &src) {
        if (e == hipSuccess) e = hipMemcpy(dst, src.data(), src.size() * sizeof(double),
                                           hipMemcpyHostToDevice);
    };
    H2D(d.tenor, p->tenor); H2D(d.delta, p->delta); H2D(d.L0, p->L0); H2D(d.vol, p->vol);
    H2D(d.strikes, p->strikes);
    if (e != hipSuccess) {
        free_tables(d);
        delete p;
        return hip_fail(e, "copying inputs to the device");
    }
    *plan_out = p;
    return LLL_OK;
}

}  // namespace

extern "C" {

int lll_plan_create(const lll_term_structure *ts, int precision, int64_t max_paths,
                    lll_plan **plan_out) {
    return create_plan(ts, precision, max_paths, 0, plan_out);
}

int lll_plan_set_timing(lll_plan *plan, int enable) {
    if (!plan) return fail(LLL_EINVAL, "plan is NULL");
    if (enable && !plan->ev[0]) {
        for (int i = 0; i < 4; ++i) {
            hipError_t e = hipEventCreate(&plan->ev[i]);
            if (e != hipSuccess) return hip_fail(e, "creating timing events");
        }
    }
    plan->timing = enable != 0;
    plan->timed = false;
    return LLL_OK;
}

int lll_plan_timing(lll_plan *plan, float *ms_host) {
    if (!plan || !ms_host) return fail(LLL_EINVAL, "NULL argument");
    if (!plan->timed) return fail(LLL_EINVAL, "no timed execute recorded");
    hipError_t e = hipEventSynchronize(plan->ev[3]);
    for (int i = 0; i < 3 && e == hipSuccess; ++i)
        e = hipEventElapsedTime(&ms_host[i], plan->ev[i], plan->ev[i + 1]);
    if (e != hipSuccess) return hip_fail(e, "reading timing events");
    return LLL_OK;
}

int lll_plan_destroy(lll_plan *plan) {
    if (!plan) return LLL_OK;
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (dev != plan->device) (void)hipSetDevice(plan->device);
    for (int i = 0; i < 4; ++i)
        if (plan->ev[i]) (void)hipEventDestroy(plan->ev[i]);
    lll::greeks_free(*plan);
    lll::mlp_plan_free(*plan);
    lll::picard_mp_free(*plan);
    free_tables(plan->d);
    if (dev != plan->device) (void)hipSetDevice(dev);
    delete plan;
    return LLL_OK;
}

int lll_plan_attach_mlp(lll_plan *plan, const lll_mlp *mlp) {
    if (!plan) return fail(LLL_EINVAL, "plan is NULL");
    plan->mlp = mlp;
    return LLL_OK;
}

int lll_plan_execute(lll_plan *plan, int scheme, int64_t n_paths, int64_t path_offset,
                     uint64_t seed, double *path_fix_dev, void *stream) {
    if (!plan) return fail(LLL_EINVAL, "plan is NULL");
    if (scheme == LLL_MLP_DRIFT) {
        if (!plan->mlp)
            return fail(LLL_EINVAL, "LLL_MLP_DRIFT needs a network attached with lll_plan_attach_mlp");
        if (path_offset != 0)
            return fail(LLL_EUNSUPPORTED, "LLL_MLP_DRIFT runs paths from 0 (path_offset=%lld)",
                        (long long)path_offset);
        return lll_plan_execute_mlp(plan, plan->mlp, 1, n_paths, seed, 0, path_fix_dev, stream);
    }
    if (scheme < LLL_FULL || scheme > LLL_EXACT)
        return fail(LLL_EINVAL, "unknown scheme %d", scheme);
    if (n_paths < 1 || n_paths > plan->max_paths)
        return fail(LLL_EINVAL, "n_paths=%lld outside 1..%lld", (long long)n_paths,
                    (long long)plan->max_paths);
    if (path_offset < 0 || path_offset > ((int64_t)1 << 62))
        return fail(LLL_EINVAL, "path_offset=%lld out of range", (long long)path_offset);
    const bool mp = scheme == LLL_PICARD_MP;
    if (!mp && plan->N > LLL_N_MAX)
        return fail(LLL_EUNSUPPORTED, "N=%d > %d rates runs only as LLL_PICARD_MP", plan->N,
                    LLL_N_MAX);
    if (mp && plan->precision != LLL_FP32)
        return fail(LLL_EUNSUPPORTED, "LLL_PICARD_MP runs on FP32 plans");
    if (mp && plan->driver != LLL_DRIVER_NIG)
        return fail(LLL_EUNSUPPORTED, "LLL_PICARD_MP is implemented for the NIG driver");
    if (mp) {
        hipError_t ea = lll::picard_mp_alloc(*plan);
        if (ea != hipSuccess) return fail(LLL_ENOMEM, "PICARD_MP buffers: %s", hipGetErrorString(ea));
    }
    const bool exact = scheme == LLL_EXACT;
    if (exact && plan->N > LLL_N_MAX_EXACT)
        return fail(LLL_EUNSUPPORTED, "LLL_EXACT sums 2^(N-1-i) terms per rate: N=%d > %d",
                    plan->N, LLL_N_MAX_EXACT);
    if (exact && (!plan->d.kex || !plan->d.xex)) {
        const size_t esz = plan->precision == LLL_FP64 ? sizeof(double) : sizeof(float);
        const int64_t nk = lll::exact_table_entries(plan->N, plan->s);
        hipError_t ea = plan->d.kex ? hipSuccess : hipMalloc(&plan->d.kex, (size_t)nk * esz);
        if (ea != hipSuccess) {
            plan->d.kex = nullptr;
            return fail(LLL_ENOMEM, "exact-drift table: %s", hipGetErrorString(ea));
        }
        ea = hipMalloc(&plan->d.xex,
                       (size_t)lll::exact_state_entries(plan->N, plan->max_paths) * esz);
        if (ea != hipSuccess) {
            plan->d.xex = nullptr;
            return fail(LLL_ENOMEM, "exact-drift path states: %s", hipGetErrorString(ea));
        }
    }
    if (scheme == LLL_FIRST_ORDER && !plan->d.k2) {
        const size_t esz = plan->precision == LLL_FP64 ? sizeof(double) : sizeof(float);
        hipError_t ea = hipMalloc(&plan->d.k2, (size_t)plan->K * plan->nmax * plan->nmax * esz);
        if (ea != hipSuccess) {
            plan->d.k2 = nullptr;
            return fail(LLL_ENOMEM, "first-order table: %s", hipGetErrorString(ea));
        }
    }
    hipStream_t st = as_stream(stream);
    const bool t = plan->timing;
    hipError_t e = t ? hipEventRecord(plan->ev[0], st) : hipSuccess;
    if (e == hipSuccess) e = lll::launch_precompute(*plan, st);
    if (e == hipSuccess && scheme == LLL_FIRST_ORDER) e = lll::launch_first_order_tables(*plan, st);
    if (e != hipSuccess) return hip_fail(e, "precompute launch");
    if (t) e = hipEventRecord(plan->ev[1], st);
    if (e == hipSuccess)
        e = mp      ? lll::launch_picard_mp(*plan, n_paths, path_offset, seed, path_fix_dev, st)
            : exact ? lll::launch_exact(*plan, n_paths, path_offset, seed, path_fix_dev, st)
                    : lll::launch_paths(*plan, scheme, n_paths, path_offset, seed, path_fix_dev, st);
    if (e != hipSuccess) return hip_fail(e, "path kernel launch");
    if (t) e = hipEventRecord(plan->ev[2], st);
    if (e == hipSuccess) e = lll::launch_reduce(*plan, n_paths, st);
    if (e != hipSuccess) return hip_fail(e, "reduction launch");
    if (t) e = hipEventRecord(plan->ev[3], st);
    if (e != hipSuccess) return hip_fail(e, "recording timing event");
    plan->timed = t;
    plan->last_n_paths = n_paths;
    plan->executed = true;
    return LLL_OK;
}

int lll_plan_results(lll_plan *plan, double *price_host, double *stderr_host,
                     double *mart_resid_host, double *mart_se_host, double *n_itm_host,
                     void *stream) {
    if (!plan) return fail(LLL_EINVAL, "plan is NULL");
    if (!plan->executed) return fail(LLL_EINVAL, "plan has not been executed");
    const size_t N = plan->N, S = plan->S;
    std::vector<double> res(3 * N * S + 2 * N);
    hipStream_t st = as_stream(stream);
    hipError_t e = hipMemcpyAsync(res.data(), plan->d.results, res.size() * sizeof(double),
                                  hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "reading results");
    const double *price = res.data(), *se = price + N * S, *itm = se + N * S;
    const double *mart = itm + N * S, *mse = mart + N;
    if (price_host) std::memcpy(price_host, price, N * S * sizeof(double));
    if (stderr_host) std::memcpy(stderr_host, se, N * S * sizeof(double));
    if (n_itm_host) std::memcpy(n_itm_host, itm, N * S * sizeof(double));
    if (mart_resid_host) std::memcpy(mart_resid_host, mart, N * sizeof(double));
    if (mart_se_host) std::memcpy(mart_se_host, mse, N * sizeof(double));
    if (!finite_all(price, N * S) || !finite_all(se, N * S)) return nonfinite_status(plan, st);
    return LLL_OK;
}

int lll_plan_set_inputs_dev(lll_plan *plan, const double *L0_dev, const double *vol_shift_dev,
                            void *stream) {
    if (!plan) return fail(LLL_EINVAL, "plan is NULL");
    if (!L0_dev && !vol_shift_dev) return LLL_OK;
    hipError_t e = hipSuccess;
    if (vol_shift_dev && !plan->d.vol_base) {
        // the curves are shifted from the table the plan was created with
        const size_t bytes = (size_t)plan->K * plan->N * sizeof(double);
        e = hipMalloc(&plan->d.vol_base, bytes);
        if (e != hipSuccess) {
            plan->d.vol_base = nullptr;
            return fail(LLL_ENOMEM, "vol table copy: %s", hipGetErrorString(e));
        }
        e = hipMemcpy(plan->d.vol_base, plan->vol.data(), bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "copying the vol table");
    }
    e = lll::launch_set_inputs(*plan, L0_dev, vol_shift_dev, as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "setting inputs");
    return LLL_OK;
}

int lll_plan_results_dev(lll_plan *plan, double *price_dev, double *stderr_dev,
                         double *mart_resid_dev, void *stream) {
    if (!plan) return fail(LLL_EINVAL, "plan is NULL");
    if (!plan->executed) return fail(LLL_EINVAL, "plan has not been executed");
    const size_t N = plan->N, S = plan->S;
    hipStream_t st = as_stream(stream);
    const double *res = plan->d.results;
    hipError_t e = hipSuccess;
    auto D2D = [&](double *dst, const double *src, size_t n) {
        if (dst && e == hipSuccess)
            e = hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, st);
    };
    D2D(price_dev, res, N * S);
    D2D(stderr_dev, res + N * S, N * S);
    D2D(mart_resid_dev, res + 3 * N * S, N);
    if (e != hipSuccess) return hip_fail(e, "copying results");
    return LLL_OK;
}

int lll_plan_sums(lll_plan *plan, double *sums_host, void *stream) {
    if (!plan || !sums_host) return fail(LLL_EINVAL, "NULL argument");
    if (!plan->executed) return fail(LLL_EINVAL, "plan has not been executed");
    const size_t n = (size_t)plan->N * (3 * plan->S + 2);
    hipStream_t st = as_stream(stream);
    hipError_t e = hipMemcpyAsync(sums_host, plan->d.sums, n * sizeof(double),
                                  hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "reading sums");
    return LLL_OK;
}

int lll_plan_partials(lll_plan *plan, double *partials_host, int64_t capacity, void *stream) {
    if (!plan || !partials_host) return fail(LLL_EINVAL, "NULL argument");
    if (!plan->executed) return fail(LLL_EINVAL, "plan has not been executed");
    const int64_t waves = (plan->last_n_paths + lll::kWaveSize - 1) / lll::kWaveSize;
    const int64_t n = waves * plan->N * (3 * plan->S + 2);
    if (capacity < n) return fail(LLL_EINVAL, "capacity %lld < %lld", (long long)capacity,
                                  (long long)n);
    hipStream_t st = as_stream(stream);
    hipError_t e = hipMemcpyAsync(partials_host, plan->d.partials, n * sizeof(double),
                                  hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "reading partials");
    return LLL_OK;
}

int lll_price_caplets(const lll_term_structure *ts, int64_t n_paths, int scheme, uint64_t seed,
                      int precision, double *price_host, double *stderr_host,
                      double *mart_resid_host, void *stream) {
    lll_plan *plan = nullptr;
    int rc = lll_plan_create(ts, precision, n_paths, &plan);
    if (rc != LLL_OK) return rc;
    rc = lll_plan_execute(plan, scheme, n_paths, 0, seed, nullptr, stream);
    if (rc == LLL_OK)
        rc = lll_plan_results(plan, price_host, stderr_host, mart_resid_host, nullptr, nullptr,
                              stream);
    lll_plan_destroy(plan);
    return rc;
}

int lll_fp32_fma_peak(double *tflops_host, void *stream) {
    if (!tflops_host) return fail(LLL_EINVAL, "tflops_host is NULL");
    hipError_t e = lll::measure_fma_peak(as_stream(stream), tflops_host);
    if (e != hipSuccess) return hip_fail(e, "FMA probe");
    return LLL_OK;
}

int lll_fp32_mix_peak(double *tflops_host, void *stream) {
    if (!tflops_host) return fail(LLL_EINVAL, "tflops_host is NULL");
    hipError_t e = lll::measure_mix_peak(as_stream(stream), tflops_host);
    if (e != hipSuccess) return hip_fail(e, "instruction-mix probe");
    return LLL_OK;
}

int lll_fp32_mfma_peak(double *tflops_host, void *stream) {
    if (!tflops_host) return fail(LLL_EINVAL, "tflops_host is NULL");
    hipError_t e = lll::measure_mfma_peak(as_stream(stream), tflops_host);
    if (e != hipSuccess) return hip_fail(e, "matrix-core probe");
    return LLL_OK;
}

int lll_philox(const uint32_t *ctr_host, const uint32_t *key_host, int64_t n, uint32_t *out_host,
               void *stream) {
    if (!ctr_host || !key_host || !out_host) return fail(LLL_EINVAL, "NULL argument");
    if (n < 1 || n > ((int64_t)1 << 28)) return fail(LLL_EINVAL, "n=%lld out of range", (long long)n);
    uint32_t *d = nullptr;
    hipError_t e = hipMalloc(&d, (size_t)n * 10 * sizeof(uint32_t));
    if (e != hipSuccess) return hip_fail(e, "allocating Philox buffers");
    hipStream_t st = as_stream(stream);
    uint32_t *dc = d, *dk = d + 4 * n, *dout = d + 6 * n;
    e = hipMemcpyAsync(dc, ctr_host, (size_t)n * 4 * sizeof(uint32_t), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dk, key_host, (size_t)n * 2 * sizeof(uint32_t), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = lll::launch_philox(dc, dk, n, dout, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out_host, dout, (size_t)n * 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d);
    if (e != hipSuccess) return hip_fail(e, "Philox kernel");
    return LLL_OK;
}

int lll_sampler_math(int fn, const double *x_host, int64_t n, double *out_host, void *stream) {
    if (!x_host || !out_host) return fail(LLL_EINVAL, "NULL argument");
    if (fn < LLL_SM_LOG || fn > LLL_SM_DIV) return fail(LLL_EINVAL, "unknown routine %d", fn);
    if (n < 1 || n > ((int64_t)1 << 26)) return fail(LLL_EINVAL, "n=%lld out of range", (long long)n);
    const int64_t nin = fn == LLL_SM_DIV ? 2 * n : n;
    for (int64_t i = 0; i < nin; ++i) {
        const double v = x_host[i];
        bool ok;
        if (fn == LLL_SM_LOG)
            ok = std::isnormal(v) && v > 0.0 && v <= 1.0;
        else if (fn == LLL_SM_SINPI || fn == LLL_SM_COSPI)
            ok = v >= 0.0 && v <= 2.0 && std::ldexp(v, 24) == std::floor(std::ldexp(v, 24));
        else if (fn == LLL_SM_SQRT)
            ok = std::isnormal(v) && v > 0.0;
        else
            ok = std::isfinite(v) && (i % 2 == 0 || (std::isnormal(v) && v > 0.0));
        if (!ok) return fail(LLL_EINVAL, "argument %lld = %g outside the routine's domain", (long long)i, v);
    }
    double *d = nullptr;
    hipError_t e = hipMalloc(&d, (size_t)(nin + n) * sizeof(double));
    if (e != hipSuccess) return hip_fail(e, "allocating sampler buffers");
    hipStream_t st = as_stream(stream);
    e = hipMemcpyAsync(d, x_host, (size_t)nin * sizeof(double), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = lll::launch_sampler_math(fn, d, n, d + nin, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out_host, d + nin, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d);
    if (e != hipSuccess) return hip_fail(e, "sampler routine kernel");
    return LLL_OK;
}

int lll_plan_increments(lll_plan *plan, int k, int64_t p0, int64_t n, uint64_t seed,
                        double *V_host, double *dH_host, void *stream) {
    if (!plan || !V_host || !dH_host) return fail(LLL_EINVAL, "NULL argument");
    if (k < 0 || k >= plan->K) return fail(LLL_EINVAL, "step %d outside 0..%d", k, plan->K - 1);
    if (n < 1 || n > ((int64_t)1 << 28) || p0 < 0) return fail(LLL_EINVAL, "bad path range");
    hipStream_t st = as_stream(stream);
    hipError_t e = lll::launch_precompute(*plan, st);
    if (e != hipSuccess) return hip_fail(e, "precompute launch");
    double *d = nullptr;
    e = hipMalloc(&d, (size_t)n * 2 * sizeof(double));
    if (e != hipSuccess) return hip_fail(e, "allocating increment buffers");
    e = lll::launch_increments(*plan, k, p0, n, seed, d, d + n, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(V_host, d, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dH_host, d + n, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d);
    if (e != hipSuccess) return hip_fail(e, "increment kernel");
    return LLL_OK;
}

int lll_plan_tables(lll_plan *plan, double *x_host, double *w_host, double *kappa_host,
                    double *E_host, double *b0_host, void *stream) {
    if (!plan) return fail(LLL_EINVAL, "plan is NULL");
    hipStream_t st = as_stream(stream);
    hipError_t e = lll::launch_precompute(*plan, st);
    if (e != hipSuccess) return hip_fail(e, "precompute launch");
    const size_t K = plan->K, N = plan->N, Q = lll::kQSize;
    auto D2H = [&](double *dst, const double *src, size_t n) {
        if (dst && e == hipSuccess)
            e = hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToHost, st);
    };
    D2H(x_host, plan->d.x, Q);
    D2H(w_host, plan->d.w, Q);
    D2H(kappa_host, plan->d.kappa, K * N);
    D2H(E_host, plan->d.E, K * N * Q);
    D2H(b0_host, plan->d.b0, K * N);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "reading tables");
    return LLL_OK;
}

int lll_plan_drift(lll_plan *plan, int k, const double *L_host, int64_t n, double *b_host,
                   void *stream) {
    if (!plan || !L_host || !b_host) return fail(LLL_EINVAL, "NULL argument");
    if (k < 0 || k >= plan->K) return fail(LLL_EINVAL, "step %d outside 0..%d", k, plan->K - 1);
    if (n < 1 || n > ((int64_t)1 << 24)) return fail(LLL_EINVAL, "n=%lld out of range", (long long)n);
    if (plan->N > LLL_N_MAX)
        return fail(LLL_EUNSUPPORTED, "the drift kernel handles N <= %d", LLL_N_MAX);
    const int first = k / plan->s;
    for (int64_t i = 0; i < n; ++i)
        for (int r = first; r < plan->N; ++r)
            if (!(L_host[i * plan->N + r] > 0.0) || !std::isfinite(L_host[i * plan->N + r]))
                return fail(LLL_EINVAL, "rates must be positive and finite");
    hipStream_t st = as_stream(stream);
    hipError_t e = lll::launch_precompute(*plan, st);
    if (e != hipSuccess) return hip_fail(e, "precompute launch");
    const size_t bytes = (size_t)n * plan->N * sizeof(double);
    double *d = nullptr;
    e = hipMalloc(&d, 2 * bytes);
    if (e != hipSuccess) return hip_fail(e, "allocating drift buffers");
    double *dL = d, *db = d + (size_t)n * plan->N;
    e = hipMemcpyAsync(dL, L_host, bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = lll::launch_drift(*plan, k, dL, n, db, st);
    if (e == hipSuccess) e = hipMemcpyAsync(b_host, db, bytes, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d);
    if (e != hipSuccess) return hip_fail(e, "drift kernel");
    return LLL_OK;
}

int lll_batch_destroy(lll_batch *batch) {
    if (!batch) return LLL_OK;
    for (lll_plan *p : batch->plans) lll_plan_destroy(p);
    if (batch->args) (void)hipFree(batch->args);
    if (batch->items) (void)hipFree(batch->items);
    if (batch->counter) (void)hipFree(batch->counter);
    for (int i = 0; i < 2; ++i)
        if (batch->ev[i]) (void)hipEventDestroy(batch->ev[i]);
    for (int k = 0; k < lll::kBatchBuckets; ++k) {
        if (batch->side[k]) (void)hipStreamDestroy(batch->side[k]);
        if (batch->join[k]) (void)hipEventDestroy(batch->join[k]);
    }
    if (batch->fork) (void)hipEventDestroy(batch->fork);
    delete batch;
    return LLL_OK;
}

int lll_batch_create(const lll_term_structure *ts, int n_ts, int64_t max_paths_each,
                     lll_batch **batch_out) {
    if (!batch_out) return fail(LLL_EINVAL, "batch_out is NULL");
    *batch_out = nullptr;
    if (!ts || n_ts < 1 || n_ts > 4096) return fail(LLL_EINVAL, "n_ts=%d outside 1..4096", n_ts);
    if (max_paths_each < 1 || max_paths_each > ((int64_t)1 << 30))
        return fail(LLL_EINVAL, "max_paths_each=%lld outside 1..2^30", (long long)max_paths_each);
    // one work item per block of 256 paths of every structure; the device
    // counter is a 32-bit int that every resident block bumps once past the
    // end, so the item count stays well below 2^31
    const int64_t items = (max_paths_each + 255) / 256 * n_ts;
    if (items > ((int64_t)1 << 30))
        return fail(LLL_EINVAL, "n_ts x max_paths_each / 256 = %lld work items exceeds 2^30",
                    (long long)items);
    for (int i = 0; i < n_ts; ++i) {
        int rc = validate(&ts[i]);
        if (rc == LLL_OK && ts[i].n_rates > LLL_N_MAX)
            rc = fail(LLL_EINVAL, "n_rates=%d outside 1..%d", ts[i].n_rates, LLL_N_MAX);
        if (rc != LLL_OK) {
            std::string msg = "structure " + std::to_string(i) + ": " + g_last_error;
            return fail(rc, "%s", msg.c_str());
        }
    }
    lll_batch *b = new (std::nothrow) lll_batch();
    if (!b) return fail(LLL_ENOMEM, "host allocation failed");
    b->max_paths_each = max_paths_each;
    for (int i = 0; i < n_ts; ++i) {
        lll_plan *p = nullptr;
        // the persistent kernels come in the 8/16/24/32/40-slot buckets
        int rc = create_plan(&ts[i], LLL_FP32, max_paths_each,
                             lll::bucket_for(ts[i].n_rates, false), &p);
        if (rc != LLL_OK) {
            lll_batch_destroy(b);
            return rc;
        }
        b->plans.push_back(p);
    }
    b->max_items = static_cast<int>(items);
    hipError_t e = hipMalloc(&b->args, n_ts * lll::batch_args_bytes());
    if (e == hipSuccess) e = hipMalloc(&b->items, (size_t)b->max_items * lll::batch_item_bytes());
    if (e == hipSuccess)
        e = hipMalloc(reinterpret_cast<void **>(&b->counter), 64 * sizeof(int) * lll::kBatchBuckets);
    if (e != hipSuccess) {
        lll_batch_destroy(b);
        return fail(LLL_ENOMEM, "device allocation: %s", hipGetErrorString(e));
    }
    e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    for (int k = 0; k < lll::kBatchBuckets && e == hipSuccess; ++k) {
        e = hipStreamCreateWithFlags(&b->side[k], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        lll_batch_destroy(b);
        return hip_fail(e, "creating the batch's streams");
    }
    *batch_out = b;
    return LLL_OK;
}

int lll_price_caplets_batched(const lll_term_structure *ts, int n_ts, int64_t n_paths_each,
                              int scheme, uint64_t seed, double *const *price_host,
                              double *const *stderr_host, void *stream) {
    if (!price_host) return fail(LLL_EINVAL, "price_host is NULL");
    for (int i = 0; i < n_ts && ts; ++i)
        if (!price_host[i]) return fail(LLL_EINVAL, "price_host[%d] is NULL", i);
    lll_batch *b = nullptr;
    int rc = lll_batch_create(ts, n_ts, n_paths_each, &b);
    if (rc != LLL_OK) return rc;
    rc = lll_batch_execute(b, scheme, n_paths_each, seed, stream);
    for (int i = 0; i < n_ts && rc == LLL_OK; ++i)
        rc = lll_batch_results(b, i, price_host[i], stderr_host ? stderr_host[i] : nullptr,
                               nullptr, nullptr, nullptr, stream);
    lll_batch_destroy(b);
    return rc;
}

int lll_batch_set_timing(lll_batch *batch, int enable) {
    if (!batch) return fail(LLL_EINVAL, "batch is NULL");
    if (enable && !batch->ev[0]) {
        for (int i = 0; i < 2; ++i) {
            hipError_t e = hipEventCreate(&batch->ev[i]);
            if (e != hipSuccess) return hip_fail(e, "creating timing events");
        }
    }
    batch->timing = enable != 0;
    batch->timed = false;
    return LLL_OK;
}

int lll_batch_timing(lll_batch *batch, float *ms_host) {
    if (!batch || !ms_host) return fail(LLL_EINVAL, "NULL argument");
    if (!batch->timed) return fail(LLL_EINVAL, "no timed execute recorded");
    hipError_t e = hipEventSynchronize(batch->ev[1]);
    if (e == hipSuccess) e = hipEventElapsedTime(ms_host, batch->ev[0], batch->ev[1]);
    if (e != hipSuccess) return hip_fail(e, "reading timing events");
    return LLL_OK;
}

int lll_batch_execute(lll_batch *batch, int scheme, int64_t n_paths_each, uint64_t seed,
                      void *stream) {
    if (!batch) return fail(LLL_EINVAL, "batch is NULL");
    if (scheme != LLL_FULL && scheme != LLL_PICARD && scheme != LLL_FROZEN)
        return fail(LLL_EINVAL, "unknown scheme %d", scheme);
    if (n_paths_each < 1 || n_paths_each > batch->max_paths_each)
        return fail(LLL_EINVAL, "n_paths_each=%lld outside 1..%lld", (long long)n_paths_each,
                    (long long)batch->max_paths_each);
    hipStream_t st = as_stream(stream);
    hipError_t e = hipSuccess;
    for (lll_plan *p : batch->plans) {
        e = lll::launch_precompute(*p, st);
        if (e != hipSuccess) return hip_fail(e, "precompute launch");
    }
    e = lll::batch_prepare(*batch, n_paths_each, seed, st);
    if (e != hipSuccess) return hip_fail(e, "preparing batch items");
    if (batch->timing) e = hipEventRecord(batch->ev[0], st);
    if (e == hipSuccess) e = lll::launch_batched(*batch, scheme, st);
    if (e != hipSuccess) return hip_fail(e, "batched kernel launch");
    if (batch->timing) e = hipEventRecord(batch->ev[1], st);
    if (e != hipSuccess) return hip_fail(e, "recording timing event");
    for (lll_plan *p : batch->plans) {
        e = lll::launch_reduce(*p, n_paths_each, st);
        if (e != hipSuccess) return hip_fail(e, "reduction launch");
        p->last_n_paths = n_paths_each;
        p->executed = true;
    }
    batch->timed = batch->timing;
    batch->n_paths_each = n_paths_each;
    batch->executed = true;
    return LLL_OK;
}

int lll_batch_results(lll_batch *batch, int index, double *price_host, double *stderr_host,
                      double *mart_resid_host, double *mart_se_host, double *n_itm_host,
                      void *stream) {
    if (!batch) return fail(LLL_EINVAL, "batch is NULL");
    if (index < 0 || index >= (int)batch->plans.size())
        return fail(LLL_EINVAL, "index %d outside 0..%d", index, (int)batch->plans.size() - 1);
    return lll_plan_results(batch->plans[index], price_host, stderr_host, mart_resid_host,
                            mart_se_host, n_itm_host, stream);
}

// Checks shared by the Greeks entry points; allocates the adjoint buffers.
static int greeks_prepare(lll_plan *plan, int64_t n_paths) {
    if (!plan) return fail(LLL_EINVAL, "plan is NULL");
    if (plan->precision != LLL_FP32)
        return fail(LLL_EUNSUPPORTED, "the adjoint runs on FP32 plans");
    if (plan->driver != LLL_DRIVER_NIG)
        return fail(LLL_EUNSUPPORTED, "the adjoint is implemented for the NIG driver");
    if (plan->N > LLL_N_MAX)
        return fail(LLL_EUNSUPPORTED, "the adjoint handles N <= %d", LLL_N_MAX);
    if (n_paths < 1 || n_paths > plan->max_paths)
        return fail(LLL_EINVAL, "n_paths=%lld outside 1..%lld", (long long)n_paths,
                    (long long)plan->max_paths);
    hipError_t e = lll::greeks_alloc(*plan);
    if (e != hipSuccess) {
        lll::greeks_free(*plan);
        return fail(e == hipErrorOutOfMemory ? LLL_ENOMEM : LLL_EHIP,
                    "allocating adjoint checkpoints: %s", hipGetErrorString(e));
    }
    return LLL_OK;
}

int lll_plan_greeks(lll_plan *plan, int64_t n_paths, uint64_t seed, void *stream) {
    const int rc = greeks_prepare(plan, n_paths);
    if (rc != LLL_OK) return rc;
    hipError_t e = hipSuccess;
    hipStream_t st = as_stream(stream);
    const bool t = plan->timing;
    // the whole Greeks pass is timed as the path stage (events 1 -> 2)
    if (t) e = hipEventRecord(plan->ev[0], st);
    if (t && e == hipSuccess) e = hipEventRecord(plan->ev[1], st);
    if (e == hipSuccess) e = lll::launch_greeks(*plan, n_paths, seed, st);
    if (e != hipSuccess) return hip_fail(e, "adjoint launch");
    if (t) {
        e = hipEventRecord(plan->ev[2], st);
        if (e == hipSuccess) e = hipEventRecord(plan->ev[3], st);
        if (e != hipSuccess) return hip_fail(e, "recording timing events");
    }
    plan->timed = t;
    plan->last_n_paths = n_paths;
    plan->executed = true;
    plan->greeks_n_paths = n_paths;
    plan->greeks_done = true;
    return LLL_OK;
}

int lll_plan_greeks_results(lll_plan *plan, double *price_host, double *dP_dL0_host,
                            double *dP_dvol_host, void *stream) {
    if (!plan) return fail(LLL_EINVAL, "plan is NULL");
    if (!plan->greeks_done) return fail(LLL_EINVAL, "no Greeks pass has run on this plan");
    const size_t N = plan->N;
    std::vector<double> out(2 * N * N + N);
    hipStream_t st = as_stream(stream);
    hipError_t e = hipMemcpyAsync(out.data(), plan->g.out, out.size() * sizeof(double),
                                  hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "reading Greeks");
    if (dP_dL0_host) std::memcpy(dP_dL0_host, out.data(), N * N * sizeof(double));
    if (dP_dvol_host) std::memcpy(dP_dvol_host, out.data() + N * N, N * N * sizeof(double));
    if (price_host) std::memcpy(price_host, out.data() + 2 * N * N, N * sizeof(double));
    if (!finite_all(out.data(), out.size())) return nonfinite_status(plan, st);
    return LLL_OK;
}

int lll_plan_greeks_vjp(lll_plan *plan, int64_t n_paths, uint64_t seed, const double *weights_host,
                        void *stream) {
    if (!weights_host) return fail(LLL_EINVAL, "weights are NULL");
    const int rc = greeks_prepare(plan, n_paths);
    if (rc != LLL_OK) return rc;
    if (!finite_all(weights_host, plan->N)) return fail(LLL_EINVAL, "non-finite weight");
    hipStream_t st = as_stream(stream);
    const bool t = plan->timing;
    hipError_t e = hipSuccess;
    if (t) e = hipEventRecord(plan->ev[0], st);
    if (t && e == hipSuccess) e = hipEventRecord(plan->ev[1], st);
    if (e == hipSuccess) e = lll::launch_greeks_vjp(*plan, n_paths, seed, weights_host, nullptr, st);
    if (e != hipSuccess) return hip_fail(e, "adjoint launch");
    if (t) {
        e = hipEventRecord(plan->ev[2], st);
        if (e == hipSuccess) e = hipEventRecord(plan->ev[3], st);
        if (e != hipSuccess) return hip_fail(e, "recording timing events");
    }
    plan->timed = t;
    plan->last_n_paths = n_paths;
    plan->executed = true;
    plan->vjp_done = true;
    return LLL_OK;
}

int lll_plan_greeks_vjp_results(lll_plan *plan, double *price_host, double *vjp_L0_host,
                                double *vjp_vol_host, void *stream) {
    if (!plan) return fail(LLL_EINVAL, "plan is NULL");
    if (!plan->vjp_done) return fail(LLL_EINVAL, "no vector-Jacobian pass has run on this plan");
    const size_t N = plan->N;
    std::vector<double> out(3 * N);
    hipStream_t st = as_stream(stream);
    hipError_t e = hipMemcpyAsync(out.data(), plan->g.vjp_out, out.size() * sizeof(double),
                                  hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "reading the vector-Jacobian product");
    if (price_host) std::memcpy(price_host, out.data(), N * sizeof(double));
    if (vjp_L0_host) std::memcpy(vjp_L0_host, out.data() + N, N * sizeof(double));
    if (vjp_vol_host) std::memcpy(vjp_vol_host, out.data() + 2 * N, N * sizeof(double));
    if (!finite_all(out.data(), out.size())) return nonfinite_status(plan, st);
    return LLL_OK;
}

int lll_plan_greeks_vjp_dev(lll_plan *plan, int64_t n_paths, uint64_t seed,
                            const double *weights_dev, void *stream) {
    if (!weights_dev) return fail(LLL_EINVAL, "weights are NULL");
    const int rc = greeks_prepare(plan, n_paths);
    if (rc != LLL_OK) return rc;
    hipStream_t st = as_stream(stream);
    const bool t = plan->timing;
    hipError_t e = hipSuccess;
    if (t) e = hipEventRecord(plan->ev[0], st);
    if (t && e == hipSuccess) e = hipEventRecord(plan->ev[1], st);
    if (e == hipSuccess) e = lll::launch_greeks_vjp(*plan, n_paths, seed, nullptr, weights_dev, st);
    if (e != hipSuccess) return hip_fail(e, "adjoint launch");
    if (t) {
        e = hipEventRecord(plan->ev[2], st);
        if (e == hipSuccess) e = hipEventRecord(plan->ev[3], st);
        if (e != hipSuccess) return hip_fail(e, "recording timing events");
    }
    plan->timed = t;
    plan->last_n_paths = n_paths;
    plan->executed = true;
    plan->vjp_done = true;
    return LLL_OK;
}

int lll_plan_greeks_vjp_results_dev(lll_plan *plan, double *price_dev, double *vjp_L0_dev,
                                    double *vjp_vol_dev, void *stream) {
    if (!plan) return fail(LLL_EINVAL, "plan is NULL");
    if (!plan->vjp_done) return fail(LLL_EINVAL, "no vector-Jacobian pass has run on this plan");
    const size_t N = plan->N;
    hipStream_t st = as_stream(stream);
    hipError_t e = hipSuccess;
    auto D2D = [&](double *dst, const double *src) {
        if (dst && e == hipSuccess)
            e = hipMemcpyAsync(dst, src, N * sizeof(double), hipMemcpyDeviceToDevice, st);
    };
    D2D(price_dev, plan->g.vjp_out);
    D2D(vjp_L0_dev, plan->g.vjp_out + N);
    D2D(vjp_vol_dev, plan->g.vjp_out + 2 * N);
    if (e != hipSuccess) return hip_fail(e, "copying the vector-Jacobian product");
    return LLL_OK;
}

int lll_plan_greeks_results_dev(lll_plan *plan, double *price_dev, double *dP_dL0_dev,
                                double *dP_dvol_dev, void *stream) {
    if (!plan) return fail(LLL_EINVAL, "plan is NULL");
    if (!plan->greeks_done) return fail(LLL_EINVAL, "no Greeks pass has run on this plan");
    const size_t N = plan->N;
    hipStream_t st = as_stream(stream);
    hipError_t e = hipSuccess;
    auto D2D = [&](double *dst, const double *src, size_t n) {
        if (dst && e == hipSuccess)
            e = hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, st);
    };
    D2D(dP_dL0_dev, plan->g.out, N * N);
    D2D(dP_dvol_dev, plan->g.out + N * N, N * N);
    D2D(price_dev, plan->g.out + 2 * N * N, N);
    if (e != hipSuccess) return hip_fail(e, "copying Greeks");
    return LLL_OK;
}

int lll_caplet_greeks(const lll_term_structure *ts, int64_t n_paths, uint64_t seed,
                      double *price_host, double *dP_dL0_host, double *dP_dvol_host,
                      void *stream) {
    lll_plan *plan = nullptr;
    int rc = lll_plan_create(ts, LLL_FP32, n_paths, &plan);
    if (rc != LLL_OK) return rc;
    rc = lll_plan_greeks(plan, n_paths, seed, stream);
    if (rc == LLL_OK) rc = lll_plan_greeks_results(plan, price_host, dP_dL0_host, dP_dvol_host, stream);
    lll_plan_destroy(plan);
    return rc;
}

}  // extern "C"
