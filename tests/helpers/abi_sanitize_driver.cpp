// Drives the C ABI's host code -- input validation, plan set-up and tear-down
// on failure, the NULL-argument and size checks of every entry point, the
// static workspace's size check -- in a build instrumented with
// AddressSanitizer and UndefinedBehaviorSanitizer, linked against host-only
// stand-ins of the kernel launchers (abi_host_stubs.cpp).  Without a GPU the
// device allocations fail and the error paths that free partial plans run.
// Prints "ok" and exits 0 when every call returned the expected status.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "lll.h"

namespace {

int failures = 0;

void expect(bool cond, const char *what) {
    if (!cond) {
        std::printf("FAIL: %s (last error: %s)\n", what, lll_last_error());
        ++failures;
    }
}

struct Inputs {
    int N, s, S;
    std::vector<double> tenor, delta, L0, vol, strikes;
    lll_term_structure ts{};
    Inputs(int N_, int s_, int S_) : N(N_), s(s_), S(S_) {
        tenor.resize(N); delta.resize(N); L0.resize(N);
        vol.assign((size_t)N * s * N, 0.0); strikes.resize((size_t)N * S);
        for (int i = 0; i < N; ++i) {
            tenor[i] = 0.5 * (i + 1);
            delta[i] = 0.5;
            L0[i] = 0.03 + 0.001 * i;
            for (int j = 0; j < S; ++j) strikes[(size_t)i * S + j] = L0[i] * (0.8 + 0.2 * j);
        }
        for (int k = 0; k < N * s; ++k)
            for (int i = k / s; i < N; ++i) vol[(size_t)k * N + i] = 0.15;
        sync();
    }
    void sync() {
        ts.n_rates = N; ts.steps_per_period = s; ts.n_strikes = S; ts.driver = LLL_DRIVER_NIG;
        ts.struct_id = 3; ts.product = LLL_CAPLETS;
        ts.tenor = tenor.data(); ts.delta = delta.data(); ts.L0 = L0.data(); ts.vol = vol.data();
        ts.strikes = strikes.data(); ts.B0_T1 = 0.0;
        ts.alpha = 18.0; ts.beta = -4.0; ts.delta_nig = 1.0; ts.c = 0.0;
    }
};

int create(const lll_term_structure *ts, int precision = LLL_FP32, int64_t paths = 1024) {
    lll_plan *p = nullptr;
    const int rc = lll_plan_create(ts, precision, paths, &p);
    if (rc == LLL_OK) lll_plan_destroy(p);
    else expect(p == nullptr, "failed create leaves no plan");
    return rc;
}

}  // namespace

int main() {
    Inputs a(10, 4, 3);
    // valid input: validation passes; without a device the allocation fails
    const int rc = create(&a.ts);
    expect(rc == LLL_OK || rc == LLL_ENOMEM || rc == LLL_EHIP, "valid structure");
    expect(create(nullptr) == LLL_EINVAL, "NULL structure");
    { Inputs b = a; b.L0[3] = -0.01; b.sync(); expect(create(&b.ts) == LLL_EINVAL, "negative L0"); }
    { Inputs b = a; b.L0[2] = NAN; b.sync(); expect(create(&b.ts) == LLL_EINVAL, "NaN L0"); }
    { Inputs b = a; b.tenor[4] = b.tenor[3]; b.sync(); expect(create(&b.ts) == LLL_EINVAL, "tenor order"); }
    { Inputs b = a; b.delta[2] = 0.3; b.sync(); expect(create(&b.ts) == LLL_EINVAL, "delta gap"); }
    { Inputs b = a; b.vol[17] = INFINITY; b.sync(); expect(create(&b.ts) == LLL_EINVAL, "inf vol"); }
    { Inputs b = a; for (double &v : b.vol) v *= 20.0; b.sync();
      expect(create(&b.ts) == LLL_EMOMENT, "moment condition"); }
    { Inputs b = a; b.ts.alpha = 3.0; expect(create(&b.ts) == LLL_EINVAL, "alpha <= |beta|"); }
    { Inputs b = a; b.ts.delta_nig = 0.0; expect(create(&b.ts) == LLL_EINVAL, "NIG delta"); }
    { Inputs b = a; b.ts.driver = 7; expect(create(&b.ts) == LLL_EINVAL, "driver"); }
    { Inputs b = a; b.ts.driver = LLL_DRIVER_BROWNIAN; b.ts.c = -1.0; expect(create(&b.ts) == LLL_EINVAL, "c < 0"); }
    { Inputs b = a; b.ts.product = 2; expect(create(&b.ts) == LLL_EINVAL, "product"); }
    { Inputs b = a; b.ts.n_strikes = 9; expect(create(&b.ts) == LLL_EINVAL, "strikes"); }
    { Inputs b = a; b.ts.n_rates = 65; expect(create(&b.ts) == LLL_EINVAL, "N > 64"); }
    { Inputs b = a; b.ts.steps_per_period = 0; expect(create(&b.ts) == LLL_EINVAL, "s = 0"); }
    { Inputs b = a; b.ts.B0_T1 = 1.5; expect(create(&b.ts) == LLL_EINVAL, "B0_T1 > 1"); }
    expect(create(&a.ts, 5) == LLL_EINVAL, "precision");
    expect(create(&a.ts, LLL_FP32, 0) == LLL_EINVAL, "max_paths");
    { Inputs big(30, 2, 1); expect(create(&big.ts, LLL_FP64) == LLL_EUNSUPPORTED, "FP64 N > 24"); }
    // every entry point rejects a NULL handle
    expect(lll_plan_execute(nullptr, 0, 64, 0, 1, nullptr, nullptr) == LLL_EINVAL, "execute NULL");
    expect(lll_plan_results(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == LLL_EINVAL, "results NULL");
    expect(lll_plan_results_dev(nullptr, nullptr, nullptr, nullptr, nullptr) == LLL_EINVAL, "results_dev NULL");
    expect(lll_plan_set_inputs_dev(nullptr, nullptr, nullptr, nullptr) == LLL_EINVAL, "set_inputs NULL");
    expect(lll_plan_greeks(nullptr, 64, 1, nullptr) == LLL_EINVAL, "greeks NULL");
    double w[10] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 1};
    expect(lll_plan_greeks_vjp(nullptr, 64, 1, w, nullptr) == LLL_EINVAL, "vjp NULL");
    expect(lll_plan_greeks_vjp_dev(nullptr, 64, 1, w, nullptr) == LLL_EINVAL, "vjp_dev NULL");
    expect(lll_plan_attach_mlp(nullptr, nullptr) == LLL_EINVAL, "attach NULL");
    expect(lll_plan_destroy(nullptr) == LLL_OK, "destroy NULL");
    expect(lll_batch_destroy(nullptr) == LLL_OK, "batch destroy NULL");
    lll_batch *bt = nullptr;
    expect(lll_batch_create(&a.ts, 0, 64, &bt) == LLL_EINVAL && !bt, "batch of 0");
    expect(lll_batch_create(&a.ts, 1, 0, &bt) == LLL_EINVAL && !bt, "batch paths 0");
    { Inputs b = a; b.L0[0] = 0.0; b.sync();
      std::vector<lll_term_structure> two = {a.ts, b.ts};
      expect(lll_batch_create(two.data(), 2, 64, &bt) == LLL_EINVAL && !bt, "batch bad structure");
      expect(std::strstr(lll_last_error(), "structure 1") != nullptr, "batch names the structure"); }
    double price[30];
    expect(lll_price_caplets_batched(&a.ts, 1, 64, 0, 1, nullptr, nullptr, nullptr) == LLL_EINVAL, "batched NULL out");
    // the static workspace: size and scheme checks happen before any device call
    { Inputs big(40, 10, 3);
      expect(lll_price_caplets_static(&big.ts, (int64_t)1 << 21, LLL_FULL, 1, LLL_FP32, price, nullptr,
                                      nullptr, nullptr) == LLL_EINVAL, "static oversize");
      expect(std::strstr(lll_last_error(), "static workspace holds") != nullptr, "static message"); }
    expect(lll_price_caplets_static(&a.ts, 64, LLL_EXACT, 1, LLL_FP32, price, nullptr, nullptr,
                                    nullptr) == LLL_EUNSUPPORTED, "static scheme");
    expect(lll_price_caplets_static(&a.ts, 0, LLL_FULL, 1, LLL_FP32, price, nullptr, nullptr,
                                    nullptr) == LLL_EINVAL, "static paths");
    expect(std::strlen(lll_version()) > 0, "version");
    std::printf(failures ? "FAILED\n" : "ok\n");
    return failures ? 1 : 0;
}
