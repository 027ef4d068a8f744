/* Runs every entry point of the C oracle on small term structures, built into
 * one translation unit with the oracle so that AddressSanitizer and
 * UndefinedBehaviorSanitizer see all of it (tests/test_oracle_sanitizers.py).
 * Shapes: N = 1, 5 and 64 (the oracle's largest), both drivers, caplets and
 * co-terminal swaptions, 1 and 3 OpenMP threads.  The quadrature rule here is a
 * plain symmetric one: the run checks memory and arithmetic safety, not values
 * (those are pinned elsewhere).  Prints "ok" and exits 0 when every call
 * returned normally and every output is finite. */
#include "../../oracle/lll_oracle.c"

#include <stdio.h>

static int all_finite(const double *a, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

static int run_case(int N, int s, int S, int driver, int product, int threads)
{
    const int K = N * s, Q = driver == ORACLE_NIG ? 64 : 0;
    double *tenor = malloc(sizeof(double) * N), *delta = malloc(sizeof(double) * N);
    double *L0 = malloc(sizeof(double) * N), *vol = calloc((size_t)K * N, sizeof(double));
    double *strikes = malloc(sizeof(double) * N * S), x[64], w[64];
    for (int i = 0; i < N; ++i) {
        tenor[i] = 0.25 * (i + 1);
        delta[i] = 0.25;
        L0[i] = 0.03 + 0.0005 * i;
        for (int j = 0; j < S; ++j) strikes[i * S + j] = L0[i] * (0.9 + 0.1 * j);
    }
    for (int k = 0; k < K; ++k)
        for (int i = k / s; i < N; ++i) vol[(size_t)k * N + i] = 0.05 + 0.001 * i;
    for (int q = 0; q < 32; ++q) {
        x[q] = 0.05 * (q + 1);
        x[32 + q] = -0.05 * (q + 1);
        w[q] = w[32 + q] = 1e-3 / (q + 1);
    }
    oracle_model m = {0};
    m.n_rates = N; m.steps_per_period = s; m.n_strikes = S; m.driver = driver; m.n_nodes = Q;
    m.stream_word = 7; m.seed = 0x123456789ull; m.product = product;
    m.tenor = tenor; m.delta = delta; m.L0 = L0; m.vol = vol; m.strikes = strikes;
    m.x = x; m.w = w; m.alpha = 18.0; m.beta = -4.0; m.delta_nig = 1.0; m.c = 0.04;
    oracle_ctx *ctx = oracle_create(&m);
    if (!ctx) return 1;
    int ok = all_finite(oracle_kappa_table(ctx), (size_t)K * N) &&
             all_finite(oracle_b0_table(ctx), (size_t)K * N) &&
             all_finite(oracle_dt_table(ctx), (size_t)K) &&
             all_finite(oracle_E_table(ctx), (size_t)K * N * (Q > 0 ? Q : 1));
    double V[5], dH[5], b[64], L[64];
    uint32_t words[4];
    oracle_increment(ctx, K - 1, 5, V, dH, words);
    oracle_increments(ctx, 0, (int64_t)1 << 33, 5, V, dH);
    ok = ok && all_finite(V, 5) && all_finite(dH, 5);
    for (int i = 0; i < N; ++i) L[i] = L0[i] * 1.1;
    for (int k = 0; k < K; k += (K > 8 ? K / 8 : 1)) {
        oracle_drift(ctx, k, k / s, L, b);
        ok = ok && all_finite(b + k / s, N - k / s);
        oracle_drift_first_order(ctx, k, k / s, L, b);
        ok = ok && all_finite(b + k / s, N - k / s);
        oracle_drift_second_order(ctx, k, k / s, L, b);
        ok = ok && all_finite(b + k / s, N - k / s);
    }
    const int64_t paths[3] = {0, 17, ((int64_t)1 << 32) + 3};
    double *Lf = malloc(sizeof(double) * 3 * N), *Df = malloc(sizeof(double) * 3 * N);
    double *sp = malloc(sizeof(double) * N * S), *sp2 = malloc(sizeof(double) * N * S);
    double *itm = malloc(sizeof(double) * N * S), *mt = malloc(sizeof(double) * N);
    double *mt2 = malloc(sizeof(double) * N);
    for (int scheme = 0; scheme <= ORACLE_SECOND_ORDER; ++scheme) {
        oracle_paths(ctx, scheme, paths, 3, Lf, Df);
        ok = ok && all_finite(Lf, 3 * (size_t)N) && all_finite(Df, 3 * (size_t)N);
        ok = ok && oracle_price_sums(ctx, scheme, 11, 7, threads, sp, sp2, itm, mt, mt2) >= 0;
        ok = ok && all_finite(sp, (size_t)N * S) && all_finite(mt2, N);
    }
    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6};
    oracle_philox4x32_10(ctr, key, words);
    ok = ok && oracle_uniform(words[0]) > 0.0 && oracle_uniform(0xFFFFFFFFu) < 1.0;
    oracle_destroy(ctx);
    free(tenor); free(delta); free(L0); free(vol); free(strikes);
    free(Lf); free(Df); free(sp); free(sp2); free(itm); free(mt); free(mt2);
    return ok ? 0 : 1;
}

int main(void)
{
    int rc = 0;
    rc |= run_case(1, 3, 1, ORACLE_NIG, ORACLE_CAPLETS, 1);
    rc |= run_case(5, 3, 2, ORACLE_NIG, ORACLE_CAPLETS, 3);
    rc |= run_case(5, 3, 2, ORACLE_NIG, ORACLE_SWAPTIONS, 3);
    rc |= run_case(5, 2, 3, ORACLE_BROWNIAN, ORACLE_CAPLETS, 1);
    rc |= run_case(5, 2, 3, ORACLE_BROWNIAN, ORACLE_SWAPTIONS, 3);
    rc |= run_case(64, 1, 1, ORACLE_NIG, ORACLE_SWAPTIONS, 3);
    printf(rc ? "FAILED\n" : "ok\n");
    return rc;
}
