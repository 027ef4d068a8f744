/*
 * lll_oracle.c -- plain FP64 CPU oracle of the Lévy LIBOR Monte Carlo path.
 *
 * TEST INFRASTRUCTURE.  Only tests/, __graft_entry__.smoke() and the CPU
 * baseline leg of bench.py may load this library.  It shares no code with the
 * HIP implementation; both are fed the same inputs (tenor, forwards, vol
 * table, driver parameters, strikes, Philox seed) and the oracle receives the
 * 64-node quadrature rule (nodes and Lévy weights) computed by oracle/rule.py.
 *
 * What it computes, in the order of Papapantoleon & Skovmand, "Numerical
 * methods for the Lévy LIBOR model":
 *
 *   - log-LIBOR rates Z_i = log L(t, T_i) under the terminal measure
 *     (Section 2, eq. (log-LIB-SIE)), stepped with an Euler scheme on a grid
 *     of s equal steps per accrual period (Section 4 uses 5 steps per period);
 *     the state kept is X_i = Z_i - Z_i(0);
 *   - the drift of eq. (LIBOR-drift-PT):
 *       b_i = -c/2 lambda_i^2 - c lambda_i sum_{l>i} ell_l lambda_l
 *             - int [ (e^{lambda_i x} - 1) prod_{l>i} beta_l(x) - lambda_i x ] F(dx),
 *     ell_l = delta_l L_l / (1 + delta_l L_l), beta_l(x) = 1 + ell_l (e^{lambda_l x} - 1)
 *     (eq. (Levy-LIBOR-beta)).  For the pure-jump NIG driver (c = 0) this is
 *       b_i = -kappa(lambda_i) - sum_q W_q E_{i,q} ( prod_{l>i} beta_l(x_q) - 1 ),
 *     kappa in closed form, the product evaluated literally for every i;
 *   - three schemes (Section 3): FULL uses the drift at the current rates;
 *     PICARD uses the drift evaluated at the second Picard iterate Z^(1)
 *     (eq. (bdrift)), itself driven by the deterministic drift at Z(0)
 *     (eq. (Picard-2)); FROZEN is Z^(1) itself; and FIRST_ORDER /
 *     SECOND_ORDER, the drift at the current rates with the product replaced
 *     by its expansion to first / second order in ell (Section 3.2, eqs.
 *     (drifta), (drifta2) with the sign of the first-order bracket as in
 *     (drifta)), in closed form through kappa;
 *   - the caplet payoff under the terminal measure (Section 3.3, eq. (caplet)):
 *       delta_i B(0,T_*) E[ prod_{l>i} (1 + delta_l L(T_i,T_l)) (L(T_i,T_i) - K)^+ ];
 *     or, for co-terminal payer swaptions (a multi-rate product the paper
 *     names as covered by the framework), expiring at T_i on the swap over
 *     the periods i..N,
 *       B(0,T_*) E[ ( sum_{l>=i} delta_l (L(T_i,T_l) - K) prod_{j>l} (1 + delta_j L(T_i,T_j)) )^+ ],
 *     the value at T_i of the swap's payments B(T_i,T_{l+1}) / B(T_i,T_*) =
 *     prod_{j>l} (1 + delta_j L(T_i,T_j)) in units of the terminal bond;
 *     this file returns path sums; the Python wrapper forms prices.
 *
 * Random numbers: the paper draws NIG increments "by the standard method"
 * (an inverse-Gaussian subordinator and a normal mixture, Glasserman 2003).
 * Uniforms come from Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11):
 * one call per (step k, path p), counter (k, p_lo, p_hi, stream_word),
 * key (seed_lo, seed_hi).  Normals by Box-Muller; the inverse Gaussian by
 * Michael, Schucany & Haas (1976) in its textbook form.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no intrinsics).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_FULL 0
#define ORACLE_PICARD 1
#define ORACLE_FROZEN 2
#define ORACLE_FIRST_ORDER 3
#define ORACLE_SECOND_ORDER 4

#define ORACLE_NIG 0
#define ORACLE_BROWNIAN 1

#define ORACLE_CAPLETS 0
#define ORACLE_SWAPTIONS 1

typedef struct {
    int32_t n_rates;          /* N */
    int32_t steps_per_period; /* s */
    int32_t n_strikes;        /* S */
    int32_t driver;           /* ORACLE_NIG or ORACLE_BROWNIAN */
    int32_t n_nodes;          /* Q (0 for the Brownian driver) */
    uint32_t stream_word;     /* fourth Philox counter word */
    uint64_t seed;            /* Philox key */
    int32_t product;          /* ORACLE_CAPLETS or ORACLE_SWAPTIONS */
    int32_t pad;
    const double *tenor;      /* T_1..T_N */
    const double *delta;      /* delta_1..delta_N */
    const double *L0;         /* L(0, T_i) */
    const double *vol;        /* lambda(t_k, T_i), [N*s][N] */
    const double *strikes;    /* [N][S] */
    const double *x;          /* quadrature nodes [Q] */
    const double *w;          /* quadrature weights incl. Lévy density [Q] */
    double alpha, beta, delta_nig; /* NIG */
    double c;                 /* Brownian variance rate */
} oracle_model;

typedef struct {
    oracle_model m;
    int K;            /* number of Euler steps N*s */
    double *dt;       /* [K] */
    double *kappa;    /* [K][N]  kappa(lambda_{k,i}) */
    double *E;        /* [K][N][Q]  e^{lambda_{k,i} x_q} - 1 */
    double *b0;       /* [K][N]  drift at the initial rates (frozen drift) */
    double gamma, mu_H;
} oracle_ctx;

/* ---------------- Philox-4x32-10 (Salmon et al. 2011) ---------------- */

void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;   /* Weyl key schedule */
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 24-bit uniform on the open interval (0, 1): ((w >> 8) + 1/2) 2^-24. */
double oracle_uniform(uint32_t w)
{
    return ((double)(w >> 8) + 0.5) * (1.0 / 16777216.0);
}

static void step_words(const oracle_ctx *ctx, int k, int64_t p, uint32_t out[4])
{
    uint32_t ctr[4], key[2];
    ctr[0] = (uint32_t)k;
    ctr[1] = (uint32_t)((uint64_t)p & 0xFFFFFFFFu);
    ctr[2] = (uint32_t)((uint64_t)p >> 32);
    ctr[3] = ctx->m.stream_word;
    key[0] = (uint32_t)(ctx->m.seed & 0xFFFFFFFFu);
    key[1] = (uint32_t)(ctx->m.seed >> 32);
    oracle_philox4x32_10(ctr, key, out);
}

/* ---------------- driver: cumulant and increments ---------------- */

/* kappa(u) = log E[e^{u H_1}] of the compensated driver (eq. (cumulant)).
 * NIG(alpha, beta, delta, mu_H) with mu_H = -delta beta / gamma so that H is
 * a martingale: kappa(u) = mu_H u + delta (gamma - sqrt(alpha^2 - (beta+u)^2)),
 * which at beta = 0 is the paper's delta alpha - delta sqrt(alpha^2 - u^2).
 * Brownian: kappa(u) = c u^2 / 2. */
static double cumulant(const oracle_ctx *ctx, double u)
{
    const oracle_model *m = &ctx->m;
    if (m->driver == ORACLE_BROWNIAN)
        return 0.5 * m->c * u * u;
    double bu = m->beta + u;
    return ctx->mu_H * u + m->delta_nig * (ctx->gamma - sqrt(m->alpha * m->alpha - bu * bu));
}

/* One driver increment Delta H over step k of path p.  Returns also the
 * subordinator draw V (0 for the Brownian driver) and the Philox words. */
void oracle_increment(const oracle_ctx *ctx, int k, int64_t p, double *V_out,
                      double *dH_out, uint32_t words_out[4])
{
    const oracle_model *m = &ctx->m;
    uint32_t w[4];
    step_words(ctx, k, p, w);
    if (words_out) memcpy(words_out, w, sizeof w);
    double u0 = oracle_uniform(w[0]);
    double u1 = oracle_uniform(w[1]);
    double u2 = oracle_uniform(w[2]);
    /* Box-Muller */
    double r = sqrt(-2.0 * log(u0));
    double z1 = r * cos(2.0 * M_PI * u1);
    double z2 = r * sin(2.0 * M_PI * u1);
    double dt = ctx->dt[k];
    if (m->driver == ORACLE_BROWNIAN) {
        if (V_out) *V_out = 0.0;
        *dH_out = sqrt(m->c * dt) * z1;
        return;
    }
    /* Inverse Gaussian IG(mean mu, shape lam) with mu = delta dt / gamma,
     * lam = (delta dt)^2 (Michael-Schucany-Haas). */
    double mu = m->delta_nig * dt / ctx->gamma;
    double lam = (m->delta_nig * dt) * (m->delta_nig * dt);
    double y = z1 * z1;
    double x = mu + mu * mu * y / (2.0 * lam)
             - mu / (2.0 * lam) * sqrt(4.0 * mu * lam * y + mu * mu * y * y);
    double V = (u2 <= mu / (mu + x)) ? x : mu * mu / x;
    if (V_out) *V_out = V;
    /* normal variance-mean mixture: NIG(alpha, beta, delta dt, mu_H dt) */
    *dH_out = ctx->mu_H * dt + m->beta * V + sqrt(V) * z2;
}

/* Increments of step k for paths p0 .. p0+n-1 (V may be NULL). */
void oracle_increments(const oracle_ctx *ctx, int k, int64_t p0, int64_t n, double *V, double *dH)
{
    for (int64_t j = 0; j < n; ++j)
        oracle_increment(ctx, k, p0 + j, V ? V + j : NULL, dH + j, NULL);
}

/* ---------------- drift (eq. (LIBOR-drift-PT)) ---------------- */

/* Drift b(t_k, T_i) of every rate i >= first, given the rates L[0..N-1]
 * (only the live ones are read).  b[i] for i < first is left untouched. */
void oracle_drift(const oracle_ctx *ctx, int k, int first, const double *L, double *b)
{
    const oracle_model *m = &ctx->m;
    const int N = m->n_rates, Q = m->n_nodes;
    const double *lam = m->vol + (size_t)k * N;
    double ell[64];
    for (int l = first; l < N; ++l)
        ell[l] = m->delta[l] * L[l] / (1.0 + m->delta[l] * L[l]);
    for (int i = first; i < N; ++i) {
        if (m->driver == ORACLE_BROWNIAN) {
            double s = 0.0;
            for (int l = i + 1; l < N; ++l)
                s += ell[l] * lam[l];
            b[i] = -0.5 * lam[i] * lam[i] * m->c - m->c * lam[i] * s;
            continue;
        }
        double coupling = 0.0;
        for (int q = 0; q < Q; ++q) {
            double prod = 1.0;
            for (int l = i + 1; l < N; ++l)
                prod *= 1.0 + ell[l] * ctx->E[((size_t)k * N + l) * Q + q];
            coupling += m->w[q] * ctx->E[((size_t)k * N + i) * Q + q] * (prod - 1.0);
        }
        b[i] = -ctx->kappa[(size_t)k * N + i] - coupling;
    }
}

/* First-order drift expansion (Section 3.2, eq. (drifta)): the product over
 * l > i truncated after its terms linear in ell, each integral in closed form,
 *   b_i = -kappa(lambda_i)
 *         - sum_{l>i} ell_l (kappa(lambda_i + lambda_l) - kappa(lambda_i) - kappa(lambda_l)).
 * For the Brownian driver the coupling is linear in ell, so this equals the
 * exact drift. */
void oracle_drift_first_order(const oracle_ctx *ctx, int k, int first, const double *L, double *b)
{
    const oracle_model *m = &ctx->m;
    const int N = m->n_rates;
    const double *lam = m->vol + (size_t)k * N;
    double ell[64];
    for (int l = first; l < N; ++l)
        ell[l] = m->delta[l] * L[l] / (1.0 + m->delta[l] * L[l]);
    for (int i = first; i < N; ++i) {
        const double ki = cumulant(ctx, lam[i]);
        double coupling = 0.0;
        for (int l = i + 1; l < N; ++l)
            coupling += ell[l] * (cumulant(ctx, lam[i] + lam[l]) - ki - cumulant(ctx, lam[l]));
        b[i] = -ki - coupling;
    }
}

/* Second-order drift expansion (Section 3.2, eq. (drifta2), its first-order
 * bracket read with the signs of eq. (drifta)): the first-order drift plus
 *   - sum_{i<k<l} ell_k ell_l ( kappa(lambda_i + lambda_k + lambda_l)
 *       - kappa(lambda_i + lambda_k) - kappa(lambda_i + lambda_l) - kappa(lambda_k + lambda_l)
 *       + kappa(lambda_i) + kappa(lambda_k) + kappa(lambda_l) ). */
void oracle_drift_second_order(const oracle_ctx *ctx, int k, int first, const double *L, double *b)
{
    const oracle_model *m = &ctx->m;
    const int N = m->n_rates;
    const double *lam = m->vol + (size_t)k * N;
    double ell[64];
    for (int l = first; l < N; ++l)
        ell[l] = m->delta[l] * L[l] / (1.0 + m->delta[l] * L[l]);
    oracle_drift_first_order(ctx, k, first, L, b);
    for (int i = first; i < N; ++i) {
        const double li = lam[i];
        double second = 0.0;
        for (int kk = i + 1; kk < N; ++kk)
            for (int l = kk + 1; l < N; ++l) {
                const double lk = lam[kk], ll = lam[l];
                const double bracket = cumulant(ctx, li + lk + ll) - cumulant(ctx, li + lk)
                                       - cumulant(ctx, li + ll) - cumulant(ctx, lk + ll)
                                       + cumulant(ctx, li) + cumulant(ctx, lk) + cumulant(ctx, ll);
                second += ell[kk] * ell[l] * bracket;
            }
        b[i] -= second;
    }
}

/* ---------------- set-up ---------------- */

oracle_ctx *oracle_create(const oracle_model *model)
{
    oracle_ctx *ctx = (oracle_ctx *)calloc(1, sizeof *ctx);
    if (!ctx) return NULL;
    ctx->m = *model;
    const int N = model->n_rates, s = model->steps_per_period, Q = model->n_nodes;
    const int K = N * s;
    ctx->K = K;
    if (model->driver == ORACLE_NIG) {
        ctx->gamma = sqrt(model->alpha * model->alpha - model->beta * model->beta);
        ctx->mu_H = -model->delta_nig * model->beta / ctx->gamma;
    }
    ctx->dt = (double *)malloc(sizeof(double) * K);
    ctx->kappa = (double *)calloc((size_t)K * N, sizeof(double));
    ctx->E = (double *)calloc((size_t)K * N * (Q > 0 ? Q : 1), sizeof(double));
    ctx->b0 = (double *)calloc((size_t)K * N, sizeof(double));
    if (!ctx->dt || !ctx->kappa || !ctx->E || !ctx->b0) {
        free(ctx->dt); free(ctx->kappa); free(ctx->E); free(ctx->b0); free(ctx);
        return NULL;
    }
    for (int mth = 0; mth < N; ++mth) {
        double Ta = (mth == 0) ? 0.0 : model->tenor[mth - 1];
        double Tb = model->tenor[mth];
        for (int j = 0; j < s; ++j)
            ctx->dt[mth * s + j] = (Tb - Ta) / s;
    }
    for (int k = 0; k < K; ++k) {
        int first = k / s;
        for (int i = first; i < N; ++i) {
            double lam = model->vol[(size_t)k * N + i];
            ctx->kappa[(size_t)k * N + i] = cumulant(ctx, lam);
            for (int q = 0; q < Q; ++q)
                ctx->E[((size_t)k * N + i) * Q + q] = expm1(lam * model->x[q]);
        }
    }
    /* Frozen drift: the drift evaluated at the initial rates Z(0) (eq. (Picard-2)). */
    for (int k = 0; k < K; ++k)
        oracle_drift(ctx, k, k / s, model->L0, ctx->b0 + (size_t)k * N);
    return ctx;
}

void oracle_destroy(oracle_ctx *ctx)
{
    if (!ctx) return;
    free(ctx->dt); free(ctx->kappa); free(ctx->E); free(ctx->b0);
    free(ctx);
}

const double *oracle_kappa_table(const oracle_ctx *ctx) { return ctx->kappa; }
const double *oracle_E_table(const oracle_ctx *ctx) { return ctx->E; }
const double *oracle_b0_table(const oracle_ctx *ctx) { return ctx->b0; }
const double *oracle_dt_table(const oracle_ctx *ctx) { return ctx->dt; }

/* ---------------- one path ---------------- */

/* Simulates path p.  For every caplet i (fixing at T_i) writes the fixed rate
 * Lfix[i] = L(T_i, T_i) and the terminal-measure factor
 * Dfix[i] = prod_{l>i} (1 + delta_l L(T_i, T_l)) of the scheme's rates; if
 * Sfix / Afix are not NULL, also the floating and fixed legs of the
 * co-terminal swap at T_i in units of B(T_i, T_*), term by term:
 *   Sfix[i] = sum_{l>=i} delta_l L(T_i,T_l) prod_{j>l} (1 + delta_j L(T_i,T_j)),
 *   Afix[i] = sum_{l>=i} delta_l prod_{j>l} (1 + delta_j L(T_i,T_j)). */
static void simulate_path(const oracle_ctx *ctx, int scheme, int64_t p, double *Lfix, double *Dfix,
                          double *Sfix, double *Afix)
{
    const oracle_model *m = &ctx->m;
    const int N = m->n_rates, s = m->steps_per_period;
    double X[64], X1[64], L[64], b[64];
    for (int i = 0; i < N; ++i) { X[i] = 0.0; X1[i] = 0.0; }
    for (int mth = 0; mth < N; ++mth) {          /* period [T_mth, T_mth+1] */
        for (int j = 0; j < s; ++j) {
            const int k = mth * s + j;
            const double *lam = m->vol + (size_t)k * N;
            const double dt = ctx->dt[k];
            double V, dH;
            oracle_increment(ctx, k, p, &V, &dH, NULL);
            if (scheme == ORACLE_FULL) {
                for (int i = mth; i < N; ++i) L[i] = m->L0[i] * exp(X[i]);
                oracle_drift(ctx, k, mth, L, b);
            } else if (scheme == ORACLE_FIRST_ORDER) {
                for (int i = mth; i < N; ++i) L[i] = m->L0[i] * exp(X[i]);
                oracle_drift_first_order(ctx, k, mth, L, b);
            } else if (scheme == ORACLE_SECOND_ORDER) {
                for (int i = mth; i < N; ++i) L[i] = m->L0[i] * exp(X[i]);
                oracle_drift_second_order(ctx, k, mth, L, b);
            } else if (scheme == ORACLE_PICARD) {
                for (int i = mth; i < N; ++i) L[i] = m->L0[i] * exp(X1[i]);
                oracle_drift(ctx, k, mth, L, b);
            } else {
                for (int i = mth; i < N; ++i) b[i] = ctx->b0[(size_t)k * N + i];
            }
            for (int i = mth; i < N; ++i)
                X[i] += b[i] * dt + lam[i] * dH;
            if (scheme == ORACLE_PICARD)
                for (int i = mth; i < N; ++i)
                    X1[i] += ctx->b0[(size_t)k * N + i] * dt + lam[i] * dH;
        }
        /* t = T_{mth+1}: the rate with maturity T_{mth+1} fixes. */
        const int c = mth;
        double Lc = m->L0[c] * exp(X[c]);
        double D = 1.0;
        for (int l = c + 1; l < N; ++l)
            D *= 1.0 + m->delta[l] * m->L0[l] * exp(X[l]);
        Lfix[c] = Lc;
        Dfix[c] = D;
        if (Sfix && Afix) {
            double fl = 0.0, fx = 0.0;
            for (int l = c; l < N; ++l) {
                double Q = 1.0;
                for (int j = l + 1; j < N; ++j) Q *= 1.0 + m->delta[j] * m->L0[j] * exp(X[j]);
                fl += m->delta[l] * m->L0[l] * exp(X[l]) * Q;
                fx += m->delta[l] * Q;
            }
            Sfix[c] = fl;
            Afix[c] = fx;
        }
    }
}

int oracle_paths(const oracle_ctx *ctx, int scheme, const int64_t *paths, int64_t n,
                 double *Lfix, double *Dfix)
{
    const int N = ctx->m.n_rates;
    for (int64_t j = 0; j < n; ++j)
        simulate_path(ctx, scheme, paths[j], Lfix + j * N, Dfix + j * N, NULL, NULL);
    return 0;
}

/* Path sums for paths p0 .. p0+n-1 with `threads` OpenMP threads (<= 0: all).
 * sum_p, sum_p2, n_itm: [N][S]; sum_mart, sum_mart2: [N] of the factor
 * prod_{l>=i}(1 + delta_l L(T_i, T_l)) and its square. */
int oracle_price_sums(const oracle_ctx *ctx, int scheme, int64_t p0, int64_t n, int threads,
                      double *sum_p, double *sum_p2, double *n_itm, double *sum_mart,
                      double *sum_mart2)
{
    const int N = ctx->m.n_rates, S = ctx->m.n_strikes;
    const size_t NS = (size_t)N * S;
    int nt = 1;
#ifdef _OPENMP
    nt = threads > 0 ? threads : omp_get_max_threads();
#endif
    double *acc = (double *)calloc((size_t)nt * (3 * NS + 2 * N), sizeof(double));
    if (!acc) return -1;
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *a = acc + (size_t)tid * (3 * NS + 2 * N);
        double Lfix[64], Dfix[64], Sfix[64], Afix[64];
        const int swaptions = ctx->m.product == ORACLE_SWAPTIONS;
        /* contiguous static chunk per thread: fixed summation order */
        int64_t lo = p0 + n * tid / nt, hi = p0 + n * (tid + 1) / nt;
        for (int64_t p = lo; p < hi; ++p) {
            simulate_path(ctx, scheme, p, Lfix, Dfix, swaptions ? Sfix : NULL,
                          swaptions ? Afix : NULL);
            for (int c = 0; c < N; ++c) {
                for (int r = 0; r < S; ++r) {
                    double K = ctx->m.strikes[(size_t)c * S + r];
                    double v = swaptions ? Sfix[c] - K * Afix[c] : Dfix[c] * (Lfix[c] - K);
                    double pay = v > 0.0 ? v : 0.0;
                    a[(size_t)c * S + r] += pay;
                    a[NS + (size_t)c * S + r] += pay * pay;
                    a[2 * NS + (size_t)c * S + r] += (v > 0.0) ? 1.0 : 0.0;
                }
                double mart = Dfix[c] * (1.0 + ctx->m.delta[c] * Lfix[c]);
                a[3 * NS + c] += mart;
                a[3 * NS + N + c] += mart * mart;
            }
        }
    }
    memset(sum_p, 0, NS * sizeof(double));
    memset(sum_p2, 0, NS * sizeof(double));
    memset(n_itm, 0, NS * sizeof(double));
    memset(sum_mart, 0, N * sizeof(double));
    memset(sum_mart2, 0, N * sizeof(double));
    for (int t = 0; t < nt; ++t) {
        const double *a = acc + (size_t)t * (3 * NS + 2 * N);
        for (size_t j = 0; j < NS; ++j) {
            sum_p[j] += a[j];
            sum_p2[j] += a[NS + j];
            n_itm[j] += a[2 * NS + j];
        }
        for (int c = 0; c < N; ++c) {
            sum_mart[c] += a[3 * NS + c];
            sum_mart2[c] += a[3 * NS + N + c];
        }
    }
    free(acc);
    return nt;
}
