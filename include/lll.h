/*
 * lll.h -- C ABI of the MI355X Monte Carlo engine for the Lévy LIBOR model
 * (Papapantoleon & Skovmand, "Numerical methods for the Lévy LIBOR model").
 *
 * One call prices caplets (paper Section 3.3, eq. (caplet)) by simulating
 * log-LIBOR rates under the terminal measure P_{T_*} (Section 2, eqs.
 * (LIBOR-dyn-PT), (LIBOR-drift-PT), (log-LIB-SIE)) with an Euler scheme and
 * one of five drift treatments (Section 3), PICARD also in a second layout:
 *
 *   LLL_FULL    the drift of eq. (LIBOR-drift-PT) at the current rates;
 *   LLL_PICARD  the drift of eq. (bdrift), evaluated at the second Picard
 *               iterate Z^(1) of eq. (Picard-2);
 *   LLL_FROZEN  Z^(1) itself (the drift frozen at the initial rates);
 *   LLL_FIRST_ORDER  the drift at the current rates with the product of eq.
 *               (LIBOR-drift-PT) expanded to first order in ell (Section 3.2,
 *               eq. (drifta)), in closed form through the cumulant (no
 *               quadrature); error O(|L|^2);
 *   LLL_SECOND_ORDER the same expansion to second order (eq. (drifta2), its
 *               first-order bracket with the signs of eq. (drifta)); the
 *               truncated product is integrated with the 64-node rule;
 *               error O(|L|^3);
 *   LLL_PICARD_MP    LLL_PICARD computed in a maturity-parallel layout: under
 *               the Picard approximation the drift of every step depends on
 *               the predictor path only (Section 3), so the drift integrals
 *               of all accrual periods are computed at once, spread over
 *               (group of 4 paths, period, quadrature node) instead of one
 *               path per lane.  The same estimator as LLL_PICARD (equal up to
 *               FP32 summation order) for runs with few paths and many rates;
 *               FP32 plans, NIG driver, N up to LLL_N_MAX_MP;
 *   LLL_EXACT   the LLL_FULL estimator with the drift taken from the exact
 *               expansion of the product over the subsets U of the later
 *               rates (Section 3.2, eq. (product)): coupling of rate i =
 *               sum_U prod_{l in U} ell_l prod_{l>i, l not in U}(1 - ell_l)
 *               [kappa(lambda_i + lambda_U) - kappa(lambda_U) - kappa(lambda_i)],
 *               closed-form cumulants and no quadrature (the paper's full
 *               solution); 2^(N-1-i) terms for rate i, so N up to
 *               LLL_N_MAX_EXACT; both precisions and drivers.  Its cumulant
 *               table (about s 2^(N+1) entries in the plan precision: 170 MB
 *               in FP32 at N = 20, s = 20) and the paths' states between
 *               periods (N max_paths values) are allocated on the first
 *               LLL_EXACT execute and kept by the plan.
 *
 * driven by a normal inverse Gaussian Lévy process (Section 4) or, as a
 * special case, by a Brownian motion.  The jump integral of the drift is the
 * closed-form cumulant plus a 64-node quadrature of the coupling term.
 *
 * Conventions
 *   - Rates are 0-indexed: entry r is the paper's rate i = r + 1 with
 *     maturity T_i; tenor[r] = T_{r+1}; delta[r] = T_{r+2} - T_{r+1}, with
 *     T_* = tenor[N-1] + delta[N-1].
 *   - The Euler grid has steps_per_period equal steps in every accrual period
 *     [T_m, T_{m+1}] (T_0 = 0); step k lies in period m = k / steps_per_period.
 *   - vol is lambda(t_k, T_{r+1}) at the left point of step k, row-major
 *     [N * steps_per_period][N]; entries of rates already fixed are ignored.
 *   - strikes are absolute, row-major [N][n_strikes].
 *   - Random numbers: one Philox-4x32-10 call per (step k, path p) with
 *     counter (k, p mod 2^32, p div 2^32, struct_id | tag << 24) and key
 *     (seed mod 2^32, seed div 2^32); tag 0 is used for pricing.
 *   - All pointers named *_host are caller-owned host memory, read or written
 *     during the call only; pointers named *_dev are device memory of the
 *     current HIP device.  `stream` is a hipStream_t (NULL = default stream).
 *
 * Errors: every function returns LLL_OK (0) or a negative lll_status and
 * never throws or aborts; lll_last_error() gives a thread-local message for
 * the last failing call on the calling thread.  Validation of the inputs
 * happens on the host before any device work.
 */
#ifndef LLL_H
#define LLL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LLL_N_MAX 40        /* largest N of the path-per-lane kernels (all schemes but
                               LLL_PICARD_MP), of batches, Greeks and the surrogate */
#define LLL_N_MAX_MP 64     /* largest N of a plan (N > LLL_N_MAX: LLL_PICARD_MP only) */
#define LLL_N_MAX_FP64 24   /* largest N for the FP64 path kernel */
#define LLL_N_MAX_EXACT 20  /* largest N of LLL_EXACT (2^(N-m) - 1 drift terms per step) */
#define LLL_S_MAX 8         /* largest number of strikes per caplet */
#define LLL_Q 64            /* quadrature nodes of the coupling integral */
#define LLL_NSTAT(S) (3 * (S) + 2) /* path statistics per caplet */

typedef enum {
    LLL_OK = 0,
    LLL_EINVAL = -1,       /* malformed input: sizes, ordering, signs, NaN */
    LLL_EMOMENT = -2,      /* exponential-moment condition fails: drift integral diverges */
    LLL_ENOMEM = -3,       /* device allocation failed */
    LLL_EHIP = -4,         /* a HIP runtime call failed (message has the HIP error) */
    LLL_EUNSUPPORTED = -5, /* valid input outside what this library implements */
    LLL_ENUMERIC = -6      /* non-finite payoffs were produced */
} lll_status;

/* Products priced at every fixing date T_i (rate r = i - 1 fixes at tenor[r]),
 * strikes[r][j] absolute:
 *   LLL_CAPLETS    delta_r B(0,T_*) E[ prod_{l>r}(1 + delta_l L_l(T_i)) (L_r(T_i) - K)^+ ]
 *                  (Section 3.3, eq. (caplet));
 *   LLL_SWAPTIONS  co-terminal payer swaptions: expiry T_i, underlying swap over
 *                  the accrual periods r..N-1 (to T_*), paid in units of the
 *                  terminal bond:
 *                  B(0,T_*) E[ ( sum_{l>=r} delta_l (L_l(T_i) - K) prod_{j>l}(1 + delta_j L_j(T_i)) )^+ ].
 * Results have the same [N][S] layout; n_itm counts positive payoffs. */
typedef enum { LLL_CAPLETS = 0, LLL_SWAPTIONS = 1 } lll_product;

typedef enum {
    LLL_FULL = 0,
    LLL_PICARD = 1,
    LLL_FROZEN = 2,
    LLL_FIRST_ORDER = 3,
    LLL_SECOND_ORDER = 4,
    LLL_PICARD_MP = 5,
    LLL_EXACT = 6,
    LLL_MLP_DRIFT = 7   /* FULL with the learned drift of an attached network (lll_plan_attach_mlp) */
} lll_scheme;
typedef enum { LLL_DRIVER_NIG = 0, LLL_DRIVER_BROWNIAN = 1 } lll_driver;
typedef enum { LLL_FP32 = 0, LLL_FP64 = 1 } lll_precision;

/* One term structure, its driver and its caplet strikes (host memory).
 * Paper Section 2: tenor 0 = T_0 < T_1 < ... < T_N < T_* (delta_i = T_{i+1} - T_i),
 * L(0, T_i) > 0 (assumption (LR2)), bounded deterministic vols lambda(., T_i)
 * (assumption (LR1)).  NIG driver: alpha > |beta|, delta_nig > 0, its drift
 * chosen so that H is a martingale; Brownian driver: c >= 0. */
typedef struct {
    int32_t n_rates;            /* N, 1..LLL_N_MAX_MP (see LLL_N_MAX) */
    int32_t steps_per_period;   /* s >= 1 */
    int32_t n_strikes;          /* S, 1..LLL_S_MAX */
    int32_t driver;             /* lll_driver */
    uint32_t struct_id;         /* fourth Philox counter word (low 24 bits) */
    int32_t product;            /* lll_product: what the strikes price */
    const double *tenor;        /* [N] T_1..T_N, strictly increasing, > 0 */
    const double *delta;        /* [N] accrual fractions, > 0, matching tenor gaps */
    const double *L0;           /* [N] L(0, T_i) > 0 */
    double B0_T1;               /* B(0, T_1); <= 0 means 1 / (1 + T_1 L(0, T_1)) */
    const double *vol;          /* [N*s][N] lambda(t_k, T_i) */
    const double *strikes;      /* [N][S] */
    double alpha, beta, delta_nig; /* NIG parameters */
    double c;                   /* Brownian variance rate */
} lll_term_structure;

/* Opaque plan: validated inputs copied to the device, precompute tables and
 * reduction buffers for up to max_paths paths.  Owned by the library. */
typedef struct lll_plan lll_plan;
typedef struct lll_mlp lll_mlp;  /* the drift surrogate (see below) */

const char *lll_version(void);
const char *lll_last_error(void);

/* Validate `ts` (host) and allocate a plan on the current device for at most
 * `max_paths` paths per execute call, computing in `precision` (lll_precision:
 * FP32 path arithmetic with FP64 increments and sums, or FP64 throughout).
 * The inputs are copied; `ts` may be freed after return.  Synchronous. */
int lll_plan_create(const lll_term_structure *ts, int precision, int64_t max_paths,
                    lll_plan **plan_out);

/* Enqueue one pricing pass on `stream` with `scheme` (lll_scheme; LLL_EINVAL
 * otherwise): FP64 precompute of the quadrature rule and of the cumulant,
 * quadrature and frozen-drift tables (LLL_FIRST_ORDER: also the per-step
 * coefficients kappa(lambda_i + lambda_l) - kappa(lambda_i) - kappa(lambda_l),
 * allocated on its first use, LLL_ENOMEM if that fails); the path kernel over
 * paths path_offset .. path_offset + n_paths - 1; the deterministic FP64
 * reduction of the payoff sums.  Asynchronous: results are read with
 * lll_plan_results.  LLL_PICARD_MP replaces the path kernel by three kernels
 * (predictor and increments, per-period drift integrals, payoffs) over chunks
 * of paths whose buffers (ell at the predictor for every step, rate and path:
 * 4 K N bytes per path, plus 4 N^2) stay within 2 GiB; they are allocated on
 * its first use (LLL_ENOMEM if that fails); LLL_EUNSUPPORTED on FP64 plans or
 * the Brownian driver.  Plans with N > LLL_N_MAX run only LLL_PICARD_MP
 * (LLL_EUNSUPPORTED for the other schemes).  If path_fix_dev is not NULL it receives, for every path
 * j of this call and caplet r, L(T_r, T_r) at [j][2r] and the terminal-measure
 * factor prod_{l>r}(1 + delta_l L(T_r, T_l)) at [j][2r+1] (FP64, n_paths x 2N). */
int lll_plan_execute(lll_plan *plan, int scheme, int64_t n_paths, int64_t path_offset,
                     uint64_t seed, double *path_fix_dev, void *stream);

/* Wait for `stream` and copy the results of the last execute to the host.
 * price_host, stderr_host, n_itm_host: [N][S]; mart_resid_host, mart_se_host: [N]
 * (mean of prod_{l>=i}(1 + delta_l L(T_i, T_l)) minus its time-0 value, and its
 * standard error).  Any output pointer may be NULL.  Returns LLL_ENUMERIC if a
 * price or standard error is not finite. */
int lll_plan_results(lll_plan *plan, double *price_host, double *stderr_host,
                     double *mart_resid_host, double *mart_se_host, double *n_itm_host,
                     void *stream);

/* ---- device-resident inputs and outputs (asynchronous on `stream`) ---- */

/* Replace the plan's initial forwards L(0, T_i) by L0_dev[N] (device FP64, or
 * NULL to keep them) and shift each rate's vol curve in parallel by
 * vol_shift_dev[N] (device FP64, or NULL): lambda(t_k, T_i) = the table the
 * plan was created with + vol_shift_dev[i] (the "vol level" of rate i, paper
 * Section 2's deterministic volatility lambda(., T_i)).  B(0, T_1), the
 * strikes and the tenor stay as created.  Enqueued on `stream` (no host
 * synchronisation): the inputs are read when the stream reaches the call and
 * apply to every later execute or Greeks pass on the plan.  The host cannot
 * check device values: the next pass checks them (positive finite forwards,
 * finite vols and the moment condition of (LR1)) and, if they fail, its
 * prices and Greeks are NaN and the host result calls return LLL_EINVAL or
 * LLL_EMOMENT.  The first call with a shift copies the creation table to the
 * device (allocation, synchronous). */
int lll_plan_set_inputs_dev(lll_plan *plan, const double *L0_dev, const double *vol_shift_dev,
                            void *stream);

/* Copy the last execute's results into device buffers on `stream`
 * (asynchronous): price_dev, stderr_dev [N][S], mart_resid_dev [N] (FP64; any
 * may be NULL).  Non-finite values are not reported here (NaN prices mark
 * invalid device inputs, see lll_plan_set_inputs_dev). */
int lll_plan_results_dev(lll_plan *plan, double *price_dev, double *stderr_dev,
                         double *mart_resid_dev, void *stream);

/* Attach the surrogate network that scheme LLL_MLP_DRIFT of lll_plan_execute
 * uses (NULL detaches); the network must outlive its use by the plan.
 * LLL_MLP_DRIFT is lll_plan_execute_mlp with use_net = 1 and no judge, from
 * path 0 (LLL_EUNSUPPORTED for path_offset != 0; LLL_EINVAL with no network).
 * The one-shot calls have no network and reject the scheme. */
int lll_plan_attach_mlp(lll_plan *plan, const lll_mlp *mlp);

/* Raw per-caplet sums of the last execute, [N][LLL_NSTAT(S)] doubles:
 * sum p_j (S), sum p_j^2 (S), in-the-money counts (S), sum M, sum M^2 with
 * p_j = prod_{l>i}(1 + delta L)(L_i - K_j)^+ and M = prod_{l>=i}(1 + delta L). */
int lll_plan_sums(lll_plan *plan, double *sums_host, void *stream);

/* Per-wavefront partial sums of the last execute ([n_waves][N][NSTAT], FP64),
 * the input of the fixed-order reduction.  n_waves = ceil(n_paths / 64). */
int lll_plan_partials(lll_plan *plan, double *partials_host, int64_t capacity, void *stream);

/* Record HIP events around the three stages of every later execute on its
 * stream (enable != 0) or stop recording (enable == 0). */
int lll_plan_set_timing(lll_plan *plan, int enable);

/* Durations in milliseconds of the last timed execute: ms_host[0] precompute,
 * ms_host[1] path kernel, ms_host[2] reduction.  Waits for the last event. */
int lll_plan_timing(lll_plan *plan, float *ms_host);

int lll_plan_destroy(lll_plan *plan);

/* One-shot convenience: create a plan, execute on `stream`, read the results,
 * destroy.  Outputs as in lll_plan_results (any may be NULL). */
int lll_price_caplets(const lll_term_structure *ts, int64_t n_paths, int scheme, uint64_t seed,
                      int precision, double *price_host, double *stderr_host,
                      double *mart_resid_host, void *stream);

/* ---- pricing without device allocation ---- */

/* Size of the library's static device workspace (bytes per GPU). */
#define LLL_STATIC_WORKSPACE_BYTES (64u << 20)

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the same
 * pass as lll_price_caplets (same arguments, same kernels, the same prices
 * bit for bit) with every device buffer taken from one static workspace of
 * LLL_STATIC_WORKSPACE_BYTES that each GPU holds from the first call on it
 * until the process ends.  Calls no hipMalloc or hipFree.  The inputs are
 * copied into the workspace on `stream`; the call waits for `stream` before
 * it returns the results to the host buffers.
 * Schemes LLL_FULL .. LLL_SECOND_ORDER (LLL_EUNSUPPORTED for LLL_PICARD_MP and
 * LLL_EXACT), N <= LLL_N_MAX (FP64: N <= LLL_N_MAX_FP64).  The workspace needed,
 * about 8 (K N Q + ceil(n_paths / 64) N (3 S + 2)) bytes plus the plan-precision
 * step tables (K = N steps_per_period), must fit LLL_STATIC_WORKSPACE_BYTES:
 * larger passes get LLL_EINVAL, with the size in the message, before any
 * device work (the N = 20, 400-step, 3-strike workload fits up to ~2.0 M paths).
 * Every call on a GPU shares that GPU's workspace: calls that overlap on one
 * GPU (from several threads, or on unordered streams) race and must be
 * serialised by the caller. */
int lll_price_caplets_static(const lll_term_structure *ts, int64_t n_paths, int scheme,
                             uint64_t seed, int precision, double *price_host,
                             double *stderr_host, double *mart_resid_host, void *stream);

/* ---- pathwise adjoint (caplet and swaption Greeks) ---- */

/* Enqueue a FULL-scheme pricing pass of paths 0 .. n_paths-1 on an FP32 plan
 * (NIG driver; LLL_EUNSUPPORTED otherwise) together with the pathwise adjoint
 * of every product price (strike 0; caplets or the co-terminal swaptions of
 * the plan's product) with respect to the initial forwards L(0, T_l) and to a parallel
 * shift of each rate's volatility curve lambda(., T_l) (all steps k).  The
 * forward pass checkpoints the live rates at every tenor date; each product's
 * reverse sweep recomputes one accrual period at a time from its checkpoint.
 * B(0, T_1) is held fixed, so dP/dL0 includes the dependence of B(0, T_*) on
 * the forwards (paper Section 3.3, eq. (caplet)).  Checkpoint and scratch
 * buffers (about (N (N+1) / 2 + N + s nmax + s) x 4 bytes per path) are
 * allocated on the first call and kept by the plan.  LLL_EUNSUPPORTED for
 * N > LLL_N_MAX.  Asynchronous. */
int lll_plan_greeks(lll_plan *plan, int64_t n_paths, uint64_t seed, void *stream);

/* Vector-Jacobian product of the same product prices (strike 0) with weights
 * g = weights_host[N] (host, read before return): out_L0[l] = sum_i g_i
 * dP_i/dL(0,T_l) and out_vol[l] = sum_i g_i dP_i/dv_l, the quantities that
 * reverse-mode differentiation of a scalar function of the prices needs.  One
 * reverse sweep, from the last fixing date to t = 0, whose state adjoint is
 * seeded with g_i times the payoff adjoint of product i at its fixing date
 * (paper Section 3.3, eq. (caplet); the swaption payoff of lll_product); per accrual period one kernel recomputes
 * the period from its tenor-date checkpoint and walks it back.  Cost: the
 * forward pass plus one recompute and one reverse pass, against one sweep per
 * product for the full Jacobian of lll_plan_greeks (same conventions, buffers
 * and restrictions; equal to g^T J up to FP32 summation order).
 * LLL_EINVAL for NULL or non-finite weights.  Asynchronous. */
int lll_plan_greeks_vjp(lll_plan *plan, int64_t n_paths, uint64_t seed, const double *weights_host,
                        void *stream);

/* lll_plan_greeks_vjp with the weights in device memory (weights_dev[N] FP64,
 * read when the stream reaches the call): no host synchronisation, for
 * reverse-mode differentiation that stays on the device. */
int lll_plan_greeks_vjp_dev(lll_plan *plan, int64_t n_paths, uint64_t seed,
                            const double *weights_dev, void *stream);

/* The last vector-Jacobian product into device buffers on `stream`
 * (asynchronous): price_dev[N] (strike 0), vjp_L0_dev[N], vjp_vol_dev[N] (FP64;
 * any may be NULL). */
int lll_plan_greeks_vjp_results_dev(lll_plan *plan, double *price_dev, double *vjp_L0_dev,
                                    double *vjp_vol_dev, void *stream);

/* The last Greeks pass into device buffers on `stream` (asynchronous):
 * price_dev[N], dP_dL0_dev[N][N], dP_dvol_dev[N][N] (FP64; any may be NULL). */
int lll_plan_greeks_results_dev(lll_plan *plan, double *price_dev, double *dP_dL0_dev,
                                double *dP_dvol_dev, void *stream);

/* Results of the last lll_plan_greeks_vjp: price_host[N] (strike 0),
 * vjp_L0_host[N], vjp_vol_host[N]; waits for `stream`.  Any pointer may be NULL. */
int lll_plan_greeks_vjp_results(lll_plan *plan, double *price_host, double *vjp_L0_host,
                                double *vjp_vol_host, void *stream);

/* Wait for `stream` and copy the last Greeks pass: price_host[N] (strike 0),
 * dP_dL0_host[N][N] and dP_dvol_host[N][N], row = product, column = input rate.
 * Any pointer may be NULL. */
int lll_plan_greeks_results(lll_plan *plan, double *price_host, double *dP_dL0_host,
                            double *dP_dvol_host, void *stream);

/* One-shot: plan, Greeks pass, results, destroy. */
int lll_caplet_greeks(const lll_term_structure *ts, int64_t n_paths, uint64_t seed,
                      double *price_host, double *dP_dL0_host, double *dP_dvol_host,
                      void *stream);

/* ---- learned drift surrogate ---- */

/* A small network that corrects the first-order drift expansion of paper
 * Section 3.2 (eq. (drifta)) towards the 64-node quadrature coupling:
 *   C_i = C'_i + sigma * net(t_k / T_N, X_{l>i}, onehot(i)),
 * C'_i = sum_{l>i} ell_l [kappa(lambda_i + lambda_l) - kappa(lambda_i) - kappa(lambda_l)],
 * 96 inputs (81 used: t, the 40 later-rate log-rate states X_l = log L_l/L_l(0),
 * the 40-wide rate one-hot), 3 hidden layers of 64 with tanh-form GELU, one
 * output; BF16 matrix-core operands with FP32 accumulation and FP32 master
 * weights.  Parameter vector (LLL_MLP_PARAMS floats): W1[64][96] b1[64]
 * W2[64][64] b2[64] W3[64][64] b3[64] w4[64] b4.  The surrogate serves plans
 * of 33..40 rates (the 40-slot register bucket), FP32, NIG driver. */
#define LLL_MLP_PARAMS 14593
#define LLL_MLP_INPUTS 96

/* Allocate a network on the current device with Glorot-uniform weights drawn
 * from Philox (key = seed, counter word 3 = tag 2) and zero biases. */
int lll_mlp_create(uint64_t seed, lll_mlp **mlp_out);
int lll_mlp_destroy(lll_mlp *mlp);

/* Copy the FP32 parameter vector to get_host and/or replace it from set_host
 * (either may be NULL; setting resets the optimiser state).  Synchronous. */
int lll_mlp_params(lll_mlp *mlp, float *get_host, const float *set_host);

/* Training pairs from the plan's term structure: n_paths FULL paths on their
 * own random stream (counter word 3 = struct_id | 1 << 24) record their state
 * at `records` staggered steps; every recorded state yields one pair per live
 * rate i with BF16 features and the FP64 label C_i - C'_i (quadrature coupling
 * minus first-order expansion), stored in FP32.  Also computes the per-rate
 * state range (the trust box of the fallback) and the label scale sigma (root
 * mean square).  Synchronous; *n_pairs_out receives the number of pairs. */
int lll_mlp_generate(lll_mlp *mlp, lll_plan *plan, int64_t n_paths, int records, uint64_t seed,
                     int64_t *n_pairs_out, void *stream);

/* info_host[81]: box minimum per rate [40], box maximum per rate [40], sigma. */
int lll_mlp_info(lll_mlp *mlp, float *info_host, int64_t *n_pairs);

/* Replace the trust box (box_host[80]: minimum per rate [40], maximum per rate
 * [40], in units of X_l = log L_l - log L_l(0)) that lll_mlp_generate set.  A
 * rate whose later rates leave the box takes the quadrature coupling; an
 * empty box (minimum above maximum) sends every coupling to the quadrature.
 * Needs generated data (LLL_EINVAL otherwise); NaN entries are rejected.
 * Synchronous. */
int lll_mlp_set_box(lll_mlp *mlp, const float *box_host);

/* For pairs[n]: the recorded state [n][40] (FP32, by rate), its step, the
 * pair's rate, its label and its features [n][96] (BF16 values as FP32).
 * Any output may be NULL. */
int lll_mlp_pairs(lll_mlp *mlp, const int64_t *pairs, int64_t n, float *state_host, int *k_host,
                  int *rate_host, float *label_host, float *feat_host);

/* n_steps Adam steps (beta 0.9 / 0.999, cosine decay of lr to lr / 100) on
 * minibatches of `batch` pairs drawn with replacement (Philox key seed, tag 2),
 * loss = mean squared error of the labels divided by sigma.  loss_host[n_steps]
 * (may be NULL) receives the minibatch losses.  Synchronous. */
int lll_mlp_train(lll_mlp *mlp, int n_steps, int batch, float lr, uint64_t seed, float *loss_host,
                  void *stream);

/* Training on caller-owned pairs in device memory: feat_dev [n_pairs][96]
 * bfloat16 bit patterns (the features of lll_mlp_generate's layout),
 * label_dev [n_pairs] FP32 raw labels, divided by `sigma` (> 0) for the loss.
 * Otherwise as lll_mlp_train: n_steps Adam steps (beta 0.9 / 0.999, eps 1e-8,
 * bias correction with the network's step count t, which continues across
 * calls and restarts when the parameters are set) at the learning rate
 * lr (0.01 + 0.99 (1 + cos(pi j / n_steps)) / 2) of step j of the call, on
 * minibatches of `batch` pairs drawn with replacement: draw i of step t is
 * (w0 2^32 + w1) mod n_pairs for the Philox words of counter (t, i, 1, 2 << 24)
 * and key seed.  loss_dev [n_steps] (FP32, may be NULL) receives the
 * minibatch losses sum (y - label / sigma)^2 / (2 batch).  Asynchronous on
 * `stream`: the inputs must stay valid until the stream reaches the end of
 * the call; nothing is copied to the host.  The optimiser's buffers are
 * allocated on first use (LLL_ENOMEM if that fails). */
int lll_mlp_train_dev(lll_mlp *mlp, const uint16_t *feat_dev, const float *label_dev,
                      int64_t n_pairs, float sigma, int n_steps, int batch, float lr, uint64_t seed,
                      float *loss_dev, void *stream);

/* Adam moments of the network after the work queued so far (waits for the
 * device): m_host and v_host [LLL_MLP_PARAMS] FP32 (either may be NULL) and the
 * step count t of the last step (step_host, may be NULL). */
int lll_mlp_optimizer_state(lll_mlp *mlp, float *m_host, float *v_host, int64_t *step_host);

/* Copy the pairs of the last lll_mlp_generate into caller device buffers on
 * `stream` (asynchronous): feat_dev [n][96] bfloat16 bit patterns, label_dev [n]
 * FP32, n = the pair count lll_mlp_info reports; LLL_EINVAL if capacity < n. */
int lll_mlp_copy_pairs_dev(lll_mlp *mlp, uint16_t *feat_dev, float *label_dev, int64_t capacity,
                           void *stream);

/* Forward pass on n host feature rows [n][96] (rounded to BF16 on the device):
 * outputs y_host[n]; with targets (target_host[n]) also the gradient of
 * loss = sum (y - target)^2 / (2 n) with respect to the parameter vector
 * (grad_host[LLL_MLP_PARAMS]) and the loss.  Synchronous. */
int lll_mlp_eval(lll_mlp *mlp, const float *feat_host, const float *target_host, int64_t n,
                 float *y_host, float *grad_host, float *loss_host, void *stream);

/* Pricing pass (as lll_plan_execute, FULL-scheme Euler steps) whose coupling
 * is C'_i + sigma * net (use_net = 1) or the first-order expansion C'_i alone
 * (use_net = 0, mlp may be NULL).  A path whose state of a later rate leaves
 * the training range takes the quadrature coupling for that rate (fallback);
 * every judge_stride-th wavefront (0: none) also evaluates the quadrature at
 * every step and records the surrogate's errors.  Asynchronous. */
int lll_plan_execute_mlp(lll_plan *plan, const lll_mlp *mlp, int use_net, int64_t n_paths,
                         uint64_t seed, int judge_stride, double *path_fix_dev, void *stream);

/* Statistics of the last surrogate pass, stats_host[8]: rate-steps evaluated,
 * fallbacks taken, judged rate-steps, sum |C - C_quad| over judged rate-steps,
 * sum |C_quad|, max |C - C_quad| / |C_quad|, 0, 0. */
int lll_plan_mlp_stats(lll_plan *plan, double *stats_host, void *stream);

/* ---- many term structures in one persistent launch ---- */

/* Opaque batch of n_ts independent term structures (FP32 path arithmetic).
 * Owned by the library. */
typedef struct lll_batch lll_batch;

/* Validate all n_ts structures (host array ts[n_ts]) and allocate their
 * device tables and buffers for up to max_paths_each paths per structure.
 * Each structure's struct_id is its fourth Philox counter word.  Limits:
 * 1 <= n_ts <= 4096, 1 <= max_paths_each <= 2^30 and n_ts x ceil(max_paths_each
 * / 256) <= 2^30 (one work item per block of 256 paths), N <= LLL_N_MAX for
 * every structure, else LLL_EINVAL.  Synchronous. */
int lll_batch_create(const lll_term_structure *ts, int n_ts, int64_t max_paths_each,
                     lll_batch **batch_out);

/* Price every structure with n_paths_each paths in one persistent kernel
 * launch on `stream` (schemes LLL_FULL, LLL_PICARD, LLL_FROZEN; LLL_EINVAL
 * otherwise): work items of 256 paths, longest tenors first, pulled
 * from a device counter by a grid sized to the GPU's resident capacity; then
 * each structure's fixed-order reduction.  Blocks the host briefly while the
 * work list is copied to the device; the pricing itself is asynchronous. */
int lll_batch_execute(lll_batch *batch, int scheme, int64_t n_paths_each, uint64_t seed,
                      void *stream);

/* Results of structure `index` of the last batch execute (as lll_plan_results). */
int lll_batch_results(lll_batch *batch, int index, double *price_host, double *stderr_host,
                      double *mart_resid_host, double *mart_se_host, double *n_itm_host,
                      void *stream);

/* Record HIP events around the persistent kernel of later executes; read the
 * duration (ms) of the last one. */
int lll_batch_set_timing(lll_batch *batch, int enable);
int lll_batch_timing(lll_batch *batch, float *ms_host);

int lll_batch_destroy(lll_batch *batch);

/* One-shot batch: create, execute once with n_paths_each paths per structure,
 * copy each structure's results and destroy (as lll_batch_create,
 * lll_batch_execute and lll_batch_results).  price_host[i] receives structure
 * i's [N_i][S_i] prices; stderr_host may be NULL, else stderr_host[i] is NULL
 * or an [N_i][S_i] buffer.  Synchronous. */
int lll_price_caplets_batched(const lll_term_structure *ts, int n_ts, int64_t n_paths_each,
                              int scheme, uint64_t seed, double *const *price_host,
                              double *const *stderr_host, void *stream);

/* ---- inspection entry points (used by the parity tests) ---- */

/* Measured roofline ceiling of the path kernels: the throughput (TFLOP/s,
 * FMA = 2) of plain non-packed FP32 FMAs on the current device -- independent
 * chains on every lane of a full grid, best of 3 timed runs.  The quoted FP32
 * vector peak counts dual-issue packed FMAs, which this library does not
 * generate.  Synchronous (waits for `stream`); allocates and frees a small
 * buffer. */
int lll_fp32_fma_peak(double *tflops_host, void *stream);

/* The attainable ceiling of the quadrature recursion (the path kernels'
 * coupling loop): throughput in TFLOP/s of its instruction mix -- per node and
 * rate two FMAs whose second operand is a wave-uniform table entry held in a
 * scalar register and one FMA on vector registers -- on every lane of a full
 * grid, best of 3 timed runs.  On gfx950 a vector instruction with a
 * scalar-register operand issues at about the single-issue rate while one on
 * vector registers alone can issue faster, so this mix sits between the plain
 * FMA probe and the quoted peak.  Synchronous; allocates a small buffer. */
int lll_fp32_mix_peak(double *tflops_host, void *stream);

/* The attainable ceiling of the exact-drift kernel's products: throughput in
 * TFLOP/s (multiply-add = 2) of a stream of independent FP32 matrix-core
 * instructions (v_mfma_f32_16x16x4f32, operands in registers, no memory
 * traffic, 16 accumulators per wavefront) on 3 wavefronts per SIMD of every
 * compute unit, best of 3 timed runs.  Synchronous; allocates a small
 * buffer. */
int lll_fp32_mfma_peak(double *tflops_host, void *stream);

/* Philox-4x32-10 words computed on the device for n counters ctr_host[n][4]
 * and keys key_host[n][2]; out_host[n][4]. */
int lll_philox(const uint32_t *ctr_host, const uint32_t *key_host, int64_t n,
               uint32_t *out_host, void *stream);

/* The FP64 routines of the driver increment (the Box-Muller and inverse-
 * Gaussian steps of Section 4's sampling of the NIG increments), evaluated on
 * the device for inspection: fn = LLL_SM_LOG log(x) for normal 0 < x <= 1;
 * LLL_SM_SINPI / LLL_SM_COSPI sin(pi t) / cos(pi t) for t in [0, 2] a multiple
 * of 2^-24 (the sampler's angles); LLL_SM_SQRT sqrt(x) for normal x > 0;
 * LLL_SM_DIV x[2i] / x[2i+1] for finite x[2i] and normal x[2i+1] > 0.
 * x_host holds n arguments (2n for LLL_SM_DIV), out_host[n] the results.
 * LLL_EINVAL (nothing computed) for an unknown fn, n outside 1 .. 2^26 or an
 * argument outside the routine's domain. */
typedef enum {
    LLL_SM_LOG = 0,
    LLL_SM_SINPI = 1,
    LLL_SM_COSPI = 2,
    LLL_SM_SQRT = 3,
    LLL_SM_DIV = 4
} lll_sampler_routine;
int lll_sampler_math(int fn, const double *x_host, int64_t n, double *out_host, void *stream);

/* Driver increments of step k for paths p0 .. p0 + n - 1 as drawn by the path
 * kernel (FP64): subordinator draws V_host[n] (0 for the Brownian driver) and
 * increments dH_host[n].  Runs the plan's precompute first. */
int lll_plan_increments(lll_plan *plan, int k, int64_t p0, int64_t n, uint64_t seed,
                        double *V_host, double *dH_host, void *stream);

/* FP64 precompute tables of the plan (after lll_plan_execute or
 * lll_plan_increments): nodes x_host[Q], weights w_host[Q] (Lévy density
 * included), kappa_host[K][N] = kappa(lambda_{k,i}), E_host[K][N][Q] =
 * e^{lambda_{k,i} x_q} - 1, b0_host[K][N] = drift at the initial rates; entries
 * of fixed rates are 0.  K = N * steps_per_period.  Any pointer may be NULL. */
int lll_plan_tables(lll_plan *plan, double *x_host, double *w_host, double *kappa_host,
                    double *E_host, double *b0_host, void *stream);

/* Drift b(t_k, T_i) of the live rates at step k for n given rate vectors
 * L_host[n][N], computed by the path kernel's own drift code in the plan's
 * precision; b_host[n][N] (entries of fixed rates are 0).  LLL_EUNSUPPORTED
 * for N > LLL_N_MAX. */
int lll_plan_drift(lll_plan *plan, int k, const double *L_host, int64_t n, double *b_host,
                   void *stream);

#ifdef __cplusplus
}
#endif

#endif /* LLL_H */
