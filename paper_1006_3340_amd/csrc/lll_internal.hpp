// lll_internal.hpp -- host-side plan and kernel launchers (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "lll.h"

namespace lll {

constexpr int kWaveSize = 64;  // CDNA wavefront
constexpr int kQSize = 64;     // quadrature nodes

// Smallest register bucket holding N rates: 8, 16, 20 (with slots20: FP32
// single-structure plans), 24, 32, 40, and 64 for the tables of the
// maturity-parallel scheme.  Rates live in register slots off .. off + N - 1
// with off = nmax - N, so that the live rates of every period are a suffix of
// the bucket and all slot indices are compile-time.
int bucket_for(int n_rates, bool slots20);

struct DeviceTables {
    // FP64 inputs (device)
    double *tenor = nullptr, *delta = nullptr, *L0 = nullptr, *vol = nullptr, *strikes = nullptr;
    // FP64 precompute, inspection layout
    double *x = nullptr, *w = nullptr;          // [Q]
    double *kappa = nullptr;                    // [K][N]
    double *E = nullptr;                        // [K][N][Q]
    double *b0 = nullptr;                       // [K][N]
    double *steps = nullptr;                    // [N][4] per-period increment constants
    double *lam_pm = nullptr;                   // [4] Lambda_+, Lambda_-, moment flag, input flag
    double *vol_base = nullptr;                 // [K][N] the creation vol table (first shifted input)
    // path-kernel layout in the plan's precision (slot columns, nmax wide)
    void *ew = nullptr;        // [K][Q][nmax][2]  (E, W E)
    void *lam = nullptr;       // [K][nmax]
    void *drift0 = nullptr;    // [K][nmax]  -kappa dt
    void *frozen = nullptr;    // [K][nmax]  b0 dt
    void *dt = nullptr;        // [K]
    void *cinv = nullptr;      // [nmax]  1 / (delta L0)
    void *k2 = nullptr;        // [K][nmax][nmax] first-order coefficients (allocated on first use)
    void *kex = nullptr;       // exact-drift cumulant table (allocated on first use)
    void *xex = nullptr;       // [N][max_paths] exact-drift path states (allocated on first use)
    // maturity-parallel PICARD (FP32, allocated on first use)
    void *mp_ewq = nullptr;       // [K][N][Q] (E, W E dt)
    float *mp_ell = nullptr;      // [chunk/4][s N (N+1)/2][4] ell at the predictor, live rates
    float *mp_z = nullptr;        // [chunk/4][N][N][4] per-period state increments
    double *mp_pay = nullptr;     // [N][S+1][chunk] per-path payoff values
    float *mp_dh = nullptr;       // [chunk/4][K][4] driver increments
    double *L0s = nullptr, *deltas = nullptr;   // [nmax] FP64 slot layout
    // reduction
    double *partials = nullptr;  // [max_waves][N][NSTAT]
    double *chunks = nullptr;    // [max_chunks][N*NSTAT]
    double *sums = nullptr;      // [N][NSTAT]
    double *results = nullptr;   // price[N*S], se[N*S], itm[N*S], mart[N], mart_se[N]
};

}  // namespace lll

namespace lll {
struct MlpBuffers {
    float *K2 = nullptr, *B1 = nullptr, *open_box = nullptr;
    void *zero_params = nullptr;  // zero FP32 + BF16 parameter vectors (first-order runs)
    double *stats = nullptr;
    int64_t stat_waves = 0;
};
struct GreeksBuffers {
    float *xe = nullptr, *dkap = nullptr, *w32 = nullptr;
    double *inv_L0 = nullptr;
    float *ckpt = nullptr, *fix = nullptr, *scr = nullptr, *scr_dh = nullptr;
    double *gpart = nullptr, *gchunks = nullptr, *gsums = nullptr, *out = nullptr;
    float *vjp_xb = nullptr;   // [N][paths] state adjoint carried between periods
    double *vjp_g = nullptr;   // [N] the weights g of the vector-Jacobian product
    float *vjp_w = nullptr;    // [N] g_i times the product's price scale (delta_i or 1)
    double *vjp_out = nullptr; // [3N] price, sum_i g_i dP_i/dL0, sum_i g_i dP_i/dvol
};
}  // namespace lll

struct lll_plan {
    int N = 0, s = 0, S = 0, K = 0, driver = 0, precision = 0, nmax = 0, off = 0;
    uint32_t struct_id = 0;
    int product = 0;  // lll_product
    double B0_T1 = 0, alpha = 0, beta = 0, delta_nig = 0, c = 0;
    int64_t max_paths = 0, max_waves = 0, max_chunks = 0;
    int64_t mp_chunk = 0;  // paths per chunk of the maturity-parallel PICARD
    int device = 0;
    std::vector<double> tenor, delta, L0, vol, strikes;
    lll::DeviceTables d;
    lll::GreeksBuffers g;
    lll::MlpBuffers mb;
    int64_t last_n_paths = 0, greeks_n_paths = 0;
    const lll_mlp *mlp = nullptr;  // network of scheme LLL_MLP_DRIFT (lll_plan_attach_mlp)
    bool mlp_done = false;
    bool greeks_done = false;
    bool vjp_done = false;
    bool executed = false;
    bool timing = false, timed = false;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
};

namespace lll {
constexpr int kBatchBuckets = 5;  // register buckets of 40, 32, 24, 16 and 8 slots
}

struct lll_batch {
    std::vector<lll_plan *> plans;   // one per structure, its own register bucket, FP32
    int64_t max_paths_each = 0, n_paths_each = 0;
    void *args = nullptr;            // device PathArgs<float>[n]
    void *items = nullptr;           // device work items, grouped by bucket
    int *counter = nullptr;          // device work counters, one per bucket (64 ints apart)
    int n_items = 0, max_items = 0;
    int bucket_begin[lll::kBatchBuckets] = {}, bucket_end[lll::kBatchBuckets] = {};
    hipStream_t side[lll::kBatchBuckets] = {};  // the buckets' launch streams (default priority)
    hipEvent_t fork = nullptr, join[lll::kBatchBuckets] = {};
    bool executed = false, timing = false, timed = false;
    hipEvent_t ev[2] = {nullptr, nullptr};
};

namespace lll {

constexpr int kStatBase = 3;  // NSTAT = 3 S + 2

// abi.hip: thread-local error text of the C ABI
int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
// abi.hip: host-side checks of a term structure (LLL_OK or a status with the
// message set) and the scalar fields of a plan for it
int validate(const lll_term_structure *ts);
void fill_plan_header(lll_plan &p, const lll_term_structure *ts, int precision, int64_t max_paths,
                      int nmax);

// precompute.hip: first-order coefficients K2 (scheme LLL_FIRST_ORDER)
hipError_t launch_first_order_tables(const lll_plan &p, hipStream_t st);

// adjoint.hip
hipError_t greeks_alloc(lll_plan &p);
void greeks_free(lll_plan &p);
hipError_t launch_greeks(const lll_plan &p, int64_t n_paths, uint64_t seed, hipStream_t st);
hipError_t launch_greeks_vjp(const lll_plan &p, int64_t n_paths, uint64_t seed,
                             const double *weights_host, const double *weights_dev, hipStream_t st);

// mlp_host.hip
void mlp_plan_free(lll_plan &p);

// batched.hip
size_t batch_item_bytes();
size_t batch_args_bytes();
hipError_t batch_prepare(lll_batch &b, int64_t n_paths_each, uint64_t seed, hipStream_t st);
hipError_t launch_batched(const lll_batch &b, int scheme, hipStream_t st);

// precompute.hip
hipError_t launch_precompute(const lll_plan &p, hipStream_t st);
// precompute.hip: replace the initial forwards (L0_dev [N], or NULL) and shift
// each rate's vol curve from the creation table (shift_dev [N], or NULL)
hipError_t launch_set_inputs(const lll_plan &p, const double *L0_dev, const double *shift_dev,
                             hipStream_t st);

// picard_mp.hip: PICARD in the maturity-parallel layout; its buffers hold at
// most kMpBufferBytes, so larger runs go in chunks of picard_mp_chunk paths
constexpr int64_t kMpBufferBytes = int64_t(2) << 30;
int64_t picard_mp_chunk(const lll_plan &p);
hipError_t picard_mp_alloc(lll_plan &p);
void picard_mp_free(lll_plan &p);
hipError_t launch_picard_mp(const lll_plan &p, int64_t n_paths, int64_t path_offset,
                            uint64_t seed, double *path_fix, hipStream_t st);

// fma_probe.hip: throughput of plain FP32 FMAs (TFLOP/s, best of 3 timed runs)
hipError_t measure_fma_peak(hipStream_t st, double *tflops);
// the same for the quadrature recursion's instruction mix (two FMAs with a
// scalar-register table operand, one on vector registers, per node and rate)
hipError_t measure_mix_peak(hipStream_t st, double *tflops);
hipError_t measure_mfma_peak(hipStream_t st, double *tflops);

// paths.hip
// LLL_EXACT: entries of the cumulant table and the launch (table build, paths).
int64_t exact_table_entries(int N, int s);
int64_t exact_state_entries(int N, int64_t max_paths);
hipError_t launch_exact(const lll_plan &p, int64_t n_paths, int64_t path_offset, uint64_t seed,
                        double *path_fix, hipStream_t st);
hipError_t launch_paths(const lll_plan &p, int scheme, int64_t n_paths, int64_t path_offset,
                        uint64_t seed, double *path_fix, hipStream_t st);
hipError_t launch_reduce(const lll_plan &p, int64_t n_paths, hipStream_t st);
hipError_t launch_drift(const lll_plan &p, int k, const double *L_dev, int64_t n, double *b_dev,
                        hipStream_t st);
hipError_t launch_increments(const lll_plan &p, int k, int64_t p0, int64_t n, uint64_t seed,
                             double *V_dev, double *dH_dev, hipStream_t st);
hipError_t launch_philox(const uint32_t *ctr_dev, const uint32_t *key_dev, int64_t n,
                         uint32_t *out_dev, hipStream_t st);
hipError_t launch_sampler_math(int fn, const double *x_dev, int64_t n, double *out_dev,
                               hipStream_t st);

}  // namespace lll
