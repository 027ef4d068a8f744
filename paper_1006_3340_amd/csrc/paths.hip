// paths.hip -- the Monte Carlo path kernel and the fixed-order reduction.
//
// One path per lane, 64 paths per wavefront.  The log-rate state X_i =
// log L(t, T_i) - log L(0, T_i) of all rates lives in registers (slots off ..
// nmax-1 of a compile-time bucket), so every period of the tenor runs code
// specialised to its number of live rates.  Per Euler step k (paper Section 2,
// eqs. (LIBOR-dyn-PT), (log-LIB-SIE); Section 3 for the schemes):
//
//   1. Philox-4x32-10 words for counter (k, p_lo, p_hi, stream word);
//   2. the driver increment dH (FP64: subordinator + normal mixture);
//   3. ell_j = delta_j L_j / (1 + delta_j L_j) of the live rates, from X
//      (FULL) or from the Picard iterate X1 (PICARD, eq. (bdrift));
//   4. the coupling C_i = sum_q W_q E_{i,q} (prod_{l>i} beta_l(x_q) - 1) by a
//      suffix recursion over the rates, node by node:
//          C_i += W_q E_{i,q} R_q,   R_q <- R_q + ell_i E_{i,q} (1 + R_q),
//      which is the product of eq. (LIBOR-drift-PT) with beta_l = 1 + ell_l E_l
//      evaluated once for all i (O(N Q) per step instead of O(N^2 Q));
//      the uniform table entries (E, W E) are wave-uniform scalar operands;
//   5. X_i += (-kappa_i - C_i) dt + lambda_i dH (PICARD also advances
//      X1_i += b0_i dt + lambda_i dH; FROZEN advances only X with b0);
//   6. at the end of period m the rate with maturity T_{m+1} fixes: the FP64
//      payoffs prod_{l>i}(1 + delta_l L_l)(L_i - K)^+ of eq. (caplet) and the
//      martingale factor are summed across the wavefront (butterfly), and lane
//      0 writes the wave's sums; a two-pass fixed-order FP64 reduction follows.
#include <hip/hip_runtime.h>

#include "lll_device.hpp"
#include "lll_internal.hpp"
#include "path_kernel.hpp"

namespace lll {
namespace {

__global__ void __launch_bounds__(kBlock) increments_kernel(const double *__restrict__ steps, int k,
                                                            int s, int64_t p0, int64_t n,
                                                            uint32_t stream_word, uint32_t key0,
                                                            uint32_t key1, double beta,
                                                            int brownian, double *__restrict__ V,
                                                            double *__restrict__ dH) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t p = p0 + i;
    const int m = k / s;
    const StepConsts cst{steps[4 * m], steps[4 * m + 1], steps[4 * m + 2], steps[4 * m + 3]};
    const uint4 w = philox4x32_10(
        make_uint4(static_cast<uint32_t>(k), static_cast<uint32_t>(p),
                   static_cast<uint32_t>(static_cast<uint64_t>(p) >> 32), stream_word),
        key0, key1);
    double v;
    dH[i] = increment(w, cst, beta, brownian != 0, &v);
    V[i] = v;
}

__global__ void __launch_bounds__(kBlock) philox_kernel(const uint32_t *__restrict__ ctr,
                                                        const uint32_t *__restrict__ key,
                                                        int64_t n, uint32_t *__restrict__ out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint4 c = make_uint4(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]);
    const uint4 r = philox4x32_10(c, key[2 * i], key[2 * i + 1]);
    out[4 * i] = r.x;
    out[4 * i + 1] = r.y;
    out[4 * i + 2] = r.z;
    out[4 * i + 3] = r.w;
}

// The increment's FP64 routines on given arguments (fn: LLL_SM_*; LLL_SM_DIV
// reads the pairs x[2i], x[2i+1]); the host has checked the domains.
__global__ void __launch_bounds__(kBlock) sampler_math_kernel(int fn, const double *__restrict__ x,
                                                              int64_t n, double *__restrict__ out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    double r = 0.0;
    if (fn == LLL_SM_LOG) {
        r = log_unit(x[i]);
    } else if (fn == LLL_SM_SINPI || fn == LLL_SM_COSPI) {
        double sn, cs;
        sincospi_unit(x[i], sn, cs);
        r = fn == LLL_SM_SINPI ? sn : cs;
    } else if (fn == LLL_SM_SQRT) {
        r = sqrt_pos(x[i]);
    } else {
        r = div_pos(x[2 * i], x[2 * i + 1]);
    }
    out[i] = r;
}

// Pass 1: block b sums rows [b*256, (b+1)*256) of the wave partials column by
// column in row order.  Pass 2: one block sums the chunk rows in order.
__global__ void __launch_bounds__(256) reduce_rows_kernel(const double *__restrict__ in,
                                                          int64_t rows, int cols,
                                                          int64_t rows_per_chunk,
                                                          double *__restrict__ out) {
    const int64_t r0 = static_cast<int64_t>(blockIdx.x) * rows_per_chunk;
    const int64_t r1 = min(rows, r0 + rows_per_chunk);
    for (int c = threadIdx.x; c < cols; c += blockDim.x) {
        double acc = 0.0;
        for (int64_t r = r0; r < r1; ++r) acc += in[r * cols + c];
        out[static_cast<int64_t>(blockIdx.x) * cols + c] = acc;
    }
}

// Prices, standard errors and martingale residuals from the sums (eq. (caplet)):
// price = delta_i B(0, T_*) mean(p), B(0, T_*) = B(0, T_1) / prod_l (1 + delta_l L_l(0)).
__global__ void __launch_bounds__(64) finalize_kernel(const double *__restrict__ sums,
                                                      const double *__restrict__ delta,
                                                      const double *__restrict__ L0, int N, int S,
                                                      double B0_T1, int64_t n_paths, int product,
                                                      const double *__restrict__ status,
                                                      double *__restrict__ res) {
    const int nstat = 3 * S + 2;
    // inputs set from device memory that fail the checks of Section 2 give NaN
    const double poison = (status[2] != 0.0 || status[3] != 0.0) ? __builtin_nan("") : 0.0;
    double prod_all = 1.0;
    for (int l = 0; l < N; ++l) prod_all *= 1.0 + delta[l] * L0[l];
    const double B0T = B0_T1 / prod_all;
    const double n = static_cast<double>(n_paths);
    const double nm1 = n > 1.0 ? n - 1.0 : 1.0;
    double *price = res, *se = res + N * S, *itm = res + 2 * N * S;
    double *mart = res + 3 * N * S, *mart_se = res + 3 * N * S + N;
    for (int r = threadIdx.x; r < N; r += blockDim.x) {
        const double *sr = sums + (size_t)r * nstat;
        // caplets pay delta_r (L - K)^+; swaption payoffs are already amounts
        const double scale = product == LLL_SWAPTIONS ? B0T : delta[r] * B0T;
        for (int t = 0; t < S; ++t) {
            const double mean = sr[t] / n;
            const double var = fmax(sr[S + t] / n - mean * mean, 0.0);
            price[r * S + t] = scale * mean + poison;
            se[r * S + t] = scale * sqrt(var / nm1) + poison;
            itm[r * S + t] = sr[2 * S + t];
        }
        double fwd = 1.0;
        for (int l = r; l < N; ++l) fwd *= 1.0 + delta[l] * L0[l];
        const double mm = sr[3 * S] / n;
        const double mv = fmax(sr[3 * S + 1] / n - mm * mm, 0.0);
        mart[r] = mm - fwd;
        mart_se[r] = sqrt(mv / nm1);
    }
}

}  // namespace

int bucket_for(int n_rates, bool slots20) {
    if (n_rates <= 8) return 8;
    if (n_rates <= 16) return 16;
    if (slots20 && n_rates <= 20) return 20;
    if (n_rates <= 24) return 24;
    if (n_rates <= 32) return 32;
    if (n_rates <= 40) return 40;
    return 64;  // tables only: the maturity-parallel PICARD
}

hipError_t launch_paths(const lll_plan &p, int scheme, int64_t n_paths, int64_t path_offset,
                        uint64_t seed, double *path_fix, hipStream_t st) {
    using namespace detail;
    if (p.precision == LLL_FP64) {
        switch (p.nmax) {
            case 8: return launch_bucket<double, 8>(p, scheme, n_paths, path_offset, seed, path_fix, st);
            case 16: return launch_bucket<double, 16>(p, scheme, n_paths, path_offset, seed, path_fix, st);
            case 24: return launch_bucket<double, 24>(p, scheme, n_paths, path_offset, seed, path_fix, st);
            default: return hipErrorInvalidValue;
        }
    }
    switch (p.nmax) {
        case 8: return launch_bucket<float, 8>(p, scheme, n_paths, path_offset, seed, path_fix, st);
        case 16: return launch_bucket<float, 16>(p, scheme, n_paths, path_offset, seed, path_fix, st);
        case 20: return launch_bucket<float, 20>(p, scheme, n_paths, path_offset, seed, path_fix, st);
        case 24: return launch_bucket<float, 24>(p, scheme, n_paths, path_offset, seed, path_fix, st);
        case 32: return launch_bucket<float, 32>(p, scheme, n_paths, path_offset, seed, path_fix, st);
        case 40: return launch_bucket<float, 40>(p, scheme, n_paths, path_offset, seed, path_fix, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_drift(const lll_plan &p, int k, const double *L_dev, int64_t n, double *b_dev,
                        hipStream_t st) {
    using namespace detail;
    if (p.precision == LLL_FP64) {
        switch (p.nmax) {
            case 8: return launch_drift_bucket<double, 8>(p, k, L_dev, n, b_dev, st);
            case 16: return launch_drift_bucket<double, 16>(p, k, L_dev, n, b_dev, st);
            case 24: return launch_drift_bucket<double, 24>(p, k, L_dev, n, b_dev, st);
            default: return hipErrorInvalidValue;
        }
    }
    switch (p.nmax) {
        case 8: return launch_drift_bucket<float, 8>(p, k, L_dev, n, b_dev, st);
        case 16: return launch_drift_bucket<float, 16>(p, k, L_dev, n, b_dev, st);
        case 20: return launch_drift_bucket<float, 20>(p, k, L_dev, n, b_dev, st);
        case 24: return launch_drift_bucket<float, 24>(p, k, L_dev, n, b_dev, st);
        case 32: return launch_drift_bucket<float, 32>(p, k, L_dev, n, b_dev, st);
        case 40: return launch_drift_bucket<float, 40>(p, k, L_dev, n, b_dev, st);
        default: return hipErrorInvalidValue;
    }
}
hipError_t launch_reduce(const lll_plan &p, int64_t n_paths, hipStream_t st) {
    const int64_t waves = (n_paths + kWave - 1) / kWave;
    const int cols = p.N * (3 * p.S + 2);
    const int64_t rows_per_chunk = 256;
    const int64_t chunks = (waves + rows_per_chunk - 1) / rows_per_chunk;
    hipLaunchKernelGGL(reduce_rows_kernel, dim3(static_cast<unsigned>(chunks)), dim3(256), 0, st,
                       p.d.partials, waves, cols, rows_per_chunk, p.d.chunks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_rows_kernel, dim3(1), dim3(256), 0, st, p.d.chunks, chunks, cols,
                       chunks, p.d.sums);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(64), 0, st, p.d.sums, p.d.delta, p.d.L0, p.N,
                       p.S, p.B0_T1, n_paths, p.product, p.d.lam_pm, p.d.results);
    return hipGetLastError();
}

hipError_t launch_increments(const lll_plan &p, int k, int64_t p0, int64_t n, uint64_t seed,
                             double *V_dev, double *dH_dev, hipStream_t st) {
    const dim3 grid(static_cast<unsigned>((n + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(increments_kernel, grid, dim3(kBlock), 0, st, p.d.steps, k, p.s, p0, n,
                       p.struct_id & 0xFFFFFFu, static_cast<uint32_t>(seed & 0xFFFFFFFFull),
                       static_cast<uint32_t>(seed >> 32), p.beta,
                       p.driver == LLL_DRIVER_BROWNIAN ? 1 : 0, V_dev, dH_dev);
    return hipGetLastError();
}

hipError_t launch_sampler_math(int fn, const double *x_dev, int64_t n, double *out_dev,
                               hipStream_t st) {
    const dim3 grid(static_cast<unsigned>((n + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(sampler_math_kernel, grid, dim3(kBlock), 0, st, fn, x_dev, n, out_dev);
    return hipGetLastError();
}

hipError_t launch_philox(const uint32_t *ctr_dev, const uint32_t *key_dev, int64_t n,
                         uint32_t *out_dev, hipStream_t st) {
    const dim3 grid(static_cast<unsigned>((n + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(philox_kernel, grid, dim3(kBlock), 0, st, ctr_dev, key_dev, n, out_dev);
    return hipGetLastError();
}

}  // namespace lll
