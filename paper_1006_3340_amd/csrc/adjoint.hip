// adjoint.hip -- host side of the pathwise caplet Greeks and their tables.
#include <hip/hip_runtime.h>

#include "adjoint_kernel.hpp"
#include "lll_device.hpp"
#include "lll_internal.hpp"

namespace lll {
namespace adj {

extern template hipError_t launch_adjoint_bucket<8>(const PathArgs<float> &, const AdjArgs &, hipStream_t);
extern template hipError_t launch_adjoint_bucket<16>(const PathArgs<float> &, const AdjArgs &, hipStream_t);
extern template hipError_t launch_adjoint_bucket<20>(const PathArgs<float> &, const AdjArgs &, hipStream_t);
extern template hipError_t launch_adjoint_bucket<24>(const PathArgs<float> &, const AdjArgs &, hipStream_t);
extern template hipError_t launch_adjoint_bucket<32>(const PathArgs<float> &, const AdjArgs &, hipStream_t);
extern template hipError_t launch_adjoint_bucket<40>(const PathArgs<float> &, const AdjArgs &, hipStream_t);
#define LLL_VJP_EXTERN(NM)                                                                         \
    extern template hipError_t launch_vjp_bucket<NM>(const PathArgs<float> &, const AdjArgs &,    \
                                                     const VjpArgs &, hipStream_t);
LLL_VJP_EXTERN(8)
LLL_VJP_EXTERN(16)
LLL_VJP_EXTERN(20)
LLL_VJP_EXTERN(24)
LLL_VJP_EXTERN(32)
LLL_VJP_EXTERN(40)
#undef LLL_VJP_EXTERN

namespace {

// Tables of the reverse sweep: x_q e^{lambda x_q} = dE/dlambda per (step, node,
// slot), kappa'(lambda) dt per (step, slot), the weights in FP32 and 1/L(0,T).
// NIG: kappa'(u) = mu_H + delta (beta + u) / sqrt(alpha^2 - (beta + u)^2).
__global__ void __launch_bounds__(64) setup_adjoint_tables_kernel(
    const double *__restrict__ tenor, const double *__restrict__ L0, const double *__restrict__ vol,
    const double *__restrict__ x_in, const double *__restrict__ w_in, int N, int s, int off,
    int nmax, double alpha, double beta, double delta_nig, float *__restrict__ xe,
    float *__restrict__ dkap, float *__restrict__ w32, double *__restrict__ inv_L0) {
    const int k = blockIdx.x;
    const int q = threadIdx.x;
    const int m = k / s;
    const double Ta = (m == 0) ? 0.0 : tenor[m - 1];
    const double dt = (tenor[m] - Ta) / s;
    const double xq = x_in[q];
    for (int j = 0; j < nmax; ++j) {
        const int r = j - off;
        double v = 0.0;
        if (r >= m) v = xq * exp(vol[(size_t)k * N + r] * xq);
        xe[((size_t)k * kQ + q) * nmax + j] = static_cast<float>(v);
    }
    if (q < nmax) {
        const int r = q - off;
        double d = 0.0;
        if (r >= m) {
            const double u = vol[(size_t)k * N + r];
            const double gamma = sqrt(alpha * alpha - beta * beta);
            const double bu = beta + u;
            d = (-delta_nig * beta / gamma + delta_nig * bu / sqrt(alpha * alpha - bu * bu)) * dt;
        }
        dkap[(size_t)k * nmax + q] = static_cast<float>(d);
    }
    if (k == 0) {
        w32[q] = static_cast<float>(w_in[q]);
        if (q < nmax) inv_L0[q] = (q - off >= 0) ? 1.0 / L0[q - off] : 0.0;
    }
}

// dP_i/dL0_l = s_i B(0,T_*) mean(L0bar) - P_i delta_l / (1 + delta_l L0_l)
// (the second term: B(0,T_*) = B(0,T_1) / prod_l (1 + delta_l L0_l) with B(0,T_1) held);
// dP_i/dvol_l = s_i B(0,T_*) mean(vbar); s_i = delta_i for caplets, 1 for swaptions.
__global__ void __launch_bounds__(64) greeks_finalize_kernel(
    const double *__restrict__ gsums, const double *__restrict__ results,
    const double *__restrict__ delta, const double *__restrict__ L0, int N, int S, double B0_T1,
    int64_t n_paths, int product, const double *__restrict__ status, double *__restrict__ out) {
    const double poison = (status[2] != 0.0 || status[3] != 0.0) ? __builtin_nan("") : 0.0;
    double prod_all = 1.0;
    for (int l = 0; l < N; ++l) prod_all *= 1.0 + delta[l] * L0[l];
    const double B0T = B0_T1 / prod_all;
    const double n = static_cast<double>(n_paths);
    double *dL = out, *dV = out + N * N, *price = out + 2 * N * N;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const double P = results[i * S];  // strike 0
        price[i] = P;
        const double scale = (product == LLL_SWAPTIONS ? 1.0 : delta[i]) * B0T / n;
        for (int l = 0; l < N; ++l) {
            dL[i * N + l] =
                scale * gsums[(size_t)i * 2 * N + l] - P * delta[l] / (1.0 + delta[l] * L0[l]) + poison;
            dV[i * N + l] = scale * gsums[(size_t)i * 2 * N + N + l] + poison;
        }
    }
}

// The vector-Jacobian product from the swept sums (seeds g_i s_i, s_i = delta_i
// for caplets, 1 for swaptions):
// sum_i g_i dP_i/dL0_l = B(0,T_*) mean(L0bar_l) - (sum_i g_i P_i) delta_l / (1 + delta_l L0_l),
// sum_i g_i dP_i/dvol_l = B(0,T_*) mean(vbar_l); out = [price (strike 0), dL0, dvol].
struct VjpWeights {
    double g[LLL_N_MAX];
};

// The weights g of a vector-Jacobian product (host values passed by value,
// or device memory) and the FP32 seeds g_i s_i of the reverse sweep.
__global__ void __launch_bounds__(64) vjp_weights_kernel(VjpWeights host, const double *__restrict__ dev,
                                                         const double *__restrict__ delta, int N,
                                                         int product, double *__restrict__ g_out,
                                                         float *__restrict__ w_out) {
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const double g = dev ? dev[i] : host.g[i];
        g_out[i] = g;
        w_out[i] = static_cast<float>(g * (product == LLL_SWAPTIONS ? 1.0 : delta[i]));
    }
}

__global__ void __launch_bounds__(64) vjp_finalize_kernel(
    const double *__restrict__ vsums, const double *__restrict__ results,
    const double *__restrict__ delta, const double *__restrict__ L0, const double *__restrict__ wg,
    int N, int S, double B0_T1, int64_t n_paths, const double *__restrict__ status,
    double *__restrict__ out) {
    const double poison = (status[2] != 0.0 || status[3] != 0.0) ? __builtin_nan("") : 0.0;
    double prod_all = 1.0, gP = 0.0;
    for (int l = 0; l < N; ++l) {
        prod_all *= 1.0 + delta[l] * L0[l];
        gP += wg[l] * results[l * S];
    }
    const double scale = B0_T1 / prod_all / static_cast<double>(n_paths);
    for (int l = threadIdx.x; l < N; l += blockDim.x) {
        out[l] = results[l * S];
        out[N + l] = scale * vsums[l] - gP * delta[l] / (1.0 + delta[l] * L0[l]) + poison;
        out[2 * N + l] = scale * vsums[N + l] + poison;
    }
}

__global__ void __launch_bounds__(256) zero_kernel(double *__restrict__ a, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i < n) a[i] = 0.0;
}

__global__ void __launch_bounds__(256) reduce_cols_kernel(const double *__restrict__ in,
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

}  // namespace
}  // namespace adj

hipError_t greeks_alloc(lll_plan &p) {
    if (p.g.ckpt) return hipSuccess;
    const size_t N = p.N, K = p.K, NM = p.nmax, P = p.max_paths, S = p.s;
    GreeksBuffers &g = p.g;
    hipError_t e = hipSuccess;
    auto A = [&](void **ptr, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc(ptr, bytes + 64);
    };
    A((void **)&g.xe, K * kQSize * NM * sizeof(float));
    A((void **)&g.dkap, K * NM * sizeof(float));
    A((void **)&g.w32, kQSize * sizeof(float));
    A((void **)&g.inv_L0, NM * sizeof(double));
    A((void **)&g.ckpt, N * (N + 1) / 2 * P * sizeof(float));
    A((void **)&g.fix, N * P * sizeof(float));
    A((void **)&g.scr, S * NM * P * sizeof(float));
    A((void **)&g.scr_dh, S * P * sizeof(float));
    A((void **)&g.gpart, (size_t)p.max_waves * N * 2 * N * sizeof(double));
    A((void **)&g.gchunks, (size_t)p.max_chunks * N * 2 * N * sizeof(double));
    A((void **)&g.gsums, N * 2 * N * sizeof(double));
    A((void **)&g.out, (2 * N * N + N) * sizeof(double));
    A((void **)&g.vjp_xb, N * P * sizeof(float));
    A((void **)&g.vjp_out, 3 * N * sizeof(double));
    A((void **)&g.vjp_g, N * sizeof(double));
    A((void **)&g.vjp_w, N * sizeof(float));
    return e;
}

void greeks_free(lll_plan &p) {
    GreeksBuffers &g = p.g;
    void *ptrs[] = {g.xe, g.dkap, g.w32, g.inv_L0, g.ckpt, g.fix, g.scr, g.scr_dh, g.gpart,
                    g.gchunks, g.gsums, g.out, g.vjp_xb, g.vjp_out, g.vjp_g, g.vjp_w};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    p.g = GreeksBuffers{};
}

namespace {

// Precompute, the adjoint tables and the kernel arguments of a Greeks pass.
hipError_t adjoint_setup(const lll_plan &p, int64_t n_paths, uint64_t seed, hipStream_t st,
                         adj::AdjArgs &g) {
    using namespace adj;
    const DeviceTables &d = p.d;
    const GreeksBuffers &gb = p.g;
    hipError_t e = launch_precompute(p, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(setup_adjoint_tables_kernel, dim3(p.K), dim3(64), 0, st, d.tenor, d.L0,
                       d.vol, d.x, d.w, p.N, p.s, p.off, p.nmax, p.alpha, p.beta, p.delta_nig,
                       gb.xe, gb.dkap, gb.w32, gb.inv_L0);
    e = hipGetLastError();
    g.xe = detail::as_const<float>(gb.xe);
    g.dkap = detail::as_const<float>(gb.dkap);
    g.w = detail::as_const<float>(gb.w32);
    g.inv_L0 = detail::as_const<double>(gb.inv_L0);
    g.ckpt = gb.ckpt;
    g.fix = gb.fix;
    g.scr = gb.scr;
    g.scr_dh = gb.scr_dh;
    g.gpart = gb.gpart;
    g.n_paths = n_paths;
    return e;
}

// Fixed-order column sums of rows x cols per-wave partials into `out` (via the
// chunk buffer).
hipError_t reduce_cols(const double *in, int64_t rows, int cols, double *chunks_buf, double *out,
                       hipStream_t st) {
    const int64_t chunks = (rows + 255) / 256;
    hipLaunchKernelGGL(adj::reduce_cols_kernel, dim3(static_cast<unsigned>(chunks)), dim3(256), 0,
                       st, in, rows, cols, 256, chunks_buf);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(adj::reduce_cols_kernel, dim3(1), dim3(256), 0, st, chunks_buf, chunks, cols,
                       chunks, out);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_greeks_vjp(const lll_plan &p, int64_t n_paths, uint64_t seed,
                             const double *weights_host, const double *weights_dev, hipStream_t st) {
    using namespace adj;
    const GreeksBuffers &gb = p.g;
    AdjArgs g;
    hipError_t e = adjoint_setup(p, n_paths, seed, st, g);
    if (e != hipSuccess) return e;
    PathArgs<float> a = detail::make_args<float>(p, seed, n_paths, 0, nullptr);
    const int64_t waves = (n_paths + kWave - 1) / kWave;
    const int64_t n_part = waves * 2 * p.N;
    hipLaunchKernelGGL(zero_kernel, dim3(static_cast<unsigned>((n_part + 255) / 256)), dim3(256), 0,
                       st, gb.gpart, n_part);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    VjpWeights wts{};
    if (weights_host)
        for (int i = 0; i < p.N; ++i) wts.g[i] = weights_host[i];
    hipLaunchKernelGGL(vjp_weights_kernel, dim3(1), dim3(64), 0, st, wts, weights_dev, p.d.delta,
                       p.N, p.product, gb.vjp_g, gb.vjp_w);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    VjpArgs v;
    v.xb = gb.vjp_xb;
    v.part = gb.gpart;
    v.w = detail::as_const<float>(gb.vjp_w);
    switch (p.nmax) {
        case 8: e = launch_vjp_bucket<8>(a, g, v, st); break;
        case 16: e = launch_vjp_bucket<16>(a, g, v, st); break;
        case 20: e = launch_vjp_bucket<20>(a, g, v, st); break;
        case 24: e = launch_vjp_bucket<24>(a, g, v, st); break;
        case 32: e = launch_vjp_bucket<32>(a, g, v, st); break;
        case 40: e = launch_vjp_bucket<40>(a, g, v, st); break;
        default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    e = launch_reduce(p, n_paths, st);  // prices
    if (e != hipSuccess) return e;
    e = reduce_cols(gb.gpart, waves, 2 * p.N, gb.gchunks, gb.gsums, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(vjp_finalize_kernel, dim3(1), dim3(64), 0, st, gb.gsums, p.d.results,
                       p.d.delta, p.d.L0, gb.vjp_g, p.N, p.S, p.B0_T1, n_paths, p.d.lam_pm,
                       gb.vjp_out);
    return hipGetLastError();
}

hipError_t launch_greeks(const lll_plan &p, int64_t n_paths, uint64_t seed, hipStream_t st) {
    using namespace adj;
    const DeviceTables &d = p.d;
    const GreeksBuffers &gb = p.g;
    AdjArgs g;
    hipError_t e = adjoint_setup(p, n_paths, seed, st, g);
    if (e != hipSuccess) return e;
    PathArgs<float> a = detail::make_args<float>(p, seed, n_paths, 0, nullptr);
    switch (p.nmax) {
        case 8: e = launch_adjoint_bucket<8>(a, g, st); break;
        case 16: e = launch_adjoint_bucket<16>(a, g, st); break;
        case 20: e = launch_adjoint_bucket<20>(a, g, st); break;
        case 24: e = launch_adjoint_bucket<24>(a, g, st); break;
        case 32: e = launch_adjoint_bucket<32>(a, g, st); break;
        case 40: e = launch_adjoint_bucket<40>(a, g, st); break;
        default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    e = launch_reduce(p, n_paths, st);  // prices
    if (e != hipSuccess) return e;
    const int64_t waves = (n_paths + kWave - 1) / kWave;
    e = reduce_cols(gb.gpart, waves, p.N * 2 * p.N, gb.gchunks, gb.gsums, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(greeks_finalize_kernel, dim3(1), dim3(64), 0, st, gb.gsums, d.results,
                       d.delta, d.L0, p.N, p.S, p.B0_T1, n_paths, p.product, d.lam_pm, gb.out);
    return hipGetLastError();
}

}  // namespace lll
