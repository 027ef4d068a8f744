// adjoint.hip -- host side of the pathwise caplet Greeks and their tables.
#include <hip/hip_runtime.h>

#include "adjoint_kernel.hpp"
#include "lll_device.hpp"
#include "lll_internal.hpp"

namespace lll {
namespace adj {

extern template hipError_t launch_adjoint_bucket<8>(const PathArgs<float> &, const AdjArgs &, hipStream_t);
extern template hipError_t launch_adjoint_bucket<16>(const PathArgs<float> &, const AdjArgs &, hipStream_t);
extern template hipError_t launch_adjoint_bucket<24>(const PathArgs<float> &, const AdjArgs &, hipStream_t);
extern template hipError_t launch_adjoint_bucket<32>(const PathArgs<float> &, const AdjArgs &, hipStream_t);
extern template hipError_t launch_adjoint_bucket<40>(const PathArgs<float> &, const AdjArgs &, hipStream_t);

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

// dP_i/dL0_l = delta_i B(0,T_*) mean(L0bar) - P_i delta_l / (1 + delta_l L0_l)
// (the second term: B(0,T_*) = B(0,T_1) / prod_l (1 + delta_l L0_l) with B(0,T_1) held);
// dP_i/dvol_l = delta_i B(0,T_*) mean(vbar).
__global__ void __launch_bounds__(64) greeks_finalize_kernel(
    const double *__restrict__ gsums, const double *__restrict__ results,
    const double *__restrict__ delta, const double *__restrict__ L0, int N, int S, double B0_T1,
    int64_t n_paths, double *__restrict__ out) {
    double prod_all = 1.0;
    for (int l = 0; l < N; ++l) prod_all *= 1.0 + delta[l] * L0[l];
    const double B0T = B0_T1 / prod_all;
    const double n = static_cast<double>(n_paths);
    double *dL = out, *dV = out + N * N, *price = out + 2 * N * N;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const double P = results[i * S];  // strike 0
        price[i] = P;
        const double scale = delta[i] * B0T / n;
        for (int l = 0; l < N; ++l) {
            dL[i * N + l] = scale * gsums[(size_t)i * 2 * N + l] - P * delta[l] / (1.0 + delta[l] * L0[l]);
            dV[i * N + l] = scale * gsums[(size_t)i * 2 * N + N + l];
        }
    }
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
    return e;
}

void greeks_free(lll_plan &p) {
    GreeksBuffers &g = p.g;
    void *ptrs[] = {g.xe, g.dkap, g.w32, g.inv_L0, g.ckpt, g.fix, g.scr, g.scr_dh, g.gpart,
                    g.gchunks, g.gsums, g.out};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    p.g = GreeksBuffers{};
}

hipError_t launch_greeks(const lll_plan &p, int64_t n_paths, uint64_t seed, hipStream_t st) {
    using namespace adj;
    const DeviceTables &d = p.d;
    const GreeksBuffers &gb = p.g;
    hipError_t e = launch_precompute(p, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(setup_adjoint_tables_kernel, dim3(p.K), dim3(64), 0, st, d.tenor, d.L0,
                       d.vol, d.x, d.w, p.N, p.s, p.off, p.nmax, p.alpha, p.beta, p.delta_nig,
                       gb.xe, gb.dkap, gb.w32, gb.inv_L0);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    PathArgs<float> a = detail::make_args<float>(p, seed, n_paths, 0, nullptr);
    AdjArgs g;
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
    switch (p.nmax) {
        case 8: e = launch_adjoint_bucket<8>(a, g, st); break;
        case 16: e = launch_adjoint_bucket<16>(a, g, st); break;
        case 24: e = launch_adjoint_bucket<24>(a, g, st); break;
        case 32: e = launch_adjoint_bucket<32>(a, g, st); break;
        case 40: e = launch_adjoint_bucket<40>(a, g, st); break;
        default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    e = launch_reduce(p, n_paths, st);  // prices
    if (e != hipSuccess) return e;
    const int64_t waves = (n_paths + kWave - 1) / kWave;
    const int cols = p.N * 2 * p.N;
    const int64_t chunks = (waves + 255) / 256;
    hipLaunchKernelGGL(reduce_cols_kernel, dim3(static_cast<unsigned>(chunks)), dim3(256), 0, st,
                       gb.gpart, waves, cols, 256, gb.gchunks);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_cols_kernel, dim3(1), dim3(256), 0, st, gb.gchunks, chunks, cols,
                       chunks, gb.gsums);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(greeks_finalize_kernel, dim3(1), dim3(64), 0, st, gb.gsums, d.results,
                       d.delta, d.L0, p.N, p.S, p.B0_T1, n_paths, gb.out);
    return hipGetLastError();
}

}  // namespace lll
