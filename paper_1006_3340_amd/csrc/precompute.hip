// precompute.hip -- FP64 precompute on the device, once per pricing pass.
//
// Paper Section 2, eq. (LIBOR-drift-PT): for the pure-jump NIG driver the
// drift of rate i at step k is
//     b_i = -kappa(lambda_i) - int (e^{lambda_i x} - 1)(prod_{l>i} beta_l(x) - 1) F(dx).
// The cumulant is closed form (Section 4 NIG cumulant, generalised to beta != 0
// with the martingale drift).  The coupling integral uses a fixed 64-node rule:
// 32 Gauss-Legendre points v_j on [0, 1] mapped by x = +-X_pm v^2 on each side,
// weights W = w_j 2 X_pm v_j f(x) with the NIG Lévy density
// f(x) = (delta alpha / pi) e^{beta x} K_1(alpha |x|) / |x|, and truncation
// X_+ = min(36 / (alpha - beta - Lambda_+), 40), X_- = min(36 / (alpha + beta - Lambda_-), 40)
// where Lambda_pm bounds the sum of the live vols' positive / negative parts.
//
// Tables (per step k and live rate slot j):
//   E[k][q][j]  = e^{lambda_{k,j} x_q} - 1 and W_q E   (path kernel, interleaved)
//   drift0      = -kappa(lambda_{k,j}) dt_k
//   frozen      = b0 dt_k, b0 the drift at the initial rates (eq. (Picard-2))
// all computed in FP64 and stored in the plan's precision.
#include <hip/hip_runtime.h>

#include "lll_device.hpp"
#include "lll_internal.hpp"

namespace lll {
namespace {

__device__ double levy_density(double x, double alpha, double beta, double delta) {
    const double pi = 3.141592653589793238462643383279502884;
    const double ax = fabs(x);
    return delta * alpha / pi * exp(beta * x - alpha * ax) * bessel_k1e(alpha * ax) / ax;
}

// One block of 64 threads: quadrature rule, Lambda_pm, per-period increment
// constants and per-slot constants.
template <typename Real>
__global__ void __launch_bounds__(64) setup_rule_kernel(
    const double *__restrict__ tenor, const double *__restrict__ delta,
    const double *__restrict__ L0, const double *__restrict__ vol, int N, int s, int off,
    int driver, double alpha, double beta, double delta_nig, double c, double *__restrict__ x_out,
    double *__restrict__ w_out, double *__restrict__ steps, double *__restrict__ lam_pm,
    Real *__restrict__ cinv, double *__restrict__ L0s, double *__restrict__ deltas, int nmax) {
    __shared__ double red_p[64], red_m[64];
    const int t = threadIdx.x;
    const int K = N * s;
    double lp = 0.0, lm = 0.0;
    int bad = 0;  // inputs the host could not check (set from device memory)
    for (int k = t; k < K; k += 64) {
        const int m = k / s;
        double sp = 0.0, sm = 0.0;
        for (int r = m; r < N; ++r) {
            const double v = vol[(size_t)k * N + r];
            bad |= !isfinite(v);
            sp += fmax(v, 0.0);
            sm += fmax(-v, 0.0);
        }
        lp = fmax(lp, sp);
        lm = fmax(lm, sm);
    }
    for (int r = t; r < N; r += 64) bad |= !(L0[r] > 0.0) || !isfinite(L0[r]);
    bad = __syncthreads_or(bad);
    red_p[t] = lp;
    red_m[t] = lm;
    __syncthreads();
    for (int o = 32; o > 0; o >>= 1) {
        if (t < o) {
            red_p[t] = fmax(red_p[t], red_p[t + o]);
            red_m[t] = fmax(red_m[t], red_m[t + o]);
        }
        __syncthreads();
    }
    const double Lp = red_p[0], Lm = red_m[0];
    if (t == 0) {
        lam_pm[0] = Lp;
        lam_pm[1] = Lm;
        // (LR1): the drift integral is finite iff Lambda_+ < alpha - beta and
        // Lambda_- < alpha + beta; the pricing pass returns NaN otherwise
        lam_pm[2] = (driver == kNig && !(Lp < alpha - beta && Lm < alpha + beta)) ? 1.0 : 0.0;
        lam_pm[3] = bad ? 1.0 : 0.0;
    }
    if (driver == kNig) {
        const double xp = fmin(kTailExponent / (alpha - beta - Lp), kXCap);
        const double xm = fmin(kTailExponent / (alpha + beta - Lm), kXCap);
        const int j = t % kGL;
        const bool right = t < kGL;
        double g, wg;
        gauss_legendre_point(kGL, j, &g, &wg);
        const double v = 0.5 * (g + 1.0);
        const double wv = 0.5 * wg;
        const double X = right ? xp : xm;
        const double xq = right ? X * v * v : -X * v * v;
        x_out[t] = xq;
        w_out[t] = wv * 2.0 * X * v * levy_density(xq, alpha, beta, delta_nig);
    } else {
        x_out[t] = 0.0;
        w_out[t] = 0.0;
    }
    if (t < N) {
        const double Ta = (t == 0) ? 0.0 : tenor[t - 1];
        const double dt = (tenor[t] - Ta) / s;
        double *sc = steps + 4 * t;
        if (driver == kNig) {
            const double gamma = sqrt(alpha * alpha - beta * beta);
            sc[0] = delta_nig * dt / gamma;                 // IG mean
            sc[1] = (delta_nig * dt) * (delta_nig * dt);    // IG shape
            sc[2] = -delta_nig * beta / gamma * dt;         // mu_H dt
            sc[3] = 0.0;
        } else {
            sc[0] = sc[1] = sc[2] = 0.0;
            sc[3] = sqrt(c * dt);
        }
    }
    if (t < nmax) {
        const int r = t - off;
        if (r >= 0) {
            cinv[t] = static_cast<Real>(1.0 / (delta[r] * L0[r]));
            L0s[t] = L0[r];
            deltas[t] = delta[r];
        } else {
            cinv[t] = Real(0);
            L0s[t] = 0.0;
            deltas[t] = 0.0;
        }
    }
}

// One block of 64 threads (one per node q) per Euler step k.
template <typename Real>
__global__ void __launch_bounds__(64) setup_tables_kernel(
    const double *__restrict__ tenor, const double *__restrict__ delta,
    const double *__restrict__ L0, const double *__restrict__ vol,
    const double *__restrict__ x_in, const double *__restrict__ w_in, int N, int s, int off,
    int nmax, int driver, double alpha, double beta, double delta_nig, double c,
    double *__restrict__ kappa_out, double *__restrict__ E_out, double *__restrict__ b0_out,
    Real *__restrict__ ew, Real *__restrict__ lam_t, Real *__restrict__ drift0,
    Real *__restrict__ frozen, Real *__restrict__ dt_t) {
    __shared__ double cq[LLL_N_MAX_MP][kQ];    // WE_q R_q contributions per rate
    __shared__ double kap[LLL_N_MAX_MP];
    const int k = blockIdx.x;
    const int q = threadIdx.x;
    const int m = k / s;
    const double Ta = (m == 0) ? 0.0 : tenor[m - 1];
    const double dt = (tenor[m] - Ta) / s;
    const double *lam = vol + (size_t)k * N;
    const double xq = x_in[q], wq = w_in[q];
    const bool nig = (driver == kNig);

    // cumulant of every live rate
    if (q < N) {
        double kv = 0.0;
        if (q >= m) {
            const double u = lam[q];
            kv = nig ? nig_cumulant(u, alpha, beta, delta_nig) : 0.5 * c * u * u;
        }
        kap[q] = kv;
        kappa_out[(size_t)k * N + q] = kv;
    }
    __syncthreads();

    // quadrature tables and the suffix recursion at the initial rates:
    // R <- R + ell0_l E_l (1 + R) from the last rate down, C_i = sum_q W E_i R_q
    double R = 0.0;
    for (int r = N - 1; r >= 0; --r) {
        const int j = r + off;
        Real *row = ew + (((size_t)k * kQ + q) * nmax + j) * 2;
        if (r >= m && nig) {
            const double E = expm1(lam[r] * xq);
            const double WE = wq * E;
            E_out[((size_t)k * N + r) * kQ + q] = E;
            row[0] = static_cast<Real>(E);
            row[1] = static_cast<Real>(WE);
            cq[r][q] = WE * R;
            const double ell0 = delta[r] * L0[r] / (1.0 + delta[r] * L0[r]);
            R = R + ell0 * E * (1.0 + R);
        } else {
            E_out[((size_t)k * N + r) * kQ + q] = 0.0;
            row[0] = Real(0);
            row[1] = Real(0);
            cq[r][q] = 0.0;
        }
    }
    for (int j = q; j < off; j += kQ) {  // unused leading slots
        Real *row = ew + (((size_t)k * kQ) * nmax + j) * 2;
        for (int qq = 0; qq < kQ; ++qq) {
            row[(size_t)qq * nmax * 2] = Real(0);
            row[(size_t)qq * nmax * 2 + 1] = Real(0);
        }
    }
    __syncthreads();
    if (q == 0) dt_t[k] = static_cast<Real>(dt);
    if (q < nmax) {
        const int j = q, r = j - off;
        double b0 = 0.0, kv = 0.0, lv = 0.0;
        if (r >= m) {
            kv = kap[r];
            lv = lam[r];
            double C = 0.0;
            if (nig) {
                for (int qq = 0; qq < kQ; ++qq) C += cq[r][qq];
            } else {
                double S = 0.0;
                for (int l = r + 1; l < N; ++l)
                    S += delta[l] * L0[l] / (1.0 + delta[l] * L0[l]) * lam[l];
                C = c * lv * S;
            }
            b0 = -kv - C;
        }
        if (r >= 0) b0_out[(size_t)k * N + r] = b0;
        lam_t[(size_t)k * nmax + j] = static_cast<Real>(lv);
        drift0[(size_t)k * nmax + j] = static_cast<Real>(-kv * dt);
        frozen[(size_t)k * nmax + j] = static_cast<Real>(b0 * dt);
    }
}

template <typename Real>
hipError_t launch_precompute_t(const lll_plan &p, hipStream_t st) {
    const DeviceTables &d = p.d;
    hipLaunchKernelGGL(setup_rule_kernel<Real>, dim3(1), dim3(64), 0, st, d.tenor, d.delta, d.L0,
                       d.vol, p.N, p.s, p.off, p.driver, p.alpha, p.beta, p.delta_nig, p.c, d.x,
                       d.w, d.steps, d.lam_pm, static_cast<Real *>(d.cinv), d.L0s, d.deltas,
                       p.nmax);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(setup_tables_kernel<Real>, dim3(p.K), dim3(64), 0, st, d.tenor, d.delta,
                       d.L0, d.vol, d.x, d.w, p.N, p.s, p.off, p.nmax, p.driver, p.alpha, p.beta,
                       p.delta_nig, p.c, d.kappa, d.E, d.b0, static_cast<Real *>(d.ew),
                       static_cast<Real *>(d.lam), static_cast<Real *>(d.drift0),
                       static_cast<Real *>(d.frozen), static_cast<Real *>(d.dt));
    return hipGetLastError();
}

// First-order expansion of the coupling (paper Section 3.2, eq. (drifta)):
// K2[k][j][l] = kappa(lambda_j + lambda_l) - kappa(lambda_j) - kappa(lambda_l)
// for live slots j < l at step k, 0 elsewhere; FP64, stored in the plan
// precision.  One block per step.
template <typename Real>
__global__ void __launch_bounds__(64) setup_first_order_kernel(
    const double *__restrict__ vol, int N, int s, int off, int nmax, int driver, double alpha,
    double beta, double delta_nig, double c, Real *__restrict__ k2) {
    const int k = blockIdx.x;
    const int m = k / s;
    const double *lam = vol + (size_t)k * N;
    const bool nig = driver == LLL_DRIVER_NIG;
    for (int e = threadIdx.x; e < nmax * nmax; e += 64) {
        const int j = e / nmax, l = e % nmax;
        const int rj = j - off, rl = l - off;
        double v = 0.0;
        if (rj >= m && rl > rj) {
            const double a = lam[rj], b = lam[rl];
            v = nig ? nig_cumulant(a + b, alpha, beta, delta_nig) -
                          nig_cumulant(a, alpha, beta, delta_nig) -
                          nig_cumulant(b, alpha, beta, delta_nig)
                    : c * a * b;  // c (a + b)^2 / 2 - c a^2 / 2 - c b^2 / 2
        }
        k2[(size_t)k * nmax * nmax + e] = static_cast<Real>(v);
    }
}

template <typename Real>
hipError_t launch_first_order_t(const lll_plan &p, hipStream_t st) {
    hipLaunchKernelGGL(setup_first_order_kernel<Real>, dim3(p.K), dim3(64), 0, st, p.d.vol, p.N,
                       p.s, p.off, p.nmax, p.driver, p.alpha, p.beta, p.delta_nig, p.c,
                       static_cast<Real *>(p.d.k2));
    return hipGetLastError();
}

}  // namespace

hipError_t launch_first_order_tables(const lll_plan &p, hipStream_t st) {
    if (!p.d.k2) return hipErrorInvalidValue;
    return p.precision == LLL_FP64 ? launch_first_order_t<double>(p, st)
                                   : launch_first_order_t<float>(p, st);
}

namespace {

// New initial forwards and a parallel shift of each rate's vol curve:
// vol[k][r] = vol_base[k][r] + shift[r] for the live rates r >= k / s.
__global__ void __launch_bounds__(256) set_inputs_kernel(const double *__restrict__ L0_in,
                                                         const double *__restrict__ shift,
                                                         const double *__restrict__ vol_base,
                                                         double *__restrict__ L0,
                                                         double *__restrict__ vol, int N, int s) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (L0_in && i < N) L0[i] = L0_in[i];
    if (shift && i < N * s * N) {
        const int k = i / N, r = i % N;
        vol[i] = vol_base[i] + (r >= k / s ? shift[r] : 0.0);
    }
}

}  // namespace

hipError_t launch_set_inputs(const lll_plan &p, const double *L0_dev, const double *shift_dev,
                             hipStream_t st) {
    const int n = shift_dev ? p.K * p.N : p.N;
    hipLaunchKernelGGL(set_inputs_kernel, dim3((n + 255) / 256), dim3(256), 0, st, L0_dev,
                       shift_dev, p.d.vol_base, p.d.L0, p.d.vol, p.N, p.s);
    return hipGetLastError();
}

hipError_t launch_precompute(const lll_plan &p, hipStream_t st) {
    return p.precision == LLL_FP64 ? launch_precompute_t<double>(p, st)
                                   : launch_precompute_t<float>(p, st);
}

}  // namespace lll
