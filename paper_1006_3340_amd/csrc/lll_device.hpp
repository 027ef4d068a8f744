// lll_device.hpp -- device-side building blocks shared by the kernels:
// the counter-based generator, the driver increment, the NIG cumulant, the
// scaled Bessel function K_1 and the Gauss-Legendre rule.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lll {

constexpr int kQ = 64;          // quadrature nodes of the coupling integral
constexpr int kGL = 32;         // Gauss-Legendre points per half line
constexpr int kWave = 64;       // CDNA wavefront
constexpr int kBlock = 256;     // threads per path block (4 wavefronts)
constexpr double kTailExponent = 36.0;  // truncate the Lévy integral where e^{-36}
constexpr double kXCap = 40.0;          // ... but never beyond |x| = 40

enum { kFull = 0, kPicard = 1, kFrozen = 2, kFirst = 3, kSecond = 4 };
enum { kNig = 0, kBrownian = 1 };

// Philox-4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two
// 32x32->64 multiplications with the Weyl key schedule.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32->64 product each (v_mad_u64_u32) rather than separate
        // low and high halves
        const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c.x;
        const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c.z;
        const uint32_t lo0 = static_cast<uint32_t>(p0), hi0 = static_cast<uint32_t>(p0 >> 32);
        const uint32_t lo1 = static_cast<uint32_t>(p1), hi1 = static_cast<uint32_t>(p1 >> 32);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// 24-bit uniform on (0, 1), exact in FP64: (k + 1/2) 2^-24 = k 2^-24 + 2^-25
// for the top 24 bits k of the word, one FMA with no rounding.
__device__ __forceinline__ double uniform24(uint32_t w) {
    return fma(static_cast<double>(w >> 8), 1.0 / 16777216.0, 1.0 / 33554432.0);
}

// Per-period constants of the increment: IG mean m = delta dt / gamma, IG shape
// lam = (delta dt)^2, drift mu_H dt, Brownian scale sqrt(c dt).
struct StepConsts {
    double m, lam, mu_dt, sqrt_c_dt;
};

// Driver increment of one Euler step from four Philox words (FP64).
// NIG(alpha, beta, delta dt, mu_H dt) as a normal variance-mean mixture over an
// inverse-Gaussian subordinator: Box-Muller normals (z1, z2), the IG draw by
// Michael-Schucany-Haas from y = z1^2 (smaller root written without
// cancellation: x = 4 m lam a / (a + sqrt(a^2 + 4 lam a))^2 with a = m y), then
// dH = mu_H dt + beta V + sqrt(V) z2.  Brownian: dH = sqrt(c dt) z1.
__device__ __forceinline__ double increment(uint4 w, const StepConsts& sc, double beta,
                                            bool brownian, double* V_out) {
    const double u0 = uniform24(w.x);
    const double u1 = uniform24(w.y);
    const double u2 = uniform24(w.z);
    const double r = sqrt(-2.0 * log(u0));
    double sn, cs;
    sincospi(2.0 * u1, &sn, &cs);
    const double z1 = r * cs;
    const double z2 = r * sn;
    if (brownian) {
        if (V_out) *V_out = 0.0;
        return sc.sqrt_c_dt * z1;
    }
    const double m = sc.m;
    const double a = m * (z1 * z1);
    const double d = sqrt(a * a + 4.0 * sc.lam * a);
    const double ad = a + d;
    const double x = (a > 0.0) ? 4.0 * m * sc.lam * a / (ad * ad) : m;
    const double V = (u2 <= m / (m + x)) ? x : m * m / x;
    if (V_out) *V_out = V;
    return sc.mu_dt + beta * V + sqrt(V) * z2;
}

// NIG cumulant kappa(u) = mu_H u + delta (gamma - sqrt(alpha^2 - (beta+u)^2)),
// mu_H = -delta beta / gamma, rearranged so that no two large terms cancel:
// kappa(u) = delta u^2 (gamma + beta (2 beta + u) / (gamma + s)) / (gamma (gamma + s)),
// s = sqrt(alpha^2 - (beta + u)^2).
__device__ __forceinline__ double nig_cumulant(double u, double alpha, double beta, double delta) {
    const double gamma = sqrt(alpha * alpha - beta * beta);
    const double bu = beta + u;
    const double s = sqrt(alpha * alpha - bu * bu);
    const double gs = gamma + s;
    return delta * u * u * (gamma + beta * (2.0 * beta + u) / gs) / (gamma * gs);
}

// Exponentially scaled K_1(z) e^z from the integral representation
// K_1(z) = int_0^inf e^{-z cosh t} cosh t dt (Abramowitz & Stegun 9.6.24),
// by the trapezoidal rule, which converges geometrically in 1/h for this
// analytic integrand; h = min(1/8, 1/(2 sqrt z)) keeps the error below e^{-60}
// for all z > 0, and the sum stops once z (cosh t - 1) exceeds 50.
__device__ inline double bessel_k1e(double z) {
    const double h = fmin(0.125, 0.5 / sqrt(z));
    double sum = 0.5;  // t = 0 term counted with weight 1/2
    for (int j = 1; j < 4000; ++j) {
        const double t = j * h;
        const double sh = sinh(0.5 * t);
        const double e = z * 2.0 * sh * sh;  // z (cosh t - 1)
        if (e > 50.0) break;
        sum += exp(-e) * cosh(t);
    }
    return h * sum;
}

// j-th point (ascending) of the n-point Gauss-Legendre rule on [-1, 1] by
// Newton's method on the three-term recurrence of P_n.
__device__ inline void gauss_legendre_point(int n, int j, double* x_out, double* w_out) {
    const double pi = 3.141592653589793238462643383279502884;
    double x = -cos(pi * (j + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = x;
        for (int k = 2; k <= n; ++k) {
            const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (x * p1 - p0) / (x * x - 1.0);
        const double dx = p1 / dp;
        x -= dx;
        if (fabs(dx) < 1e-16) break;
    }
    // derivative at the converged root for the weight
    double p0 = 1.0, p1 = x;
    for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
    }
    dp = n * (x * p1 - p0) / (x * x - 1.0);
    *x_out = x;
    *w_out = 2.0 / ((1.0 - x * x) * dp * dp);
}

}  // namespace lll
