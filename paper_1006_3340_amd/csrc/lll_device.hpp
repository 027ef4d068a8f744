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
        // three-input XORs as one v_bitop3_b32 each (truth table 0x96)
        c = make_uint4(__builtin_amdgcn_bitop3_b32(hi1, c.y, k0, 0x96), lo1,
                       __builtin_amdgcn_bitop3_b32(hi0, c.w, k1, 0x96), lo0);
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

// FP64 arithmetic of the increment on its own argument ranges (all operands
// positive and normal), each a textbook construction with at most 2 ulp of
// error against the correctly rounded result -- a third of the instructions
// of the general-purpose library routines, whose double-double steps and
// special-value paths the sampler does not need.

// a / b for b > 0 normal: hardware reciprocal estimate, two Newton steps
// r <- r + r (1 - b r), then one residual correction q <- q + r (a - b q)
// (each residual exact by FMA).
__device__ __forceinline__ double div_pos(double a, double b) {
    double r = __builtin_amdgcn_rcp(b);
    r = fma(fma(-b, r, 1.0), r, r);
    r = fma(fma(-b, r, 1.0), r, r);
    const double q = a * r;
    return fma(fma(-b, q, a), r, q);
}

// sqrt(x) for x > 0 normal: from the hardware 1/sqrt estimate y, g = x y and
// h = y / 2 refined by two coupled Newton (Goldschmidt) steps, then
// g <- g + h (x - g^2).
__device__ __forceinline__ double sqrt_pos(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const double r = fma(-g, h, 0.5);
        g = fma(g, r, g);
        h = fma(h, r, h);
    }
    return fma(fma(-g, g, x), h, g);
}

// log(x) for 0 < x <= 1 normal: x = f 2^e with f in [1/sqrt 2, sqrt 2),
// log f = 2 atanh(z) = 2 z (1 + z^2/3 + z^4/5 + ...), z = (f - 1) / (f + 1),
// |z| <= 0.172 (terms through z^19: truncation below 3e-17 relative), and
// e log 2 with log 2 split into 32 leading bits (e times it is exact) and the
// FP64 rest.
__device__ __forceinline__ double log_unit(double x) {
    constexpr double kLn2Hi = 0x1.62e42ffp-1;             // log 2 to 32 bits
    constexpr double kLn2Lo = -4.2009150726810846e-11;    // log 2 - kLn2Hi
    double f = __builtin_amdgcn_frexp_mant(x);             // [1/2, 1)
    int e = __builtin_amdgcn_frexp_exp(x);
    if (f < 0.7071067811865476) {
        f *= 2.0;
        --e;
    }
    const double z = div_pos(f - 1.0, f + 1.0);
    const double w = z * z;
    double s = 1.0 / 19.0;
#pragma unroll
    for (int j = 7; j >= 0; --j) s = fma(s, w, 1.0 / (2 * j + 3));
    const double tz = 2.0 * z;
    const double lf = fma(tz * w, s, tz);
    const double de = static_cast<double>(e);
    return fma(de, kLn2Hi, fma(de, kLn2Lo, lf));
}

// sin(pi t) and cos(pi t) for 0 <= t <= 2 with t a multiple of 2^-24: with
// v = 2 t, q = rint(v) and r = (v - q) / 2 (both steps exact), pi t =
// q pi/2 + pi r, |r| <= 1/4; sin(pi r) and cos(pi r) by their Taylor series
// through r^17 and r^18 (coefficients (-1)^k pi^n / n!; truncation below
// 1e-18), then the quadrant q mod 4.
__device__ __forceinline__ void sincospi_unit(double t, double &sn, double &cs) {
    const double v = 2.0 * t;
    const double q = __builtin_rint(v);
    const double r = (v - q) * 0.5;
    const double x = r * r;
    double ps = 7.952054001475513e-07;
    ps = fma(ps, x, -2.1915353447830217e-05);
    ps = fma(ps, x, 0.00046630280576761255);
    ps = fma(ps, x, -0.0073704309457143504);
    ps = fma(ps, x, 0.08214588661112823);
    ps = fma(ps, x, -0.5992645293207921);
    ps = fma(ps, x, 2.5501640398773455);
    ps = fma(ps, x, -5.16771278004997);
    ps = fma(ps, x, 3.141592653589793);
    double pc = -1.3878952462213771e-07;
    pc = fma(pc, x, 4.303069587032947e-06);
    pc = fma(pc, x, -0.0001046381049248457);
    pc = fma(pc, x, 0.0019295743094039231);
    pc = fma(pc, x, -0.02580689139001406);
    pc = fma(pc, x, 0.2353306303588932);
    pc = fma(pc, x, -1.3352627688545895);
    pc = fma(pc, x, 4.0587121264167685);
    pc = fma(pc, x, -4.934802200544679);
    pc = fma(pc, x, 1.0);
    const double s = r * ps;
    const int qi = static_cast<int>(q) & 3;
    const bool odd = (qi & 1) != 0;
    sn = odd ? pc : s;
    cs = odd ? s : pc;
    if (qi & 2) sn = -sn;
    if (qi == 1 || qi == 2) cs = -cs;
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
    const double r = sqrt_pos(-2.0 * log_unit(u0));
    double sn, cs;
    sincospi_unit(2.0 * u1, sn, cs);
    const double z1 = r * cs;
    const double z2 = r * sn;
    if (brownian) {
        if (V_out) *V_out = 0.0;
        return sc.sqrt_c_dt * z1;
    }
    const double m = sc.m;
    const double a = m * (z1 * z1);
    const double d = sqrt_pos(a * a + 4.0 * sc.lam * a);
    const double ad = a + d;
    const double x = (a > 0.0) ? div_pos(4.0 * m * sc.lam * a, ad * ad) : m;
    const double V = (u2 <= div_pos(m, m + x)) ? x : div_pos(m * m, x);
    if (V_out) *V_out = V;
    return sc.mu_dt + beta * V + sqrt_pos(V) * z2;
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
