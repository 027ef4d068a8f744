// adjoint_kernel.hpp -- pathwise adjoint of the caplet prices (FULL scheme, FP32).
//
// Caplet i's price is delta_i B(0, T_*) E[f_i], f_i = D_i (L_i(T_i) - K)^+,
// D_i = prod_{l>i}(1 + delta_l L_l(T_i)) (paper Section 3.3, eq. (caplet)).
// For every path the kernel differentiates f_i with respect to the initial
// forwards L(0, T_l) and to a parallel shift of each rate's volatility curve
// lambda(., T_l), by reverse-mode differentiation of the Euler recursion
//     X_l <- X_l - kappa(lambda_l) dt - C_l dt + lambda_l dH,
//     C_l = sum_q W_q E_{l,q} (P_{l,q} - 1),  P_{l,q} = prod_{m>l} (1 + ell_m E_{m,q}),
// (eq. (LIBOR-drift-PT) with the quadrature rule), E_{l,q} = e^{lambda_l x_q} - 1,
// ell_l = delta_l L_l / (1 + delta_l L_l), L_l = L(0, T_l) e^{X_l}.
//
// Rate i depends only on rates l >= i, so the sweep of caplet i carries only
// those.  Memory: the forward pass checkpoints the live rates at every tenor
// date (packed, N (N+1) / 2 floats per path) and the fixing of every rate;
// each sweep recomputes one period at a time from its checkpoint into a
// per-period scratch (steps_per_period states per path) and walks it back.
//
// Reverse of one step, per node q (the suffix products P by a downward pass,
// then an upward pass with F_l = sum_{i<l} Cbar_i W E_{i,q} prod_{i<m<l} beta_m):
//     ellbar_l += E_{l,q} P_l F_l
//     Ebar_l    = Cbar_l W_q (P_l - 1) + ell_l P_l F_l,  lambdabar_l += x_q e^{lambda_l x_q} Ebar_l
//     F_{l+1}   = (1 + ell_l E_{l,q}) F_l + Cbar_l W_q E_{l,q},     Cbar_l = -dt Xbar_l,
// then Xbar_l += ellbar_l ell_l (1 - ell_l), L0bar_l += ellbar_l ell_l (1 - ell_l) / L(0, T_l),
// lambdabar_l += Xbar_l (dH - kappa'(lambda_l) dt).  The per-lane L0 accumulators
// sum the unscaled increments ellbar_l ell_l (1 - ell_l); the factor 1 / L(0, T_l),
// the same for every step, multiplies their wavefront sum (no per-step constant
// held in registers).
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

#include "lll_device.hpp"
#include "lll_internal.hpp"
#include "path_kernel.hpp"

namespace lll {
namespace adj {

using detail::cptr;
using detail::PathArgs;

constexpr int kAdjBlock = 64;  // one wavefront per block: per-lane accumulators in LDS

struct AdjArgs {
    cptr<float> xe;        // [K][Q][nmax]  x_q e^{lambda x_q}
    cptr<float> dkap;      // [K][nmax]     kappa'(lambda) dt
    cptr<float> w;         // [Q]           quadrature weights
    cptr<double> inv_L0;   // [nmax]        1 / L(0, T)
    float *ckpt;           // [N (N+1) / 2][n_paths] live rates at the start of each period
    float *fix;            // [N][n_paths]  X_i at its fixing
    float *scr;            // [s][nmax][n_paths] states within one period
    float *scr_dh;         // [s][n_paths]
    double *gpart;         // [waves][N][2N] per-wave sums of L0bar (first N) and vbar
    int64_t n_paths;
};

// Packed checkpoint row of rate r at the start of period m (r >= m).
__device__ __forceinline__ int64_t ckpt_row(int N, int m, int r) {
    return static_cast<int64_t>(m) * N - (static_cast<int64_t>(m) * (m - 1)) / 2 + (r - m);
}

__device__ __forceinline__ float increment_f(const PathArgs<float> &a, int k, int m, uint32_t p_lo,
                                             uint32_t p_hi) {
    const cptr<double> sc = a.steps + 4 * m;
    const StepConsts cst{sc[0], sc[1], sc[2], sc[3]};
    const uint4 w = philox4x32_10(make_uint4(static_cast<uint32_t>(k), p_lo, p_hi, a.stream_word),
                                  a.key0, a.key1);
    return static_cast<float>(increment(w, cst, a.beta, a.brownian != 0, nullptr));
}

template <int NMAX, int J0>
__device__ __forceinline__ void store_ckpt(const PathArgs<float> &a, const AdjArgs &g, int m,
                                           int64_t gid, bool active, const float (&X)[NMAX]) {
    if (!active) return;
#pragma unroll
    for (int j = J0; j < NMAX; ++j)
        g.ckpt[ckpt_row(a.N, m, j - a.off) * g.n_paths + gid] = X[j];
}

template <int NMAX, int... Js>
__device__ __forceinline__ void dispatch_ckpt(std::integer_sequence<int, Js...>, int j0,
                                              const PathArgs<float> &a, const AdjArgs &g, int m,
                                              int64_t gid, bool active, const float (&X)[NMAX]) {
    (void)((j0 == Js ? (store_ckpt<NMAX, Js>(a, g, m, gid, active, X), 0) : 0) + ...);
}

// Forward FULL pass with checkpoints; also the price partials of PRODUCT
// (LLL_CAPLETS or LLL_SWAPTIONS, fixed at compile time: the product's payoff
// code is inlined at every fixing date).
template <int NMAX, int PRODUCT>
__device__ void forward(const PathArgs<float> &a, const AdjArgs &g, int64_t gid, bool active) {
    const int64_t p = a.path_offset + gid;
    const uint32_t p_lo = static_cast<uint32_t>(p);
    const uint32_t p_hi = static_cast<uint32_t>(static_cast<uint64_t>(p) >> 32);
    float X[NMAX], X1[NMAX];
#pragma unroll
    for (int j = 0; j < NMAX; ++j) {
        X[j] = 0.0f;
        X1[j] = 0.0f;
    }
    for (int m = 0; m < a.N; ++m) {
        const int j0 = a.off + m;
        dispatch_ckpt<NMAX>(std::make_integer_sequence<int, NMAX>{}, j0, a, g, m, gid, active, X);
        for (int js = 0; js < a.s; ++js) {
            const int k = m * a.s + js;
            const float dH = increment_f(a, k, m, p_lo, p_hi);
            detail::dispatch_step<float, NMAX, kFull>(std::make_integer_sequence<int, NMAX>{}, j0,
                                                      a, k, dH, X, X1);
        }
        if (active) {
            // X of the rate that fixes now (slot j0), selected from registers
            float xf = 0.0f;
#pragma unroll
            for (int j = 0; j < NMAX; ++j) xf = (j == j0) ? X[j] : xf;
            g.fix[static_cast<int64_t>(m) * g.n_paths + gid] = xf;
        }
        detail::dispatch_payoff<float, NMAX, PRODUCT>(std::make_integer_sequence<int, NMAX>{}, j0,
                                                      a, m, gid, active, X);
    }
}

// The same forward pass with the state in the block's LDS columns, as the
// plain FP32 FULL path kernels of the 24- to 40-slot buckets run it (same
// step and payoff code, so the same prices bit for bit): X, ell and the
// coupling sums do not all fit the registers of two wavefronts per SIMD.
template <int NMAX, int PRODUCT>
__device__ void forward_lds(const PathArgs<float> &a, const AdjArgs &g, int64_t gid, bool active) {
    float *xs = detail::state_lds<float, NMAX>() + threadIdx.x;
    const int64_t p = a.path_offset + gid;
    const uint32_t p_lo = static_cast<uint32_t>(p);
    const uint32_t p_hi = static_cast<uint32_t>(static_cast<uint64_t>(p) >> 32);
    float X1[NMAX];
#pragma unroll
    for (int j = 0; j < NMAX; ++j) {
        xs[j * kBlock] = 0.0f;
        X1[j] = 0.0f;
    }
    for (int m = 0; m < a.N; ++m) {
        const int j0 = a.off + m;
        if (active)
            for (int j = j0; j < NMAX; ++j)
                g.ckpt[ckpt_row(a.N, m, j - a.off) * g.n_paths + gid] = xs[j * kBlock];
        for (int js = 0; js < a.s; ++js) {
            const int k = m * a.s + js;
            const float dH = increment_f(a, k, m, p_lo, p_hi);
            detail::dispatch_step_lds<float, NMAX, kFull>(std::make_integer_sequence<int, NMAX>{}, j0,
                                                          a, k, dH, xs, X1);
        }
        if (active) g.fix[static_cast<int64_t>(m) * g.n_paths + gid] = xs[j0 * kBlock];
        detail::payoff_lds<float, NMAX, PRODUCT>(a, m, gid, active, xs, j0);
    }
}

// Reverse of Euler step k for the slots JC .. NMAX-1, given the state X at the
// start of the step and Xb = adjoint of the state at its end (updated in place
// to the adjoint at the start).  Parameter adjoints go to the LDS accumulators.
template <int NMAX, int JC>
__device__ __forceinline__ void reverse_step(const PathArgs<float> &a, const AdjArgs &g, int k,
                                             float dH, const float (&X)[NMAX], float (&Xb)[NMAX],
                                             float *__restrict__ accL0, float *__restrict__ accV) {
    // Cbar = -dt Xbar: the factor -dt is applied once after the node loop
    // (lb and vb below are the adjoints divided by -dt).
    const int lane = threadIdx.x;
    const float mdt = -a.dt[k];
    const cptr<float> dk = g.dkap + (size_t)k * NMAX;
    float ell[NMAX], lb[NMAX], vb[NMAX], P[NMAX];
#pragma unroll
    for (int j = JC; j < NMAX; ++j) {
        ell[j] = detail::ell_of(X[j], a.cinv[j]);
        lb[j] = 0.0f;
        vb[j] = Xb[j] * (dH - dk[j]) / mdt;
    }
    cptr<float> row = a.ew + (size_t)k * kQ * NMAX * 2;
    cptr<float> xrow = g.xe + (size_t)k * kQ * NMAX;
#pragma unroll 1
    for (int q = 0; q < kQ; ++q, row += NMAX * 2, xrow += NMAX) {
        const float W = g.w[q];
        P[NMAX - 1] = 1.0f;
#pragma unroll
        for (int j = NMAX - 2; j >= JC; --j)
            P[j] = P[j + 1] * fmaf(ell[j + 1], row[2 * (j + 1)], 1.0f);
        float F = 0.0f;
#pragma unroll
        for (int j = JC; j < NMAX; ++j) {
            const float E = row[2 * j];
            const float WE = row[2 * j + 1];
            const float G = P[j] * F;
            lb[j] = fmaf(E, G, lb[j]);
            const float WR = fmaf(P[j], W, -W);  // W (P - 1)
            const float Eb = fmaf(Xb[j], WR, ell[j] * G);
            vb[j] = fmaf(xrow[j], Eb, vb[j]);
            F = fmaf(fmaf(ell[j], E, 1.0f), F, Xb[j] * WE);
        }
    }
#pragma unroll
    for (int j = JC; j < NMAX; ++j) {
        const float t = lb[j] * mdt * ell[j] * (1.0f - ell[j]);
        Xb[j] += t;
        accL0[(j - JC) * kAdjBlock + lane] += t;
        accV[(j - JC) * kAdjBlock + lane] += vb[j] * mdt;
    }
}

// Adds w times the payoff adjoint of product c (strike 0; slot JC = off + c)
// at its fixing date T_{c+1} to the state adjoint Xb and the L0 accumulators,
// and loads the fixing state into X.
//   caplet:   f = D (L_c - K)^+, D = prod_{l>c}(1 + delta_l L_l);
//   swaption: f = (Q - 1 - K A)^+, Q = prod_{l>=c} b_l, b_l = 1 + delta_l L_l,
//             A = sum_{l>=c} delta_l prod_{j>l} b_j, so that with
//             S_l = sum_{c<=m<l} delta_m prod_{j>m} b_j = sum_{c<=m<l} delta_m Q / prod_{c<=j<=m} b_j
//             df/dX_l = ell_l (Q - K S_l) where the payoff is positive.
// The direct L0 terms are df/dX_l / L(0, T_l) (L = L(0,T) e^X at fixed X); the
// accumulators hold the df/dX_l terms, scaled by 1 / L(0, T_l) after the wave sum.
template <int NMAX, int JC>
__device__ __forceinline__ void seed_caplet(const PathArgs<float> &a, const AdjArgs &g, int64_t gl,
                                            bool active, float w, float (&X)[NMAX],
                                            float (&Xb)[NMAX], float *__restrict__ accL0) {
    const int lane = threadIdx.x;
    const int c = JC - a.off;
    X[JC] = g.fix[static_cast<int64_t>(c) * g.n_paths + gl];
#pragma unroll
    for (int j = JC + 1; j < NMAX; ++j)
        X[j] = g.ckpt[ckpt_row(a.N, c + 1, j - a.off) * g.n_paths + gl];
    if (a.product == LLL_SWAPTIONS) {
        double Q = 1.0, A = 0.0;
#pragma unroll
        for (int j = NMAX - 1; j >= JC; --j) {
            const double b = 1.0 + a.deltas[j] * (a.L0s[j] * static_cast<double>(expf(X[j])));
            A = fma(a.deltas[j], Q, A);
            Q *= b;
        }
        const double K = a.strikes[c * a.S];
        const bool itm = active && ((Q - 1.0) - K * A > 0.0);
        double pre = 1.0, S = 0.0;
#pragma unroll
        for (int j = JC; j < NMAX; ++j) {
            const double L = a.L0s[j] * static_cast<double>(expf(X[j]));
            const double b = 1.0 + a.deltas[j] * L;
            const float t = itm ? w * static_cast<float>(a.deltas[j] * L / b * (Q - K * S)) : 0.0f;
            Xb[j] += t;
            accL0[(j - JC) * kAdjBlock + lane] += t;
            pre *= b;
            S = fma(a.deltas[j], Q / pre, S);
        }
        return;
    }
    double D = 1.0;
    float ellf[NMAX];
#pragma unroll
    for (int j = JC + 1; j < NMAX; ++j) {
        const double L = a.L0s[j] * static_cast<double>(expf(X[j]));
        D *= 1.0 + a.deltas[j] * L;
        ellf[j] = static_cast<float>(a.deltas[j] * L / (1.0 + a.deltas[j] * L));
    }
    const double Lc = a.L0s[JC] * static_cast<double>(expf(X[JC]));
    const double K = a.strikes[c * a.S];
    const bool itm = active && (Lc > K);
    const float dXc = itm ? w * static_cast<float>(D * Lc) : 0.0f;
    const float dD = itm ? w * static_cast<float>(Lc - K) : 0.0f;
    const float Df = static_cast<float>(D);
    Xb[JC] += dXc;
    accL0[lane] += dXc;
#pragma unroll
    for (int j = JC + 1; j < NMAX; ++j) {
        const float t = dD * Df * ellf[j];
        Xb[j] += t;
        accL0[(j - JC) * kAdjBlock + lane] += t;
    }
}

// Reverse of period m for the slots JC .. NMAX-1: recompute the period from
// its checkpoint, keeping every step's state in the scratch, then walk the
// steps back, updating Xb from the adjoint at the period's end to the one at
// its start.
template <int NMAX, int JC>
__device__ __forceinline__ void reverse_period(const PathArgs<float> &a, const AdjArgs &g, int m,
                                               int64_t gl, bool active, uint32_t p_lo,
                                               uint32_t p_hi, float (&X)[NMAX], float (&X1)[NMAX],
                                               float (&Xb)[NMAX], float *__restrict__ accL0,
                                               float *__restrict__ accV) {
#pragma unroll
    for (int j = JC; j < NMAX; ++j) X[j] = g.ckpt[ckpt_row(a.N, m, j - a.off) * g.n_paths + gl];
    for (int js = 0; js < a.s; ++js) {
        const int k = m * a.s + js;
        const float dH = increment_f(a, k, m, p_lo, p_hi);
        if (active) {
#pragma unroll
            for (int j = JC; j < NMAX; ++j)
                g.scr[(static_cast<int64_t>(js) * NMAX + j) * g.n_paths + gl] = X[j];
            g.scr_dh[static_cast<int64_t>(js) * g.n_paths + gl] = dH;
        }
        detail::step<float, NMAX, kFull, JC>(a, k, dH, X, X1);
    }
    for (int js = a.s - 1; js >= 0; --js) {
        const int k = m * a.s + js;
#pragma unroll
        for (int j = JC; j < NMAX; ++j)
            X[j] = g.scr[(static_cast<int64_t>(js) * NMAX + j) * g.n_paths + gl];
        const float dH = g.scr_dh[static_cast<int64_t>(js) * g.n_paths + gl];
        reverse_step<NMAX, JC>(a, g, k, dH, X, Xb, accL0, accV);
    }
}

// Sweep of the caplet fixing in slot JC (rate c = JC - off, period c).
template <int NMAX, int JC>
__device__ __forceinline__ void sweep(const PathArgs<float> &a, const AdjArgs &g, int64_t gid, bool active,
                      float *__restrict__ accL0, float *__restrict__ accV) {
    const int lane = threadIdx.x;
    const int c = JC - a.off;
    const int N = a.N;
    const int64_t p = a.path_offset + gid;
    const uint32_t p_lo = static_cast<uint32_t>(p);
    const uint32_t p_hi = static_cast<uint32_t>(static_cast<uint64_t>(p) >> 32);
    const int64_t gl = active ? gid : 0;  // lanes past the end read path 0 and contribute 0
#pragma unroll
    for (int j = JC; j < NMAX; ++j) {
        accL0[(j - JC) * kAdjBlock + lane] = 0.0f;
        accV[(j - JC) * kAdjBlock + lane] = 0.0f;
    }
    float X[NMAX], X1[NMAX], Xb[NMAX];
#pragma unroll
    for (int j = 0; j < NMAX; ++j) {
        X[j] = 0.0f;
        X1[j] = 0.0f;
        Xb[j] = 0.0f;
    }
    seed_caplet<NMAX, JC>(a, g, gl, active, 1.0f, X, Xb, accL0);
    // skip the sweep when no lane of the wavefront has a nonzero adjoint
    bool any = false;
#pragma unroll
    for (int j = JC; j < NMAX; ++j) any = any || (Xb[j] != 0.0f);
    if (__any(any)) {
        for (int m = c; m >= 0; --m)
            reverse_period<NMAX, JC>(a, g, m, gl, active, p_lo, p_hi, X, X1, Xb, accL0, accV);
    }
    // wavefront sums of this caplet's adjoints
    const int64_t wave = gid / kWave;
    double *out = g.gpart + (static_cast<int64_t>(wave) * N + c) * 2 * N;
    for (int j = JC; j < NMAX; ++j) {
        const double l0 =
            detail::wave_sum(active ? accL0[(j - JC) * kAdjBlock + lane] : 0.0f) * g.inv_L0[j];
        const double vv = detail::wave_sum(active ? accV[(j - JC) * kAdjBlock + lane] : 0.0f);
        if (lane == 0) {
            out[j - a.off] = l0;
            out[N + j - a.off] = vv;
        }
    }
    if (lane == 0)
        for (int r = 0; r < c; ++r) {
            out[r] = 0.0;
            out[N + r] = 0.0;
        }
}

// Vector-Jacobian product: one reverse sweep for sum_c g_c f_c.  The kernel of
// period m (slot JC = off + m) continues the sweep from the end of period m:
// it takes the state adjoint carried from period m+1 (xb, by rate), adds the
// seed of caplet m (weight w_m = g_m delta_m) at its fixing, reverses the
// period and stores the adjoint at the period's start; the wavefront sums of
// its parameter adjoints are added to the per-wave partials (periods in
// launch order, so the sums are deterministic).
struct VjpArgs {
    float *xb;      // [N][n_paths] state adjoint by rate, carried between periods
    double *part;   // [waves][2N] sums of L0bar (first N) and vbar
    detail::cptr<float> w;  // [N] seeds g_m s_m of the products (device memory)
};

template <int NMAX, int JC>
__device__ __forceinline__ void vjp_period(const PathArgs<float> &a, const AdjArgs &g,
                                           const VjpArgs &v, int64_t gid, bool active,
                                           float *__restrict__ accL0, float *__restrict__ accV) {
    const int lane = threadIdx.x;
    const int m = JC - a.off;
    const float w = v.w[m];
    const int N = a.N;
    const int64_t p = a.path_offset + gid;
    const uint32_t p_lo = static_cast<uint32_t>(p);
    const uint32_t p_hi = static_cast<uint32_t>(static_cast<uint64_t>(p) >> 32);
    const int64_t gl = active ? gid : 0;
#pragma unroll
    for (int j = JC; j < NMAX; ++j) {
        accL0[(j - JC) * kAdjBlock + lane] = 0.0f;
        accV[(j - JC) * kAdjBlock + lane] = 0.0f;
    }
    float X[NMAX], X1[NMAX], Xb[NMAX];
#pragma unroll
    for (int j = 0; j < NMAX; ++j) {
        X[j] = 0.0f;
        X1[j] = 0.0f;
        Xb[j] = 0.0f;
    }
    // rate m is fixed after period m: only the later rates carry an adjoint
#pragma unroll
    for (int j = JC + 1; j < NMAX; ++j)
        Xb[j] = active ? v.xb[static_cast<int64_t>(j - a.off) * g.n_paths + gid] : 0.0f;
    seed_caplet<NMAX, JC>(a, g, gl, active, w, X, Xb, accL0);
    bool any = false;
#pragma unroll
    for (int j = JC; j < NMAX; ++j) any = any || (Xb[j] != 0.0f);
    if (__any(any)) reverse_period<NMAX, JC>(a, g, m, gl, active, p_lo, p_hi, X, X1, Xb, accL0, accV);
    if (active) {
#pragma unroll
        for (int j = JC; j < NMAX; ++j) v.xb[static_cast<int64_t>(j - a.off) * g.n_paths + gid] = Xb[j];
    }
    double *out = v.part + (gid / kWave) * 2 * N;
    for (int j = JC; j < NMAX; ++j) {
        const double l0 =
            detail::wave_sum(active ? accL0[(j - JC) * kAdjBlock + lane] : 0.0f) * g.inv_L0[j];
        const double vv = detail::wave_sum(active ? accV[(j - JC) * kAdjBlock + lane] : 0.0f);
        if (lane == 0) {
            out[j - a.off] += l0;
            out[N + j - a.off] += vv;
        }
    }
}

// One launch per caplet (slot JC): each sweep is its own kernel so that its
// register allocation covers only its own live set.
template <int NMAX, int JC>
__global__ void __launch_bounds__(kAdjBlock) sweep_kernel(PathArgs<float> a, AdjArgs g) {
    // per-lane accumulators of the carried slots JC..NMAX-1 only (LDS bounds
    // the resident wavefronts of the long sweeps)
    __shared__ float accL0[(NMAX - JC) * kAdjBlock];
    __shared__ float accV[(NMAX - JC) * kAdjBlock];
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * kAdjBlock + threadIdx.x;
    const int64_t wave_first = gid - threadIdx.x;
    if (wave_first >= a.n_paths) return;
    sweep<NMAX, JC>(a, g, gid, gid < a.n_paths, accL0, accV);
}

template <int NMAX, int JC>
__global__ void __launch_bounds__(kAdjBlock) vjp_period_kernel(PathArgs<float> a, AdjArgs g,
                                                               VjpArgs v) {
    __shared__ float accL0[(NMAX - JC) * kAdjBlock];
    __shared__ float accV[(NMAX - JC) * kAdjBlock];
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * kAdjBlock + threadIdx.x;
    const int64_t wave_first = gid - threadIdx.x;
    if (wave_first >= a.n_paths) return;
    vjp_period<NMAX, JC>(a, g, v, gid, gid < a.n_paths, accL0, accV);
}

template <int NMAX, int PRODUCT>
__global__ void __launch_bounds__(kAdjBlock) forward_kernel(PathArgs<float> a, AdjArgs g) {
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * kAdjBlock + threadIdx.x;
    const int64_t wave_first = gid - threadIdx.x;
    if (wave_first >= a.n_paths) return;
    forward<NMAX, PRODUCT>(a, g, gid, gid < a.n_paths);
}

template <int NMAX, int JC>
hipError_t launch_one_sweep(dim3 grid, const PathArgs<float> &a, const AdjArgs &g, hipStream_t st) {
    hipLaunchKernelGGL((sweep_kernel<NMAX, JC>), grid, dim3(kAdjBlock), 0, st, a, g);
    return hipGetLastError();
}

template <int NMAX, int... Js>
hipError_t launch_sweep(std::integer_sequence<int, Js...>, int jc, dim3 grid,
                        const PathArgs<float> &a, const AdjArgs &g, hipStream_t st) {
    hipError_t e = hipErrorInvalidValue;
    (void)((jc == Js ? (e = launch_one_sweep<NMAX, Js>(grid, a, g, st), 0) : 0) + ...);
    return e;
}

template <int NMAX, int JC>
hipError_t launch_one_vjp(dim3 grid, const PathArgs<float> &a, const AdjArgs &g, const VjpArgs &v,
                          hipStream_t st) {
    hipLaunchKernelGGL((vjp_period_kernel<NMAX, JC>), grid, dim3(kAdjBlock), 0, st, a, g, v);
    return hipGetLastError();
}

template <int NMAX, int... Js>
hipError_t launch_vjp(std::integer_sequence<int, Js...>, int jc, dim3 grid, const PathArgs<float> &a,
                      const AdjArgs &g, const VjpArgs &v, hipStream_t st) {
    hipError_t e = hipErrorInvalidValue;
    (void)((jc == Js ? (e = launch_one_vjp<NMAX, Js>(grid, a, g, v, st), 0) : 0) + ...);
    return e;
}

template <int NMAX, int PRODUCT>
__global__ void __launch_bounds__(kBlock) forward_lds_kernel(PathArgs<float> a, AdjArgs g) {
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int64_t wave_first = gid - (threadIdx.x % kWave);
    if (wave_first >= a.n_paths) return;
    forward_lds<NMAX, PRODUCT>(a, g, gid, gid < a.n_paths);
}

template <int NMAX>
hipError_t launch_forward(dim3 grid, const PathArgs<float> &a, const AdjArgs &g, hipStream_t st) {
    if constexpr (detail::kStateInLds<float, NMAX, kFull>) {
        const dim3 lgrid(static_cast<unsigned>((a.n_paths + kBlock - 1) / kBlock));
        if (a.product == LLL_SWAPTIONS)
            hipLaunchKernelGGL((forward_lds_kernel<NMAX, LLL_SWAPTIONS>), lgrid, dim3(kBlock), 0, st,
                               a, g);
        else
            hipLaunchKernelGGL((forward_lds_kernel<NMAX, LLL_CAPLETS>), lgrid, dim3(kBlock), 0, st, a,
                               g);
    } else {
        if (a.product == LLL_SWAPTIONS)
            hipLaunchKernelGGL((forward_kernel<NMAX, LLL_SWAPTIONS>), grid, dim3(kAdjBlock), 0, st, a,
                               g);
        else
            hipLaunchKernelGGL((forward_kernel<NMAX, LLL_CAPLETS>), grid, dim3(kAdjBlock), 0, st, a, g);
    }
    return hipGetLastError();
}

// Forward pass with checkpoints, then the periods from the last to the first
// (v.w[m] = weight of product m times its price scale; v.part must be zero).
template <int NMAX>
hipError_t launch_vjp_bucket(const PathArgs<float> &a, const AdjArgs &g, const VjpArgs &v,
                             hipStream_t st) {
    const dim3 grid(static_cast<unsigned>((a.n_paths + kAdjBlock - 1) / kAdjBlock));
    hipError_t e = launch_forward<NMAX>(grid, a, g, st);
    for (int m = a.N - 1; m >= 0 && e == hipSuccess; --m)
        e = launch_vjp<NMAX>(std::make_integer_sequence<int, NMAX>{}, a.off + m, grid, a, g, v, st);
    return e;
}

// Forward pass with checkpoints, then one sweep launch per caplet.
template <int NMAX>
hipError_t launch_adjoint_bucket(const PathArgs<float> &a, const AdjArgs &g, hipStream_t st) {
    const dim3 grid(static_cast<unsigned>((a.n_paths + kAdjBlock - 1) / kAdjBlock));
    hipError_t e = launch_forward<NMAX>(grid, a, g, st);
    for (int c = 0; c < a.N && e == hipSuccess; ++c)
        e = launch_sweep<NMAX>(std::make_integer_sequence<int, NMAX>{}, a.off + c, grid, a, g, st);
    return e;
}

}  // namespace adj
}  // namespace lll
