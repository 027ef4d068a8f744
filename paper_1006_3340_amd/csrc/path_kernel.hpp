// path_kernel.hpp -- the Monte Carlo path kernel (templates, one bucket per TU).
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
//      (FULL) or of the Picard iterate X1 (PICARD, eq. (bdrift): the kernel
//      carries that ell itself from step to step, see pred_init);
//   4. the coupling C_i = sum_q W_q E_{i,q} (prod_{l>i} beta_l(x_q) - 1) by a
//      suffix recursion over the rates, node by node:
//          C_i += W_q E_{i,q} R_q,   R_q <- R_q + ell_i E_{i,q} (1 + R_q),
//      which is the product of eq. (LIBOR-drift-PT) with beta_l = 1 + ell_l E_l
//      evaluated once for all i (O(N Q) per step instead of O(N^2 Q));
//      the uniform table entries (E, W E) are wave-uniform scalar operands;
//   5. X_i += (-kappa_i - C_i) dt + lambda_i dH (PICARD also advances its
//      iterate by b0_i dt + lambda_i dH; FROZEN advances only X with b0);
//   6. at the end of period m the rate with maturity T_{m+1} fixes: the FP64
//      payoffs prod_{l>i}(1 + delta_l L_l)(L_i - K)^+ of eq. (caplet) and the
//      martingale factor are summed across the wavefront (butterfly), and lane
//      0 writes the wave's sums; a two-pass fixed-order FP64 reduction follows.
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

#include "lll_device.hpp"
#include "lll_internal.hpp"

namespace lll {
namespace detail {

// Read-only tables are addressed through the constant address space: they are
// not written while a path kernel runs, so wave-uniform reads of them become
// scalar loads whose results are SGPR operands of the vector FMAs.
template <typename T>
using cptr = const __attribute__((address_space(4))) T *;

template <typename T>
__host__ __device__ inline cptr<T> as_const(const T *p) {
    return (cptr<T>)(p);
}

template <typename Real>
struct PathArgs {
    cptr<Real> ew;         // [K][Q][nmax][2]
    cptr<Real> lam;        // [K][nmax]
    cptr<Real> drift0;     // [K][nmax]
    cptr<Real> frozen;     // [K][nmax]
    cptr<Real> dt;         // [K]
    cptr<Real> cinv;       // [nmax]
    cptr<Real> k2;         // [K][nmax][nmax] first-order coefficients, or null
    cptr<double> L0s;      // [nmax]
    cptr<double> deltas;   // [nmax]
    cptr<double> strikes;  // [N][S]
    cptr<double> steps;    // [N][4]
    double *__restrict__ partials;     // [waves][N][NSTAT]
    double *__restrict__ path_fix;     // [n_paths][2N] or null
    int64_t n_paths, path_offset;
    int N, s, S, off, brownian, product;
    uint32_t stream_word, key0, key1;
    double beta, c;
};

__device__ __forceinline__ float ell_of(float x, float cinv) {
    // delta L / (1 + delta L) = 1 / (1 + e^{-X} / (delta L0))
    return __builtin_amdgcn_rcpf(fmaf(cinv, __expf(-x), 1.0f));
}
__device__ __forceinline__ double ell_of(double x, double cinv) {
    return 1.0 / fma(cinv, exp(-x), 1.0);
}

// ell after the state moves by d: with L' = L e^d, ell' = delta L' / (1 + delta L')
// = ell / (ell + (1 - ell) e^{-d}).  PICARD carries the predictor's ell this
// way instead of its state, which saves one register per rate.
__device__ __forceinline__ float ell_advance(float ell, float d) {
    const float e = __expf(-d);
    return ell * __builtin_amdgcn_rcpf(fmaf(ell, 1.0f - e, e));
}
__device__ __forceinline__ double ell_advance(double ell, double d) {
    const double e = exp(-d);
    return ell / fma(ell, 1.0 - e, e);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Coupling sums C[j], j = J0 .. nmax-2, of the jump drift for the live slots
// J0 .. nmax-1 at step k (row = table of step k).  C[nmax-1] = 0.
template <typename Real, int NMAX, int J0>
__device__ __forceinline__ void quad_coupling(cptr<Real> row, const Real (&ell)[NMAX],
                                              Real (&C)[NMAX]) {
#pragma unroll
    for (int j = J0; j < NMAX; ++j) C[j] = Real(0);
    if constexpr (J0 < NMAX - 1) {
        for (int q = 0; q < kQ; ++q, row += NMAX * 2) {
            Real R = ell[NMAX - 1] * row[2 * (NMAX - 1)];
#pragma unroll
            for (int j = NMAX - 2; j >= J0; --j) {
                const Real E = row[2 * j];
                const Real WE = row[2 * j + 1];
                C[j] = fma(WE, R, C[j]);
                if (j > J0) R = fma(ell[j], fma(E, R, E), R);
            }
        }
    }
}

// Brownian driver: C_i = c lambda_i sum_{l>i} ell_l lambda_l.
template <typename Real, int NMAX, int J0>
__device__ __forceinline__ void brownian_coupling(cptr<Real> lamk, Real cR,
                                                  const Real (&ell)[NMAX], Real (&C)[NMAX]) {
    Real S = Real(0);
#pragma unroll
    for (int j = NMAX - 1; j >= J0; --j) {
        const Real lj = lamk[j];
        C[j] = cR * lj * S;
        S = fma(ell[j], lj, S);
    }
}

// First-order expansion of the coupling (Section 3.2, eq. (drifta)):
// C_j = sum_{l>j} ell_l K2_{k,j,l}, K2 = kappa(lambda_j + lambda_l) - kappa(lambda_j)
// - kappa(lambda_l) from the step's table (wave-uniform scalar operands).
template <typename Real, int NMAX, int J0>
__device__ __forceinline__ void first_order_coupling(cptr<Real> k2k, const Real (&ell)[NMAX],
                                                     Real (&C)[NMAX]) {
#pragma unroll
    for (int j = J0; j < NMAX; ++j) {
        Real c = Real(0);
#pragma unroll
        for (int l = j + 1; l < NMAX; ++l) c = fma(ell[l], k2k[j * NMAX + l], c);
        C[j] = c;
    }
}

// Second-order expansion of the coupling (Section 3.2, eq. (drifta2)): the
// product prod_{l>i}(1 + ell_l E_l) truncated after its terms of degree 2 in
// ell, e1 + e2 (elementary symmetric sums of the ell_l E_l, l > i), integrated
// with the same 64-node rule.  Per node, from the top slot down, with
// u = 1 + e1 and s = e1 + e2 of the slots above j:
//     C_j += W E_j s,   t = ell_j E_j,   s += t u,   u += t.
template <typename Real, int NMAX, int J0>
__device__ __forceinline__ void quad_coupling2(cptr<Real> row, const Real (&ell)[NMAX],
                                               Real (&C)[NMAX]) {
#pragma unroll
    for (int j = J0; j < NMAX; ++j) C[j] = Real(0);
    if constexpr (J0 < NMAX - 1) {
        for (int q = 0; q < kQ; ++q, row += NMAX * 2) {
            Real t = ell[NMAX - 1] * row[2 * (NMAX - 1)];
            Real s = t;
            Real u = Real(1) + t;
#pragma unroll
            for (int j = NMAX - 2; j >= J0; --j) {
                const Real E = row[2 * j];
                const Real WE = row[2 * j + 1];
                C[j] = fma(WE, s, C[j]);
                if (j > J0) {
                    t = ell[j] * E;
                    s = fma(t, u, s);
                    u = u + t;
                }
            }
        }
    }
}

// Coupling sums of the scheme: the first-order expansion, the Brownian
// closed form (exact, hence also the second-order expansion), the truncated
// product or the full product on the 64-node rule.
template <typename Real, int NMAX, int SCHEME, int J0>
__device__ __forceinline__ void coupling(const PathArgs<Real> &a, int k, const Real (&ell)[NMAX],
                                         Real (&C)[NMAX]) {
    if constexpr (SCHEME == kFirst)
        first_order_coupling<Real, NMAX, J0>(a.k2 + (size_t)k * NMAX * NMAX, ell, C);
    else if (a.brownian)
        brownian_coupling<Real, NMAX, J0>(a.lam + (size_t)k * NMAX, static_cast<Real>(a.c), ell, C);
    else if constexpr (SCHEME == kSecond)
        quad_coupling2<Real, NMAX, J0>(a.ew + (size_t)k * kQ * NMAX * 2, ell, C);
    else
        quad_coupling<Real, NMAX, J0>(a.ew + (size_t)k * kQ * NMAX * 2, ell, C);
}

// PICARD's predictor (the frozen-drift path, paper Section 3.1) enters the
// drift only through its ell, so the kernels carry that ell per slot (pred,
// initialised by pred_init) and move it by each step's frozen-drift
// increment with ell_advance.  The other schemes leave pred alone.
template <typename Real, int NMAX, int SCHEME>
__device__ __forceinline__ void pred_init(const PathArgs<Real> &a, Real (&pred)[NMAX]) {
#pragma unroll
    for (int j = 0; j < NMAX; ++j)
        pred[j] = SCHEME == kPicard ? ell_of(Real(0), a.cinv[j]) : Real(0);
}

// One Euler step for the live slots J0 .. NMAX-1 (drift and state update).
template <typename Real, int NMAX, int SCHEME, int J0>
__device__ __forceinline__ void step(const PathArgs<Real> &a, int k, Real dH, Real (&X)[NMAX],
                                     Real (&pred)[NMAX]) {
    const cptr<Real> lamk = a.lam + (size_t)k * NMAX;
    const cptr<Real> frzk = a.frozen + (size_t)k * NMAX;
    if constexpr (SCHEME == kFrozen) {
#pragma unroll
        for (int j = J0; j < NMAX; ++j) X[j] += fma(lamk[j], dH, frzk[j]);
    } else {
        Real ell[NMAX];
#pragma unroll
        for (int j = J0; j < NMAX; ++j)
            ell[j] = SCHEME == kPicard ? pred[j] : ell_of(X[j], a.cinv[j]);
        Real C[NMAX];
        coupling<Real, NMAX, SCHEME, J0>(a, k, ell, C);
        const Real dt = a.dt[k];
        const cptr<Real> d0k = a.drift0 + (size_t)k * NMAX;
#pragma unroll
        for (int j = J0; j < NMAX; ++j) {
            const Real lam = lamk[j];
            X[j] += fma(lam, dH, fma(-C[j], dt, d0k[j]));
            if constexpr (SCHEME == kPicard) pred[j] = ell_advance(pred[j], fma(lam, dH, frzk[j]));
        }
    }
}

// Payoff before the positive part of strike K at the fixing of rate r:
// swaption (Q - 1) - K A, caplet D (L_r - K) (quantities as in fixing_sums).
__device__ __forceinline__ double payoff_value(bool swaption, double K, double Q, double A,
                                              double D, double Lc) {
    return swaption ? (Q - 1.0) - K * A : D * (Lc - K);
}

// Wavefront sums (FP64) of the payoffs of the fixing of rate r, given
// Q = prod_{l>=r}(1 + delta_l L_l), A = sum_{l>=r} delta_l prod_{j>l}(1 + delta_j L_j),
// D = prod_{l>r}(1 + delta_l L_l) and L_r: per strike the sum, the sum of
// squares and the count of positive payoffs, then the martingale factor Q.
template <typename Real>
__device__ __forceinline__ void fixing_sums(const PathArgs<Real> &a, int r, int64_t gid,
                                            bool active, bool swaption, double Q, double A,
                                            double D, double Lc) {
    if (!swaption && a.path_fix != nullptr && active) {
        a.path_fix[gid * 2 * a.N + 2 * r] = Lc;
        a.path_fix[gid * 2 * a.N + 2 * r + 1] = D;
    }
    const int S = a.S;
    double *out = a.partials + ((size_t)(gid / kWave) * a.N + r) * (3 * S + 2);
    const bool lane0 = (threadIdx.x % kWave) == 0;
    for (int t = 0; t < S; ++t) {
        const double K = a.strikes[r * S + t];
        const double v = payoff_value(swaption, K, Q, A, D, Lc);
        const double pay = active ? fmax(v, 0.0) : 0.0;
        const double s1 = wave_sum(pay);
        const double s2 = wave_sum(pay * pay);
        const double ni = wave_sum((active && v > 0.0) ? 1.0 : 0.0);
        if (lane0) {
            out[t] = s1;
            out[S + t] = s2;
            out[2 * S + t] = ni;
        }
    }
    const double M = active ? Q : 0.0;
    const double m1 = wave_sum(M);
    const double m2 = wave_sum(M * M);
    if (lane0) {
        out[3 * S] = m1;
        out[3 * S + 1] = m2;
    }
}

// Product of a kernel: LLL_CAPLETS or LLL_SWAPTIONS fixed at compile time (the
// plain path kernels, so each carries only its own payoff code), or read from
// the arguments (kAnyProduct: the batched and surrogate kernels).
constexpr int kAnyProduct = -1;

// Payoffs at the end of period m (the rate in slot J0 fixes), in units of the
// terminal bond, and the martingale factor M = prod_{l>=c}(1 + delta_l L_l),
// summed over the wavefront; FP64.  Caplets: D (L_c - K)^+ with
// D = prod_{l>c}(1 + delta_l L_l).  Co-terminal payer swaptions: the swap's
// value sum_{l>=c} delta_l (L_l - K) Q_l with Q_l = prod_{j>l}(1 + delta_j L_j);
// its floating leg telescopes, sum_{l>=c} delta_l L_l Q_l = M - 1, and its
// fixed leg is K A with A = sum_{l>=c} delta_l Q_l.
template <typename Real, int NMAX, int J0>
__device__ __forceinline__ void caplet_payoff(const PathArgs<Real> &a, int m, int64_t gid,
                                              bool active, const Real (&X)[NMAX]) {
    const int r = m;  // caplet on the rate with maturity T_{m+1}
    double D = 1.0;
#pragma unroll
    for (int j = J0 + 1; j < NMAX; ++j)
        D *= 1.0 + a.deltas[j] * a.L0s[j] * static_cast<double>(exp(X[j]));
    const double Lc = a.L0s[J0] * static_cast<double>(exp(X[J0]));
    if (a.path_fix != nullptr && active) {
        a.path_fix[gid * 2 * a.N + 2 * r] = Lc;
        a.path_fix[gid * 2 * a.N + 2 * r + 1] = D;
    }
    const int S = a.S;
    const int nstat = 3 * S + 2;
    const int64_t wave = gid / kWave;
    double *out = a.partials + ((size_t)wave * a.N + r) * nstat;
    const bool lane0 = (threadIdx.x % kWave) == 0;
    for (int t = 0; t < S; ++t) {
        const double K = a.strikes[r * S + t];
        const double pay = active ? D * fmax(Lc - K, 0.0) : 0.0;
        const double s1 = wave_sum(pay);
        const double s2 = wave_sum(pay * pay);
        const double ni = wave_sum((active && Lc > K) ? 1.0 : 0.0);
        if (lane0) {
            out[t] = s1;
            out[S + t] = s2;
            out[2 * S + t] = ni;
        }
    }
    const double M = active ? D * (1.0 + a.deltas[J0] * Lc) : 0.0;
    const double m1 = wave_sum(M);
    const double m2 = wave_sum(M * M);
    if (lane0) {
        out[3 * S] = m1;
        out[3 * S + 1] = m2;
    }
}

template <typename Real, int NMAX, int J0, int PRODUCT>
__device__ __forceinline__ void payoff(const PathArgs<Real> &a, int m, int64_t gid, bool active,
                                       const Real (&X)[NMAX]) {
    if constexpr (PRODUCT == LLL_CAPLETS) {
        caplet_payoff<Real, NMAX, J0>(a, m, gid, active, X);
        return;
    }
    // Same arithmetic as payoff_lds (so the kernels that read the product at
    // run time reproduce the LDS kernels bit for bit): one pass from the last
    // rate down, Q = prod_{j>l}(1 + delta_j L_j) before slot l is multiplied
    // in; D = Q at slot J0, M = Q at the end.
    const int r = m;  // the rate with maturity T_{m+1}
    const bool swaption =
        PRODUCT == kAnyProduct ? a.product == LLL_SWAPTIONS : PRODUCT == LLL_SWAPTIONS;
    double Q = 1.0, A = 0.0, D = 1.0, Lc = 0.0;
#pragma unroll
    for (int j = NMAX - 1; j >= J0; --j) {
        const double L = a.L0s[j] * static_cast<double>(exp(X[j]));
        if (j == J0) {
            D = Q;
            Lc = L;
        }
        A = fma(a.deltas[j], Q, A);
        Q *= 1.0 + a.deltas[j] * L;
    }
    fixing_sums(a, r, gid, active, swaption, Q, A, D, Lc);
}

// Payoffs of the LDS-state kernels: the state is read from the thread's LDS
// column (slot stride STRIDE) slot by slot in a loop, so no register copy of
// all slots (whose unrolled FP64 products would otherwise set the kernel's
// register count: 86 -> 58 VGPRs for FULL at 24 slots).  Same quantities as
// payoff(): Q, A, D and L_r of fixing_sums.
template <typename Real, int NMAX, int STRIDE = kBlock>
__device__ __forceinline__ void fixing_quantities_lds(const PathArgs<Real> &a, const Real *xs,
                                                      int j0, double &Q, double &A, double &D,
                                                      double &Lc) {
    Q = 1.0;
    A = 0.0;
    D = 1.0;
    Lc = 0.0;
    for (int j = NMAX - 1; j >= j0; --j) {
        const double L = a.L0s[j] * static_cast<double>(exp(xs[j * STRIDE]));
        if (j == j0) {
            D = Q;
            Lc = L;
        }
        A = fma(a.deltas[j], Q, A);
        Q *= 1.0 + a.deltas[j] * L;
    }
}

template <typename Real, int NMAX, int PRODUCT>
__device__ __forceinline__ void payoff_lds(const PathArgs<Real> &a, int m, int64_t gid,
                                           bool active, const Real *xs, int j0) {
    const bool swaption =
        PRODUCT == kAnyProduct ? a.product == LLL_SWAPTIONS : PRODUCT == LLL_SWAPTIONS;
    double Q, A, D, Lc;
    fixing_quantities_lds<Real, NMAX>(a, xs, j0, Q, A, D, Lc);
    fixing_sums(a, m, gid, active, swaption, Q, A, D, Lc);
}

// The same step with the state X held in LDS (column `xs`, stride kBlock) for
// the wide buckets: X is read twice and written once per step, while ell and
// the coupling sums stay in registers.  A compiler-only fence keeps the second
// read from being merged with the first, which would pin X in registers
// across the node loop again.
template <typename Real, int NMAX, int SCHEME, int J0>
__device__ __forceinline__ void step_lds(const PathArgs<Real> &a, int k, Real dH, Real *xs,
                                         Real (&pred)[NMAX]) {
    const cptr<Real> lamk = a.lam + (size_t)k * NMAX;
    const cptr<Real> frzk = a.frozen + (size_t)k * NMAX;
    Real ell[NMAX];
#pragma unroll
    for (int j = J0; j < NMAX; ++j)
        ell[j] = SCHEME == kPicard ? pred[j] : ell_of(xs[j * kBlock], a.cinv[j]);
    __asm__ volatile("" ::: "memory");
    Real C[NMAX];
    coupling<Real, NMAX, SCHEME, J0>(a, k, ell, C);
    const Real dt = a.dt[k];
    const cptr<Real> d0k = a.drift0 + (size_t)k * NMAX;
    // each slot's table entries (lambda, -kappa dt, b0 dt) are used together,
    // so few of them are live in scalar registers at once
#pragma unroll
    for (int j = J0; j < NMAX; ++j) {
        const Real lam = lamk[j];
        xs[j * kBlock] += fma(lam, dH, fma(-C[j], dt, d0k[j]));
        if constexpr (SCHEME == kPicard) pred[j] = ell_advance(pred[j], fma(lam, dH, frzk[j]));
    }
}

template <typename Real, int NMAX, int SCHEME, int... Js>
__device__ __forceinline__ void dispatch_step_lds(std::integer_sequence<int, Js...>, int j0,
                                                  const PathArgs<Real> &a, int k, Real dH,
                                                  Real *xs, Real (&pred)[NMAX]) {
    (void)((j0 == Js ? (step_lds<Real, NMAX, SCHEME, Js>(a, k, dH, xs, pred), 0) : 0) + ...);
}

template <typename Real, int NMAX, int SCHEME, int... Js>
__device__ __forceinline__ void dispatch_step(std::integer_sequence<int, Js...>, int j0,
                                              const PathArgs<Real> &a, int k, Real dH,
                                              Real (&X)[NMAX], Real (&pred)[NMAX]) {
    (void)((j0 == Js ? (step<Real, NMAX, SCHEME, Js>(a, k, dH, X, pred), 0) : 0) + ...);
}

template <typename Real, int NMAX, int PRODUCT, int... Js>
__device__ __forceinline__ void dispatch_payoff(std::integer_sequence<int, Js...>, int j0,
                                                const PathArgs<Real> &a, int m, int64_t gid,
                                                bool active, const Real (&X)[NMAX]) {
    (void)((j0 == Js ? (payoff<Real, NMAX, Js, PRODUCT>(a, m, gid, active, X), 0) : 0) + ...);
}

// The block's LDS state, [slot][thread]: one allocation per kernel that uses
// it, NMAX slots (the batched kernel, whose structures differ in N).
template <typename Real, int NMAX>
__device__ __forceinline__ Real *state_lds() {
    __shared__ Real sX[NMAX * kBlock];
    return sX;
}

// The path kernel's LDS state: rows for the structure's N rates only (slot j
// in row j - off), sized at launch (N x 256 x 4 B), so that N = 20 in the
// 24-slot bucket takes 20 KB per block, not 24 KB: 8 blocks per CU instead
// of 6.  Returns the thread's column, indexed by slot (slots >= off only).
template <typename Real>
__device__ __forceinline__ Real *state_lds_dynamic(int off) {
    extern __shared__ __attribute__((aligned(16))) unsigned char lll_state_dyn[];
    return reinterpret_cast<Real *>(lll_state_dyn) + threadIdx.x - off * kBlock;
}

template <typename Real, int NMAX, int SCHEME, int PRODUCT>
__device__ __forceinline__ void simulate_lds(const PathArgs<Real> &a, int64_t gid, Real *xs) {
    const bool active = gid < a.n_paths;
    const int64_t p = a.path_offset + gid;
    const uint32_t p_lo = static_cast<uint32_t>(p);
    const uint32_t p_hi = static_cast<uint32_t>(static_cast<uint64_t>(p) >> 32);
    const bool brownian = a.brownian != 0;
    Real pred[NMAX];
    pred_init<Real, NMAX, SCHEME>(a, pred);
#pragma unroll
    for (int j = 0; j < NMAX; ++j)
        if (j >= a.off) xs[j * kBlock] = Real(0);
    int m = 0, js = 0;
    const int K = a.N * a.s;
    for (int k = 0; k < K; ++k) {
        const cptr<double> sc = a.steps + 4 * m;
        const StepConsts cst{sc[0], sc[1], sc[2], sc[3]};
        const uint4 w = philox4x32_10(
            make_uint4(static_cast<uint32_t>(k), p_lo, p_hi, a.stream_word), a.key0, a.key1);
        const Real dH = static_cast<Real>(increment(w, cst, a.beta, brownian, nullptr));
        const int j0 = a.off + m;
        dispatch_step_lds<Real, NMAX, SCHEME>(std::make_integer_sequence<int, NMAX>{}, j0, a, k, dH,
                                              xs, pred);
        if (++js == a.s) {
            payoff_lds<Real, NMAX, PRODUCT>(a, m, gid, active, xs, j0);
            js = 0;
            ++m;
        }
    }
}

// FP32 FULL / PICARD kernels of the 24- to 40-slot buckets keep X in LDS
// (NMAX x 256 x 4 B per block): with X, ell and the coupling sums all in
// registers they need 100-180 VGPRs, one wavefront per SIMD fewer than with X
// in LDS (measured: N = 20 FULL 22.7 -> 21.2 ms, N = 40 FULL 50.0 -> 42.7 ms,
// N = 40 PICARD 70.6 -> 58.0 ms at 2^20 paths).
template <typename Real, int NMAX, int SCHEME>
constexpr bool kStateInLds = sizeof(Real) == 4 && NMAX >= 20 && SCHEME != kFrozen;

// Simulates path `gid` (0-based within the structure; lanes past n_paths run
// but contribute nothing) through all periods, writing the wave's payoff sums.
// Every lane of the wavefront must call this together (wave reductions), and
// every thread of the block index its own LDS column (threadIdx.x < kBlock).
// ALLOW_LDS = false keeps the state in registers; PRODUCT is LLL_CAPLETS,
// LLL_SWAPTIONS or kAnyProduct (see payoff).
template <typename Real, int NMAX, int SCHEME, bool ALLOW_LDS, int PRODUCT, bool DYN_LDS = false>
__device__ __forceinline__ void simulate(const PathArgs<Real> &a, int64_t gid) {
    if constexpr (ALLOW_LDS && kStateInLds<Real, NMAX, SCHEME>) {
        if constexpr (DYN_LDS)
            simulate_lds<Real, NMAX, SCHEME, PRODUCT>(a, gid, state_lds_dynamic<Real>(a.off));
        else
            simulate_lds<Real, NMAX, SCHEME, PRODUCT>(a, gid, state_lds<Real, NMAX>() + threadIdx.x);
        return;
    }
    const bool active = gid < a.n_paths;
    const int64_t p = a.path_offset + gid;
    const uint32_t p_lo = static_cast<uint32_t>(p);
    const uint32_t p_hi = static_cast<uint32_t>(static_cast<uint64_t>(p) >> 32);
    const bool brownian = a.brownian != 0;
    Real X[NMAX], pred[NMAX];
    pred_init<Real, NMAX, SCHEME>(a, pred);
#pragma unroll
    for (int j = 0; j < NMAX; ++j) X[j] = Real(0);
    int m = 0, js = 0;
    const int K = a.N * a.s;
    for (int k = 0; k < K; ++k) {
        const cptr<double> sc = a.steps + 4 * m;
        const StepConsts cst{sc[0], sc[1], sc[2], sc[3]};
        const uint4 w = philox4x32_10(
            make_uint4(static_cast<uint32_t>(k), p_lo, p_hi, a.stream_word), a.key0, a.key1);
        const Real dH = static_cast<Real>(increment(w, cst, a.beta, brownian, nullptr));
        const int j0 = a.off + m;
        dispatch_step<Real, NMAX, SCHEME>(std::make_integer_sequence<int, NMAX>{}, j0, a, k, dH, X,
                                          pred);
        if (++js == a.s) {
            dispatch_payoff<Real, NMAX, PRODUCT>(std::make_integer_sequence<int, NMAX>{}, j0, a, m, gid,
                                        active, X);
            js = 0;
            ++m;
        }
    }
}

// LDS state (dynamic, launch_scheme sizes it by N) for the wide FP32
// buckets, registers otherwise.
template <typename Real, int NMAX, int SCHEME, int PRODUCT>
__global__ void __launch_bounds__(kBlock) path_kernel(PathArgs<Real> a) {
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int64_t wave_first = gid - (threadIdx.x % kWave);
    if (wave_first >= a.n_paths) return;  // whole wavefront past the end
    simulate<Real, NMAX, SCHEME, true, PRODUCT, true>(a, gid);
}

// Drift of the live rates at step k for given rate vectors (inspection): the
// same coupling code as the path kernel, one state per lane.
template <typename Real, int NMAX, int J0>
__device__ void drift_one(const PathArgs<Real> &a, int k, const double *__restrict__ L,
                          const double *__restrict__ kappa, double *__restrict__ b) {
    Real ell[NMAX], C[NMAX];
#pragma unroll
    for (int j = J0; j < NMAX; ++j) {
        const int r = j - a.off;
        const Real x = static_cast<Real>(log(L[r] / a.L0s[j]));
        ell[j] = ell_of(x, a.cinv[j]);
    }
    if (a.brownian)
        brownian_coupling<Real, NMAX, J0>(a.lam + (size_t)k * NMAX, static_cast<Real>(a.c), ell, C);
    else
        quad_coupling<Real, NMAX, J0>(a.ew + (size_t)k * kQ * NMAX * 2, ell, C);
#pragma unroll
    for (int j = J0; j < NMAX; ++j) {
        const int r = j - a.off;
        b[r] = -kappa[(size_t)k * a.N + r] - static_cast<double>(C[j]);
    }
}

template <typename Real, int NMAX, int... Js>
__device__ void dispatch_drift(std::integer_sequence<int, Js...>, int j0, const PathArgs<Real> &a,
                               int k, const double *L, const double *kappa, double *b) {
    (void)((j0 == Js ? (drift_one<Real, NMAX, Js>(a, k, L, kappa, b), 0) : 0) + ...);
}

template <typename Real, int NMAX>
__global__ void __launch_bounds__(kBlock) drift_kernel(PathArgs<Real> a, int k,
                                                       const double *__restrict__ L,
                                                       const double *__restrict__ kappa,
                                                       double *__restrict__ b, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    const int m = k / a.s;
    for (int r = 0; r < a.N; ++r) b[i * a.N + r] = 0.0;
    dispatch_drift<Real, NMAX>(std::make_integer_sequence<int, NMAX>{}, a.off + m, a, k,
                               L + i * a.N, kappa, b + i * a.N);
}

template <typename Real>
inline PathArgs<Real> make_args(const lll_plan &p, uint64_t seed, int64_t n_paths, int64_t path_offset,
                         double *path_fix) {
    const DeviceTables &d = p.d;
    PathArgs<Real> a;
    a.ew = as_const(static_cast<const Real *>(d.ew));
    a.lam = as_const(static_cast<const Real *>(d.lam));
    a.drift0 = as_const(static_cast<const Real *>(d.drift0));
    a.frozen = as_const(static_cast<const Real *>(d.frozen));
    a.dt = as_const(static_cast<const Real *>(d.dt));
    a.cinv = as_const(static_cast<const Real *>(d.cinv));
    a.k2 = as_const(static_cast<const Real *>(d.k2));
    a.L0s = as_const<double>(d.L0s);
    a.deltas = as_const<double>(d.deltas);
    a.strikes = as_const<double>(d.strikes);
    a.steps = as_const<double>(d.steps);
    a.partials = d.partials;
    a.path_fix = path_fix;
    a.n_paths = n_paths;
    a.path_offset = path_offset;
    a.N = p.N;
    a.s = p.s;
    a.S = p.S;
    a.off = p.off;
    a.brownian = p.driver == LLL_DRIVER_BROWNIAN;
    a.product = p.product;
    a.stream_word = p.struct_id & 0xFFFFFFu;
    a.key0 = static_cast<uint32_t>(seed & 0xFFFFFFFFull);
    a.key1 = static_cast<uint32_t>(seed >> 32);
    a.beta = p.beta;
    a.c = p.c;
    return a;
}

// Dynamic LDS of path_kernel<Real, NMAX, SCHEME>: the state rows of the N rates.
template <typename Real, int NMAX, int SCHEME>
size_t state_lds_bytes(const PathArgs<Real> &a) {
    return kStateInLds<Real, NMAX, SCHEME> ? size_t(a.N) * kBlock * sizeof(Real) : 0;
}

template <typename Real, int NMAX, int PRODUCT, int SCHEME>
void launch_one_scheme(const PathArgs<Real> &a, dim3 grid, hipStream_t st) {
    const size_t lds = state_lds_bytes<Real, NMAX, SCHEME>(a);
    hipLaunchKernelGGL((path_kernel<Real, NMAX, SCHEME, PRODUCT>), grid, dim3(kBlock), lds, st, a);
}

template <typename Real, int NMAX, int PRODUCT>
void launch_scheme(const PathArgs<Real> &a, int scheme, dim3 grid, hipStream_t st) {
    switch (scheme) {
        case kFull: launch_one_scheme<Real, NMAX, PRODUCT, kFull>(a, grid, st); break;
        case kPicard: launch_one_scheme<Real, NMAX, PRODUCT, kPicard>(a, grid, st); break;
        case kFirst: launch_one_scheme<Real, NMAX, PRODUCT, kFirst>(a, grid, st); break;
        case kSecond: launch_one_scheme<Real, NMAX, PRODUCT, kSecond>(a, grid, st); break;
        default: launch_one_scheme<Real, NMAX, PRODUCT, kFrozen>(a, grid, st); break;
    }
}

template <typename Real, int NMAX>
hipError_t launch_paths_n(const PathArgs<Real> &a, int scheme, int64_t n_paths, hipStream_t st) {
    const dim3 grid(static_cast<unsigned>((n_paths + kBlock - 1) / kBlock));
    if (a.product == LLL_SWAPTIONS)
        launch_scheme<Real, NMAX, LLL_SWAPTIONS>(a, scheme, grid, st);
    else
        launch_scheme<Real, NMAX, LLL_CAPLETS>(a, scheme, grid, st);
    return hipGetLastError();
}

template <typename Real, int NMAX>
hipError_t launch_drift_n(const PathArgs<Real> &a, int k, const double *L, const double *kappa,
                          double *b, int64_t n, hipStream_t st) {
    const dim3 grid(static_cast<unsigned>((n + kBlock - 1) / kBlock));
    hipLaunchKernelGGL((drift_kernel<Real, NMAX>), grid, dim3(kBlock), 0, st, a, k, L, kappa, b, n);
    return hipGetLastError();
}

// Launchers of one bucket.  Each (Real, NMAX) pair is instantiated in its
// own translation unit (bucket_*.hip) so that the buckets compile in parallel.
template <typename Real, int NMAX>
hipError_t launch_bucket(const lll_plan &p, int scheme, int64_t n_paths, int64_t path_offset,
                         uint64_t seed, double *path_fix, hipStream_t st) {
    return launch_paths_n<Real, NMAX>(make_args<Real>(p, seed, n_paths, path_offset, path_fix),
                                      scheme, n_paths, st);
}

template <typename Real, int NMAX>
hipError_t launch_drift_bucket(const lll_plan &p, int k, const double *L, int64_t n, double *b,
                               hipStream_t st) {
    return launch_drift_n<Real, NMAX>(make_args<Real>(p, 0, 0, 0, nullptr), k, L, p.d.kappa, b, n,
                                      st);
}

#define LLL_BUCKET_DECL(EXT, REAL, NMAX)                                                          \
    EXT template hipError_t launch_bucket<REAL, NMAX>(const lll_plan &, int, int64_t, int64_t,   \
                                                      uint64_t, double *, hipStream_t);          \
    EXT template hipError_t launch_drift_bucket<REAL, NMAX>(const lll_plan &, int,               \
                                                            const double *, int64_t, double *,   \
                                                            hipStream_t);

#define LLL_BUCKET_LIST(X)                                                                        \
    X(float, 8) X(float, 16) X(float, 20) X(float, 24) X(float, 32) X(float, 40) X(double, 8)    \
        X(double, 16) X(double, 24)

#define LLL_BUCKET_EXTERN(REAL, NMAX) LLL_BUCKET_DECL(extern, REAL, NMAX)
#ifndef LLL_BUCKET_TU
LLL_BUCKET_LIST(LLL_BUCKET_EXTERN)
#endif

}  // namespace detail
}  // namespace lll
