// mlp_path.hip -- path kernel with the learned drift (and the first-order
// expansion alone), quadrature fallback and quadrature judge.
//
// Per Euler step the coupling of every live rate i is
//     C_i = C'_i + sigma * net(t, X_{l>i}, i)                (mlp.hpp)
// with C'_i = sum_{l>i} ell_l K2_{k,i,l}, K2_{k,i,l} = kappa(lambda_i + lambda_l)
// - kappa(lambda_i) - kappa(lambda_l) (paper Section 3.2, eq. (drifta)).  With
// use_net = 0 the kernel runs the first-order drift expansion alone.
//
// All three layers run on the matrix cores (v_mfma_f32_16x16x32_bf16, FP32
// accumulation) for the wavefront's 64 paths at once, as Z^T = W . H^T: the
// weights are the A operand (LDS, shared by the block), the activations the B
// operand, the accumulators start from the biases.  Layer 1 reads the BF16
// states from a per-wavefront LDS tile written once per step with the rates
// l <= i of the step's first coupled rate i zeroed; the rates are taken in
// ascending order and each zeroes one more column of the tile (its bias,
// b1 + the time column x t_k/T_N + rate i's one-hot column, is a per-(step,
// rate) table).  A lane's accumulator tile holds units 16 mt + 4 g + e of
// paths 16 nt + c (lane = 16 g + c); with the hidden units of the next layer's
// K dimension permuted accordingly (perm_unit), those GELU outputs are
// already that layer's B operand, so the hidden activations never leave the
// registers.  The output unit (64 -> 1) runs on the matrix cores as well: its
// FP32 weights split exactly into three BF16 terms (A operand rows 4 g + p),
// whose products with the BF16 activations are exact and summed in FP32.
// Nothing is shared between wavefronts inside the step loop.
//
// Fallback: a path whose later-rate state leaves the range seen in training
// (per rate) takes the 64-node quadrature coupling for that rate instead.
// Judge: every judge_stride-th wavefront also evaluates the quadrature at every
// step and records the surrogate's absolute and relative drift errors.
#include <hip/hip_runtime.h>

#include <utility>

#include "lll_device.hpp"
#include "lll_internal.hpp"
#include "mlp.hpp"
#define LLL_BUCKET_TU
#include "path_kernel.hpp"

namespace lll {
namespace mlp {
namespace {

using detail::cptr;
using detail::PathArgs;

constexpr int kSlots = kRates;  // the surrogate runs in the 40-slot bucket
constexpr int kNStat = 8;
constexpr int kLd = 72;         // padded row length (BF16) of the LDS tiles

struct MlpArgs {
    cptr<float> wf;     // FP32 parameter vector (biases, w4, b4)
    const float *wfv;   // the same, for per-lane loads
    const __bf16 *wbf;  // BF16 parameter vector
    cptr<float> K2;     // [K][40][40]
    cptr<float> lo;     // [40] trust box per slot
    cptr<float> hi;
    const float *B1;    // [K][40][64] first-layer bias of (step, rate)
    double *stats;      // [waves][kNStat]
    float sigma;
    int use_net;
    int judge_stride;
};

// Hidden unit behind K slot ks of a hidden layer's input: slot (kt, g, e) of
// lane group g holds the unit that group's accumulators produced for row
// tile mt = 2 kt + e / 4, element e % 4.
__host__ __device__ constexpr int perm_unit(int ks) {
    return 16 * (2 * (ks / 32) + (ks % 8) / 4) + 4 * ((ks % 32) / 8) + ks % 4;
}

// Orders this wavefront's LDS accesses across its lanes.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Term p (0, 1, 2) of the exact split of an FP32 weight into three BF16
// values, w = hi + mid + lo (each term takes the next 8 significant bits of
// what the previous ones leave; the differences are exact in FP32).
__device__ __forceinline__ __bf16 w4_term(float w, int p) {
    const __bf16 hi = static_cast<__bf16>(w);
    const float r1 = w - static_cast<float>(hi);
    const __bf16 mid = static_cast<__bf16>(r1);
    const __bf16 lo = static_cast<__bf16>(r1 - static_cast<float>(mid));
    return p == 0 ? hi : p == 1 ? mid : lo;
}

// Start of a step for the live slots J0..: the trust-box test of the state and
// the first-order couplings C_j = sum_{l>j} ell_l K2_{k,j,l} of every live rate.
template <int J0>
__device__ __forceinline__ void first_order(const PathArgs<float> &a, const MlpArgs &g, int k,
                                            const float (&X)[kSlots], float (&C)[kSlots],
                                            uint64_t &oob) {
    float ell[kSlots];
    oob = 0;
#pragma unroll
    for (int j = J0; j < kSlots; ++j) {
        ell[j] = detail::ell_of(X[j], a.cinv[j]);
        const bool out = (X[j] < g.lo[j]) || (X[j] > g.hi[j]);
        oob |= static_cast<uint64_t>(out) << j;
    }
    const cptr<float> K2k = g.K2 + (size_t)k * kSlots * kSlots;
#pragma unroll
    for (int j = J0; j < kSlots; ++j) {
        float c1 = 0.0f;
#pragma unroll
        for (int l = j + 1; l < kSlots; ++l) c1 = fmaf(ell[l], K2k[j * kSlots + l], c1);
        C[j] = c1;
    }
}

template <int... Js>
__device__ __forceinline__ void dispatch_first_order(std::integer_sequence<int, Js...>, int j0,
                                                     const PathArgs<float> &a, const MlpArgs &g,
                                                     int k, const float (&X)[kSlots],
                                                     float (&C)[kSlots], uint64_t &oob) {
    (void)((j0 == Js ? (first_order<Js>(a, g, k, X, C, oob), 0) : 0) + ...);
}

// Quadrature coupling for the judge and the fallback (ell recomputed from the
// state, which this step has not changed yet), then the state update.
template <int J0>
__device__ __forceinline__ void finish_step(const PathArgs<float> &a, int k, float dH,
                                            bool need_quad, bool judge, uint64_t oob,
                                            float (&C)[kSlots], float (&X)[kSlots],
                                            float (&st)[kNStat]) {
    if (need_quad) {
        float ell[kSlots], Cq[kSlots];
#pragma unroll
        for (int j = J0; j < kSlots; ++j) ell[j] = detail::ell_of(X[j], a.cinv[j]);
        detail::quad_coupling<float, kSlots, J0>(a.ew + (size_t)k * kQ * kSlots * 2, ell, Cq);
#pragma unroll
        for (int j = J0; j < kSlots; ++j) {
            if (judge) {
                const float e = fabsf(C[j] - Cq[j]);
                st[2] += 1.0f;
                st[3] += e;
                st[4] += fabsf(Cq[j]);
                if (Cq[j] != 0.0f) st[5] = fmaxf(st[5], e / fabsf(Cq[j]));
            }
            const bool fb = (oob >> (j + 1)) != 0;
            st[1] += fb ? 1.0f : 0.0f;
            C[j] = fb ? Cq[j] : C[j];
        }
    }
    const cptr<float> lamk = a.lam + (size_t)k * kSlots;
    const cptr<float> d0k = a.drift0 + (size_t)k * kSlots;
    const float dt = a.dt[k];
#pragma unroll
    for (int j = J0; j < kSlots; ++j) X[j] += fma(lamk[j], dH, fma(-C[j], dt, d0k[j]));
    st[0] += static_cast<float>(kSlots - J0);
}

template <int... Js>
__device__ __forceinline__ void dispatch_finish(std::integer_sequence<int, Js...>, int j0,
                                                const PathArgs<float> &a, int k, float dH,
                                                bool need_quad, bool judge, uint64_t oob,
                                                float (&C)[kSlots], float (&X)[kSlots],
                                                float (&st)[kNStat]) {
    (void)((j0 == Js ? (finish_step<Js>(a, k, dH, need_quad, judge, oob, C, X, st), 0) : 0) + ...);
}

// acc[mt] = the biases of this lane's units 16 mt + 4 grp + e (reloaded at
// every use, see layer2).
__device__ __forceinline__ void bias_init(const float *b, int grp, floatx4 (&acc)[4]) {
    __asm__ volatile("" ::: "memory");
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) acc[mt] = *reinterpret_cast<const floatx4 *>(b + 16 * mt + 4 * grp);
}

// B operands of the next layer from a finished accumulator tile: GELU, BF16,
// K slots (kt, grp, e) = units of row tiles 2 kt and 2 kt + 1.
__device__ __forceinline__ void activate(const floatx4 (&acc)[4], bf16x8 (&h)[2]) {
#pragma unroll
    for (int kt = 0; kt < 2; ++kt)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            h[kt][e] = static_cast<__bf16>(gelu(acc[2 * kt][e]));
            h[kt][4 + e] = static_cast<__bf16>(gelu(acc[2 * kt + 1][e]));
        }
}

// One layer for two column tiles (32 paths): acc[t][mt] += W[mt rows] . B[t].
// The weight fragments are read from LDS at every use: the compiler-only
// memory fence keeps them from being hoisted out of the rate loop, where the
// three layers' fragments would pin 96 registers.
__device__ __forceinline__ void layer2(const __bf16 *Wp, int lane, const bf16x8 (&B)[2][2],
                                       floatx4 (&acc)[2][4]) {
    __asm__ volatile("" ::: "memory");
#pragma unroll
    for (int kt = 0; kt < 2; ++kt)
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const bf16x8 w = *reinterpret_cast<const bf16x8 *>(
                Wp + (16 * mt + lane % 16) * kLd + 32 * kt + 8 * (lane / 16));
#pragma unroll
            for (int t = 0; t < 2; ++t) acc[t][mt] = mfma16(w, B[t][kt], acc[t][mt]);
        }
}

// Two wavefronts per SIMD (256 registers each, two 65 KiB blocks per CU): left
// to itself the compiler takes ~300 registers and one wavefront per SIMD,
// which ran the pass 1.6x slower at 2^20 paths.
template <int SCHEME>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2)))
mlp_path_kernel(PathArgs<float> a, MlpArgs g) {
    // 65 KiB: three padded weight tiles and the output unit's A operand
    // (shared), one state tile per wavefront
    __shared__ __attribute__((aligned(16))) __bf16 W1p[kHid * kLd];
    __shared__ __attribute__((aligned(16))) __bf16 W2p[kHid * kLd];
    __shared__ __attribute__((aligned(16))) __bf16 W3p[kHid * kLd];
    __shared__ __attribute__((aligned(16))) __bf16 W4p[16 * kLd];
    __shared__ __attribute__((aligned(16))) __bf16 Ft[kBlock / kWave][kWave * kLd];
    const int tid = threadIdx.x;
    for (int e = tid; e < kHid * kLd; e += kBlock) {
        const int o = e / kLd, ks = e % kLd;
        const __bf16 z = static_cast<__bf16>(0.0f);
        // layer 1's K slots are register slots: slot ks holds rate ks - off
        const int rate = ks - a.off;
        W1p[e] = (ks < kSlots && rate >= 0) ? g.wbf[kOffW1 + o * kIn + 1 + rate] : z;
        W2p[e] = (ks < kHid) ? g.wbf[kOffW2 + o * kHid + perm_unit(ks)] : z;
        W3p[e] = (ks < kHid) ? g.wbf[kOffW3 + o * kHid + perm_unit(ks)] : z;
    }
    for (int e = tid; e < 16 * kLd; e += kBlock) {
        const int row = e / kLd, ks = e % kLd;
        W4p[e] = (ks < kHid && row % 4 < 3) ? w4_term(g.wf[kOffW4 + perm_unit(ks)], row % 4)
                                            : static_cast<__bf16>(0.0f);
    }
    __syncthreads();  // the only block-wide barrier: the weights are read-only after it
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * kBlock + tid;
    const int lane = tid % kWave;
    const int grp = lane / 16;
    const int64_t wave = gid / kWave;
    if (gid - lane >= a.n_paths) return;  // whole wavefront past the end
    const bool active = gid < a.n_paths;
    const bool judge = g.judge_stride > 0 && (wave % g.judge_stride) == 0;
    const int64_t p = a.path_offset + gid;
    const uint32_t p_lo = static_cast<uint32_t>(p);
    const uint32_t p_hi = static_cast<uint32_t>(static_cast<uint64_t>(p) >> 32);
    __bf16 *F = Ft[tid / kWave];
    float X[kSlots];
#pragma unroll
    for (int j = 0; j < kSlots; ++j) X[j] = 0.0f;
    float st[kNStat];
#pragma unroll
    for (int i = 0; i < kNStat; ++i) st[i] = 0.0f;
    int m = 0, js = 0;
    const int K = a.N * a.s;
    for (int k = 0; k < K; ++k) {
        const cptr<double> sc = a.steps + 4 * m;
        const StepConsts cst{sc[0], sc[1], sc[2], sc[3]};
        const uint4 w = philox4x32_10(
            make_uint4(static_cast<uint32_t>(k), p_lo, p_hi, a.stream_word), a.key0, a.key1);
        const float dH = static_cast<float>(increment(w, cst, a.beta, false, nullptr));
        const int j0 = a.off + m;
        float C[kSlots];
        uint64_t oob = 0;
        dispatch_first_order(std::make_integer_sequence<int, kSlots>{}, j0, a, g, k, X, C, oob);
        // the last live slot has no later rate: its coupling stays exactly 0
        if (g.use_net && j0 < kSlots - 1) {
            // this lane's row of the state tile: BF16 X of slot l at column l for
            // the rates l > j0 (the features of the first coupled rate), zero
            // at the other columns
            wave_sync();  // the previous step's reads of the tile are done
#pragma unroll
            for (int c0 = 0; c0 < kSlots; c0 += 8) {
                bf16x8 v;
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    v[e] = static_cast<__bf16>(c0 + e > j0 ? X[c0 + e] : 0.0f);
                *reinterpret_cast<bf16x8 *>(F + lane * kLd + c0) = v;
            }
            *reinterpret_cast<bf16x8 *>(F + lane * kLd + 40) = bf16x8{};
            *reinterpret_cast<bf16x8 *>(F + lane * kLd + 48) = bf16x8{};
            *reinterpret_cast<bf16x8 *>(F + lane * kLd + 56) = bf16x8{};
            wave_sync();
            const float *B1k = g.B1 + (size_t)k * kRates * kHid;
            // rates in ascending slot order: after rate j the tile's column j + 1
            // is zeroed, so rate j + 1 reads exactly the states l > j + 1
            for (int j = j0; j < kSlots - 1; ++j) {
                const int r = j - a.off;
                float mine = 0.0f;
#pragma unroll 1
                for (int np = 0; np < 2; ++np) {
                    bf16x8 B[2][2];
                    floatx4 acc[2][4];
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        const int nt = 2 * np + t;
#pragma unroll
                        for (int kt = 0; kt < 2; ++kt)
                            B[t][kt] = *reinterpret_cast<const bf16x8 *>(
                                F + (16 * nt + lane % 16) * kLd + 32 * kt + 8 * grp);
                        bias_init(B1k + r * kHid, grp, acc[t]);
                    }
                    layer2(W1p, lane, B, acc);
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        activate(acc[t], B[t]);
                        bias_init(g.wfv + kOffB2, grp, acc[t]);
                    }
                    layer2(W2p, lane, B, acc);
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        activate(acc[t], B[t]);
                        bias_init(g.wfv + kOffB3, grp, acc[t]);
                    }
                    layer2(W3p, lane, B, acc);
#pragma unroll
                    for (int t = 0; t < 2; ++t) activate(acc[t], B[t]);
                    // output unit on the matrix cores: every lane group's rows
                    // 4 g + p hold term p of w4, so element p of a lane's
                    // accumulator is term p's dot product with the 64 units of
                    // path 16 nt + c; lane 16 grp + c keeps column tile grp
                    __asm__ volatile("" ::: "memory");
                    floatx4 out[2] = {floatx4{}, floatx4{}};
#pragma unroll
                    for (int kt = 0; kt < 2; ++kt) {
                        const bf16x8 w = *reinterpret_cast<const bf16x8 *>(
                            W4p + (lane % 16) * kLd + 32 * kt + 8 * grp);
#pragma unroll
                        for (int t = 0; t < 2; ++t) out[t] = mfma16(w, B[t][kt], out[t]);
                    }
#pragma unroll
                    for (int t = 0; t < 2; ++t)
                        mine = (grp == 2 * np + t) ? (out[t][0] + out[t][1]) + out[t][2] : mine;
                }
                const float sy = g.sigma * (g.wf[kOffB4] + mine);
#pragma unroll
                for (int jj = 0; jj < kSlots - 1; ++jj) C[jj] += (jj == j) ? sy : 0.0f;
                // the next rate's features leave out this lane's state at column j + 1
                F[lane * kLd + j + 1] = static_cast<__bf16>(0.0f);
                wave_sync();
            }
        }
        const bool need_quad = judge || __any((oob >> (j0 + 1)) != 0);
        dispatch_finish(std::make_integer_sequence<int, kSlots>{}, j0, a, k, dH, need_quad, judge,
                        oob, C, X, st);
        if (++js == a.s) {
            detail::dispatch_payoff<float, kSlots, detail::kAnyProduct>(std::make_integer_sequence<int, kSlots>{}, j0, a,
                                                   m, gid, active, X);
            js = 0;
            ++m;
        }
    }
    double tot[kNStat];
#pragma unroll
    for (int i = 0; i < kNStat; ++i) tot[i] = detail::wave_sum(active ? static_cast<double>(st[i]) : 0.0);
    double mx = active ? static_cast<double>(st[5]) : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, kWave));
    tot[5] = mx;
    if (lane == 0)
        for (int i = 0; i < kNStat; ++i) g.stats[wave * kNStat + i] = tot[i];
}

// Per-step tables of the surrogate: first-order coefficients K2 (FP64 -> FP32)
// and the first-layer bias of every (step, rate) -- b1 + the time column x
// t_k / T_N + the rate's one-hot column -- with the weights and the time
// feature BF16-rounded as in training.
__global__ void __launch_bounds__(64) mlp_tables_kernel(
    const double *__restrict__ tenor, const double *__restrict__ vol, int N, int s, int off,
    double alpha, double beta, double delta_nig, const float *__restrict__ wts,
    float *__restrict__ K2, float *__restrict__ B1) {
    const int k = blockIdx.x;
    const int t = threadIdx.x;
    const int m = k / s;
    const double *lam = vol + (size_t)k * N;
    for (int e = t; e < kSlots * kSlots; e += 64) {
        const int j = e / kSlots, l = e % kSlots;
        const int ri = j - off, rl = l - off;
        double v = 0.0;
        if (ri >= m && rl > ri)
            v = nig_cumulant(lam[ri] + lam[rl], alpha, beta, delta_nig) -
                nig_cumulant(lam[ri], alpha, beta, delta_nig) -
                nig_cumulant(lam[rl], alpha, beta, delta_nig);
        K2[(size_t)k * kSlots * kSlots + e] = static_cast<float>(v);
    }
    const double Ta = (m == 0) ? 0.0 : tenor[m - 1];
    const double tk = Ta + (k - m * s) * (tenor[m] - Ta) / s;
    const float tb = static_cast<float>(static_cast<__bf16>(static_cast<float>(tk / tenor[N - 1])));
    const float w0 = static_cast<float>(static_cast<__bf16>(wts[kOffW1 + t * kIn]));
    const float bt = fmaf(w0, tb, wts[kOffB1 + t]);
    for (int r = 0; r < kRates; ++r) {
        const float wi = static_cast<float>(static_cast<__bf16>(wts[kOffW1 + t * kIn + 1 + kRates + r]));
        B1[((size_t)k * kRates + r) * kHid + t] = bt + wi;
    }
}

}  // namespace

hipError_t launch_mlp_tables(const lll_plan &p, const float *wts, float *K2, float *B1,
                             hipStream_t st) {
    static_assert(kHid == 64, "one thread per hidden unit");
    hipLaunchKernelGGL(mlp_tables_kernel, dim3(p.K), dim3(64), 0, st, p.d.tenor, p.d.vol, p.N, p.s,
                       p.off, p.alpha, p.beta, p.delta_nig, wts, K2, B1);
    return hipGetLastError();
}

hipError_t launch_mlp_paths(const lll_plan &p, const float *wts, const __bf16 *wbf,
                            const float *K2, const float *B1, const float *box, float sigma,
                            int use_net, int judge_stride, int64_t n_paths, uint64_t seed,
                            double *path_fix, double *stats, hipStream_t st) {
    if (p.nmax != kSlots) return hipErrorInvalidValue;
    PathArgs<float> a = detail::make_args<float>(p, seed, n_paths, 0, path_fix);
    MlpArgs g;
    g.wf = detail::as_const(wts);
    g.wfv = wts;
    g.wbf = wbf;
    g.K2 = detail::as_const(K2);
    // the trust box arrays are per rate; the kernel indexes them by slot
    g.lo = detail::as_const(box) - p.off;
    g.hi = detail::as_const(box + kRates) - p.off;
    g.B1 = B1;
    g.stats = stats;
    g.sigma = sigma;
    g.use_net = use_net;
    g.judge_stride = judge_stride;
    const dim3 grid(static_cast<unsigned>((n_paths + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(mlp_path_kernel<kFull>, grid, dim3(kBlock), 0, st, a, g);
    return hipGetLastError();
}

}  // namespace mlp
}  // namespace lll
