// mlp_path.hip -- path kernel with the learned drift (and the first-order
// expansion alone), quadrature fallback and quadrature judge.
//
// Per Euler step the coupling of every live rate i is
//     C_i = C'_i + sigma * net(t, X_{l>i}, i)                (mlp.hpp)
// with C'_i = sum_{l>i} ell_l K2_{k,i,l}, K2_{k,i,l} = kappa(lambda_i + lambda_l)
// - kappa(lambda_i) - kappa(lambda_l) (paper Section 3.2, eq. (drifta)).  With
// use_net = 0 the kernel runs the first-order drift expansion alone.
//
// The network's first layer is a suffix sum over the rates (the features of
// rate i are the states of the rates l > i), so it costs 64 FMAs per rate plus
// one add of a per-(step, rate) bias table (b1 + the time and one-hot
// columns); the two hidden 64x64 layers run on the matrix cores for the
// wave's 64 paths at once: Z^T = W . H^T with W from LDS (shared by the
// block) and H staged per wave in LDS, v_mfma_f32_16x16x32_bf16, FP32
// accumulation.  The state X and the couplings C live in LDS columns (one per
// thread), so a rate's state and coupling are addressed by the loop index
// without register selects.  Nothing is shared between wavefronts inside the
// step loop, so the waves synchronise only with themselves.
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

struct MlpArgs {
    cptr<float> W1T;    // [96][64] first layer, transposed (BF16-rounded values)
    cptr<float> wf;     // FP32 parameter vector (biases, w4, b4)
    const __bf16 *W2;   // [64][64]
    const __bf16 *W3;   // [64][64]
    cptr<float> K2;     // [K][40][40]
    cptr<float> lo;     // [40] trust box per slot
    cptr<float> hi;
    cptr<float> B1;     // [K][40][64] first-layer bias of (step, rate)
    double *stats;      // [waves][kNStat]
    float sigma;
    int use_net;
    int judge_stride;
};

// LDS of one wavefront's LDS-resident per-lane state: column `lane` of
// [slot][kWave] arrays.
struct LaneLds {
    float *x;  // X_j at x[j * kWave]
    float *c;  // C_j at c[j * kWave]
};

// Orders this wavefront's LDS accesses across lanes (all LDS data used inside
// the step loop is private to the wavefront).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int J0>
__device__ __forceinline__ void ell_and_box(const PathArgs<float> &a, const MlpArgs &g,
                                            const LaneLds &s, float (&ell)[kSlots], uint64_t &oob) {
    oob = 0;
#pragma unroll
    for (int j = 0; j < kSlots; ++j) {
        if (j >= J0) {
            const float x = s.x[j * kWave];
            ell[j] = detail::ell_of(x, a.cinv[j]);
            const bool out = (x < g.lo[j]) || (x > g.hi[j]);
            oob |= static_cast<uint64_t>(out) << j;
        } else {
            ell[j] = 0.0f;
        }
    }
}

template <int... Js>
__device__ __forceinline__ void dispatch_ell(std::integer_sequence<int, Js...>, int j0,
                                             const PathArgs<float> &a, const MlpArgs &g,
                                             const LaneLds &s, float (&ell)[kSlots], uint64_t &oob) {
    (void)((j0 == Js ? (ell_and_box<Js>(a, g, s, ell, oob), 0) : 0) + ...);
}

// Quadrature coupling for the judge and the fallback, plus the state update.
template <int J0>
__device__ __forceinline__ void finish_step(const PathArgs<float> &a, const MlpArgs &g, int k,
                                            float dH, bool need_quad, bool judge, uint64_t oob,
                                            const float (&ell)[kSlots], const LaneLds &s,
                                            float (&st)[kNStat]) {
    float C[kSlots];
#pragma unroll
    for (int j = J0; j < kSlots; ++j) C[j] = s.c[j * kWave];
    if (need_quad) {
        float Cq[kSlots];
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
    for (int j = J0; j < kSlots; ++j) s.x[j * kWave] += fma(lamk[j], dH, fma(-C[j], dt, d0k[j]));
    st[0] += static_cast<float>(kSlots - J0);
}

template <int... Js>
__device__ __forceinline__ void dispatch_finish(std::integer_sequence<int, Js...>, int j0,
                                                const PathArgs<float> &a, const MlpArgs &g, int k,
                                                float dH, bool need_quad, bool judge, uint64_t oob,
                                                const float (&ell)[kSlots], const LaneLds &s,
                                                float (&st)[kNStat]) {
    (void)((j0 == Js ? (finish_step<Js>(a, g, k, dH, need_quad, judge, oob, ell, s, st), 0)
                     : 0) + ...);
}

// One hidden 64x64 layer for the wave's 64 paths: Hout[m][o] = gelu(sum_k W[o][k] Hin[m][k] + b[o]).
__device__ __forceinline__ void hidden_layer(const __bf16 *Ws, const __bf16 *Hin, cptr<float> b,
                                             __bf16 *Hout, int lane) {
#pragma unroll 1
    for (int mt = 0; mt < 4; ++mt) {
        floatx4 acc[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[nt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int kt = 0; kt < 2; ++kt) {
            const int k0 = 32 * kt + 8 * (lane / 16);
            const bf16x8 av = *reinterpret_cast<const bf16x8 *>(Ws + (16 * mt + lane % 16) * kHid + k0);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const bf16x8 bv =
                    *reinterpret_cast<const bf16x8 *>(Hin + (16 * nt + lane % 16) * kHid + k0);
                acc[nt] = mfma16(av, bv, acc[nt]);
            }
        }
        const int o0 = 16 * mt + 4 * (lane / 16);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const int m = 16 * nt + lane % 16;
            typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
            bf16x4 h;
#pragma unroll
            for (int e = 0; e < 4; ++e) h[e] = static_cast<__bf16>(gelu(acc[nt][e] + b[o0 + e]));
            *reinterpret_cast<bf16x4 *>(Hout + m * kHid + o0) = h;
        }
    }
}

template <int SCHEME>
__global__ void __launch_bounds__(kBlock) mlp_path_kernel(PathArgs<float> a, MlpArgs g) {
    // 160 KiB: the weights (16 KiB), two activation tiles per wavefront
    // (64 KiB) and the per-lane state and coupling columns (2 x 40 KiB)
    __shared__ __attribute__((aligned(16))) __bf16 W2s[kHid * kHid];
    __shared__ __attribute__((aligned(16))) __bf16 W3s[kHid * kHid];
    __shared__ __attribute__((aligned(16))) __bf16 Hb[kBlock / kWave][2][kWave * kHid];
    __shared__ float Xs[kBlock / kWave][kSlots * kWave];
    __shared__ float Cs[kBlock / kWave][kSlots * kWave];
    const int tid = threadIdx.x;
    for (int e = tid; e < kHid * kHid; e += kBlock) {
        W2s[e] = g.W2[e];
        W3s[e] = g.W3[e];
    }
    __syncthreads();  // the only block-wide barrier: the weights are read-only after it
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * kBlock + tid;
    const int lane = tid % kWave;
    const int wv = tid / kWave;
    const int64_t wave = gid / kWave;
    if (gid - lane >= a.n_paths) return;  // whole wavefront past the end
    const bool active = gid < a.n_paths;
    const bool judge = g.judge_stride > 0 && (wave % g.judge_stride) == 0;
    const int64_t p = a.path_offset + gid;
    const uint32_t p_lo = static_cast<uint32_t>(p);
    const uint32_t p_hi = static_cast<uint32_t>(static_cast<uint64_t>(p) >> 32);
    __bf16 *H0 = Hb[wv][0];
    __bf16 *H1 = Hb[wv][1];
    const LaneLds s{Xs[wv] + lane, Cs[wv] + lane};
    const cptr<float> b2 = g.wf + kOffB2;
    const cptr<float> b3 = g.wf + kOffB3;
#pragma unroll
    for (int j = 0; j < kSlots; ++j) s.x[j * kWave] = 0.0f;
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
        float ell[kSlots];
        uint64_t oob = 0;
        dispatch_ell(std::make_integer_sequence<int, kSlots>{}, j0, a, g, s, ell, oob);
        float S[kHid];
#pragma unroll
        for (int h = 0; h < kHid; ++h) S[h] = 0.0f;
        const cptr<float> K2k = g.K2 + (size_t)k * kSlots * kSlots;
        const cptr<float> B1k = g.B1 + (size_t)k * kRates * kHid;
        for (int j = kSlots - 1; j >= j0; --j) {
            const int r = j - a.off;
            // first-order expansion
            float c1 = 0.0f;
            const cptr<float> K2row = K2k + j * kSlots;
#pragma unroll
            for (int jj = 0; jj < kSlots; ++jj) c1 = fmaf(ell[jj], K2row[jj], c1);
            float y = 0.0f;
            // the last live slot has no later rate: its coupling is exactly 0
            if (g.use_net && j < kSlots - 1) {
                // layer 1 from the suffix sum of the later rates
                const cptr<float> bias = B1k + r * kHid;
                __bf16 *row = H0 + lane * kHid;
#pragma unroll
                for (int h = 0; h < kHid; h += 8) {
                    bf16x8 v;
#pragma unroll
                    for (int e = 0; e < 8; ++e) v[e] = static_cast<__bf16>(gelu(S[h + e] + bias[h + e]));
                    *reinterpret_cast<bf16x8 *>(row + h) = v;
                }
                wave_sync();
                hidden_layer(W2s, H0, b2, H1, lane);
                wave_sync();
                hidden_layer(W3s, H1, b3, H0, lane);
                wave_sync();
                y = g.wf[kOffB4];
#pragma unroll
                for (int h = 0; h < kHid; h += 8) {
                    const bf16x8 v = *reinterpret_cast<const bf16x8 *>(row + h);
#pragma unroll
                    for (int e = 0; e < 8; ++e) y = fmaf(g.wf[kOffW4 + h + e], static_cast<float>(v[e]), y);
                }
                wave_sync();  // row is rewritten by the next rate
            }
            if (g.use_net) {
                // this rate's state joins the suffix sum of the next (lower) rate,
                // rounded as the BF16 features are
                const float xj = static_cast<float>(static_cast<__bf16>(s.x[j * kWave]));
                const cptr<float> wx = g.W1T + (1 + r) * kHid;
#pragma unroll
                for (int h = 0; h < kHid; ++h) S[h] = fmaf(wx[h], xj, S[h]);
            }
            s.c[j * kWave] = fmaf(g.sigma, y, c1);
        }
        const bool need_quad = judge || __any((oob >> (j0 + 1)) != 0);
        dispatch_finish(std::make_integer_sequence<int, kSlots>{}, j0, a, g, k, dH, need_quad,
                        judge, oob, ell, s, st);
        if (++js == a.s) {
            float X[kSlots];
#pragma unroll
            for (int j = 0; j < kSlots; ++j) X[j] = s.x[j * kWave];
            detail::dispatch_payoff<float, kSlots>(std::make_integer_sequence<int, kSlots>{}, j0, a,
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

// Per-step tables of the surrogate: first-order coefficients K2 (FP64 -> FP32),
// the first-layer bias of every (step, rate) -- b1 + the time column x t_k / T_N
// + the rate's one-hot column -- and the transposed first layer, with the
// weights and the time feature BF16-rounded as in training.
__global__ void __launch_bounds__(64) mlp_tables_kernel(
    const double *__restrict__ tenor, const double *__restrict__ vol, int N, int s, int off,
    double alpha, double beta, double delta_nig, const float *__restrict__ wts,
    float *__restrict__ K2, float *__restrict__ B1, float *__restrict__ W1T) {
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
    if (k == 0)
        for (int e = t; e < kIn * kHid; e += 64) {
            const int c = e / kHid, h = e % kHid;
            W1T[e] = static_cast<float>(static_cast<__bf16>(wts[kOffW1 + h * kIn + c]));
        }
}

}  // namespace

hipError_t launch_mlp_tables(const lll_plan &p, const float *wts, float *K2, float *B1,
                             float *W1T, hipStream_t st) {
    static_assert(kHid == 64, "one thread per hidden unit");
    hipLaunchKernelGGL(mlp_tables_kernel, dim3(p.K), dim3(64), 0, st, p.d.tenor, p.d.vol, p.N, p.s,
                       p.off, p.alpha, p.beta, p.delta_nig, wts, K2, B1, W1T);
    return hipGetLastError();
}

hipError_t launch_mlp_paths(const lll_plan &p, const float *wts, const __bf16 *wbf,
                            const float *K2, const float *B1, const float *W1T,
                            const float *box, float sigma, int use_net, int judge_stride,
                            int64_t n_paths, uint64_t seed, double *path_fix, double *stats,
                            hipStream_t st) {
    if (p.nmax != kSlots) return hipErrorInvalidValue;
    PathArgs<float> a = detail::make_args<float>(p, seed, n_paths, 0, path_fix);
    MlpArgs g;
    g.W1T = detail::as_const(W1T);
    g.wf = detail::as_const(wts);
    g.W2 = wbf + kOffW2;
    g.W3 = wbf + kOffW3;
    g.K2 = detail::as_const(K2);
    g.lo = detail::as_const(box);
    g.hi = detail::as_const(box + kRates);
    g.B1 = detail::as_const(B1);
    g.stats = stats;
    g.sigma = sigma;
    g.use_net = use_net;
    g.judge_stride = judge_stride;
    // the trust box arrays are per rate; the kernel indexes them by slot
    g.lo = g.lo - p.off;
    g.hi = g.hi - p.off;
    const dim3 grid(static_cast<unsigned>((n_paths + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(mlp_path_kernel<kFull>, grid, dim3(kBlock), 0, st, a, g);
    return hipGetLastError();
}

}  // namespace mlp
}  // namespace lll
