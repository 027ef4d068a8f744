// mlp_train.hip -- data generation, BF16-MFMA forward/backward and Adam for
// the drift surrogate (layout and target in mlp.hpp).
//
// Training data: FULL paths (their own random stream, Philox tag 1) record
// their state at a staggered set of steps; for every recorded state and live
// rate i an FP64 kernel forms the features and the label
//     (C_i - C'_i), C_i = sum_q W_q E_{i,q} (prod_{l>i}(1 + ell_l E_{l,q}) - 1)
// (the quadrature coupling of eq. (LIBOR-drift-PT)) and C'_i its first-order
// expansion (eq. (drifta)).  Training: minibatches drawn with replacement by
// Philox (tag 2); one block of 256 threads per 64 samples runs the three
// hidden layers forward and backward on v_mfma_f32_16x16x32_bf16 and writes
// its gradient; a second kernel sums the block gradients in a fixed order and
// applies Adam to the FP32 master weights, refreshing their BF16 copies.
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

constexpr int kTile = 64;      // samples per block
constexpr int kTrainBlock = 256;

// ---------------------------------------------------------------- data ----

// FULL paths recording their state (all NMAX slots; fixed rates 0) at steps
// k_r = r * (K / R) + (p mod (K / R)), r = 0..R-1.
template <int NMAX>
__global__ void __launch_bounds__(kBlock) record_kernel(PathArgs<float> a, int R,
                                                        float *__restrict__ states,
                                                        int *__restrict__ kidx) {
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int64_t wave_first = gid - (threadIdx.x % kWave);
    if (wave_first >= a.n_paths) return;
    const bool active = gid < a.n_paths;
    const int64_t p = a.path_offset + gid;
    const uint32_t p_lo = static_cast<uint32_t>(p);
    const uint32_t p_hi = static_cast<uint32_t>(static_cast<uint64_t>(p) >> 32);
    const int K = a.N * a.s;
    const int stride = K / R;
    const int phase = static_cast<int>(gid % stride);
    float X[NMAX], X1[NMAX];
#pragma unroll
    for (int j = 0; j < NMAX; ++j) {
        X[j] = 0.0f;
        X1[j] = 0.0f;
    }
    int r = 0;
    for (int k = 0; k < K; ++k) {
        const int m = k / a.s;
        const int j0 = a.off + m;
        if (r < R && k == r * stride + phase) {   // divergent: per-lane phase
            if (active) {
                float *dst = states + (gid * R + r) * NMAX;
#pragma unroll
                for (int j = 0; j < NMAX; ++j) dst[j] = (j >= j0) ? X[j] : 0.0f;
                kidx[gid * R + r] = k;
            }
            ++r;
        }
        const cptr<double> sc = a.steps + 4 * m;
        const StepConsts cst{sc[0], sc[1], sc[2], sc[3]};
        const uint4 w = philox4x32_10(
            make_uint4(static_cast<uint32_t>(k), p_lo, p_hi, a.stream_word), a.key0, a.key1);
        const float dH = static_cast<float>(increment(w, cst, a.beta, false, nullptr));
        detail::dispatch_step<float, NMAX, kFull>(std::make_integer_sequence<int, NMAX>{}, j0, a,
                                                  k, dH, X, X1);
    }
}

// FP64 labels and BF16 features of every live rate of one recorded state.
__global__ void __launch_bounds__(64) label_kernel(
    const float *__restrict__ states, const int *__restrict__ kidx, const int64_t *__restrict__ poff,
    int64_t n_states, int nmax, int off, int N, int s, const double *__restrict__ tenor,
    const double *__restrict__ delta, const double *__restrict__ L0, const double *__restrict__ vol,
    const double *__restrict__ E, const double *__restrict__ w, double alpha, double beta,
    double delta_nig, __bf16 *__restrict__ feat, float *__restrict__ label) {
    const int64_t st = static_cast<int64_t>(blockIdx.x) * 64 + threadIdx.x;
    if (st >= n_states) return;
    const int k = kidx[st];
    const int first = k / s;
    const float *X = states + st * nmax;
    const double *lam = vol + (size_t)k * N;
    const double t = (first == 0 ? 0.0 : tenor[first - 1]) +
                     (k - first * s) * (tenor[first] - (first == 0 ? 0.0 : tenor[first - 1])) / s;
    const double tn = t / tenor[N - 1];
    double ell[kRates], C[kRates];
    for (int r = first; r < N; ++r) {
        const double L = L0[r] * exp(static_cast<double>(X[r + off]));
        ell[r] = delta[r] * L / (1.0 + delta[r] * L);
        C[r] = 0.0;
    }
    for (int q = 0; q < kQ; ++q) {
        double R = 0.0;
        for (int r = N - 1; r >= first; --r) {
            const double e = E[((size_t)k * N + r) * kQ + q];
            C[r] += w[q] * e * R;
            R += ell[r] * e * (1.0 + R);
        }
    }
    int64_t pi = poff[st];
    for (int i = first; i < N; ++i, ++pi) {
        double c1 = 0.0;
        const double ki = nig_cumulant(lam[i], alpha, beta, delta_nig);
        for (int l = i + 1; l < N; ++l)
            c1 += ell[l] * (nig_cumulant(lam[i] + lam[l], alpha, beta, delta_nig) - ki -
                            nig_cumulant(lam[l], alpha, beta, delta_nig));
        label[pi] = static_cast<float>(C[i] - c1);
        __bf16 *f = feat + pi * kIn;
        for (int c = 0; c < kIn; ++c) f[c] = static_cast<__bf16>(0.0f);
        f[0] = static_cast<__bf16>(static_cast<float>(tn));
        for (int l = i + 1; l < N; ++l) f[1 + l] = static_cast<__bf16>(X[l + off]);
        f[1 + kRates + i] = static_cast<__bf16>(1.0f);
    }
}

// Per-slot range of the state over the data (the surrogate's trust box) and
// the root mean square of the labels; one block, fixed reduction order.
__global__ void __launch_bounds__(256) stats_kernel(const float *__restrict__ states,
                                                    const int *__restrict__ kidx, int64_t n_states,
                                                    int nmax, int off, int s,
                                                    const float *__restrict__ label,
                                                    int64_t n_pairs, float *__restrict__ out) {
    __shared__ float lo[256], hi[256];
    __shared__ double ss[256];
    const int t = threadIdx.x;
    for (int r = 0; r < kRates; ++r) {
        const int j = r + off;
        float l = 3.0e38f, h = -3.0e38f;
        if (j < nmax)
            for (int64_t st = t; st < n_states; st += 256) {
                if (kidx[st] / s > r) continue;  // rate already fixed in this state
                const float v = states[st * nmax + j];
                l = fminf(l, v);
                h = fmaxf(h, v);
            }
        lo[t] = l;
        hi[t] = h;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (t < o) {
                lo[t] = fminf(lo[t], lo[t + o]);
                hi[t] = fmaxf(hi[t], hi[t + o]);
            }
            __syncthreads();
        }
        if (t == 0) {
            out[r] = lo[0];
            out[kRates + r] = hi[0];
        }
        __syncthreads();
    }
    double acc = 0.0;
    for (int64_t p = t; p < n_pairs; p += 256) acc += static_cast<double>(label[p]) * label[p];
    ss[t] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) ss[t] += ss[t + o];
        __syncthreads();
    }
    if (t == 0) out[2 * kRates] = static_cast<float>(sqrt(ss[0] / static_cast<double>(n_pairs)));
}

// ------------------------------------------------------------ training ----

__global__ void __launch_bounds__(256) init_kernel(float *__restrict__ wts, __bf16 *__restrict__ wbf,
                                                   float *__restrict__ adam, uint32_t key0,
                                                   uint32_t key1) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= kParams) return;
    float a = 0.0f;
    if (p < kOffB1) a = sqrtf(6.0f / (kIn + kHid));
    else if (p >= kOffW2 && p < kOffB2) a = sqrtf(6.0f / (2 * kHid));
    else if (p >= kOffW3 && p < kOffB3) a = sqrtf(6.0f / (2 * kHid));
    else if (p >= kOffW4 && p < kOffB4) a = sqrtf(6.0f / (kHid + 1));
    const uint4 r = philox4x32_10(make_uint4(static_cast<uint32_t>(p), 0u, 0u, 2u << 24), key0, key1);
    const float u = static_cast<float>(uniform24(r.x));
    const float v = a * (2.0f * u - 1.0f);
    wts[p] = v;
    wbf[p] = static_cast<__bf16>(v);
    adam[p] = 0.0f;
    adam[kParams + p] = 0.0f;
}

__global__ void __launch_bounds__(256) batch_index_kernel(int *__restrict__ idx, int B,
                                                          int64_t n_pairs, uint32_t step,
                                                          uint32_t key0, uint32_t key1) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= B) return;
    const uint4 r = philox4x32_10(make_uint4(step, static_cast<uint32_t>(j), 1u, 2u << 24), key0, key1);
    const uint64_t x = (static_cast<uint64_t>(r.x) << 32) | r.y;
    idx[j] = static_cast<int>(x % static_cast<uint64_t>(n_pairs));
}

struct TileArgs {
    const __bf16 *feat;   // [P][96]
    const float *target;  // [P] raw labels (scaled by inv_sigma here)
    const int *idx;       // [B] sample indices, or null for rows 0..B-1
    int B;
    float inv_sigma;
    float inv_B;
    const __bf16 *wbf;    // BF16 copy of the parameter vector
    const float *wf;      // FP32 parameter vector
    float *gpart;         // [tiles][kParams] or null (forward only)
    float *lpart;         // [tiles] loss partials or null
    float *yout;          // [B] outputs (normalised units) or null
};

__device__ __forceinline__ bf16x8 frag_contig(const __bf16 *p) {
    bf16x8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = p[e];
    return v;
}
__device__ __forceinline__ bf16x8 frag_strided(const __bf16 *p, int stride) {
    bf16x8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = p[e * stride];
    return v;
}
__device__ __forceinline__ bf16x8 frag_f32_contig(const float *p) {
    bf16x8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = static_cast<__bf16>(p[e]);
    return v;
}
__device__ __forceinline__ bf16x8 frag_f32_strided(const float *p, int stride) {
    bf16x8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = static_cast<__bf16>(p[e * stride]);
    return v;
}

// One hidden layer forward for the block's 64 samples: Z^T = W . H^T (+ b),
// wave w computes hidden units 16w .. 16w+15 for all 64 samples.
template <int KIN>
__device__ __forceinline__ void layer_fwd(const __bf16 *Ws, const __bf16 *Hin, const float *bias,
                                          float *Zout, __bf16 *Hout) {
    const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
    floatx4 acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kt = 0; kt < KIN / 32; ++kt) {
        const int k0 = 32 * kt + 8 * (lane / 16);
        const bf16x8 a = frag_contig(Ws + (16 * w + lane % 16) * KIN + k0);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const bf16x8 b = frag_contig(Hin + (16 * nt + lane % 16) * KIN + k0);
            acc[nt] = mfma16(a, b, acc[nt]);
        }
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int o = 16 * w + 4 * (lane / 16) + e, m = 16 * nt + lane % 16;
            const float z = acc[nt][e] + bias[o];
            Zout[m * kHid + o] = z;
            Hout[m * kHid + o] = static_cast<__bf16>(gelu(z));
        }
}

// dW[o][i] = sum_m dZ[m][o] Hin[m][i] for the block; wave w rows o = 16w..,
// NT column tiles of 16; written to the block's gradient slice.
template <int NT, int HSTRIDE>
__device__ __forceinline__ void weight_grad(const float *dZ, const __bf16 *Hin, float *g) {
    const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
    floatx4 acc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[nt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kt = 0; kt < kTile / 32; ++kt) {
        const int m0 = 32 * kt + 8 * (lane / 16);
        const bf16x8 a = frag_f32_strided(dZ + m0 * kHid + 16 * w + lane % 16, kHid);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const bf16x8 b = frag_strided(Hin + m0 * HSTRIDE + 16 * nt + lane % 16, HSTRIDE);
            acc[nt] = mfma16(a, b, acc[nt]);
        }
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int o = 16 * w + 4 * (lane / 16) + e, i = 16 * nt + lane % 16;
            g[o * HSTRIDE + i] = acc[nt][e];
        }
}

// dH^T[i][m] = sum_o W[o][i] dZ[m][o]; returns the wave's 4 tiles
// (i = 16w + 4(lane/16) + e, m = 16nt + lane%16).
__device__ __forceinline__ void input_grad(const __bf16 *Ws, const float *dZ, floatx4 (&acc)[4]) {
    const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kt = 0; kt < kHid / 32; ++kt) {
        const int o0 = 32 * kt + 8 * (lane / 16);
        const bf16x8 a = frag_strided(Ws + o0 * kHid + 16 * w + lane % 16, kHid);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const bf16x8 b = frag_f32_contig(dZ + (16 * nt + lane % 16) * kHid + o0);
            acc[nt] = mfma16(a, b, acc[nt]);
        }
    }
}

__global__ void __launch_bounds__(kTrainBlock) tile_kernel(TileArgs t) {
    __shared__ __bf16 Xs[kTile * kIn];
    __shared__ __bf16 W1s[kHid * kIn];
    __shared__ __bf16 W2s[kHid * kHid];
    __shared__ __bf16 W3s[kHid * kHid];
    __shared__ __bf16 Hs[3][kTile * kHid];
    __shared__ float Zs[3][kTile * kHid];
    __shared__ float dZ[kTile * kHid];
    __shared__ float dyS[kTile];
    __shared__ float red[kTile];
    const int tid = threadIdx.x;
    const int lane = tid % 64, w = tid / 64;
    const int64_t row0 = static_cast<int64_t>(blockIdx.x) * kTile;
    const float *wf = t.wf;
    for (int e = tid; e < kTile * kIn; e += kTrainBlock) {
        const int m = e / kIn, c = e % kIn;
        const int64_t r = row0 + m;
        __bf16 v = static_cast<__bf16>(0.0f);
        if (r < t.B) {
            const int64_t smp = t.idx ? t.idx[r] : r;
            v = t.feat[smp * kIn + c];
        }
        Xs[e] = v;
    }
    for (int e = tid; e < kHid * kIn; e += kTrainBlock) W1s[e] = t.wbf[kOffW1 + e];
    for (int e = tid; e < kHid * kHid; e += kTrainBlock) {
        W2s[e] = t.wbf[kOffW2 + e];
        W3s[e] = t.wbf[kOffW3 + e];
    }
    __syncthreads();
    layer_fwd<kIn>(W1s, Xs, wf + kOffB1, Zs[0], Hs[0]);
    __syncthreads();
    layer_fwd<kHid>(W2s, Hs[0], wf + kOffB2, Zs[1], Hs[1]);
    __syncthreads();
    layer_fwd<kHid>(W3s, Hs[1], wf + kOffB3, Zs[2], Hs[2]);
    __syncthreads();
    if (tid < kTile) {
        const int64_t r = row0 + tid;
        const bool valid = r < t.B;
        float y = wf[kOffB4];
        for (int o = 0; o < kHid; ++o) y = fmaf(wf[kOffW4 + o], static_cast<float>(Hs[2][tid * kHid + o]), y);
        float target = 0.0f;
        if (valid) {
            const int64_t smp = t.idx ? t.idx[r] : r;
            target = t.target[smp] * t.inv_sigma;
            if (t.yout) t.yout[r] = y;
        }
        const float d = valid ? (y - target) : 0.0f;
        dyS[tid] = d * t.inv_B;
        red[tid] = 0.5f * d * d * t.inv_B;
    }
    __syncthreads();
    if (t.lpart && tid == 0) {
        float s = 0.0f;
        for (int m = 0; m < kTile; ++m) s += red[m];
        t.lpart[blockIdx.x] = s;
    }
    if (!t.gpart) return;
    float *g = t.gpart + static_cast<int64_t>(blockIdx.x) * kParams;
    // output layer and dZ3
    if (tid < kHid) {
        float s = 0.0f;
        for (int m = 0; m < kTile; ++m) s = fmaf(dyS[m], static_cast<float>(Hs[2][m * kHid + tid]), s);
        g[kOffW4 + tid] = s;
    } else if (tid == kHid) {
        float s = 0.0f;
        for (int m = 0; m < kTile; ++m) s += dyS[m];
        g[kOffB4] = s;
    }
    for (int e = tid; e < kTile * kHid; e += kTrainBlock) {
        const int m = e / kHid, o = e % kHid;
        dZ[e] = dyS[m] * wf[kOffW4 + o] * gelu_grad(Zs[2][e]);
    }
    __syncthreads();
    // layer 3: dW3, db3, dH2
    weight_grad<4, kHid>(dZ, Hs[1], g + kOffW3);
    if (tid < kHid) {
        float s = 0.0f;
        for (int m = 0; m < kTile; ++m) s += dZ[m * kHid + tid];
        g[kOffB3 + tid] = s;
    }
    floatx4 acc[4];
    input_grad(W3s, dZ, acc);
    __syncthreads();
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int i = 16 * w + 4 * (lane / 16) + e, m = 16 * nt + lane % 16;
            dZ[m * kHid + i] = acc[nt][e] * gelu_grad(Zs[1][m * kHid + i]);
        }
    __syncthreads();
    // layer 2: dW2, db2, dH1
    weight_grad<4, kHid>(dZ, Hs[0], g + kOffW2);
    if (tid < kHid) {
        float s = 0.0f;
        for (int m = 0; m < kTile; ++m) s += dZ[m * kHid + tid];
        g[kOffB2 + tid] = s;
    }
    input_grad(W2s, dZ, acc);
    __syncthreads();
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int i = 16 * w + 4 * (lane / 16) + e, m = 16 * nt + lane % 16;
            dZ[m * kHid + i] = acc[nt][e] * gelu_grad(Zs[0][m * kHid + i]);
        }
    __syncthreads();
    // layer 1: dW1, db1
    weight_grad<kIn / 16, kIn>(dZ, Xs, g + kOffW1);
    if (tid < kHid) {
        float s = 0.0f;
        for (int m = 0; m < kTile; ++m) s += dZ[m * kHid + tid];
        g[kOffB1 + tid] = s;
    }
}

// Sum of the tile gradients and, with lr > 0, an Adam step of the FP32 master
// weights (and a refresh of the BF16 copy).  A block takes 32 parameters; each
// parameter's tiles are split into 8 contiguous slices summed by 8 threads at
// once (coalesced rows of 32 parameters), then the slices in slice order: a
// fixed summation order, the same in every call.  Block 0 sums the tile losses
// the same way.
constexpr int kSlices = 8;
constexpr int kParamsPerBlock = 256 / kSlices;

__global__ void __launch_bounds__(256) reduce_adam_kernel(const float *__restrict__ gpart,
                                                          int tiles, const float *__restrict__ lpart,
                                                          float *__restrict__ loss_out,
                                                          float *__restrict__ wts,
                                                          __bf16 *__restrict__ wbf,
                                                          float *__restrict__ adam,
                                                          float *__restrict__ grad_out, float lr,
                                                          float bc1, float bc2) {
    __shared__ float part[kSlices][kParamsPerBlock];
    __shared__ float lsum[kSlices];
    const int pl = threadIdx.x % kParamsPerBlock, sl = threadIdx.x / kParamsPerBlock;
    const int p = blockIdx.x * kParamsPerBlock + pl;
    const int per = (tiles + kSlices - 1) / kSlices;
    const int t0 = sl * per, t1 = min(tiles, t0 + per);
    float s = 0.0f;
    if (p < kParams)
        for (int i = t0; i < t1; ++i) s += gpart[static_cast<int64_t>(i) * kParams + p];
    part[sl][pl] = s;
    if (blockIdx.x == 0 && loss_out && pl == 0) {
        float l = 0.0f;
        for (int i = t0; i < t1; ++i) l += lpart[i];
        lsum[sl] = l;
    }
    __syncthreads();
    if (blockIdx.x == 0 && loss_out && threadIdx.x == 0) {
        float l = lsum[0];
        for (int k = 1; k < kSlices; ++k) l += lsum[k];
        *loss_out = l;
    }
    if (sl != 0 || p >= kParams) return;
    float gsum = part[0][pl];
#pragma unroll
    for (int k = 1; k < kSlices; ++k) gsum += part[k][pl];
    if (grad_out) grad_out[p] = gsum;
    if (lr > 0.0f) {
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        const float m = b1 * adam[p] + (1.0f - b1) * gsum;
        const float v = b2 * adam[kParams + p] + (1.0f - b2) * gsum * gsum;
        adam[p] = m;
        adam[kParams + p] = v;
        const float wv = wts[p] - lr * (m * bc1) / (sqrtf(v * bc2) + eps);
        wts[p] = wv;
        wbf[p] = static_cast<__bf16>(wv);
    }
}

__global__ void refresh_bf16_kernel(const float *__restrict__ wts, __bf16 *__restrict__ wbf) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p < kParams) wbf[p] = static_cast<__bf16>(wts[p]);
}

}  // namespace

// ----------------------------------------------------------- launchers ----

hipError_t launch_record(const lll_plan &p, int64_t n_paths, int R, uint64_t seed, float *states,
                         int *kidx, hipStream_t st) {
    PathArgs<float> a = detail::make_args<float>(p, seed, n_paths, 0, nullptr);
    a.stream_word = (p.struct_id & 0xFFFFFFu) | (1u << 24);  // tag 1: training data
    const dim3 grid(static_cast<unsigned>((n_paths + kBlock - 1) / kBlock));
    if (p.nmax != kRates) return hipErrorInvalidValue;
    hipLaunchKernelGGL(record_kernel<kRates>, grid, dim3(kBlock), 0, st, a, R, states, kidx);
    return hipGetLastError();
}

hipError_t launch_labels(const lll_plan &p, const float *states, const int *kidx,
                         const int64_t *poff, int64_t n_states, __bf16 *feat, float *label,
                         hipStream_t st) {
    const dim3 grid(static_cast<unsigned>((n_states + 63) / 64));
    hipLaunchKernelGGL(label_kernel, grid, dim3(64), 0, st, states, kidx, poff, n_states, p.nmax,
                       p.off, p.N, p.s, p.d.tenor, p.d.delta, p.d.L0, p.d.vol, p.d.E, p.d.w,
                       p.alpha, p.beta, p.delta_nig, feat, label);
    return hipGetLastError();
}

hipError_t launch_stats(const lll_plan &p, const float *states, const int *kidx, int64_t n_states,
                        const float *label, int64_t n_pairs, float *out, hipStream_t st) {
    hipLaunchKernelGGL(stats_kernel, dim3(1), dim3(256), 0, st, states, kidx, n_states, p.nmax,
                       p.off, p.s, label, n_pairs, out);
    return hipGetLastError();
}

hipError_t launch_init(float *wts, __bf16 *wbf, float *adam, uint64_t seed, hipStream_t st) {
    hipLaunchKernelGGL(init_kernel, dim3((kParams + 255) / 256), dim3(256), 0, st, wts, wbf, adam,
                       static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
    return hipGetLastError();
}

hipError_t launch_refresh(const float *wts, __bf16 *wbf, hipStream_t st) {
    hipLaunchKernelGGL(refresh_bf16_kernel, dim3((kParams + 255) / 256), dim3(256), 0, st, wts, wbf);
    return hipGetLastError();
}

// One pass over B samples: forward (and backward when gpart != null), then the
// fixed-order reduction (and an Adam step when lr > 0).
hipError_t launch_tiles(const __bf16 *feat, const float *target, const int *idx, int B,
                        float inv_sigma, const float *wts, const __bf16 *wbf, float *gpart,
                        float *lpart, float *yout, float *loss_out, float *wts_mut,
                        __bf16 *wbf_mut, float *adam, float *grad_out, float lr, float bc1,
                        float bc2, hipStream_t st) {
    const int tiles = (B + kTile - 1) / kTile;
    TileArgs t{feat, target, idx, B, inv_sigma, 1.0f / static_cast<float>(B), wbf, wts, gpart,
               lpart, yout};
    hipLaunchKernelGGL(tile_kernel, dim3(tiles), dim3(kTrainBlock), 0, st, t);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !gpart) return e;
    hipLaunchKernelGGL(reduce_adam_kernel, dim3((kParams + kParamsPerBlock - 1) / kParamsPerBlock),
                       dim3(256), 0, st, gpart,
                       tiles, lpart, loss_out, wts_mut, wbf_mut, adam, grad_out, lr, bc1, bc2);
    return hipGetLastError();
}

hipError_t launch_batch_index(int *idx, int B, int64_t n_pairs, uint32_t step, uint64_t seed,
                              hipStream_t st) {
    hipLaunchKernelGGL(batch_index_kernel, dim3((B + 255) / 256), dim3(256), 0, st, idx, B,
                       n_pairs, step, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
    return hipGetLastError();
}

}  // namespace mlp
}  // namespace lll
