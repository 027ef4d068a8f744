// picard_mp.hip -- PICARD in a maturity-parallel layout (few paths, many rates).
//
// Paper Section 3 (eqs. (Picard-2), (bdrift)) and its parallelism remark: under
// the Picard approximation the drift of every rate at step k is evaluated at
// the predictor X1(t_k), which is a function of the driver increments alone and
// never of the other rates' main states.  So the drift integrals of different
// periods (maturity windows) are independent, and the main state of every rate
// at the tenor dates is a plain sum:
//
//   X_i(T_{m+1}) = sum_{m' <= m} Z_{m',i},
//   Z_{m,i}      = sum_{k in period m} (lambda_{k,i} dH_k - kappa_{k,i} dt_k)
//                - sum_{k in period m} dt_k C_i(ell(X1(t_k)))   (C_{N-1} = 0),
//
// with C_i the coupling of eq. (LIBOR-drift-PT) on the 64-node rule.  With one
// path per lane (the path kernel) a run of 10^4 paths fills 157 wavefronts,
// a sixth of the SIMDs; here the work of a path spreads over (period, node):
//
//   0. increments -- one thread per (path, step): the driver increments;
//   1. prologue -- one wavefront per group of 4 paths, lane = rate: the
//      predictor X1 advanced with the same FP32 updates as the path kernel,
//      ell^ = ell(X1(t_k)) stored for every (step, live rate), and the first
//      sum of Z;
//   2. items -- one wavefront per (group, period m), lane = quadrature node q:
//      the suffix recursion of the path kernel over the rates, for all steps
//      of the period at once, the 4 paths of the group sharing every table
//      load; each rate's per-node sums are transposed through LDS, summed over
//      the 64 nodes and subtracted from Z;
//   3. payoffs -- one lane per path: the states at the tenor dates as running
//      sums of Z, the payoff quantities and formula of the path kernel, and
//      per wavefront the sums of the path kernel's partial-sum layout.
//
// Items run period-major: the wavefronts resident together read the same
// period's tables (held in L2), and the items with the most live rates start
// first.  Paths are processed in chunks so that the ell^ buffer stays bounded.
#include <hip/hip_runtime.h>

#include "path_kernel.hpp"

namespace lll {
namespace {

using detail::as_const;
using detail::cptr;

constexpr int kGroup = 4;                 // paths per group (lanes of one item)
constexpr int kRateBlock = 4;             // rates per LDS transposition
constexpr int kRows = kRateBlock * kGroup;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kMaxChunk = 16;             // steps per item chunk

struct MpArgs {
    cptr<float> lam, drift0, frozen, cinv;  // [K][nmax], [K][nmax], [K][nmax], [nmax]
    cptr<double> steps;                     // [N][4]
    const float2 *__restrict__ ewq;         // [K][N][Q]: (E, W E dt)
    float *__restrict__ ellhat;             // [G][ell_entries][kGroup]: (step, live rate)
    float *__restrict__ z;                  // [G][N][N][kGroup]: group, period, rate, path
    float *__restrict__ dh;                 // [G][K][kGroup] driver increments
    int64_t path_base;                      // global index of the chunk's first path
    int G, N, s, K, off, nmax;
    uint32_t stream_word, key0, key1;
    double beta;
};

// ell^ is stored for the live rates only: step k of period m holds rates
// m .. N-1, at entry ell_entry(k) + i - m of its group (s N (N+1) / 2 entries).
__host__ __device__ inline size_t ell_entry(int k, int s, int N) {
    const int m = k / s;
    return (size_t)s * ((size_t)m * N - (size_t)m * (m - 1) / 2) + (size_t)(k - m * s) * (N - m);
}
__host__ __device__ inline size_t ell_entries(int s, int N) { return (size_t)s * N * (N + 1) / 2; }
// Z per group: N x N entries (of kGroup floats each).
__host__ __device__ inline size_t z_entries(int N) { return (size_t)N * N; }

// Cross-lane exchange through LDS within one wavefront: the writes of every
// lane are complete and visible before any lane reads.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// (E, W_q E dt_k) of every (step, rate, node), from the FP64 tables of the
// precompute ([K][N][Q], 0 for fixed rates).  One block of 64 nodes per step.
__global__ void __launch_bounds__(64) mp_tables_kernel(const double *__restrict__ E,
                                                       const double *__restrict__ w,
                                                       const double *__restrict__ tenor, int N,
                                                       int s, float2 *__restrict__ ewq) {
    const int k = blockIdx.x, q = threadIdx.x;
    const int m = k / s;
    const double Ta = m == 0 ? 0.0 : tenor[m - 1];
    const double wdt = w[q] * ((tenor[m] - Ta) / s);
    for (int r = 0; r < N; ++r) {
        const size_t i = ((size_t)k * N + r) * kQ + q;
        const double e = E[i];
        ewq[i] = make_float2(static_cast<float>(e), static_cast<float>(wdt * e));
    }
}

// Driver increments of the chunk's paths, one thread per (path, step) (the
// FP64 sampler needs the occupancy of a flat grid), FP32 as the path kernel
// uses them; layout [group][step][path of the group].
__global__ void __launch_bounds__(kBlock) mp_increments_kernel(MpArgs a) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (e >= (int64_t)a.G * a.K * kGroup) return;
    const int p = static_cast<int>(e % kGroup);
    const int64_t gk = e / kGroup;
    const int k = static_cast<int>(gk % a.K);
    const int64_t g = gk / a.K;
    const uint64_t path = static_cast<uint64_t>(a.path_base + g * kGroup + p);
    const cptr<double> sc = a.steps + 4 * (k / a.s);
    const StepConsts cst{sc[0], sc[1], sc[2], sc[3]};
    const uint4 w = philox4x32_10(make_uint4(static_cast<uint32_t>(k), static_cast<uint32_t>(path),
                                             static_cast<uint32_t>(path >> 32), a.stream_word),
                                  a.key0, a.key1);
    a.dh[e] = static_cast<float>(increment(w, cst, a.beta, false, nullptr));
}

// Table values and driver increments of steps kb .. kb+3 (clamped to the last
// step): vol, cumulant term and frozen drift of slot j (byte offsets into the
// K x nmax tables stay below 2^32: K <= 2^24, nmax <= 64), and the 4 paths'
// increments (one 16-byte load, the same address on every lane).
struct Steps4 {
    float lam[4], d0[4], frz[4];
    float4 dh[4];
};
__device__ __forceinline__ void load_steps4(const MpArgs &a, const float4 *dh_g, int kb,
                                            unsigned j, Steps4 &t) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int k = min(kb + u, a.K - 1);
        const unsigned b = ((unsigned)k * (unsigned)a.nmax + j) * 4u;
        t.lam[u] = *(cptr<float>)((cptr<char>)a.lam + b);
        t.d0[u] = *(cptr<float>)((cptr<char>)a.drift0 + b);
        t.frz[u] = *(cptr<float>)((cptr<char>)a.frozen + b);
        t.dh[u] = dh_g[k];
    }
}

// Predictor state of one group: X1 and the running first sums A of the 4
// paths, the period m of the next step and the step's place kk in it, and e,
// the ell^ entry of that step's first live rate (ell_entry(k, s, N)).
struct Predictor {
    float X1[kGroup], A[kGroup];
    int m, kk;
    size_t e;
};

// Steps kb .. kb+3 (those below K) of one group: ell^ at the predictor, then
// the predictor and the first sums advanced; Z's first sums stored at each
// period's last step.
__device__ __forceinline__ void prologue_steps4(const MpArgs &a, const Steps4 &t, int kb, int lane,
                                                int r, float ci, float4 *ell_g, float4 *z_g,
                                                Predictor &q) {
    const int N = a.N;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        if (kb + u < a.K) {
            const bool live = lane >= q.m && lane < N;
            if (live)
                ell_g[q.e + (r - q.m)] =
                    make_float4(detail::ell_of(q.X1[0], ci), detail::ell_of(q.X1[1], ci),
                                detail::ell_of(q.X1[2], ci), detail::ell_of(q.X1[3], ci));
            const float d[kGroup] = {t.dh[u].x, t.dh[u].y, t.dh[u].z, t.dh[u].w};
#pragma unroll
            for (int p = 0; p < kGroup; ++p) {
                q.A[p] += fmaf(t.lam[u], d[p], t.d0[u]);
                q.X1[p] += fmaf(t.lam[u], d[p], t.frz[u]);
            }
            q.e += N - q.m;
            if (++q.kk == a.s) {  // last step of period m
                if (live) z_g[(size_t)q.m * N + r] = make_float4(q.A[0], q.A[1], q.A[2], q.A[3]);
#pragma unroll
                for (int p = 0; p < kGroup; ++p) q.A[p] = 0.0f;
                q.kk = 0;
                ++q.m;
            }
        }
    }
}

// One wavefront per group of 4 paths, lane = rate.  The steps run in order
// with the period and the step within it carried along, so that ell^'s entry
// and the period's live lanes advance by additions; the loads of the next 4
// steps are issued while the current 4 steps compute (a step's own loads
// would otherwise wait a full L2 round trip), into two register sets used in
// turn.  A fixed rate's vol, cumulant and frozen drift are 0, so its updates
// add nothing.  Stores are 16 B per lane, contiguous over the live rates.
__global__ void __launch_bounds__(kBlock) mp_prologue_kernel(MpArgs a) {
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x % kWave;
    const int g = blockIdx.x * kWavesPerBlock + wv;
    if (g >= a.G) return;  // whole wavefront
    const int N = a.N, K = a.K, s = a.s;
    // rate of this lane (N <= 64); lanes past the last rate repeat it and
    // store nothing
    const int r = lane < N ? lane : N - 1;
    const unsigned j = static_cast<unsigned>(a.off + r);
    const float ci = a.cinv[j];
    const float4 *dh_g = reinterpret_cast<const float4 *>(a.dh) + (size_t)g * K;
    float4 *ell_g = reinterpret_cast<float4 *>(a.ellhat) + (size_t)g * ell_entries(s, N);
    float4 *z_g = reinterpret_cast<float4 *>(a.z) + (size_t)g * z_entries(N);
    Predictor q;
#pragma unroll
    for (int p = 0; p < kGroup; ++p) q.X1[p] = q.A[p] = 0.0f;
    q.m = q.kk = 0;
    q.e = 0;
    Steps4 t0, t1;
    load_steps4(a, dh_g, 0, j, t0);
    for (int k0 = 0; k0 < K; k0 += 8) {
        load_steps4(a, dh_g, k0 + 4, j, t1);
        prologue_steps4(a, t0, k0, lane, r, ci, ell_g, z_g, q);
        if (k0 + 4 >= K) break;
        load_steps4(a, dh_g, k0 + 8, j, t0);
        prologue_steps4(a, t1, k0 + 4, lane, r, ci, ell_g, z_g, q);
    }
}

// One block = the 4 items (groups g0 .. g0+3) of one period m; G is a
// multiple of 4, so the wavefronts of a block run the same steps and rates in
// lockstep.  Per rate i the block stages in LDS the table entries (E, W E dt)
// of the chunk's steps at all 64 nodes and the 4 groups' ell^, double-buffered:
// the loads for rate i-1 are issued before the arithmetic of rate i and stored
// after it, one barrier per rate.  Each table entry is read from L2 once per
// block instead of once per wavefront, and the latency of the ell^ reads (HBM)
// is covered by a rate's arithmetic.  The chunk length SC is a compile-time
// constant (steps past the period's end are staged as zeros and add nothing),
// so the step loops carry no branches.  R[p][kk] is prod_{l>i}(1 + ell^_l
// E_{l,q}) - 1 for path p at step c0+kk, advanced from the last rate down as
// in the path kernel; acc[p] sums W E dt R over the steps for rate i; every
// kRateBlock rates the per-node sums are transposed through LDS, summed over
// the nodes and subtracted from Z.
template <int SC>
struct ItemLds {
    float2 ew[2][SC][kQ];               // (E, W E dt) per step and node
    float4 ell[2][SC][kWavesPerBlock];  // ell^ of the 4 paths of each group
    float red[kWavesPerBlock][kRows][kWave + 1];
};

// Global loads of the staging of rate i by thread t of the block: up to two
// float4 of table pairs and one float4 of ell^ (zeros for steps kk >= nk).
template <int SC>
__device__ __forceinline__ void stage_load(const MpArgs &a, int g0, int c0, int nk, int i, int t,
                                           float4 (&v)[3]) {
    const float4 *ew4 = reinterpret_cast<const float4 *>(a.ewq);
    const float4 zero = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int f = t + u * kBlock;
        const int kk = f / (kQ / 2);
        v[u] = zero;
        if (kk < nk) v[u] = ew4[((size_t)(c0 + kk) * a.N + i) * (kQ / 2) + f % (kQ / 2)];
    }
    v[2] = zero;
    if (t < SC * kWavesPerBlock) {
        const int kk = t % SC, w = t / SC;
        if (kk < nk)
            v[2] = reinterpret_cast<const float4 *>(
                a.ellhat)[(size_t)(g0 + w) * ell_entries(a.s, a.N) + ell_entry(c0 + kk, a.s, a.N) +
                          (i - (c0 + kk) / a.s)];
    }
}

template <int SC>
__device__ __forceinline__ void stage_store(ItemLds<SC> &L, int buf, int t, const float4 (&v)[3]) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int f = t + u * kBlock;
        if (f < SC * (kQ / 2))
            *reinterpret_cast<float4 *>(&L.ew[buf][f / (kQ / 2)][2 * (f % (kQ / 2))]) = v[u];
    }
    if (t < SC * kWavesPerBlock) L.ell[buf][t % SC][t / SC] = v[2];
}

// Rate i's sums of one wavefront's 4 paths: acc[p] into row `row` of the
// transposition buffer; after kRateBlock rates (or the last rate) every row is
// summed over the 64 nodes (four lanes per row, a quarter each) and
// subtracted from Z.  Returns the number of rows still pending.
__device__ __forceinline__ int push_rate_sums(float (*red)[kWave + 1], float *z_gm, int q,
                                              int row, int i, bool last,
                                              const float (&acc)[kGroup]) {
#pragma unroll
    for (int p = 0; p < kGroup; ++p) red[row * kGroup + p][q] = acc[p];
    ++row;
    if (row < kRateBlock && !last) return row;
    // rows 0 .. row*kGroup-1 hold rates i+row-1 down to i
    wave_sync();
    const int rr = q % kRows, h = q / kRows;
    const bool used = rr < row * kGroup;
    float sum = 0.0f;
    if (used) {
#pragma unroll
        for (int u = 0; u < kWave / 4; ++u) sum += red[rr][h * (kWave / 4) + u];
    }
    sum += __shfl_xor(sum, kWave / 4, kWave);
    sum += __shfl_xor(sum, kWave / 2, kWave);
    if (used && h == 0) z_gm[(i + row - 1 - rr / kGroup) * kGroup + rr % kGroup] -= sum;
    wave_sync();
    return 0;
}

template <int SC>
__global__ void __launch_bounds__(kBlock) mp_item_kernel(MpArgs a) {
    __shared__ ItemLds<SC> L;
    const int t = threadIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane(t / kWave);
    const int q = t % kWave;
    const int64_t item0 = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock;
    if (item0 >= (int64_t)(a.N - 1) * a.G) return;  // whole block
    const int m = static_cast<int>(item0 / a.G), g0 = static_cast<int>(item0 % a.G);
    const int N = a.N, s = a.s;
    float *z_gm = a.z + ((size_t)(g0 + wv) * z_entries(N) + (size_t)m * N) * kGroup;
    float(*red)[kWave + 1] = L.red[wv];
    for (int c0 = m * s; c0 < (m + 1) * s; c0 += SC) {
        const int nk = min(SC, (m + 1) * s - c0);
        float4 v[3];
        float R[kGroup][SC];
        // the last rate starts the products: R = ell^_{N-1} E_{N-1}
        stage_load<SC>(a, g0, c0, nk, N - 1, t, v);
        stage_store<SC>(L, 0, t, v);
        __syncthreads();
        stage_load<SC>(a, g0, c0, nk, N - 2, t, v);
#pragma unroll
        for (int kk = 0; kk < SC; ++kk) {
            const float e = L.ew[0][kk][q].x;
            const float4 l = L.ell[0][kk][wv];
            R[0][kk] = l.x * e;
            R[1][kk] = l.y * e;
            R[2][kk] = l.z * e;
            R[3][kk] = l.w * e;
        }
        stage_store<SC>(L, 1, t, v);
        __syncthreads();
        int row = 0;
        // rates N-2 .. m+1: sums and the product update
        for (int i = N - 2; i > m; --i) {
            const int buf = (N - 1 - i) & 1;
            stage_load<SC>(a, g0, c0, nk, i - 1, t, v);
            float acc[kGroup] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int kk = 0; kk < SC; ++kk) {
                const float2 ew = L.ew[buf][kk][q];
                const float4 l = L.ell[buf][kk][wv];
#pragma unroll
                for (int p = 0; p < kGroup; ++p) acc[p] = fmaf(ew.y, R[p][kk], acc[p]);
                R[0][kk] = fmaf(l.x, fmaf(ew.x, R[0][kk], ew.x), R[0][kk]);
                R[1][kk] = fmaf(l.y, fmaf(ew.x, R[1][kk], ew.x), R[1][kk]);
                R[2][kk] = fmaf(l.z, fmaf(ew.x, R[2][kk], ew.x), R[2][kk]);
                R[3][kk] = fmaf(l.w, fmaf(ew.x, R[3][kk], ew.x), R[3][kk]);
            }
            row = push_rate_sums(red, z_gm, q, row, i, false, acc);
            stage_store<SC>(L, buf ^ 1, t, v);
            __syncthreads();
        }
        // rate m: sums only
        {
            const int buf = (N - 1 - m) & 1;
            float acc[kGroup] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int kk = 0; kk < SC; ++kk) {
                const float w = L.ew[buf][kk][q].y;
#pragma unroll
                for (int p = 0; p < kGroup; ++p) acc[p] = fmaf(w, R[p][kk], acc[p]);
            }
            push_rate_sums(red, z_gm, q, row, m, true, acc);
        }
        __syncthreads();  // the next chunk restages buffer 0
    }
}

// Payoff values of the chunk's paths: lane = path, the 4 wavefronts of a block
// take the same 64 paths and every fourth fixing each (the FP64 payoff
// quantities dominate; a 10^4-path run so has 628 wavefronts, not 157), the
// states of the plan's slots in LDS advanced by Z period by period; per fixing
// the quantities Q, A, D, L_r and the payoff formula of the path kernel, stored
// path-contiguous ([rate][t][path] with pay_t = max(v_t, 0) for the S strikes,
// t = S for Q; zs paths per row) and summed over each
// wavefront's 64 paths by mp_wave_sums_kernel: no cross-lane reduction here,
// so the 157 wavefronts of a 10^4-path run do not wait on shuffles.
template <int NMAX>
__global__ void __launch_bounds__(kBlock) mp_payoff_kernel(detail::PathArgs<float> a,
                                                           const float *__restrict__ z,
                                                           double *__restrict__ pays,
                                                           int64_t chunk_first, int64_t zs) {
    __shared__ float sX[kWavesPerBlock][NMAX * kWave];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x % kWave;
    const int64_t lp = static_cast<int64_t>(blockIdx.x) * kWave + lane;
    const int64_t gid = chunk_first + lp;
    if (gid - lane >= a.n_paths) return;  // whole wavefront past the end
    float *xs = sX[wv] + lane;
    const bool active = gid < a.n_paths;
    const bool swaption = a.product == LLL_SWAPTIONS;
    const int N = a.N, S = a.S;
    const float *zp = z + (size_t)(lp / kGroup) * z_entries(N) * kGroup + lp % kGroup;
    double *pp = pays + lp;  // [m][t][path], t = 0..S
#pragma unroll
    for (int j = 0; j < NMAX; ++j) xs[j * kWave] = 0.0f;
    for (int m = 0; m < N; ++m) {
#pragma unroll 8
        for (int r = m; r < N; ++r) xs[(a.off + r) * kWave] += zp[((size_t)m * N + r) * kGroup];
        if (m % kWavesPerBlock != wv) continue;  // the block's wavefronts share the fixings
        double Q, A, D, Lc;
        detail::fixing_quantities_lds<float, NMAX, kWave>(a, xs, a.off + m, Q, A, D, Lc);
        if (active && !swaption && a.path_fix != nullptr) {
            a.path_fix[gid * 2 * N + 2 * m] = Lc;
            a.path_fix[gid * 2 * N + 2 * m + 1] = D;
        }
        for (int t = 0; t < S; ++t) {
            const double v = detail::payoff_value(swaption, a.strikes[m * S + t], Q, A, D, Lc);
            pp[((size_t)m * (S + 1) + t) * zs] = active ? fmax(v, 0.0) : 0.0;
        }
        pp[((size_t)m * (S + 1) + S) * zs] = active ? Q : 0.0;
    }
}

// Per (wavefront w of the chunk, rate r): the sums of the wavefront's 64 path
// values in lane order, in the partial-sum layout of the path kernel (per
// strike the sum, the sum of squares and the count of positive payoffs, then
// the sum and sum of squares of Q).
__global__ void __launch_bounds__(kBlock) mp_wave_sums_kernel(const double *__restrict__ pays,
                                                             int N, int S, int64_t n_waves,
                                                             int64_t zs, int64_t wave0,
                                                             double *__restrict__ partials) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (e >= n_waves * N) return;
    const int64_t w = e / N;
    const int r = static_cast<int>(e % N);
    double *out = partials + ((size_t)(wave0 + w) * N + r) * (3 * S + 2);
    for (int t = 0; t <= S; ++t) {
        const double *pv = pays + ((size_t)r * (S + 1) + t) * zs + (size_t)w * kWave;
        double s1 = 0.0, s2 = 0.0, ni = 0.0;
        for (int l = 0; l < kWave; ++l) {
            const double v = pv[l];
            s1 += v;
            s2 += v * v;
            ni += v > 0.0 ? 1.0 : 0.0;
        }
        if (t < S) {
            out[t] = s1;
            out[S + t] = s2;
            out[2 * S + t] = ni;
        } else {
            out[3 * S] = s1;
            out[3 * S + 1] = s2;
        }
    }
}

template <int NMAX>
void launch_mp_payoff(const detail::PathArgs<float> &a, const float *z, double *pays,
                      int64_t chunk_first, int64_t n_chunk, int64_t zs, hipStream_t st) {
    const dim3 grid(static_cast<unsigned>((n_chunk + kWave - 1) / kWave));
    hipLaunchKernelGGL(mp_payoff_kernel<NMAX>, grid, dim3(kBlock), 0, st, a, z, pays, chunk_first,
                       zs);
}

template <int SC>
void launch_items(const MpArgs &a, hipStream_t st) {
    const int64_t items = (int64_t)(a.N - 1) * a.G;
    const dim3 grid(static_cast<unsigned>((items + kWavesPerBlock - 1) / kWavesPerBlock));
    hipLaunchKernelGGL(mp_item_kernel<SC>, grid, dim3(kBlock), 0, st, a);
}

}  // namespace

int64_t picard_mp_chunk(const lll_plan &p) {
    // paths per chunk: a multiple of 256 with ell^, Z and the payoff values
    // within kMpBufferBytes
    const int64_t per_path = ((int64_t)ell_entries(p.s, p.N) + (int64_t)z_entries(p.N)) *
                                 (int64_t)sizeof(float) +
                             (int64_t)p.N * (p.S + 1) * (int64_t)sizeof(double) +
                             (int64_t)p.K * (int64_t)sizeof(float);
    int64_t c = kMpBufferBytes / per_path / kBlock * kBlock;
    if (c < kBlock) c = kBlock;
    const int64_t need = (p.max_paths + kBlock - 1) / kBlock * kBlock;
    return c < need ? c : need;
}

hipError_t picard_mp_alloc(lll_plan &p) {
    if (p.d.mp_ell) return hipSuccess;
    const int64_t chunk = picard_mp_chunk(p);
    const size_t G = (size_t)chunk / kGroup;
    hipError_t e = hipMalloc(&p.d.mp_ewq, (size_t)p.K * p.N * kQ * sizeof(float2));
    if (e == hipSuccess) e = hipMalloc(&p.d.mp_ell, G * ell_entries(p.s, p.N) * kGroup * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&p.d.mp_z, G * z_entries(p.N) * kGroup * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&p.d.mp_pay, (size_t)chunk * p.N * (p.S + 1) * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&p.d.mp_dh, (size_t)chunk * p.K * sizeof(float));
    if (e != hipSuccess) {
        picard_mp_free(p);
        return e;
    }
    p.mp_chunk = chunk;
    return hipSuccess;
}

void picard_mp_free(lll_plan &p) {
    (void)hipFree(p.d.mp_ewq);
    (void)hipFree(p.d.mp_ell);
    (void)hipFree(p.d.mp_z);
    (void)hipFree(p.d.mp_pay);
    (void)hipFree(p.d.mp_dh);
    p.d.mp_pay = nullptr;
    p.d.mp_dh = nullptr;
    p.d.mp_ewq = nullptr;
    p.d.mp_ell = nullptr;
    p.d.mp_z = nullptr;
    p.mp_chunk = 0;
}

hipError_t launch_picard_mp(const lll_plan &p, int64_t n_paths, int64_t path_offset,
                            uint64_t seed, double *path_fix, hipStream_t st) {
    const detail::PathArgs<float> pa =
        detail::make_args<float>(p, seed, n_paths, path_offset, path_fix);
    float2 *ewq = static_cast<float2 *>(p.d.mp_ewq);
    hipLaunchKernelGGL(mp_tables_kernel, dim3(p.K), dim3(kQ), 0, st, p.d.E, p.d.w, p.d.tenor,
                       p.N, p.s, ewq);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    MpArgs a;
    a.lam = pa.lam;
    a.drift0 = pa.drift0;
    a.frozen = pa.frozen;
    a.cinv = pa.cinv;
    a.steps = pa.steps;
    a.ewq = ewq;
    a.ellhat = p.d.mp_ell;
    a.z = p.d.mp_z;
    a.dh = p.d.mp_dh;
    a.N = p.N;
    a.s = p.s;
    a.K = p.K;
    a.off = p.off;
    a.nmax = p.nmax;
    a.stream_word = pa.stream_word;
    a.key0 = pa.key0;
    a.key1 = pa.key1;
    a.beta = p.beta;
    for (int64_t first = 0; first < n_paths; first += p.mp_chunk) {
        const int64_t n_chunk = n_paths - first < p.mp_chunk ? n_paths - first : p.mp_chunk;
        a.path_base = path_offset + first;
        a.G = static_cast<int>((n_chunk + kWave - 1) / kWave * (kWave / kGroup));
        const int64_t n_inc = (int64_t)a.G * p.K * kGroup;
        hipLaunchKernelGGL(mp_increments_kernel, dim3(static_cast<unsigned>((n_inc + kBlock - 1) / kBlock)),
                           dim3(kBlock), 0, st, a);
        hipLaunchKernelGGL(mp_prologue_kernel, dim3(a.G / kWavesPerBlock), dim3(kBlock), 0, st, a);
        if (p.N > 1) {
            // steps per chunk: the period in ceil(s / 16) chunks of equal length
            // (the last one padded)
            const int nch = (p.s + kMaxChunk - 1) / kMaxChunk;
            switch ((p.s + nch - 1) / nch) {
                case 1: launch_items<1>(a, st); break;
                case 2: launch_items<2>(a, st); break;
                case 3: launch_items<3>(a, st); break;
                case 4: launch_items<4>(a, st); break;
                case 5: launch_items<5>(a, st); break;
                case 6: launch_items<6>(a, st); break;
                case 7: launch_items<7>(a, st); break;
                case 8: launch_items<8>(a, st); break;
                case 9: launch_items<9>(a, st); break;
                case 10: launch_items<10>(a, st); break;
                case 11: launch_items<11>(a, st); break;
                case 12: launch_items<12>(a, st); break;
                case 13: launch_items<13>(a, st); break;
                case 14: launch_items<14>(a, st); break;
                case 15: launch_items<15>(a, st); break;
                default: launch_items<16>(a, st); break;
            }
        }
        double *pays = p.d.mp_pay;
        const int64_t zs = (int64_t)a.G * kGroup;
        switch (p.nmax) {
            case 8: launch_mp_payoff<8>(pa, a.z, pays, first, n_chunk, zs, st); break;
            case 16: launch_mp_payoff<16>(pa, a.z, pays, first, n_chunk, zs, st); break;
            case 20: launch_mp_payoff<20>(pa, a.z, pays, first, n_chunk, zs, st); break;
            case 24: launch_mp_payoff<24>(pa, a.z, pays, first, n_chunk, zs, st); break;
            case 32: launch_mp_payoff<32>(pa, a.z, pays, first, n_chunk, zs, st); break;
            case 40: launch_mp_payoff<40>(pa, a.z, pays, first, n_chunk, zs, st); break;
            case 64: launch_mp_payoff<64>(pa, a.z, pays, first, n_chunk, zs, st); break;
            default: return hipErrorInvalidValue;
        }
        const int64_t waves = (n_chunk + kWave - 1) / kWave;
        hipLaunchKernelGGL(mp_wave_sums_kernel,
                           dim3(static_cast<unsigned>((waves * p.N + kBlock - 1) / kBlock)),
                           dim3(kBlock), 0, st, pays, p.N, p.S, waves, zs, first / kWave,
                           pa.partials);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace lll
