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
//   1. prologue -- one wavefront per group of 4 paths, lane = rate: the lanes
//      draw the increments 64 steps at a time, then advance the predictor X1
//      with the same FP32 updates as the path kernel, store
//      ell^ = ell(X1(t_k)) for every (step, live rate) and the first sum of Z;
//   2. items -- one wavefront per (group, period m), lane = quadrature node q:
//      the suffix recursion of the path kernel over the rates, for all steps
//      of the period at once, the 4 paths of the group sharing every table
//      load; each rate's per-node sums are transposed through LDS, summed over
//      the 64 nodes and subtracted from Z;
//   3. payoffs -- one lane per path: the states at the tenor dates as running
//      sums of Z, then the payoffs and wavefront sums of the path kernel.
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
constexpr int kRateBlock = 8;             // rates per LDS transposition
constexpr int kRows = kRateBlock * kGroup;
constexpr int kWavesPerBlock = kBlock / kWave;

struct MpArgs {
    cptr<float> lam, drift0, frozen, cinv;  // [K][nmax], [K][nmax], [K][nmax], [nmax]
    cptr<double> steps;                     // [N][4]
    const float2 *__restrict__ ewq;         // [K][N][Q]: (E, W E dt)
    float *__restrict__ ellhat;             // [G][K][N][kGroup]
    float *__restrict__ z;                  // [G][N][N][kGroup]
    int64_t path_base;                      // global index of the chunk's first path
    int G, N, s, K, off, nmax;
    uint32_t stream_word, key0, key1;
    double beta;
};

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

__global__ void __launch_bounds__(kBlock) mp_prologue_kernel(MpArgs a) {
    __shared__ float sdh[kWavesPerBlock][kGroup][kWave];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x % kWave;
    const int g = blockIdx.x * kWavesPerBlock + wv;
    if (g >= a.G) return;  // whole wavefront
    float(*dh)[kWave] = sdh[wv];
    const int N = a.N, K = a.K, s = a.s;
    const int r = lane;  // rate of this lane (N <= 64)
    const int j = a.off + (r < N ? r : 0);
    const float ci = a.cinv[j];
    float X1[kGroup], A[kGroup];
#pragma unroll
    for (int p = 0; p < kGroup; ++p) X1[p] = A[p] = 0.0f;
    const int64_t path0 = a.path_base + (int64_t)g * kGroup;
    float *ell_g = a.ellhat + (size_t)g * K * N * kGroup;
    float *z_g = a.z + (size_t)g * N * N * kGroup;
    for (int k0 = 0; k0 < K; k0 += kWave) {
        const int kd = k0 + lane;
        if (kd < K) {
            const cptr<double> sc = a.steps + 4 * (kd / s);
            const StepConsts cst{sc[0], sc[1], sc[2], sc[3]};
#pragma unroll
            for (int p = 0; p < kGroup; ++p) {
                const uint64_t path = static_cast<uint64_t>(path0 + p);
                const uint4 w = philox4x32_10(
                    make_uint4(static_cast<uint32_t>(kd), static_cast<uint32_t>(path),
                               static_cast<uint32_t>(path >> 32), a.stream_word),
                    a.key0, a.key1);
                dh[p][lane] = static_cast<float>(increment(w, cst, a.beta, false, nullptr));
            }
        }
        wave_sync();
        const int kn = min(kWave, K - k0);
        for (int kk = 0; kk < kn; ++kk) {
            const int k = k0 + kk;
            const int m = k / s;
            if (r < N && r >= m) {
                const size_t t = (size_t)k * a.nmax + j;
                const float lam = a.lam[t], d0 = a.drift0[t], frz = a.frozen[t];
                float4 e;
                e.x = detail::ell_of(X1[0], ci);
                e.y = detail::ell_of(X1[1], ci);
                e.z = detail::ell_of(X1[2], ci);
                e.w = detail::ell_of(X1[3], ci);
                *reinterpret_cast<float4 *>(ell_g + ((size_t)k * N + r) * kGroup) = e;
#pragma unroll
                for (int p = 0; p < kGroup; ++p) {
                    const float d = dh[p][kk];
                    A[p] += fmaf(lam, d, d0);
                    X1[p] += fmaf(lam, d, frz);
                }
                if ((k + 1) % s == 0) {
                    *reinterpret_cast<float4 *>(z_g + ((size_t)m * N + r) * kGroup) =
                        make_float4(A[0], A[1], A[2], A[3]);
#pragma unroll
                    for (int p = 0; p < kGroup; ++p) A[p] = 0.0f;
                }
            }
        }
        wave_sync();
    }
}

// One item: group g, period m, steps c0 .. c0+nk-1 of that period.  R[p][kk]
// is prod_{l>i}(1 + ell^_l E_{l,q}) - 1 for path p at step c0+kk, advanced from
// the last rate down as in the path kernel; acc[p] sums W E dt R over the
// steps for the current rate i.
template <int SC>
__device__ __forceinline__ void mp_item_steps(const MpArgs &a, int g, int m, int c0, int nk,
                                              float (*red)[kWave + 1], int q) {
    const int N = a.N;
    const cptr<float> ell_g = as_const<float>(a.ellhat + (size_t)g * a.K * N * kGroup);
    float *z_gm = a.z + ((size_t)g * N + m) * N * kGroup;
    float R[kGroup][SC];
#pragma unroll
    for (int kk = 0; kk < SC; ++kk) {
        if (kk < nk) {
            const int k = c0 + kk;
            const float2 ew = a.ewq[((size_t)k * N + (N - 1)) * kQ + q];
            const cptr<float> l = ell_g + ((size_t)k * N + (N - 1)) * kGroup;
#pragma unroll
            for (int p = 0; p < kGroup; ++p) R[p][kk] = l[p] * ew.x;
        }
    }
    int row = 0;
    for (int i = N - 2; i >= m; --i) {
        float acc[kGroup] = {0.0f, 0.0f, 0.0f, 0.0f};
        const bool more = i > m;
#pragma unroll
        for (int kk = 0; kk < SC; ++kk) {
            if (kk < nk) {
                const int k = c0 + kk;
                const float2 ew = a.ewq[((size_t)k * N + i) * kQ + q];
#pragma unroll
                for (int p = 0; p < kGroup; ++p) acc[p] = fmaf(ew.y, R[p][kk], acc[p]);
                if (more) {
                    const cptr<float> l = ell_g + ((size_t)k * N + i) * kGroup;
#pragma unroll
                    for (int p = 0; p < kGroup; ++p)
                        R[p][kk] = fmaf(l[p], fmaf(ew.x, R[p][kk], ew.x), R[p][kk]);
                }
            }
        }
#pragma unroll
        for (int p = 0; p < kGroup; ++p) red[row * kGroup + p][q] = acc[p];
        ++row;
        if (row == kRateBlock || !more) {
            // rows 0 .. row*kGroup-1 hold rates i+row-1 down to i; lanes rr and
            // rr + 32 each sum half of row rr over the nodes
            wave_sync();
            const int rr = q % kRows, h = q / kRows;
            const bool used = rr < row * kGroup;
            float v = 0.0f;
            if (used) {
#pragma unroll 8
                for (int t = 0; t < kWave / 2; ++t) v += red[rr][h * (kWave / 2) + t];
            }
            v += __shfl_xor(v, kWave / 2, kWave);
            if (used && h == 0) {
                const int rate = i + row - 1 - rr / kGroup;
                z_gm[rate * kGroup + rr % kGroup] -= v;
            }
            wave_sync();
            row = 0;
        }
    }
}

template <int SC>
__global__ void __launch_bounds__(kBlock) mp_item_kernel(MpArgs a) {
    __shared__ float sred[kWavesPerBlock][kRows][kWave + 1];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int q = threadIdx.x % kWave;
    const int64_t item = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wv;
    if (item >= (int64_t)(a.N - 1) * a.G) return;  // whole wavefront
    const int m = static_cast<int>(item / a.G), g = static_cast<int>(item % a.G);
    const int s = a.s;
    const int nch = (s + SC - 1) / SC;
    const int csz = (s + nch - 1) / nch;
    for (int c0 = m * s; c0 < (m + 1) * s; c0 += csz)
        mp_item_steps<SC>(a, g, m, c0, min(csz, (m + 1) * s - c0), sred[wv], q);
}

// Payoffs of the chunk's paths: lane = path, the states of the plan's slots
// in LDS (as the LDS-state path kernels hold them), advanced by Z period by
// period; the payoff code and partial-sum layout are the path kernel's.
template <int NMAX>
__global__ void __launch_bounds__(kBlock) mp_payoff_kernel(detail::PathArgs<float> a,
                                                           const float *__restrict__ z,
                                                           int64_t chunk_first) {
    const int64_t lp = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int64_t gid = chunk_first + lp;
    if (gid - (threadIdx.x % kWave) >= a.n_paths) return;  // whole wavefront past the end
    float *xs = detail::state_lds<float, NMAX>() + threadIdx.x;
    const bool active = gid < a.n_paths;
    const int N = a.N;
    const float *zp = z + (size_t)(lp / kGroup) * N * N * kGroup + lp % kGroup;
#pragma unroll
    for (int j = 0; j < NMAX; ++j) xs[j * kBlock] = 0.0f;
    for (int m = 0; m < N; ++m) {
        for (int r = m; r < N; ++r) xs[(a.off + r) * kBlock] += zp[((size_t)m * N + r) * kGroup];
        detail::payoff_lds<float, NMAX, detail::kAnyProduct>(a, m, gid, active, xs, a.off + m);
    }
}

template <int NMAX>
void launch_mp_payoff(const detail::PathArgs<float> &a, const float *z, int64_t chunk_first,
                      int64_t n_chunk, hipStream_t st) {
    const dim3 grid(static_cast<unsigned>((n_chunk + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(mp_payoff_kernel<NMAX>, grid, dim3(kBlock), 0, st, a, z, chunk_first);
}

}  // namespace

int64_t picard_mp_chunk(const lll_plan &p) {
    // paths per chunk: a multiple of 256 with ell^ and Z within kMpBufferBytes
    const int64_t per_path = ((int64_t)p.K * p.N + (int64_t)p.N * p.N) * (int64_t)sizeof(float);
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
    if (e == hipSuccess) e = hipMalloc(&p.d.mp_ell, G * p.K * p.N * kGroup * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&p.d.mp_z, G * p.N * p.N * kGroup * sizeof(float));
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
        hipLaunchKernelGGL(mp_prologue_kernel, dim3((a.G + kWavesPerBlock - 1) / kWavesPerBlock),
                           dim3(kBlock), 0, st, a);
        const int64_t items = (int64_t)(p.N - 1) * a.G;
        if (items > 0) {
            const dim3 grid(static_cast<unsigned>((items + kWavesPerBlock - 1) / kWavesPerBlock));
            if (p.s <= 8)
                hipLaunchKernelGGL(mp_item_kernel<8>, grid, dim3(kBlock), 0, st, a);
            else
                hipLaunchKernelGGL(mp_item_kernel<16>, grid, dim3(kBlock), 0, st, a);
        }
        switch (p.nmax) {
            case 8: launch_mp_payoff<8>(pa, a.z, first, n_chunk, st); break;
            case 16: launch_mp_payoff<16>(pa, a.z, first, n_chunk, st); break;
            case 24: launch_mp_payoff<24>(pa, a.z, first, n_chunk, st); break;
            case 32: launch_mp_payoff<32>(pa, a.z, first, n_chunk, st); break;
            case 40: launch_mp_payoff<40>(pa, a.z, first, n_chunk, st); break;
            case 64: launch_mp_payoff<64>(pa, a.z, first, n_chunk, st); break;
            default: return hipErrorInvalidValue;
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace lll
