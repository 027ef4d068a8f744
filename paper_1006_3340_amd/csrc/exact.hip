// exact.hip -- the FULL Euler scheme with the drift of its exact subset expansion.
//
// Writing beta_l(x) = (1 - ell_l) + ell_l e^{lambda_l x} in the product of
// eq. (LIBOR-drift-PT) and expanding the product over the subsets U of the
// later rates (paper Section 3.2, eq. (product)) turns the jump integral of
// the drift into closed-form cumulants:
//     b_i = -kappa(lambda_i) - C_i,   C_i = sum_U p_U K_i(U),
//     p_U = prod_{l in U} ell_l prod_{l > i, l not in U} (1 - ell_l),
//     K_i(U) = kappa(lambda_i + lambda_U) - kappa(lambda_U) - kappa(lambda_i),
// lambda_U = sum_{l in U} lambda_l (K_i of the empty set is 0).  This is the
// paper's exact ("full") drift: no quadrature, 2^{N-1-i} terms for rate i.
//
// The coefficients K are the same for every path: one FP64 table per Euler
// step, built on the device and stored in the plan precision.  Step k of
// period m holds the live rates i = m .. N-1 one after the other, rate i with
// 2^M entries (M = N-1-i later rates).  Entry e of rate i names U by bits: for
// M <= 4, bit b of e is rate i+1+b; for M > 4, e = 16 t + lo with lo's bits
// the rates i+1 .. i+4 and t's bit b the rate i+5+b.  Offsets:
//     step k = m s + js:  s (2^{N+1} - 2^{N+1-m} - m) + js (2^{N-m} - 1),
//     rate i in the step: 2^{N-m} - 2^{N-i},
// s (2^{N+1} - 2 - N) entries in all.
//
// The path kernel (one path per lane, state in registers, the same random
// numbers, payoffs and reduction as the other path kernels) evaluates, per
// rate, p_U = q_i prod_{l in U} r_l with q_i = prod_{l > i}(1 - ell_l) and
// r_l = ell_l / (1 - ell_l): the 16 products over the first four later rates
// are formed once per rate and step, and the remaining rates are enumerated in
// binary order (t) with a stack of prefix products P_b = prod over the bits
// >= b of t, so that every p_U is a product of at most M rounded factors.  The
// table rows are the same for every lane: a rate with at most 16 entries reads
// them as scalar loads, a longer one through the wavefront's LDS in 1 KiB
// chunks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>

#include "lll_device.hpp"
#include "lll_internal.hpp"
#include "path_kernel.hpp"

namespace lll {
namespace {

using detail::cptr;
using detail::PathArgs;

constexpr int kLo = 4;  // later rates whose products are formed in registers

// The coefficients of a rate with more than four later rates (more than 16
// entries) are staged through the wavefront's own LDS buffers in chunks of
// 1 KiB (64 lanes x 16 B), loaded kAhead chunks ahead with coalesced vector
// loads: wave-uniform scalar loads of the same rows left the kernel waiting on
// memory latency.
constexpr int kAhead = 3;
template <typename Real>
constexpr int kPer = 16 / sizeof(Real);  // values per lane and chunk
template <typename Real>
constexpr int kChunk = kWave * kPer<Real>;

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Entries of step k's table before step k (period m = k / s, js = k % s).
__host__ __device__ inline int64_t exact_step_base(int N, int s, int k) {
    const int m = k / s, js = k % s;
    const int64_t one = 1;
    return static_cast<int64_t>(s) * ((one << (N + 1)) - (one << (N + 1 - m)) - m) +
           static_cast<int64_t>(js) * ((one << (N - m)) - 1);
}

// One thread per table entry of step k (blockIdx.y strides over the steps).
template <typename Real>
__global__ void __launch_bounds__(256) exact_table_kernel(const double *__restrict__ vol, int N,
                                                          int s, int K, int driver, double alpha,
                                                          double beta, double delta_nig, double c,
                                                          Real *__restrict__ kex) {
    const bool nig = driver == LLL_DRIVER_NIG;
    for (int k = blockIdx.y; k < K; k += gridDim.y) {
        const int m = k / s;
        const int64_t n_step = (static_cast<int64_t>(1) << (N - m)) - 1;
        int64_t q = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
        if (q >= n_step) continue;
        const int64_t flat = exact_step_base(N, s, k) + q;
        const double *lam = vol + static_cast<size_t>(k) * N;
        int i = m;
        while (q >= (static_cast<int64_t>(1) << (N - 1 - i))) {
            q -= static_cast<int64_t>(1) << (N - 1 - i);
            ++i;
        }
        const int M = N - 1 - i;
        double lu = 0.0;
        if (M <= kLo) {
            for (int b = 0; b < M; ++b)
                if ((q >> b) & 1) lu += lam[i + 1 + b];
        } else {
            for (int b = 0; b < kLo; ++b)
                if ((q >> b) & 1) lu += lam[i + 1 + b];
            const int64_t t = q >> kLo;
            for (int b = 0; b < M - kLo; ++b)
                if ((t >> b) & 1) lu += lam[i + 1 + kLo + b];
        }
        const double li = lam[i];
        const double v = nig ? nig_cumulant(li + lu, alpha, beta, delta_nig) -
                                   nig_cumulant(lu, alpha, beta, delta_nig) -
                                   nig_cumulant(li, alpha, beta, delta_nig)
                             : c * li * lu;  // c (li + lu)^2 / 2 - c lu^2 / 2 - c li^2 / 2
        kex[flat] = static_cast<Real>(v);
    }
}

// sum_U (prod_{l in U} r_l) K_J(U) over the subsets U of the slots after J,
// kj = the table entries of slot J at this step, wbuf = the wavefront's two
// LDS chunk buffers.
template <typename Real, int NMAX, int J>
__device__ __forceinline__ Real subset_sum(const Real (&r)[NMAX], cptr<Real> kj, Real *wbuf) {
    constexpr int M = NMAX - 1 - J;
    constexpr int h = M < kLo ? M : kLo;
    constexpr int H = M - h;
    Real plo[1 << h];
    plo[0] = Real(1);
#pragma unroll
    for (int b = 0; b < h; ++b)
#pragma unroll
        for (int e = 0; e < (1 << b); ++e) plo[e | (1 << b)] = plo[e] * r[J + 1 + b];
    if constexpr (H == 0) {
        Real sum = Real(0);
#pragma unroll
        for (int e = 0; e < (1 << h); ++e) sum = fma(plo[e], kj[e], sum);
        return sum;
    } else {
        // t = 2^hm u + v: v's (up to two) bits in registers (qm), u's bits on
        // the stack P[b] = prod over the set bits b' >= b of u of r of slot
        // J+1+kLo+hm+b'
        constexpr int hm = H < 2 ? H : 2;
        constexpr int Hs = H - hm;
        Real qm[1 << hm];
        qm[0] = Real(1);
#pragma unroll
        for (int b = 0; b < hm; ++b)
#pragma unroll
            for (int v = 0; v < (1 << b); ++v) qm[v | (1 << b)] = qm[v] * r[J + 1 + kLo + b];
        Real P[Hs + 1];
#pragma unroll
        for (int b = 0; b <= Hs; ++b) P[b] = Real(1);
        constexpr int n = 1 << M;                      // entries of slot J
        constexpr int chunk = kChunk<Real>;
        constexpr int nch = n > chunk ? n / chunk : 1;  // n is a multiple of chunk
        constexpr int per = n > chunk ? chunk : n;      // entries per chunk
        constexpr int tpc = per / (1 << kLo);           // blocks of 16 per chunk
        const int lane = threadIdx.x % kWave;
        // value i of a lane is entry i * 64 + lane of its chunk
        Real pre[kAhead][kPer<Real>];
#pragma unroll
        for (int d = 0; d < kAhead; ++d)
#pragma unroll
            for (int i = 0; i < kPer<Real>; ++i) {
                const int pos = i * kWave + lane;
                pre[d][i] = (d < nch && pos < per) ? kj[static_cast<size_t>(d) * chunk + pos] : Real(0);
            }
        Real total = Real(0);
        int u = 0;
#pragma unroll 1
        for (int c = 0; c < nch; ++c) {
            Real *buf = wbuf + (c & 1) * chunk;
#pragma unroll
            for (int i = 0; i < kPer<Real>; ++i) {
                const int pos = i * kWave + lane;
                if (pos < per) buf[pos] = pre[0][i];
            }
#pragma unroll
            for (int d = 0; d + 1 < kAhead; ++d)
#pragma unroll
                for (int i = 0; i < kPer<Real>; ++i) pre[d][i] = pre[d + 1][i];
            const int cn = c + kAhead;
#pragma unroll
            for (int i = 0; i < kPer<Real>; ++i) {
                const int pos = i * kWave + lane;
                pre[kAhead - 1][i] =
                    (cn < nch && pos < per) ? kj[static_cast<size_t>(cn) * chunk + pos] : Real(0);
            }
            wave_sync();  // the chunk's LDS values are visible to every lane
#pragma unroll 1
            for (int tt = 0; tt < tpc; tt += 1 << hm, ++u) {
                // 2^hm blocks of 16, each as four independent FMA chains (one
                // wavefront per SIMD is common here, so long chains would
                // leave the ALU waiting)
                Real grp = Real(0);
#pragma unroll
                for (int v = 0; v < (1 << hm); ++v) {
                    const Real *kt = buf + (tt + v) * (1 << kLo);
                    Real in4[4] = {Real(0), Real(0), Real(0), Real(0)};
#pragma unroll
                    for (int e = 0; e < (1 << kLo); ++e)
                        in4[e & 3] = fma(plo[e], kt[e], in4[e & 3]);
                    grp = fma(qm[v], (in4[0] + in4[1]) + (in4[2] + in4[3]), grp);
                }
                total = fma(P[0], grp, total);
                // u -> u + 1: bit cb is set, the bits below it are cleared
                const int cb = __builtin_ctz(static_cast<unsigned>(u + 1));
#pragma unroll
                for (int b = Hs - 1; b >= 0; --b) {
                    if (b == cb)
                        P[b] = P[b + 1] * r[J + 1 + kLo + hm + b];
                    else if (b < cb)
                        P[b] = P[b + 1];
                }
            }
        }
        wave_sync();  // the last reads are done before the buffers are reused
        return total;
    }
}

// Slots J, J-1, .., J0: coupling of slot J (q = prod over the later slots of
// 1 - ell) and its Euler update; the ell of every slot were taken before.
template <typename Real, int NMAX, int J, int J0>
__device__ __forceinline__ void exact_rates(const PathArgs<Real> &a, cptr<Real> kstep, int k,
                                            Real dH, const Real (&r)[NMAX], const Real (&om)[NMAX],
                                            Real q, Real (&X)[NMAX], Real *wbuf) {
    if constexpr (J >= J0) {
        constexpr int64_t off = (static_cast<int64_t>(1) << (NMAX - J0)) -
                                (static_cast<int64_t>(1) << (NMAX - J));
        const Real C = q * subset_sum<Real, NMAX, J>(r, kstep + off, wbuf);
        const Real dt = a.dt[k];
        X[J] += fma(a.lam[(size_t)k * NMAX + J], dH, fma(-C, dt, a.drift0[(size_t)k * NMAX + J]));
        exact_rates<Real, NMAX, J - 1, J0>(a, kstep, k, dH, r, om, q * om[J], X, wbuf);
    }
}

template <typename Real, int NMAX, int J0>
__device__ __forceinline__ void exact_step(const PathArgs<Real> &a, cptr<Real> kstep, int k, Real dH,
                                           Real (&X)[NMAX], Real *wbuf) {
    Real r[NMAX], om[NMAX];
#pragma unroll
    for (int j = J0; j < NMAX; ++j) {
        const Real ce = a.cinv[j] * exp(-X[j]);  // 1 / (delta L)
        r[j] = Real(1) / ce;                     // ell / (1 - ell) = delta L
        om[j] = ce / (Real(1) + ce);             // 1 - ell
    }
    exact_rates<Real, NMAX, NMAX - 1, J0>(a, kstep, k, dH, r, om, Real(1), X, wbuf);
}

// The first live slot j0 = NMAX - N + m is at least NMAX - LLL_N_MAX_EXACT:
// only those slots get code (J0 = kExactLow + Js).
template <int NMAX>
constexpr int kExactLow = NMAX > LLL_N_MAX_EXACT ? NMAX - LLL_N_MAX_EXACT : 0;

template <typename Real, int NMAX, int... Js>
__device__ __forceinline__ void dispatch_exact_step(std::integer_sequence<int, Js...>, int j0,
                                                    const PathArgs<Real> &a, cptr<Real> kstep,
                                                    int k, Real dH, Real (&X)[NMAX], Real *wbuf) {
    constexpr int lo = kExactLow<NMAX>;
    (void)((j0 == lo + Js ? (exact_step<Real, NMAX, lo + Js>(a, kstep, k, dH, X, wbuf), 0) : 0) +
           ...);
}

template <typename Real, int NMAX, int PRODUCT>
__global__ void __launch_bounds__(kBlock) exact_kernel(PathArgs<Real> a, cptr<Real> kex) {
    __shared__ Real kbuf[kBlock / kWave][2 * kChunk<Real>];  // per wavefront, two chunks
    Real *wbuf = kbuf[threadIdx.x / kWave];
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int64_t wave_first = gid - (threadIdx.x % kWave);
    if (wave_first >= a.n_paths) return;  // whole wavefront past the end
    const bool active = gid < a.n_paths;
    const int64_t p = a.path_offset + gid;
    const uint32_t p_lo = static_cast<uint32_t>(p);
    const uint32_t p_hi = static_cast<uint32_t>(static_cast<uint64_t>(p) >> 32);
    const bool brownian = a.brownian != 0;
    Real X[NMAX];
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
        dispatch_exact_step<Real, NMAX>(std::make_integer_sequence<int, NMAX - kExactLow<NMAX>>{}, j0,
                                        a, kex + exact_step_base(a.N, a.s, k), k, dH, X, wbuf);
        if (++js == a.s) {
            detail::dispatch_payoff<Real, NMAX, PRODUCT>(std::make_integer_sequence<int, NMAX>{}, j0,
                                                         a, m, gid, active, X);
            js = 0;
            ++m;
        }
    }
}

template <typename Real, int NMAX>
hipError_t launch_exact_n(const PathArgs<Real> &a, cptr<Real> kex, int64_t n_paths, hipStream_t st) {
    const dim3 grid(static_cast<unsigned>((n_paths + kBlock - 1) / kBlock));
    if (a.product == LLL_SWAPTIONS)
        hipLaunchKernelGGL((exact_kernel<Real, NMAX, LLL_SWAPTIONS>), grid, dim3(kBlock), 0, st, a,
                           kex);
    else
        hipLaunchKernelGGL((exact_kernel<Real, NMAX, LLL_CAPLETS>), grid, dim3(kBlock), 0, st, a,
                           kex);
    return hipGetLastError();
}

template <typename Real>
hipError_t launch_exact_t(const lll_plan &p, int64_t n_paths, int64_t path_offset, uint64_t seed,
                          double *path_fix, hipStream_t st) {
    Real *kex = static_cast<Real *>(p.d.kex);
    const int64_t max_step = (static_cast<int64_t>(1) << p.N) - 1;
    const dim3 tgrid(static_cast<unsigned>((max_step + 255) / 256),
                     static_cast<unsigned>(std::min(p.K, 65535)));
    hipLaunchKernelGGL(exact_table_kernel<Real>, tgrid, dim3(256), 0, st, p.d.vol, p.N, p.s, p.K,
                       p.driver, p.alpha, p.beta, p.delta_nig, p.c, kex);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const PathArgs<Real> a = detail::make_args<Real>(p, seed, n_paths, path_offset, path_fix);
    const cptr<Real> kc = detail::as_const(static_cast<const Real *>(kex));
    switch (p.nmax) {
        case 8: return launch_exact_n<Real, 8>(a, kc, n_paths, st);
        case 16: return launch_exact_n<Real, 16>(a, kc, n_paths, st);
        case 24: return launch_exact_n<Real, 24>(a, kc, n_paths, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int64_t exact_table_entries(int N, int s) {
    return static_cast<int64_t>(s) * ((static_cast<int64_t>(1) << (N + 1)) - 2 - N);
}

hipError_t launch_exact(const lll_plan &p, int64_t n_paths, int64_t path_offset, uint64_t seed,
                        double *path_fix, hipStream_t st) {
    if (!p.d.kex || p.N > LLL_N_MAX_EXACT || p.N < 1) return hipErrorInvalidValue;
    return p.precision == LLL_FP64 ? launch_exact_t<double>(p, n_paths, path_offset, seed, path_fix, st)
                                   : launch_exact_t<float>(p, n_paths, path_offset, seed, path_fix, st);
}

}  // namespace lll
