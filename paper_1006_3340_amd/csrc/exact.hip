// exact.hip -- the FULL Euler scheme with the drift of its exact subset
// expansion, the subset sums on the matrix cores.
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
// Factorisation.  With r_l = ell_l / (1 - ell_l) = delta_l L_l and
// q_i = prod_{l > i} (1 - ell_l), p_U = q_i prod_{l in U} r_l.  Split the
// later rates of rate i into the low group -- the last G = 6 rates of the
// tenor -- and the high rates between (h of them).  A subset U is a pair
// (t, u) of a low subset t (64 of them) and a high subset u (2^h), and
//     C_i = q_i sum_t R(t) sum_u K_i[t][u] P(u),
//     R(t) = prod_{l in t} r_l,  P(u) = prod_{l in u} r_l.
// The coefficients K_i are the same for every path, so for 16 paths at once
// the inner sum is a matrix product Y = K_i (64 x 2^h) . P (2^h x 16 paths),
// run on v_mfma_f32_16x16x4f32 (FP64 plans: v_mfma_f64_16x16x4f64), and
// C_i = q_i sum_t R(t) Y[t] per path (16 products per lane and two lane
// exchanges; the two instructions place the result rows differently over a
// lane's elements and the lane groups).  With non-negative lambda every term
// is non-negative (kappa is convex with kappa(0) = 0, so superadditive on the
// positive axis) and the sums have no cancellation.
//
// Rates are held in NX = LLL_N_MAX_EXACT slots with the last rate in slot
// NX-1 (slot J is rate J - (NX - N)), so that the low group is always slots
// NX-6 .. NX-1 and every slot index in the code is a compile-time constant.
//
// Table (one per Euler step, built on the device in FP64 and stored in the
// plan precision): the coupled live slots J = j0 .. NX-2 one after the other,
// slot J with U_J = max(4, 2^h_J) columns (h_J = NX-7-J high rates; padded to
// the matrix cores' K step of 4), laid out as the A-operand fragments of the
// 16x16x4 products: [u / 4][t / 16][lane], lane = t % 16 + 16 (u % 4).  An
// entry whose subset names a slot at or before J (a low-group bit) or a
// padding column is 0.  Slot J's offset inside a step is cum(J) - cum(j0)
// with cum(J) = sum_{J' < J} 64 U_J'.
//
// One launch per period, every wavefront at the same step at about the same
// time, so each step's table is shared through the L2: a wavefront takes 16 T
// paths (T column tiles of 16); lane 16 g + n holds path n of each tile.  It
// moves the paths' states ([N][paths] in HBM) into its LDS for the period,
// and per step draws their increments, forms r, runs the products of every
// coupled slot and updates the states.  A payoff kernel (one path per lane,
// the path kernels' payoff code, so the same reduction) then reads them.
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

constexpr int kNX = LLL_N_MAX_EXACT;  // slots
constexpr int kG = 6;                 // low group: the last kG slots, the 64 rows
constexpr int kRows = 1 << kG;
// Table chunks (4 columns, 256 entries) loaded ahead of the products; the
// table is padded by as many chunks so that these loads need no bound.
constexpr int kAhead = 4;
constexpr int64_t kTablePad = kAhead * 256;

// High rates of slot J (slots J+1 .. NX-G-1).
__host__ __device__ constexpr int high_rates(int J) {
    return kNX - kG - 1 - J > 0 ? kNX - kG - 1 - J : 0;
}
// Columns of slot J (high subsets, padded to the matrix K step of 4).
__host__ __device__ constexpr int slot_cols(int J) {
    return high_rates(J) <= 2 ? 4 : (1 << high_rates(J));
}
// Entries of slots 0 .. J-1: the slots with 2^h columns (h >= 3) sum to a
// geometric series, the others have 4 columns each.
__host__ __device__ constexpr int64_t slot_cum(int J) {
    constexpr int H0 = kNX - kG - 1;                 // high rates of slot 0
    const int a = J < H0 - 2 ? J : H0 - 2;           // slots with 2^h columns
    const int64_t geo = (int64_t(1) << (H0 + 1)) - (int64_t(1) << (H0 + 1 - a));
    return kRows * geo + int64_t(kRows) * 4 * (J > H0 - 2 ? J - (H0 - 2) : 0);
}
constexpr bool slot_cum_checks() {
    int64_t c = 0;
    for (int J = 0; J <= kNX; ++J) {
        if (slot_cum(J) != c) return false;
        c += static_cast<int64_t>(kRows) * slot_cols(J);
    }
    return true;
}
static_assert(slot_cum_checks(), "slot offsets");
// Entries of one step of period m (coupled live slots j0 .. NX-2, j0 = NX - N + m).
__host__ __device__ inline int64_t step_entries(int N, int m) {
    return slot_cum(kNX - 1) - slot_cum(kNX - N + m);
}
// Entries of the steps before step k.
__host__ __device__ inline int64_t step_base(int N, int s, int k) {
    const int m = k / s, js = k % s;
    int64_t b = 0;
    for (int mm = 0; mm < m; ++mm) b += static_cast<int64_t>(s) * step_entries(N, mm);
    return b + static_cast<int64_t>(js) * step_entries(N, m);
}

template <typename Real>
struct Mfma;
// Result rows of a lane: lane 16 g + n holds column n of rows 4 g + e (FP32
// instruction) or rows g + 4 e (FP64 instruction), e = 0..3 its result
// element.  kElemLow: the element index gives the row's low two bits.
template <>
struct Mfma<float> {
    typedef float vec4 __attribute__((ext_vector_type(4)));
    static constexpr bool kElemLow = true;
    __device__ static vec4 run(float a, float b, vec4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <>
struct Mfma<double> {
    typedef double vec4 __attribute__((ext_vector_type(4)));
    static constexpr bool kElemLow = false;
    __device__ static vec4 run(double a, double b, vec4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

// One thread per table entry.  A step's entries are a whole number of blocks
// (64 rows times a multiple of 4 columns per slot), so every block lies in one
// step: the block finds its period, step and offset (uniform work).
template <typename Real>
__global__ void __launch_bounds__(256) exact_table_kernel(const double *__restrict__ vol, int N,
                                                          int s, int driver, double alpha,
                                                          double beta, double delta_nig, double c,
                                                          Real *__restrict__ kex) {
    const bool nig = driver == LLL_DRIVER_NIG;
    const int offx = kNX - N;
    int64_t b = blockIdx.x, base = 0;  // base: entries of the periods before m
    int m = 0;
    int64_t bm = step_entries(N, 0) / 256;  // blocks per step of period m
    while (m < N - 1 && b >= s * bm) {
        b -= s * bm;
        base += s * bm * 256;
        ++m;
        bm = step_entries(N, m) / 256;
    }
    if (bm == 0) return;
    const int js = static_cast<int>(b / bm);
    const int k = m * s + js;
    int64_t q = (b % bm) * 256 + threadIdx.x;
    const int64_t flat = base + js * bm * 256 + q;
    const int j0 = offx + m;
    {
        int J = j0;
        while (q >= static_cast<int64_t>(kRows) * slot_cols(J)) {
            q -= static_cast<int64_t>(kRows) * slot_cols(J);
            ++J;
        }
        // q = ((u / 4) * 4 + t / 16) * 64 + t % 16 + 16 (u % 4)
        const int lane = static_cast<int>(q % 64);
        const int t = 16 * static_cast<int>((q / 64) % 4) + lane % 16;
        const int64_t u = 4 * (q / 256) + lane / 16;
        const int h = high_rates(J);
        const double *lam = vol + static_cast<size_t>(k) * N;  // rate index = slot - offx
        bool valid = u < (static_cast<int64_t>(1) << h);
        double lu = 0.0;
        for (int b = 0; b < h && valid; ++b)
            if ((u >> b) & 1) lu += lam[J + 1 + b - offx];
        for (int b = 0; b < kG && valid; ++b) {
            if (!((t >> b) & 1)) continue;
            const int slot = kNX - kG + b;
            if (slot <= J) valid = false;  // not a later rate (or no rate at all)
            else lu += lam[slot - offx];
        }
        double v = 0.0;
        if (valid) {
            const double li = lam[J - offx];
            v = nig ? nig_cumulant(li + lu, alpha, beta, delta_nig) -
                          nig_cumulant(lu, alpha, beta, delta_nig) -
                          nig_cumulant(li, alpha, beta, delta_nig)
                    : c * li * lu;  // c (li + lu)^2 / 2 - c lu^2 / 2 - c li^2 / 2
        }
        kex[flat] = static_cast<Real>(v);
    }
}

// Where period m's steps sit in the table (entries): the first step, the
// step size and the offset of the first live slot within a step's layout.
struct PeriodTable {
    int64_t base, step, cum0;
};

template <typename Real, int T>
struct StepState {
    Real r[T][kNX];                  // delta L of every slot (0 if fixed or absent)
    Real q[T];                       // prod over the slots after the current one of 1 - ell
    Real pe[T][4], pg[T], pt[T][4];  // factors of R(t): element, lane group, row tile
};

// sum_t R(t) sum_u K_J[t][u] P(u) of each tile's path (the same value in the
// four lanes of a path).
// pre: this slot's first table chunk, loaded before the call; on return it
// holds the next slot's (knext, when has_next), loaded while this slot runs.
template <typename Real, int T, int J>
__device__ __forceinline__ void slot_sum(const StepState<Real, T> &st, cptr<Real> kslot, int lane,
                                         Real (&pre)[4], cptr<Real> knext, bool has_next,
                                         Real (&out)[T]) {
    typedef typename Mfma<Real>::vec4 vec4;
    constexpr int h = high_rates(J);
    constexpr int hk = h > 2 ? h - 2 : 0;  // bits of the column-chunk index kc (chunks of 4)
    constexpr int lb = hk < 3 ? hk : 3;    // low bits of kc: the unrolled inner loop
    constexpr int hb = hk - lb;            // high bits of kc: the outer loop
    constexpr int ni = 1 << lb, no = 1 << hb, nkc = ni * no;
    constexpr int D = ni < kAhead ? ni : kAhead;  // chunks of the table in flight
    const int g = lane / 16;
    // P(u) of column u = 4 kc + g = bin[kc % ni] stk[0]: the two low bits of u
    // from g (slots J+1, J+2) and the low bits of kc (slots J+3 ..) in bin, the
    // high bits of kc in the prefix products stk[b] = prod over the set bits
    // b' >= b of kc / ni of r of slot J+3+lb+b'
    Real bin[T][ni], stk[T][hb + 1];
#pragma unroll
    for (int c = 0; c < T; ++c) {
        Real f0 = Real(1), f1 = Real(1);
        if constexpr (h > 0) {
            if (g & 1) f0 = st.r[c][J + 1];
        } else {
            if (g & 1) f0 = Real(0);
        }
        if constexpr (h > 1) {
            if (g & 2) f1 = st.r[c][J + 2];
        } else {
            if (g & 2) f1 = Real(0);
        }
        bin[c][0] = f0 * f1;
#pragma unroll
        for (int b = 0; b < lb; ++b)
#pragma unroll
            for (int i = 0; i < (1 << b); ++i) bin[c][i | (1 << b)] = bin[c][i] * st.r[c][J + 3 + b];
#pragma unroll
        for (int b = 0; b <= hb; ++b) stk[c][b] = Real(1);
    }
    // FP32: two accumulator sets, even and odd chunks, so that a product's
    // accumulator is reused 16 products later instead of 8 (8 accumulators
    // per wavefront reach 128 TFLOP/s of 16x16x4 FP32 products at two
    // wavefronts per SIMD, 16 reach 150).  FP64 keeps one set: its registers
    // hold one wavefront per SIMD either way.
    constexpr int NS = (ni > 1 && sizeof(Real) == 4) ? 2 : 1;
    vec4 acc[NS][4][T];
#pragma unroll
    for (int h2 = 0; h2 < NS; ++h2)
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int c = 0; c < T; ++c) acc[h2][rt][c] = vec4{0, 0, 0, 0};
    const cptr<Real> kp = kslot + lane;
    Real A[D][4];  // ring of table fragments, D chunks ahead of the products
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) A[0][rt] = pre[rt];
#pragma unroll
    for (int d = 1; d < D; ++d)
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) A[d][rt] = kp[(d * 4 + rt) * kWave];
    if (has_next) {
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) pre[rt] = knext[lane + rt * kWave];
    }
#pragma unroll 1
    for (int ko = 0; ko < no; ++ko) {
#pragma unroll
        for (int i = 0; i < ni; ++i) {
            // keep each chunk's products and its ring load together: left to
            // itself the scheduler hoists the loads to the iteration's top and
            // drains them at its end, which breaks the ring at the back edge
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int c = 0; c < T; ++c) {
                const Real B = bin[c][i] * stk[c][0];
#pragma unroll
                for (int rt = 0; rt < 4; ++rt)
                    acc[i % NS][rt][c] = Mfma<Real>::run(A[i % D][rt], B, acc[i % NS][rt][c]);
            }
            // the chunk this ring slot takes next: past the slot's end it reads
            // the next slot's entries or the table's padding, never used
            const int kn = ko * ni + i + D;
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) A[i % D][rt] = kp[(kn * 4 + rt) * kWave];
        }
        if constexpr (hb > 0) {
            // ko -> ko + 1: bit cb is set and the bits below it cleared
            const int cb = __builtin_ctz(static_cast<unsigned>(ko + 1));
#pragma unroll
            for (int c = 0; c < T; ++c)
#pragma unroll
                for (int b = hb - 1; b >= 0; --b) {
                    if (b == cb)
                        stk[c][b] = stk[c][b + 1] * st.r[c][J + 3 + lb + b];
                    else if (b < cb)
                        stk[c][b] = stk[c][b + 1];
                }
        }
    }
    // result rows of the lane: R(t) = pe[e] pg pt[rt] (element e, row tile rt)
#pragma unroll
    for (int c = 0; c < T; ++c) {
        Real sum = Real(0);
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) {
            Real row = Real(0);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                Real y = acc[0][rt][c][e];
                if constexpr (NS > 1) y += acc[1][rt][c][e];
                row = fma(st.pe[c][e], y, row);
            }
            sum = fma(st.pt[c][rt], row, sum);
        }
        sum *= st.pg[c];
        sum += __shfl_xor(sum, 16, kWave);
        sum += __shfl_xor(sum, 32, kWave);
        out[c] = sum;
    }
}

// Slots J, J-1, .., j0 (descending): the coupling sum of slot J, then the
// Euler update of its state in the wavefront's LDS (every slot's r was taken
// at the start of the step).  The four lanes of a path update the same state
// to the same value and each reads it back at the next step: every lane sees
// its own write.
template <typename Real, int T, int J>
__device__ __forceinline__ void exact_slots(const PathArgs<Real> &a, StepState<Real, T> &st,
                                            cptr<Real> kstep, int64_t cum0, int k, int j0, int offx,
                                            int lane, const Real (&dH)[T], Real (*xw)[16 * T],
                                            Real (&pre)[4]) {
    if constexpr (J >= 0) {
        if (J < j0) return;
        Real C[T];
        if constexpr (J == kNX - 1) {
#pragma unroll
            for (int c = 0; c < T; ++c) C[c] = Real(0);  // the last rate has no coupling
        } else {
            // the next slot (J - 1) is coupled when it is live
            constexpr int Jn = J > 0 ? J - 1 : 0;
            slot_sum<Real, T, J>(st, kstep + (slot_cum(J) - cum0), lane, pre,
                                 kstep + (slot_cum(Jn) - cum0), J > 0 && J - 1 >= j0, C);
#pragma unroll
            for (int c = 0; c < T; ++c) {
                st.q[c] *= Real(1) / (Real(1) + st.r[c][J + 1]);  // 1 - ell of slot J+1
                C[c] *= st.q[c];
            }
        }
        const size_t col = static_cast<size_t>(k) * (a.off + a.N) + (J - offx + a.off);
        const Real dt = a.dt[k], lam = a.lam[col], d0 = a.drift0[col];
        const int n = lane % 16;
#pragma unroll
        for (int c = 0; c < T; ++c) xw[J][16 * c + n] += fma(lam, dH[c], fma(-C[c], dt, d0));
        exact_slots<Real, T, J - 1>(a, st, kstep, cum0, k, j0, offx, lane, dH, xw, pre);
    }
}

// The s Euler steps of period m for 16 T paths per wavefront, the states in
// the wavefront's LDS for the period (slot-major, compile-time offsets).
// Two wavefronts per SIMD for FP32 plans (256 registers each; left to itself
// the compiler takes ~300 and one), one for FP64.
template <typename Real>
constexpr int kWavesPerSimd = sizeof(Real) == 4 ? 2 : 1;

template <typename Real, int T>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kWavesPerSimd<Real>)))
exact_period_kernel(PathArgs<Real> a, cptr<Real> kex,
                                                              Real *__restrict__ xs, int m,
                                                              PeriodTable pt) {
    __shared__ Real xl[kBlock / kWave][kNX][16 * T];
    const int lane = threadIdx.x % kWave;
    const int64_t wave = (static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x) / kWave;
    const int64_t p0 = wave * 16 * T;
    if (p0 >= a.n_paths) return;  // whole wavefront past the end
    Real(*xw)[16 * T] = xl[threadIdx.x / kWave];
    const int n = lane % 16, g = lane / 16;
    const int offx = kNX - a.N;
    const int j0 = offx + m;
    int64_t pidx[T];
    bool act[T];
#pragma unroll
    for (int c = 0; c < T; ++c) {
        pidx[c] = p0 + 16 * c + n;
        act[c] = pidx[c] < a.n_paths;
        if (g == 0)
#pragma unroll
            for (int J = 0; J < kNX; ++J)
                xw[J][16 * c + n] = (J >= j0 && act[c])
                                        ? xs[static_cast<int64_t>(J - offx) * a.n_paths + pidx[c]]
                                        : Real(0);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const cptr<double> sc = a.steps + 4 * m;
    const StepConsts cst{sc[0], sc[1], sc[2], sc[3]};
    // R(t) factors of the lane's result rows: bits 0-1 of t are slots NX-6,
    // NX-5, bits 2-3 slots NX-4, NX-3 (the element index e carries one pair,
    // the lane group g the other), bits 4-5 (row tile rt) slots NX-2, NX-1
    constexpr int se = Mfma<Real>::kElemLow ? kNX - 6 : kNX - 4;
    constexpr int sg = Mfma<Real>::kElemLow ? kNX - 4 : kNX - 6;
    const int64_t cum0 = pt.cum0;
    // Driver increments: the four lane groups hold T tiles x SB steps, so each
    // lane draws one increment per SB steps (lane group g: tile g % T, step
    // g / T of the batch) and the steps read them with lane shuffles.
    constexpr int SB = 4 / T;
    Real inc = Real(0);
#pragma unroll 1
    for (int js = 0; js < a.s; ++js) {
        const int k = m * a.s + js;
        if (js % SB == 0) {
            const int jd = js + g / T;
            if (jd < a.s) {
                const int64_t p = a.path_offset + p0 + 16 * (g % T) + n;
                const uint4 w = philox4x32_10(
                    make_uint4(static_cast<uint32_t>(m * a.s + jd), static_cast<uint32_t>(p),
                               static_cast<uint32_t>(static_cast<uint64_t>(p) >> 32),
                               a.stream_word),
                    a.key0, a.key1);
                inc = static_cast<Real>(increment(w, cst, a.beta, a.brownian != 0, nullptr));
            }
        }
        Real dH[T];
        StepState<Real, T> st;
#pragma unroll
        for (int c = 0; c < T; ++c) {
            dH[c] = __shfl(inc, 16 * ((js % SB) * T + c) + n, kWave);
            st.q[c] = Real(1);
#pragma unroll
            for (int J = 0; J < kNX; ++J) {  // delta L of the live slots, 0 for the others
                Real rr = Real(0);
                if (J >= j0) {
                    const int sl = J - offx + a.off;
                    rr = static_cast<Real>(a.deltas[sl] * a.L0s[sl]) * exp(xw[J][16 * c + n]);
                }
                st.r[c][J] = rr;
            }
            const Real *r = st.r[c];
#pragma unroll
            for (int e = 0; e < 4; ++e)
                st.pe[c][e] = ((e & 1) ? r[se] : Real(1)) * ((e & 2) ? r[se + 1] : Real(1));
            st.pg[c] = ((g & 1) ? r[sg] : Real(1)) * ((g & 2) ? r[sg + 1] : Real(1));
#pragma unroll
            for (int rt = 0; rt < 4; ++rt)
                st.pt[c][rt] =
                    ((rt & 1) ? r[kNX - 2] : Real(1)) * ((rt & 2) ? r[kNX - 1] : Real(1));
        }
        const cptr<Real> kstep = kex + pt.base + js * pt.step;
        // first table chunk of the first coupled slot (NX - 2), when it is live
        Real pre[4] = {Real(0), Real(0), Real(0), Real(0)};
        if (kNX - 2 >= j0) {
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) pre[rt] = kstep[slot_cum(kNX - 2) - cum0 + lane + rt * kWave];
        }
        exact_slots<Real, T, kNX - 1>(a, st, kstep, cum0, k, j0, offx, lane, dH, xw, pre);
    }
    if (g == 0) {
#pragma unroll
        for (int c = 0; c < T; ++c)
            if (act[c]) {
#pragma unroll
                for (int J = 0; J < kNX; ++J)
                    if (J >= j0) xs[static_cast<int64_t>(J - offx) * a.n_paths + pidx[c]] = xw[J][16 * c + n];
            }
    }
}

// Payoffs at the end of period m from the states in HBM: one path per lane
// and the path kernels' payoff code (per-wavefront partials).  The first live
// slot is j0 = off + m >= NMAX - LLL_N_MAX_EXACT (N <= LLL_N_MAX_EXACT), so
// only the slots from kJ0Min on get a copy of the payoff code.
template <int NMAX>
constexpr int kJ0Min = NMAX > LLL_N_MAX_EXACT ? NMAX - LLL_N_MAX_EXACT : 0;

template <typename Real, int NMAX, int PRODUCT, int... Js>
__device__ __forceinline__ void exact_payoff_dispatch(std::integer_sequence<int, Js...>, int j0,
                                                      const PathArgs<Real> &a, int m, int64_t gid,
                                                      bool active, const Real (&X)[NMAX]) {
    (void)((j0 == kJ0Min<NMAX> + Js
                ? (detail::payoff<Real, NMAX, kJ0Min<NMAX> + Js, PRODUCT>(a, m, gid, active, X), 0)
                : 0) +
           ...);
}

template <typename Real, int NMAX, int PRODUCT>
__global__ void __launch_bounds__(kBlock) exact_payoff_kernel(PathArgs<Real> a,
                                                              const Real *__restrict__ xs, int m) {
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const int64_t wave_first = gid - (threadIdx.x % kWave);
    if (wave_first >= a.n_paths) return;  // whole wavefront past the end
    const bool active = gid < a.n_paths;
    const int j0 = a.off + m;
    Real X[NMAX];
#pragma unroll
    for (int j = 0; j < NMAX; ++j)
        X[j] = (j >= j0 && active) ? xs[static_cast<int64_t>(j - a.off) * a.n_paths + gid] : Real(0);
    exact_payoff_dispatch<Real, NMAX, PRODUCT>(
        std::make_integer_sequence<int, NMAX - kJ0Min<NMAX>>{}, j0, a, m, gid, active, X);
}

template <typename Real>
__global__ void __launch_bounds__(256) zero_state_kernel(Real *__restrict__ xs, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i < n) xs[i] = Real(0);
}

template <typename Real, int NMAX>
hipError_t launch_payoff_n(const PathArgs<Real> &a, const Real *xs, int m, hipStream_t st) {
    const dim3 grid(static_cast<unsigned>((a.n_paths + kBlock - 1) / kBlock));
    if (a.product == LLL_SWAPTIONS)
        hipLaunchKernelGGL((exact_payoff_kernel<Real, NMAX, LLL_SWAPTIONS>), grid, dim3(kBlock), 0,
                           st, a, xs, m);
    else
        hipLaunchKernelGGL((exact_payoff_kernel<Real, NMAX, LLL_CAPLETS>), grid, dim3(kBlock), 0,
                           st, a, xs, m);
    return hipGetLastError();
}

// 16-path column tiles per wavefront: two in FP32 (each table fragment feeds
// two products), one in FP64.
template <typename Real>
constexpr int kTiles = sizeof(Real) == 4 ? 2 : 1;

template <typename Real>
hipError_t launch_exact_t(const lll_plan &p, int64_t n_paths, int64_t path_offset, uint64_t seed,
                          double *path_fix, hipStream_t st) {
    Real *kex = static_cast<Real *>(p.d.kex);
    Real *xs = static_cast<Real *>(p.d.xex);
    hipError_t e = hipSuccess;
    const int64_t blocks = step_base(p.N, p.s, p.K) / 256;
    if (blocks > 0) {
        hipLaunchKernelGGL(exact_table_kernel<Real>, dim3(static_cast<unsigned>(blocks)), dim3(256),
                           0, st, p.d.vol, p.N, p.s, p.driver, p.alpha, p.beta, p.delta_nig, p.c,
                           kex);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int64_t n_state = static_cast<int64_t>(p.N) * n_paths;
    hipLaunchKernelGGL(zero_state_kernel<Real>, dim3(static_cast<unsigned>((n_state + 255) / 256)),
                       dim3(256), 0, st, xs, n_state);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const PathArgs<Real> a = detail::make_args<Real>(p, seed, n_paths, path_offset, path_fix);
    const cptr<Real> kc = detail::as_const(static_cast<const Real *>(kex));
    constexpr int T = kTiles<Real>;
    const int64_t waves = (n_paths + 16 * T - 1) / (16 * T);
    const dim3 grid(static_cast<unsigned>((waves * kWave + kBlock - 1) / kBlock));
    for (int m = 0; m < p.N && e == hipSuccess; ++m) {
        const PeriodTable pt{step_base(p.N, p.s, m * p.s), step_entries(p.N, m),
                             slot_cum(kNX - p.N + m)};
        hipLaunchKernelGGL((exact_period_kernel<Real, T>), grid, dim3(kBlock), 0, st, a, kc, xs, m,
                           pt);
        e = hipGetLastError();
        if (e == hipSuccess) {
            switch (p.nmax) {
                case 8: e = launch_payoff_n<Real, 8>(a, xs, m, st); break;
                case 16: e = launch_payoff_n<Real, 16>(a, xs, m, st); break;
                case 20: e = launch_payoff_n<Real, 20>(a, xs, m, st); break;
                case 24: e = launch_payoff_n<Real, 24>(a, xs, m, st); break;
                default: e = hipErrorInvalidValue;
            }
        }
    }
    return e;
}

}  // namespace

int64_t exact_table_entries(int N, int s) { return step_base(N, s, N * s) + kTablePad; }

int64_t exact_state_entries(int N, int64_t max_paths) {
    return static_cast<int64_t>(N) * max_paths;
}

hipError_t launch_exact(const lll_plan &p, int64_t n_paths, int64_t path_offset, uint64_t seed,
                        double *path_fix, hipStream_t st) {
    if (!p.d.kex || !p.d.xex || p.N > LLL_N_MAX_EXACT || p.N < 1 || n_paths > p.max_paths)
        return hipErrorInvalidValue;
    return p.precision == LLL_FP64
               ? launch_exact_t<double>(p, n_paths, path_offset, seed, path_fix, st)
               : launch_exact_t<float>(p, n_paths, path_offset, seed, path_fix, st);
}

}  // namespace lll
