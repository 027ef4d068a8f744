// fma_probe.hip -- measured ceiling of the roofline: the throughput of plain
// (non-packed) FP32 FMAs on the current GPU, the instruction the path kernels'
// coupling recursion is made of.  Every thread runs 8 independent FMA chains
// of kIters steps; 32 blocks of 256 threads per compute unit keep every SIMD
// busy.  The quoted 157.3 TFLOP/s vector peak counts dual-issue packed FMAs,
// which this library does not use.
#include <hip/hip_runtime.h>

#include "lll_internal.hpp"

namespace lll {
namespace {

constexpr int kIters = 4096;
constexpr int kChains = 8;

__global__ void __launch_bounds__(256) fma_probe_kernel(float *__restrict__ out, float b, float c) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    float a[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) a[j] = t * 1e-7f + j * 1e-7f;
    for (int i = 0; i < kIters; ++i) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) a[j] = fmaf(a[j], b, c);
    }
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += a[j];
    out[t] = s;  // keeps the chains live
}

// The quadrature recursion's instruction mix (path_kernel.hpp, quad_coupling):
// per (node, rate) C += W E R and R += ell E (1 + R), i.e. two FMAs that read a
// wave-uniform table entry as a scalar-register operand and one FMA on vector
// registers only.  The table rows are read through the constant address space
// as the path kernels read theirs; 8 rates per node, 8 independent R chains.
constexpr int kMixRates = 8;
constexpr int kMixNodes = 64;

__global__ void __launch_bounds__(256) mix_probe_kernel(
    const __attribute__((address_space(4))) float *__restrict__ tab, float *__restrict__ out,
    int reps) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    float ell[kMixRates], C[kMixRates];
#pragma unroll
    for (int j = 0; j < kMixRates; ++j) {
        ell[j] = 0.01f + t * 1e-9f + j * 1e-4f;
        C[j] = 0.0f;
    }
    for (int r = 0; r < reps; ++r) {
        for (int q = 0; q < kMixNodes; ++q) {
            const auto *row = tab + q * kMixRates * 2;
            float R = ell[kMixRates - 1] * row[2 * (kMixRates - 1)];
#pragma unroll
            for (int j = kMixRates - 2; j >= 0; --j) {
                const float E = row[2 * j], WE = row[2 * j + 1];
                C[j] = fmaf(WE, R, C[j]);
                R = fmaf(ell[j], fmaf(E, R, E), R);
            }
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < kMixRates; ++j) s += C[j];
    out[t] = s;
}

// The matrix-core ceiling of the exact-drift kernel's products: a stream of
// independent v_mfma_f32_16x16x4f32 (operands in registers, no memory
// traffic).  A product's accumulator must not be reused before 16 others have
// issued (8 independent accumulators per wavefront stay near 128 TFLOP/s at
// two wavefronts per SIMD), so each wavefront cycles through 16, three
// wavefronts per SIMD.
constexpr int kMfmaAcc = 16;

__global__ void __launch_bounds__(256) mfma_probe_kernel(float *__restrict__ out, float a0, float b0,
                                                         int iters) {
    typedef float vec4 __attribute__((ext_vector_type(4)));
    vec4 acc[kMfmaAcc];
#pragma unroll
    for (int j = 0; j < kMfmaAcc; ++j) acc[j] = vec4{0.0f, 0.0f, 0.0f, 0.0f};
    const float a = a0 + threadIdx.x * 1e-7f, b = b0;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < kMfmaAcc; ++j)
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[j], 0, 0, 0);
    }
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < kMfmaAcc; ++j) s += (acc[j][0] + acc[j][1]) + (acc[j][2] + acc[j][3]);
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;  // keeps the products live
}

}  // namespace

hipError_t measure_mfma_peak(hipStream_t st, double *tflops) {
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const int blocks = cus * 3, threads = 256, iters = 1024;
    float *out = nullptr;
    e = hipMalloc(&out, (size_t)blocks * threads * sizeof(float));
    if (e != hipSuccess) return e;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    double best = 0.0;
    for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {
        e = hipEventRecord(e0, st);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(mfma_probe_kernel, dim3(blocks), dim3(threads), 0, st, out, 1e-3f, 0.5f,
                           iters);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        // 16 x 16 x 4 multiply-adds per instruction and wavefront
        const double fl =
            (double)blocks * (threads / kWaveSize) * iters * kMfmaAcc * (16.0 * 16 * 4 * 2);
        if (e == hipSuccess && rep > 0 && ms > 0.0f) best = fmax(best, fl / (ms * 1e-3) / 1e12);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    *tflops = best;
    return e;
}

hipError_t measure_mix_peak(hipStream_t st, double *tflops) {
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const int blocks = cus * 32, threads = 256, reps = 64;
    float *buf = nullptr;
    const size_t tab_n = kMixNodes * kMixRates * 2;
    e = hipMalloc(&buf, ((size_t)blocks * threads + tab_n) * sizeof(float));
    if (e != hipSuccess) return e;
    float *out = buf, *tab = buf + (size_t)blocks * threads;
    float host[kMixNodes * kMixRates * 2];
    for (size_t i = 0; i < tab_n; ++i) host[i] = 1e-3f * static_cast<float>(i % 97) - 0.04f;
    e = hipMemcpyAsync(tab, host, sizeof host, hipMemcpyHostToDevice, st);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    double best = 0.0;
    for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {
        e = hipEventRecord(e0, st);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(mix_probe_kernel, dim3(blocks), dim3(threads), 0, st,
                           (const __attribute__((address_space(4))) float *)(tab), out, reps);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        // per node: 1 multiply (the top rate) + 3 FMAs per lower rate = 6 (R - 1) + 1 flops
        const double fl = (double)blocks * threads * reps * kMixNodes * (6.0 * (kMixRates - 1) + 1.0);
        if (e == hipSuccess && rep > 0 && ms > 0.0f) best = fmax(best, fl / (ms * 1e-3) / 1e12);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(buf);
    *tflops = best;
    return e;
}

hipError_t measure_fma_peak(hipStream_t st, double *tflops) {
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const int blocks = cus * 32, threads = 256;
    float *out = nullptr;
    e = hipMalloc(&out, (size_t)blocks * threads * sizeof(float));
    if (e != hipSuccess) return e;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    double best = 0.0;
    for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {
        e = hipEventRecord(e0, st);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(fma_probe_kernel, dim3(blocks), dim3(threads), 0, st, out, 0.999999f, 1e-7f);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        const double fl = (double)blocks * threads * kIters * kChains * 2.0;
        if (e == hipSuccess && rep > 0 && ms > 0.0f) best = fmax(best, fl / (ms * 1e-3) / 1e12);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    *tflops = best;
    return e;
}

}  // namespace lll
