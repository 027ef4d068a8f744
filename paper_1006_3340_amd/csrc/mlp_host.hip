// mlp_host.hip -- lifetime, data generation, training and inference calls of
// the drift surrogate (C ABI part).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "lll.h"
#include "lll_internal.hpp"
#include "mlp.hpp"

namespace lll {
namespace mlp {
hipError_t launch_record(const lll_plan &p, int64_t n_paths, int R, uint64_t seed, float *states,
                         int *kidx, hipStream_t st);
hipError_t launch_labels(const lll_plan &p, const float *states, const int *kidx,
                         const int64_t *poff, int64_t n_states, __bf16 *feat, float *label,
                         hipStream_t st);
hipError_t launch_stats(const lll_plan &p, const float *states, const int *kidx, int64_t n_states,
                        const float *label, int64_t n_pairs, float *out, hipStream_t st);
hipError_t launch_init(float *wts, __bf16 *wbf, float *adam, uint64_t seed, hipStream_t st);
hipError_t launch_refresh(const float *wts, __bf16 *wbf, hipStream_t st);
hipError_t launch_tiles(const __bf16 *feat, const float *target, const int *idx, int B,
                        float inv_sigma, const float *wts, const __bf16 *wbf, float *gpart,
                        float *lpart, float *yout, float *loss_out, float *wts_mut,
                        __bf16 *wbf_mut, float *adam, float *grad_out, float lr, float bc1,
                        float bc2, hipStream_t st);
hipError_t launch_batch_index(int *idx, int B, int64_t n_pairs, uint32_t step, uint64_t seed,
                              hipStream_t st);
hipError_t launch_mlp_tables(const lll_plan &p, const float *wts, float *K2, float *B1,
                             hipStream_t st);
hipError_t launch_mlp_paths(const lll_plan &p, const float *wts, const __bf16 *wbf,
                            const float *K2, const float *B1, const float *box, float sigma,
                            int use_net, int judge_stride, int64_t n_paths, uint64_t seed,
                            double *path_fix, double *stats, hipStream_t st);

namespace {
__global__ void to_bf16_kernel(const float *__restrict__ in, __bf16 *__restrict__ out, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i < n) out[i] = static_cast<__bf16>(in[i]);
}
}  // namespace
}  // namespace mlp

void mlp_plan_free(lll_plan &p) {
    MlpBuffers &b = p.mb;
    void *ptrs[] = {b.K2, b.B1, b.open_box, b.stats, b.zero_params};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    p.mb = MlpBuffers{};
}

}  // namespace lll

using lll::fail;
using lll::hip_fail;
using namespace lll::mlp;

struct lll_mlp {
    float *wts = nullptr;
    __bf16 *wbf = nullptr;
    float *adam = nullptr;
    int64_t adam_steps = 0;
    // training data
    int N = 0, s = 0;
    __bf16 *feat = nullptr;
    float *label = nullptr;
    float *states = nullptr;
    int *kidx = nullptr;
    int64_t *poff_dev = nullptr;
    std::vector<int64_t> poff;
    std::vector<int> kidx_host;
    int64_t n_pairs = 0, n_states = 0;
    float *info = nullptr;           // device [2*40 + 1]: box lo, box hi, sigma
    float info_host[2 * kRates + 1] = {};
    bool have_data = false;
    // training scratch
    int *idx = nullptr;
    float *gpart = nullptr, *lpart = nullptr, *loss = nullptr;
    int batch_cap = 0, loss_cap = 0;
};

namespace {

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

void free_data(lll_mlp *m) {
    void *ptrs[] = {m->feat, m->label, m->states, m->kidx, m->poff_dev};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    m->feat = nullptr;
    m->label = nullptr;
    m->states = nullptr;
    m->kidx = nullptr;
    m->poff_dev = nullptr;
    m->poff.clear();
    m->kidx_host.clear();
    m->n_pairs = m->n_states = 0;
    m->have_data = false;
}

int ensure_train_scratch(lll_mlp *m, int batch, int n_steps) {
    hipError_t e = hipSuccess;
    if (batch > m->batch_cap) {
        if (m->idx) (void)hipFree(m->idx);
        if (m->gpart) (void)hipFree(m->gpart);
        if (m->lpart) (void)hipFree(m->lpart);
        m->idx = nullptr;
        m->gpart = m->lpart = nullptr;
        const int tiles = (batch + 63) / 64;
        e = hipMalloc(&m->idx, sizeof(int) * batch);
        if (e == hipSuccess) e = hipMalloc(&m->gpart, sizeof(float) * (size_t)tiles * kParams);
        if (e == hipSuccess) e = hipMalloc(&m->lpart, sizeof(float) * tiles);
        if (e != hipSuccess) return fail(LLL_ENOMEM, "training scratch: %s", hipGetErrorString(e));
        m->batch_cap = batch;
    }
    if (n_steps > m->loss_cap) {
        if (m->loss) (void)hipFree(m->loss);
        m->loss = nullptr;
        e = hipMalloc(&m->loss, sizeof(float) * n_steps);
        if (e != hipSuccess) return fail(LLL_ENOMEM, "loss buffer: %s", hipGetErrorString(e));
        m->loss_cap = n_steps;
    }
    return LLL_OK;
}

}  // namespace

extern "C" {

int lll_mlp_destroy(lll_mlp *m) {
    if (!m) return LLL_OK;
    free_data(m);
    void *ptrs[] = {m->wts, m->wbf, m->adam, m->info, m->idx, m->gpart, m->lpart, m->loss};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    delete m;
    return LLL_OK;
}

int lll_mlp_create(uint64_t seed, lll_mlp **out) {
    if (!out) return fail(LLL_EINVAL, "out is NULL");
    *out = nullptr;
    lll_mlp *m = new (std::nothrow) lll_mlp();
    if (!m) return fail(LLL_ENOMEM, "host allocation failed");
    hipError_t e = hipMalloc(&m->wts, sizeof(float) * kParams);
    if (e == hipSuccess) e = hipMalloc(&m->wbf, sizeof(__bf16) * kParams);
    if (e == hipSuccess) e = hipMalloc(&m->adam, sizeof(float) * 2 * kParams);
    if (e == hipSuccess) e = hipMalloc(&m->info, sizeof(float) * (2 * kRates + 1));
    if (e == hipSuccess) e = launch_init(m->wts, m->wbf, m->adam, seed, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        lll_mlp_destroy(m);
        return hip_fail(e, "creating the surrogate");
    }
    *out = m;
    return LLL_OK;
}

int lll_mlp_params(lll_mlp *m, float *get_host, const float *set_host) {
    if (!m) return fail(LLL_EINVAL, "mlp is NULL");
    hipError_t e = hipSuccess;
    if (set_host) {
        e = hipMemcpy(m->wts, set_host, sizeof(float) * kParams, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = launch_refresh(m->wts, m->wbf, nullptr);
        if (e == hipSuccess) e = hipMemset(m->adam, 0, sizeof(float) * 2 * kParams);
        m->adam_steps = 0;
    }
    if (e == hipSuccess && get_host)
        e = hipMemcpy(get_host, m->wts, sizeof(float) * kParams, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "surrogate parameters");
    return LLL_OK;
}

int lll_mlp_generate(lll_mlp *m, lll_plan *plan, int64_t n_paths, int records, uint64_t seed,
                     int64_t *n_pairs_out, void *stream) {
    if (!m || !plan) return fail(LLL_EINVAL, "NULL argument");
    if (plan->nmax != kRates || plan->precision != LLL_FP32 || plan->driver != LLL_DRIVER_NIG)
        return fail(LLL_EUNSUPPORTED, "the surrogate needs an FP32 NIG plan with 33..40 rates");
    if (n_paths < 1 || n_paths > (1 << 24) || records < 1 || records > plan->K)
        return fail(LLL_EINVAL, "n_paths or records out of range");
    hipStream_t st = as_stream(stream);
    free_data(m);
    m->N = plan->N;
    m->s = plan->s;
    const int K = plan->K;
    const int stride = K / records;
    m->n_states = n_paths * records;
    m->poff.resize(m->n_states + 1);
    m->kidx_host.resize(m->n_states);
    int64_t acc = 0;
    for (int64_t g = 0; g < n_paths; ++g)
        for (int r = 0; r < records; ++r) {
            const int k = r * stride + static_cast<int>(g % stride);
            const int64_t si = g * records + r;
            m->kidx_host[si] = k;
            m->poff[si] = acc;
            acc += plan->N - k / plan->s;
        }
    m->poff[m->n_states] = acc;
    m->n_pairs = acc;
    hipError_t e = hipMalloc(&m->states, sizeof(float) * m->n_states * kRates);
    if (e == hipSuccess) e = hipMalloc(&m->kidx, sizeof(int) * m->n_states);
    if (e == hipSuccess) e = hipMalloc(&m->poff_dev, sizeof(int64_t) * (m->n_states + 1));
    if (e == hipSuccess) e = hipMalloc(&m->feat, sizeof(__bf16) * m->n_pairs * kIn);
    if (e == hipSuccess) e = hipMalloc(&m->label, sizeof(float) * m->n_pairs);
    if (e != hipSuccess) {
        free_data(m);
        return fail(LLL_ENOMEM, "training data (%lld pairs): %s", (long long)acc,
                    hipGetErrorString(e));
    }
    e = hipMemcpyAsync(m->poff_dev, m->poff.data(), sizeof(int64_t) * (m->n_states + 1),
                       hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = lll::launch_precompute(*plan, st);
    if (e == hipSuccess) e = launch_record(*plan, n_paths, records, seed, m->states, m->kidx, st);
    if (e == hipSuccess)
        e = launch_labels(*plan, m->states, m->kidx, m->poff_dev, m->n_states, m->feat, m->label, st);
    if (e == hipSuccess)
        e = launch_stats(*plan, m->states, m->kidx, m->n_states, m->label, m->n_pairs, m->info, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(m->info_host, m->info, sizeof(float) * (2 * kRates + 1),
                           hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        free_data(m);
        return hip_fail(e, "generating training pairs");
    }
    // kernel-computed k must match the host's offsets
    std::vector<int> kd(m->n_states);
    e = hipMemcpy(kd.data(), m->kidx, sizeof(int) * m->n_states, hipMemcpyDeviceToHost);
    if (e != hipSuccess || kd != m->kidx_host) {
        free_data(m);
        return fail(LLL_EHIP, "recorded steps disagree with the pair offsets");
    }
    if (!(m->info_host[2 * kRates] > 0.0f)) {
        free_data(m);
        return fail(LLL_ENUMERIC, "degenerate labels (zero scale)");
    }
    m->have_data = true;
    if (n_pairs_out) *n_pairs_out = m->n_pairs;
    return LLL_OK;
}

int lll_mlp_info(lll_mlp *m, float *info_host, int64_t *n_pairs) {
    if (!m || !info_host) return fail(LLL_EINVAL, "NULL argument");
    if (!m->have_data) return fail(LLL_EINVAL, "no training data generated");
    std::memcpy(info_host, m->info_host, sizeof(m->info_host));
    if (n_pairs) *n_pairs = m->n_pairs;
    return LLL_OK;
}

int lll_mlp_set_box(lll_mlp *m, const float *box_host) {
    if (!m || !box_host) return fail(LLL_EINVAL, "NULL argument");
    if (!m->have_data) return fail(LLL_EINVAL, "no training data generated");
    for (int i = 0; i < 2 * kRates; ++i)
        if (std::isnan(box_host[i])) return fail(LLL_EINVAL, "box entry %d is NaN", i);
    hipError_t e = hipMemcpy(m->info, box_host, sizeof(float) * 2 * kRates, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "setting the trust box");
    std::memcpy(m->info_host, box_host, sizeof(float) * 2 * kRates);
    return LLL_OK;
}

int lll_mlp_pairs(lll_mlp *m, const int64_t *pairs, int64_t n, float *state_host, int *k_host,
                  int *rate_host, float *label_host, float *feat_host) {
    if (!m || !pairs) return fail(LLL_EINVAL, "NULL argument");
    if (!m->have_data) return fail(LLL_EINVAL, "no training data generated");
    std::vector<__bf16> f(kIn);
    for (int64_t j = 0; j < n; ++j) {
        const int64_t p = pairs[j];
        if (p < 0 || p >= m->n_pairs) return fail(LLL_EINVAL, "pair %lld out of range", (long long)p);
        // state holding pair p: last offset <= p
        int64_t lo = 0, hi = m->n_states;
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) / 2;
            if (m->poff[mid] <= p) lo = mid; else hi = mid;
        }
        const int k = m->kidx_host[lo];
        const int rate = k / m->s + static_cast<int>(p - m->poff[lo]);
        if (k_host) k_host[j] = k;
        if (rate_host) rate_host[j] = rate;
        hipError_t e = hipSuccess;
        if (state_host)
            e = hipMemcpy(state_host + j * kRates, m->states + lo * kRates, sizeof(float) * kRates,
                          hipMemcpyDeviceToHost);
        if (e == hipSuccess && label_host)
            e = hipMemcpy(label_host + j, m->label + p, sizeof(float), hipMemcpyDeviceToHost);
        if (e == hipSuccess && feat_host) {
            e = hipMemcpy(f.data(), m->feat + p * kIn, sizeof(__bf16) * kIn, hipMemcpyDeviceToHost);
            for (int c = 0; c < kIn; ++c) feat_host[j * kIn + c] = static_cast<float>(f[c]);
        }
        if (e != hipSuccess) return hip_fail(e, "reading training pairs");
    }
    return LLL_OK;
}

int lll_mlp_train(lll_mlp *m, int n_steps, int batch, float lr, uint64_t seed, float *loss_host,
                  void *stream) {
    if (!m) return fail(LLL_EINVAL, "mlp is NULL");
    if (!m->have_data) return fail(LLL_EINVAL, "no training data generated");
    if (n_steps < 1 || n_steps > 1000000 || batch < 64 || batch > (1 << 20) || !(lr > 0.0f))
        return fail(LLL_EINVAL, "bad training arguments");
    int rc = ensure_train_scratch(m, batch, n_steps);
    if (rc != LLL_OK) return rc;
    hipStream_t st = as_stream(stream);
    const float inv_sigma = 1.0f / m->info_host[2 * kRates];
    hipError_t e = hipSuccess;
    for (int t = 0; t < n_steps && e == hipSuccess; ++t) {
        // cosine decay from lr to lr / 100
        const double c = 0.5 * (1.0 + std::cos(3.141592653589793 * t / n_steps));
        const float lr_t = static_cast<float>(lr * (0.01 + 0.99 * c));
        const int64_t tt = ++m->adam_steps;
        const float bc1 = static_cast<float>(1.0 / (1.0 - std::pow(0.9, (double)tt)));
        const float bc2 = static_cast<float>(1.0 / (1.0 - std::pow(0.999, (double)tt)));
        e = launch_batch_index(m->idx, batch, m->n_pairs, static_cast<uint32_t>(tt), seed, st);
        if (e == hipSuccess)
            e = launch_tiles(m->feat, m->label, m->idx, batch, inv_sigma, m->wts, m->wbf, m->gpart,
                             m->lpart, nullptr, m->loss + t, m->wts, m->wbf, m->adam, nullptr,
                             lr_t, bc1, bc2, st);
    }
    if (e == hipSuccess && loss_host)
        e = hipMemcpyAsync(loss_host, m->loss, sizeof(float) * n_steps, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "training");
    return LLL_OK;
}

int lll_mlp_train_dev(lll_mlp *m, const uint16_t *feat_dev, const float *label_dev,
                      int64_t n_pairs, float sigma, int n_steps, int batch, float lr, uint64_t seed,
                      float *loss_dev, void *stream) {
    if (!m || !feat_dev || !label_dev) return fail(LLL_EINVAL, "NULL argument");
    if (n_pairs < 1 || n_pairs > ((int64_t)1 << 31) - 1)
        return fail(LLL_EINVAL, "n_pairs=%lld outside 1..2^31-1", (long long)n_pairs);
    if (!(sigma > 0.0f) || !std::isfinite(sigma)) return fail(LLL_EINVAL, "sigma must be > 0");
    if (n_steps < 1 || n_steps > 1000000 || batch < 64 || batch > (1 << 20) || !(lr > 0.0f))
        return fail(LLL_EINVAL, "bad training arguments");
    int rc = ensure_train_scratch(m, batch, n_steps);
    if (rc != LLL_OK) return rc;
    hipStream_t st = as_stream(stream);
    const __bf16 *feat = reinterpret_cast<const __bf16 *>(feat_dev);
    float *loss = loss_dev ? loss_dev : m->loss;
    hipError_t e = hipSuccess;
    for (int t = 0; t < n_steps && e == hipSuccess; ++t) {
        const double c = 0.5 * (1.0 + std::cos(3.141592653589793 * t / n_steps));
        const float lr_t = static_cast<float>(lr * (0.01 + 0.99 * c));
        const int64_t tt = ++m->adam_steps;
        const float bc1 = static_cast<float>(1.0 / (1.0 - std::pow(0.9, (double)tt)));
        const float bc2 = static_cast<float>(1.0 / (1.0 - std::pow(0.999, (double)tt)));
        e = launch_batch_index(m->idx, batch, n_pairs, static_cast<uint32_t>(tt), seed, st);
        if (e == hipSuccess)
            e = launch_tiles(feat, label_dev, m->idx, batch, 1.0f / sigma, m->wts, m->wbf, m->gpart,
                             m->lpart, nullptr, loss + t, m->wts, m->wbf, m->adam, nullptr, lr_t,
                             bc1, bc2, st);
    }
    if (e != hipSuccess) return hip_fail(e, "training");
    return LLL_OK;
}

int lll_mlp_optimizer_state(lll_mlp *m, float *m_host, float *v_host, int64_t *step_host) {
    if (!m) return fail(LLL_EINVAL, "mlp is NULL");
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess && m_host)
        e = hipMemcpy(m_host, m->adam, sizeof(float) * kParams, hipMemcpyDeviceToHost);
    if (e == hipSuccess && v_host)
        e = hipMemcpy(v_host, m->adam + kParams, sizeof(float) * kParams, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "reading the optimiser state");
    if (step_host) *step_host = m->adam_steps;
    return LLL_OK;
}

int lll_mlp_copy_pairs_dev(lll_mlp *m, uint16_t *feat_dev, float *label_dev, int64_t capacity,
                           void *stream) {
    if (!m || !feat_dev || !label_dev) return fail(LLL_EINVAL, "NULL argument");
    if (!m->have_data) return fail(LLL_EINVAL, "no training data generated");
    if (capacity < m->n_pairs)
        return fail(LLL_EINVAL, "capacity %lld < %lld pairs", (long long)capacity,
                    (long long)m->n_pairs);
    hipStream_t st = as_stream(stream);
    hipError_t e = hipMemcpyAsync(feat_dev, m->feat, sizeof(__bf16) * m->n_pairs * kIn,
                                  hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(label_dev, m->label, sizeof(float) * m->n_pairs, hipMemcpyDeviceToDevice,
                           st);
    if (e != hipSuccess) return hip_fail(e, "copying training pairs");
    return LLL_OK;
}

int lll_mlp_eval(lll_mlp *m, const float *feat_host, const float *target_host, int64_t n,
                 float *y_host, float *grad_host, float *loss_host, void *stream) {
    if (!m || !feat_host) return fail(LLL_EINVAL, "NULL argument");
    if (n < 1 || n > (1 << 20)) return fail(LLL_EINVAL, "n out of range");
    if ((grad_host || loss_host) && !target_host) return fail(LLL_EINVAL, "gradients need targets");
    hipStream_t st = as_stream(stream);
    const int tiles = static_cast<int>((n + 63) / 64);
    float *f32 = nullptr, *tgt = nullptr, *y = nullptr, *gp = nullptr, *lp = nullptr, *gout = nullptr,
          *lout = nullptr;
    __bf16 *fb = nullptr;
    hipError_t e = hipMalloc(&f32, sizeof(float) * n * kIn);
    if (e == hipSuccess) e = hipMalloc(&fb, sizeof(__bf16) * n * kIn);
    if (e == hipSuccess) e = hipMalloc(&tgt, sizeof(float) * n);
    if (e == hipSuccess) e = hipMalloc(&y, sizeof(float) * n);
    if (e == hipSuccess) e = hipMalloc(&gp, sizeof(float) * (size_t)tiles * kParams);
    if (e == hipSuccess) e = hipMalloc(&lp, sizeof(float) * tiles);
    if (e == hipSuccess) e = hipMalloc(&gout, sizeof(float) * kParams);
    if (e == hipSuccess) e = hipMalloc(&lout, sizeof(float));
    if (e == hipSuccess)
        e = hipMemcpyAsync(f32, feat_host, sizeof(float) * n * kIn, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && target_host)
        e = hipMemcpyAsync(tgt, target_host, sizeof(float) * n, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(to_bf16_kernel, dim3(static_cast<unsigned>((n * kIn + 255) / 256)),
                           dim3(256), 0, st, f32, fb, n * kIn);
        e = hipGetLastError();
    }
    const bool grads = target_host != nullptr;
    if (e == hipSuccess)
        e = launch_tiles(fb, grads ? tgt : y, nullptr, static_cast<int>(n), 1.0f, m->wts, m->wbf,
                         grads ? gp : nullptr, grads ? lp : nullptr, y, grads ? lout : nullptr,
                         m->wts, m->wbf, m->adam, gout, 0.0f, 1.0f, 1.0f, st);
    if (e == hipSuccess && y_host)
        e = hipMemcpyAsync(y_host, y, sizeof(float) * n, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && grads && grad_host)
        e = hipMemcpyAsync(grad_host, gout, sizeof(float) * kParams, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && grads && loss_host)
        e = hipMemcpyAsync(loss_host, lout, sizeof(float), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    void *ptrs[] = {f32, fb, tgt, y, gp, lp, gout, lout};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    if (e != hipSuccess) return hip_fail(e, "evaluating the surrogate");
    return LLL_OK;
}

int lll_plan_execute_mlp(lll_plan *plan, const lll_mlp *m, int use_net, int64_t n_paths,
                         uint64_t seed, int judge_stride, double *path_fix_dev, void *stream) {
    if (!plan) return fail(LLL_EINVAL, "plan is NULL");
    if (plan->nmax != kRates || plan->precision != LLL_FP32 || plan->driver != LLL_DRIVER_NIG)
        return fail(LLL_EUNSUPPORTED, "the surrogate needs an FP32 NIG plan with 33..40 rates");
    if (use_net && (!m || !m->have_data))
        return fail(LLL_EINVAL, "use_net needs a surrogate with training data (box and scale)");
    if (use_net && (m->N != plan->N || m->s != plan->s))
        return fail(LLL_EINVAL, "the surrogate was trained on another term structure shape");
    if (n_paths < 1 || n_paths > plan->max_paths)
        return fail(LLL_EINVAL, "n_paths=%lld outside 1..%lld", (long long)n_paths,
                    (long long)plan->max_paths);
    if (judge_stride < 0) return fail(LLL_EINVAL, "judge_stride < 0");
    lll::MlpBuffers &b = plan->mb;
    hipError_t e = hipSuccess;
    if (!b.K2) {
        e = hipMalloc(&b.K2, sizeof(float) * (size_t)plan->K * kRates * kRates);
        if (e == hipSuccess) e = hipMalloc(&b.B1, sizeof(float) * (size_t)plan->K * kRates * kHid);
        if (e == hipSuccess) e = hipMalloc(&b.open_box, sizeof(float) * 2 * kRates);
        if (e == hipSuccess) e = hipMalloc(&b.stats, sizeof(double) * plan->max_waves * 8);
        const size_t zbytes = (sizeof(float) + sizeof(__bf16)) * kParams;
        if (e == hipSuccess) e = hipMalloc(&b.zero_params, zbytes);
        if (e == hipSuccess) e = hipMemset(b.zero_params, 0, zbytes);
        if (e == hipSuccess) {
            float box[2 * kRates];
            for (int i = 0; i < kRates; ++i) {
                box[i] = -INFINITY;
                box[kRates + i] = INFINITY;
            }
            e = hipMemcpy(b.open_box, box, sizeof box, hipMemcpyHostToDevice);
        }
        if (e != hipSuccess) {
            lll::mlp_plan_free(*plan);
            return fail(LLL_ENOMEM, "surrogate tables: %s", hipGetErrorString(e));
        }
        b.stat_waves = plan->max_waves;
    }
    hipStream_t st = as_stream(stream);
    // without a network the kernel still stages (zero) weights it never applies
    const float *zw = static_cast<const float *>(b.zero_params);
    const float *wts = m ? m->wts : zw;
    const __bf16 *wbf = m ? m->wbf : reinterpret_cast<const __bf16 *>(zw + kParams);
    // timing stages as in lll_plan_execute: tables, path kernel, reduction
    const bool t = plan->timing;
    e = t ? hipEventRecord(plan->ev[0], st) : hipSuccess;
    if (e == hipSuccess) e = lll::launch_precompute(*plan, st);
    if (e == hipSuccess) e = launch_mlp_tables(*plan, wts, b.K2, b.B1, st);
    const float *box = use_net ? m->info : b.open_box;
    const float sigma = use_net ? m->info_host[2 * kRates] : 0.0f;
    if (e == hipSuccess && t) e = hipEventRecord(plan->ev[1], st);
    if (e == hipSuccess)
        e = launch_mlp_paths(*plan, wts, wbf, b.K2, b.B1, box, sigma, use_net,
                             judge_stride, n_paths, seed, path_fix_dev, b.stats, st);
    if (e == hipSuccess && t) e = hipEventRecord(plan->ev[2], st);
    if (e == hipSuccess) e = lll::launch_reduce(*plan, n_paths, st);
    if (e == hipSuccess && t) e = hipEventRecord(plan->ev[3], st);
    if (e != hipSuccess) return hip_fail(e, "surrogate path launch");
    plan->timed = t;
    plan->last_n_paths = n_paths;
    plan->executed = true;
    plan->mlp_done = true;
    return LLL_OK;
}

int lll_plan_mlp_stats(lll_plan *plan, double *stats_host, void *stream) {
    if (!plan || !stats_host) return fail(LLL_EINVAL, "NULL argument");
    if (!plan->mlp_done) return fail(LLL_EINVAL, "no surrogate pass has run on this plan");
    const int64_t waves = (plan->last_n_paths + 63) / 64;
    std::vector<double> w(waves * 8);
    hipStream_t st = as_stream(stream);
    hipError_t e = hipMemcpyAsync(w.data(), plan->mb.stats, sizeof(double) * w.size(),
                                  hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "reading surrogate statistics");
    double out[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t i = 0; i < waves; ++i) {
        for (int j = 0; j < 8; ++j) {
            if (j == 5) out[5] = std::fmax(out[5], w[i * 8 + 5]);
            else out[j] += w[i * 8 + j];
        }
    }
    std::memcpy(stats_host, out, sizeof out);
    return LLL_OK;
}

}  // extern "C"
