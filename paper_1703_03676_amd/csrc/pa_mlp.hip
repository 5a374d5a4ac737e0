// Training and inference kernels of the learned temperature-step proposer
// (MLP 8 -> 64 -> 64 -> 1, ReLU; layout in pa_mlp_dev.h).
//
// Training is FP32 with a deterministic fixed-order gradient reduction: one
// thread per parameter sums its per-sample terms in sample order, so a
// training run is reproducible bit for bit.  SGD with momentum updates the FP32
// master weights and refreshes the BF16 copy used for inference.  The loss is
// the mean squared error on the normalised target.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "pa.h"
#include "pa_mlp_dev.h"

namespace pa {
namespace mlp {
namespace {

// x_all [n][8], t_all [n] raw -> xn [B][8], tn [B] normalised, for the samples idx[0..B).
__global__ void k_gather_norm(const float* __restrict__ x_all, const float* __restrict__ t_all,
                              const int32_t* __restrict__ idx, int B, const float* __restrict__ norm,
                              float* __restrict__ xn, float* __restrict__ tn)
{
    const int s = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (s >= B) return;
    const int i = idx ? idx[s] : s;
    for (int k = 0; k < kIn; ++k) xn[s * kIn + k] = (x_all[i * kIn + k] - norm[k]) / norm[kIn + k];
    if (t_all) tn[s] = (t_all[i] - norm[2 * kIn]) / norm[2 * kIn + 1];
}

// One block of 64 threads per sample: hidden activations and the output.
__global__ __launch_bounds__(64) void k_forward(const float* __restrict__ xn, const float* __restrict__ p,
                                                float* __restrict__ h1o, float* __restrict__ h2o,
                                                float* __restrict__ y)
{
    __shared__ float h[kHid];
    const int s = (int)blockIdx.x, t = (int)threadIdx.x;
    float a = p[kB1 + t];
    for (int k = 0; k < kIn; ++k) a += p[kW1 + t * kIn + k] * xn[s * kIn + k];
    const float h1 = a > 0.0f ? a : 0.0f;
    h[t] = h1;
    h1o[s * kHid + t] = h1;
    __syncthreads();
    float a2 = p[kB2 + t];
    for (int v = 0; v < kHid; ++v) a2 += p[kW2 + t * kHid + v] * h[v];
    const float h2 = a2 > 0.0f ? a2 : 0.0f;
    h2o[s * kHid + t] = h2;
    __syncthreads();
    h[t] = p[kW3 + t] * h2;
    __syncthreads();
    if (t == 0) {
        float o = p[kB3];
        for (int v = 0; v < kHid; ++v) o += h[v];
        y[s] = o;
    }
}

// Per-sample deltas of the mean squared error L = (1/B) sum_s (y_s - t_s)^2.
__global__ __launch_bounds__(64) void k_backward(const float* __restrict__ p, const float* __restrict__ h1,
                                                 const float* __restrict__ h2, const float* __restrict__ y,
                                                 const float* __restrict__ tn, int B, float* __restrict__ dy,
                                                 float* __restrict__ d1, float* __restrict__ d2)
{
    __shared__ float sd2[kHid];
    const int s = (int)blockIdx.x, t = (int)threadIdx.x;
    const float g = 2.0f * (y[s] - tn[s]) / (float)B;
    if (t == 0) dy[s] = g;
    const float e2 = (h2[s * kHid + t] > 0.0f) ? g * p[kW3 + t] : 0.0f;
    sd2[t] = e2;
    d2[s * kHid + t] = e2;
    __syncthreads();
    float acc = 0.0f;
    for (int u = 0; u < kHid; ++u) acc += p[kW2 + u * kHid + t] * sd2[u];
    d1[s * kHid + t] = (h1[s * kHid + t] > 0.0f) ? acc : 0.0f;
}

// One thread per parameter: sum of its per-sample gradient terms in sample
// order.  Thread kParams computes the loss.
__global__ __launch_bounds__(256) void k_gradient(const float* __restrict__ xn, const float* __restrict__ h1,
                                                  const float* __restrict__ h2, const float* __restrict__ d1,
                                                  const float* __restrict__ d2, const float* __restrict__ dy,
                                                  const float* __restrict__ y, const float* __restrict__ tn, int B,
                                                  float* __restrict__ grad, float* __restrict__ loss_acc)
{
    const int q = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (q > kParams) return;
    float g = 0.0f;
    if (q < kB1) {
        const int u = q / kIn, k = q % kIn;
        for (int s = 0; s < B; ++s) g += d1[s * kHid + u] * xn[s * kIn + k];
    } else if (q < kW2) {
        const int u = q - kB1;
        for (int s = 0; s < B; ++s) g += d1[s * kHid + u];
    } else if (q < kB2) {
        const int u = (q - kW2) / kHid, v = (q - kW2) % kHid;
        for (int s = 0; s < B; ++s) g += d2[s * kHid + u] * h1[s * kHid + v];
    } else if (q < kW3) {
        const int u = q - kB2;
        for (int s = 0; s < B; ++s) g += d2[s * kHid + u];
    } else if (q < kB3) {
        const int u = q - kW3;
        for (int s = 0; s < B; ++s) g += dy[s] * h2[s * kHid + u];
    } else if (q == kB3) {
        for (int s = 0; s < B; ++s) g += dy[s];
    } else {
        float l = 0.0f;
        for (int s = 0; s < B; ++s) {
            const float d = y[s] - tn[s];
            l += d * d;
        }
        if (loss_acc) *loss_acc += l / (float)B;
        return;
    }
    grad[q] = g;
}

// SGD with momentum on the FP32 master weights; refreshes the BF16 copy.
__global__ void k_sgd(float* __restrict__ p, const float* __restrict__ grad, float* __restrict__ mom, float lr,
                      float momentum, __hip_bfloat16* __restrict__ wb)
{
    const int q = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (q >= kParams) return;
    const float m = momentum * mom[q] + grad[q];
    mom[q] = m;
    const float w = p[q] - lr * m;
    p[q] = w;
    wb[q] = __float2bfloat16(w);
}

__global__ void k_to_bf16(const float* __restrict__ p, __hip_bfloat16* __restrict__ wb)
{
    const int q = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (q < kParams) wb[q] = __float2bfloat16(p[q]);
}

// Inference on raw features: BF16 weights and activations (bf16 = 1) or the
// FP32 master weights (bf16 = 0).  One block of 64 threads per sample.
__global__ __launch_bounds__(64) void k_infer(const float* __restrict__ x, const float* __restrict__ p,
                                              const __hip_bfloat16* __restrict__ wb, const float* __restrict__ norm,
                                              int bf16, float* __restrict__ y)
{
    __shared__ float h[kHid];
    const int s = (int)blockIdx.x, t = (int)threadIdx.x;
    if (bf16) {
        const float o = forward_bf16(x + s * kIn, wb, norm, h, t);
        if (t == 0) y[s] = o;
        return;
    }
    float a = p[kB1 + t];
    for (int k = 0; k < kIn; ++k) a += p[kW1 + t * kIn + k] * ((x[s * kIn + k] - norm[k]) / norm[kIn + k]);
    h[t] = a > 0.0f ? a : 0.0f;
    __syncthreads();
    float a2 = p[kB2 + t];
    for (int v = 0; v < kHid; ++v) a2 += p[kW2 + t * kHid + v] * h[v];
    const float h2 = a2 > 0.0f ? a2 : 0.0f;
    __syncthreads();
    h[t] = p[kW3 + t] * h2;
    __syncthreads();
    if (t == 0) {
        float o = p[kB3];
        for (int v = 0; v < kHid; ++v) o += h[v];
        y[s] = o * norm[2 * kIn + 1] + norm[2 * kIn];
    }
}

// Mean and standard deviation of each feature and of the target (FP64,
// sequential over samples): one thread per variable.
__global__ void k_fit_norm(const float* __restrict__ x, const float* __restrict__ t, int n, float* __restrict__ norm)
{
    const int v = (int)threadIdx.x;
    if (v > kIn) return;
    double s = 0.0, s2 = 0.0;
    for (int i = 0; i < n; ++i) {
        const double z = (v < kIn) ? (double)x[i * kIn + v] : (double)t[i];
        s += z;
        s2 += z * z;
    }
    const double mean = s / n;
    double var = s2 / n - mean * mean;
    double sd = var > 1e-24 ? sqrt(var) : 1.0;
    if (v < kIn) {
        norm[v] = (float)mean;
        norm[kIn + v] = (float)sd;
    } else {
        norm[2 * kIn] = (float)mean;
        norm[2 * kIn + 1] = (float)sd;
    }
}

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t params, grad, mom, wb, norm, xn, tn, h1, h2, d1, d2, dy, y, loss, idx, total;
};

Layout layout(int max_batch)
{
    Layout l;
    size_t o = 0;
    auto take = [&](size_t b) {
        const size_t at = o;
        o = align_up(o + b);
        return at;
    };
    const size_t B = (size_t)max_batch;
    l.params = take(kParams * 4);
    l.grad = take(kParams * 4);
    l.mom = take(kParams * 4);
    l.wb = take(kParams * 2);
    l.norm = take(kNorm * 4);
    l.xn = take(B * kIn * 4);
    l.tn = take(B * 4);
    l.h1 = take(B * kHid * 4);
    l.h2 = take(B * kHid * 4);
    l.d1 = take(B * kHid * 4);
    l.d2 = take(B * kHid * 4);
    l.dy = take(B * 4);
    l.y = take(B * 4);
    l.loss = take(16);
    l.idx = take(B * 4);
    l.total = o;
    return l;
}

}  // namespace
}  // namespace mlp
}  // namespace pa

using namespace pa::mlp;

struct pa_mlp {
    int max_batch;
    hipStream_t stream;
    Layout lo;
    uint8_t* ws;
    float *p, *grad, *mom, *norm, *xn, *tn, *h1, *h2, *d1, *d2, *dy, *y, *loss;
    __hip_bfloat16* wb;
    int32_t* idx;
    bool broken;
    std::string last_error;
};

namespace {

pa_status mfail(pa_mlp* m, hipError_t e, const char* what)
{
    m->broken = true;
    m->last_error = std::string(what) + ": " + hipGetErrorString(e);
    return PA_EHIP;
}

#define MCHK(expr)                                           \
    do {                                                     \
        const hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess) return mfail(m, e_, #expr);    \
    } while (0)

// forward + backward + gradient for the B samples already normalised in xn/tn
pa_status grad_pass(pa_mlp* m, int B, float* loss_acc)
{
    const hipStream_t s = m->stream;
    hipLaunchKernelGGL(k_forward, dim3(B), dim3(64), 0, s, m->xn, m->p, m->h1, m->h2, m->y);
    MCHK(hipGetLastError());
    hipLaunchKernelGGL(k_backward, dim3(B), dim3(64), 0, s, m->p, m->h1, m->h2, m->y, m->tn, B, m->dy, m->d1, m->d2);
    MCHK(hipGetLastError());
    hipLaunchKernelGGL(k_gradient, dim3((kParams + 1 + 255) / 256), dim3(256), 0, s, m->xn, m->h1, m->h2, m->d1,
                       m->d2, m->dy, m->y, m->tn, B, m->grad, loss_acc);
    MCHK(hipGetLastError());
    return PA_OK;
}

}  // namespace

extern "C" {

size_t pa_mlp_workspace_bytes(int32_t max_batch)
{
    if (max_batch < 1 || max_batch > (1 << 20)) return 0;
    return layout(max_batch).total;
}

pa_status pa_mlp_create(int32_t max_batch, uint64_t seed, void* d_workspace, size_t bytes, void* hip_stream,
                        pa_mlp** out)
{
    if (!out) return PA_EINVAL;
    *out = nullptr;
    if (max_batch < 1 || max_batch > (1 << 20) || !d_workspace || ((uintptr_t)d_workspace) % 256) return PA_EINVAL;
    const Layout lo = layout(max_batch);
    if (bytes < lo.total) return PA_ENOMEM;
    pa_mlp* m = new (std::nothrow) pa_mlp();
    if (!m) return PA_ENOMEM;
    m->max_batch = max_batch;
    m->stream = (hipStream_t)hip_stream;
    m->lo = lo;
    uint8_t* w = (uint8_t*)d_workspace;
    m->ws = w;
    m->p = (float*)(w + lo.params);
    m->grad = (float*)(w + lo.grad);
    m->mom = (float*)(w + lo.mom);
    m->wb = (__hip_bfloat16*)(w + lo.wb);
    m->norm = (float*)(w + lo.norm);
    m->xn = (float*)(w + lo.xn);
    m->tn = (float*)(w + lo.tn);
    m->h1 = (float*)(w + lo.h1);
    m->h2 = (float*)(w + lo.h2);
    m->d1 = (float*)(w + lo.d1);
    m->d2 = (float*)(w + lo.d2);
    m->dy = (float*)(w + lo.dy);
    m->y = (float*)(w + lo.y);
    m->loss = (float*)(w + lo.loss);
    m->idx = (int32_t*)(w + lo.idx);
    // He initialisation from the seed; biases zero; identity normalisation.
    std::vector<float> p(kParams, 0.0f), zero(kParams, 0.0f), norm(kNorm, 0.0f);
    std::mt19937_64 rng(seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    for (int i = 0; i < kHid * kIn; ++i) p[kW1 + i] = (float)(nd(rng) * std::sqrt(2.0 / kIn));
    for (int i = 0; i < kHid * kHid; ++i) p[kW2 + i] = (float)(nd(rng) * std::sqrt(2.0 / kHid));
    for (int i = 0; i < kHid; ++i) p[kW3 + i] = (float)(nd(rng) * std::sqrt(1.0 / kHid));
    for (int k = 0; k < kIn; ++k) norm[kIn + k] = 1.0f;
    norm[2 * kIn + 1] = 1.0f;
    *out = m;
    MCHK(hipMemcpyAsync(m->p, p.data(), kParams * 4, hipMemcpyHostToDevice, m->stream));
    MCHK(hipMemcpyAsync(m->mom, zero.data(), kParams * 4, hipMemcpyHostToDevice, m->stream));
    MCHK(hipMemcpyAsync(m->norm, norm.data(), kNorm * 4, hipMemcpyHostToDevice, m->stream));
    hipLaunchKernelGGL(k_to_bf16, dim3((kParams + 255) / 256), dim3(256), 0, m->stream, m->p, m->wb);
    MCHK(hipGetLastError());
    MCHK(hipStreamSynchronize(m->stream));
    return PA_OK;
}

pa_status pa_mlp_set_params(pa_mlp* m, const float* params, const float* norm)
{
    if (!m || (!params && !norm)) return PA_EINVAL;
    if (m->broken) return PA_ESTATE;
    if (params) {
        MCHK(hipMemcpyAsync(m->p, params, kParams * 4, hipMemcpyHostToDevice, m->stream));
        hipLaunchKernelGGL(k_to_bf16, dim3((kParams + 255) / 256), dim3(256), 0, m->stream, m->p, m->wb);
        MCHK(hipGetLastError());
    }
    if (norm) MCHK(hipMemcpyAsync(m->norm, norm, kNorm * 4, hipMemcpyHostToDevice, m->stream));
    MCHK(hipStreamSynchronize(m->stream));
    return PA_OK;
}

pa_status pa_mlp_get_params(pa_mlp* m, float* params, float* norm)
{
    if (!m || (!params && !norm)) return PA_EINVAL;
    if (m->broken) return PA_ESTATE;
    if (params) MCHK(hipMemcpyAsync(params, m->p, kParams * 4, hipMemcpyDeviceToHost, m->stream));
    if (norm) MCHK(hipMemcpyAsync(norm, m->norm, kNorm * 4, hipMemcpyDeviceToHost, m->stream));
    MCHK(hipStreamSynchronize(m->stream));
    return PA_OK;
}

pa_status pa_mlp_fit_norm(pa_mlp* m, const float* d_x, const float* d_t, int32_t n)
{
    if (!m || !d_x || !d_t || n < 2) return PA_EINVAL;
    if (m->broken) return PA_ESTATE;
    hipLaunchKernelGGL(k_fit_norm, dim3(1), dim3(64), 0, m->stream, d_x, d_t, n, m->norm);
    MCHK(hipGetLastError());
    MCHK(hipStreamSynchronize(m->stream));
    return PA_OK;
}

pa_status pa_mlp_forward(pa_mlp* m, const float* d_x, int32_t n, float* d_y, int32_t bf16)
{
    if (!m || !d_x || !d_y || n < 0) return PA_EINVAL;
    if (m->broken) return PA_ESTATE;
    if (n == 0) return PA_OK;
    hipLaunchKernelGGL(k_infer, dim3(n), dim3(64), 0, m->stream, d_x, m->p, m->wb, m->norm, bf16 ? 1 : 0, d_y);
    MCHK(hipGetLastError());
    MCHK(hipStreamSynchronize(m->stream));
    return PA_OK;
}

pa_status pa_mlp_gradient(pa_mlp* m, const float* d_x, const float* d_t, int32_t n, float* grad, float* loss)
{
    if (!m || !d_x || !d_t || n < 1 || n > m->max_batch) return PA_EINVAL;
    if (m->broken) return PA_ESTATE;
    hipLaunchKernelGGL(k_gather_norm, dim3((n + 255) / 256), dim3(256), 0, m->stream, d_x, d_t, (const int32_t*)nullptr,
                       n, m->norm, m->xn, m->tn);
    MCHK(hipGetLastError());
    MCHK(hipMemsetAsync(m->loss, 0, 4, m->stream));
    const pa_status st = grad_pass(m, n, m->loss);
    if (st != PA_OK) return st;
    if (grad) MCHK(hipMemcpyAsync(grad, m->grad, kParams * 4, hipMemcpyDeviceToHost, m->stream));
    if (loss) MCHK(hipMemcpyAsync(loss, m->loss, 4, hipMemcpyDeviceToHost, m->stream));
    MCHK(hipStreamSynchronize(m->stream));
    return PA_OK;
}

pa_status pa_mlp_train(pa_mlp* m, const float* d_x, const float* d_t, int32_t n, int32_t batch, int32_t epochs,
                       float lr, float momentum, uint64_t seed, float* epoch_loss)
{
    if (!m || !d_x || !d_t || n < 1 || batch < 1 || batch > m->max_batch || epochs < 0 || !(lr > 0.0f)) return PA_EINVAL;
    if (m->broken) return PA_ESTATE;
    std::mt19937_64 rng(seed);
    std::vector<int32_t> perm((size_t)n);
    const int nb = n / batch;  // full minibatches only
    if (nb < 1) return PA_EINVAL;
    for (int e = 0; e < epochs; ++e) {
        for (int i = 0; i < n; ++i) perm[(size_t)i] = i;
        std::shuffle(perm.begin(), perm.end(), rng);
        MCHK(hipMemsetAsync(m->loss, 0, 4, m->stream));
        for (int k = 0; k < nb; ++k) {
            MCHK(hipMemcpyAsync(m->idx, perm.data() + (size_t)k * batch, (size_t)batch * 4, hipMemcpyHostToDevice,
                                m->stream));
            hipLaunchKernelGGL(k_gather_norm, dim3((batch + 255) / 256), dim3(256), 0, m->stream, d_x, d_t, m->idx,
                               batch, m->norm, m->xn, m->tn);
            MCHK(hipGetLastError());
            const pa_status st = grad_pass(m, batch, m->loss);
            if (st != PA_OK) return st;
            hipLaunchKernelGGL(k_sgd, dim3((kParams + 255) / 256), dim3(256), 0, m->stream, m->p, m->grad, m->mom, lr,
                               momentum, m->wb);
            MCHK(hipGetLastError());
            // the index buffer is reused by the next minibatch: wait for this one
            MCHK(hipStreamSynchronize(m->stream));
        }
        float l = 0.0f;
        MCHK(hipMemcpyAsync(&l, m->loss, 4, hipMemcpyDeviceToHost, m->stream));
        MCHK(hipStreamSynchronize(m->stream));
        if (epoch_loss) epoch_loss[e] = l / (float)nb;
    }
    return PA_OK;
}

const char* pa_mlp_last_error(const pa_mlp* m) { return m ? m->last_error.c_str() : ""; }

pa_status pa_mlp_free(pa_mlp* m)
{
    delete m;
    return PA_OK;
}

}  // extern "C"
