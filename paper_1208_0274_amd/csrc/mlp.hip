// Work predictor for frontier ordering: a small fully connected network
// (ALAE_MLP_FEATURES -> 32 -> 32 -> 1, ReLU) mapping a chain item's
// features to log2(1 + measured work).  Forward, backward and Adam run in
// these kernels; the network only orders the queues the walkers drain, so the
// hit set never depends on it.
//
// Parameter layout (flat, fp32): W1[32][F] (row = output unit), b1[32],
// W2[32][32], b2[32], W3[32], b3.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <random>
#include <vector>

#include "alae_internal.h"
#include "mlp_internal.h"

namespace alae {

constexpr int kF = ALAE_MLP_FEATURES;
constexpr int kH = ALAE_MLP_HIDDEN;
constexpr int kP = ALAE_MLP_PARAMS;
constexpr int oW1 = 0, oB1 = kH * kF, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH, oB3 = oW3 + kH;
static_assert(oB3 + 1 == kP, "parameter count");

#define MLP_TRY(expr)                                                                            \
    do {                                                                                         \
        hipError_t _e = (expr);                                                                  \
        if (_e != hipSuccess) {                                                                  \
            set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, __LINE__); \
            return ALAE_E_DEVICE;                                                                \
        }                                                                                        \
    } while (0)

__device__ inline float wave_sum_f32(float v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Forward pass of one sample; h1, h2 keep the hidden activations.
__device__ inline float mlp_forward(const float *p, const float *x, float *h1, float *h2) {
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        float s = p[oB1 + j];
#pragma unroll
        for (int k = 0; k < kF; ++k) s += p[oW1 + j * kF + k] * x[k];
        h1[j] = s > 0.f ? s : 0.f;
    }
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        float s = p[oB2 + j];
#pragma unroll
        for (int k = 0; k < kH; ++k) s += p[oW2 + j * kH + k] * h1[k];
        h2[j] = s > 0.f ? s : 0.f;
    }
    float y = p[oB3];
#pragma unroll
    for (int j = 0; j < kH; ++j) y += p[oW3 + j] * h2[j];
    return y;
}

__global__ void __launch_bounds__(256) k_mlp_predict(const float *params, const float *x, uint32_t n, float *y) {
    __shared__ float p[kP];
    for (int i = threadIdx.x; i < kP; i += blockDim.x) p[i] = params[i];
    __syncthreads();
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    float xs[kF], h1[kH], h2[kH];
#pragma unroll
    for (int k = 0; k < kF; ++k) xs[k] = x[(size_t)s * kF + k];
    y[s] = mlp_forward(p, xs, h1, h2);
}

// Loss 0.5 * sum_i (y_i - t_i)^2 / scale over the samples idx[0..n) (idx may be
// null: samples 0..n), gradient accumulated into grad (kP floats), loss into
// loss_acc.  Per-parameter sums are reduced over the wave, then over the
// block in LDS, then added to global memory once per block.
__global__ void __launch_bounds__(256) k_mlp_grad(const float *params, const float *x, const float *t,
                                                  const uint32_t *idx, uint32_t n, float scale, float *grad,
                                                  double *loss_acc) {
    __shared__ float p[kP];
    __shared__ float g[kP];
    for (int i = threadIdx.x; i < kP; i += blockDim.x) {
        p[i] = params[i];
        g[i] = 0.f;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = s < n;
    const uint32_t row = valid ? (idx ? idx[s] : s) : 0u;
    float xs[kF], h1[kH], h2[kH];
#pragma unroll
    for (int k = 0; k < kF; ++k) xs[k] = valid ? x[(size_t)row * kF + k] : 0.f;
    const float y = mlp_forward(p, xs, h1, h2);
    const float err = valid ? (y - t[row]) : 0.f;
    const float gy = err / scale;  // dL/dy
    // loss
    const float l = wave_sum_f32(0.5f * err * err / scale);
    if (lane == 0) atomicAdd(loss_acc, (double)l);
    // output layer
    {
        const float r = wave_sum_f32(gy);
        if (lane == 0) atomicAdd(&g[oB3], r);
    }
    float dh2[kH];
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        const float r = wave_sum_f32(gy * h2[j]);
        if (lane == 0) atomicAdd(&g[oW3 + j], r);
        dh2[j] = h2[j] > 0.f ? gy * p[oW3 + j] : 0.f;
    }
    // second hidden layer
    float dh1[kH];
#pragma unroll
    for (int k = 0; k < kH; ++k) dh1[k] = 0.f;
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        const float rb = wave_sum_f32(dh2[j]);
        if (lane == 0) atomicAdd(&g[oB2 + j], rb);
#pragma unroll
        for (int k = 0; k < kH; ++k) {
            const float r = wave_sum_f32(dh2[j] * h1[k]);
            if (lane == 0) atomicAdd(&g[oW2 + j * kH + k], r);
            dh1[k] += dh2[j] * p[oW2 + j * kH + k];
        }
    }
    // first hidden layer
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        const float d = h1[j] > 0.f ? dh1[j] : 0.f;
        const float rb = wave_sum_f32(d);
        if (lane == 0) atomicAdd(&g[oB1 + j], rb);
#pragma unroll
        for (int k = 0; k < kF; ++k) {
            const float r = wave_sum_f32(d * xs[k]);
            if (lane == 0) atomicAdd(&g[oW1 + j * kF + k], r);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kP; i += blockDim.x) atomicAdd(&grad[i], g[i]);
}

// Adam (Kingma and Ba), bias-corrected, one thread per parameter.
__global__ void k_mlp_adam(float *params, const float *grad, float *m1, float *m2, float lr, float b1, float b2,
                           float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kP) return;
    const float gi = grad[i];
    const float a = b1 * m1[i] + (1.f - b1) * gi;
    const float v = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = v;
    params[i] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

__global__ void k_fill_f32(float *p, float v, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_f64(double *p, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// Predictions for n feature rows already on the device (used by the search).
alae_status mlp_predict_device(const alae_mlp *net, const float *d_x, uint32_t n, float *d_y, hipStream_t s) {
    if (n == 0) return ALAE_OK;
    k_mlp_predict<<<(n + 255) / 256, 256, 0, s>>>(net->d_params, d_x, n, d_y);
    MLP_TRY(hipGetLastError());
    return ALAE_OK;
}

// Device buffers for host-side training and checking calls.
static alae_status stage_data(alae_mlp *net, const float *x, const float *t, size_t n) {
    if (n > net->data_cap) {
        hipFree(net->d_x);
        hipFree(net->d_t);
        hipFree(net->d_idx);
        net->d_x = nullptr;
        net->d_t = nullptr;
        net->d_idx = nullptr;
        net->data_cap = 0;
        MLP_TRY(hipMalloc(&net->d_x, n * kF * sizeof(float)));
        MLP_TRY(hipMalloc(&net->d_t, n * sizeof(float)));
        MLP_TRY(hipMalloc(&net->d_idx, n * sizeof(uint32_t)));
        net->data_cap = n;
    }
    MLP_TRY(hipMemcpy(net->d_x, x, n * kF * sizeof(float), hipMemcpyHostToDevice));
    if (t) MLP_TRY(hipMemcpy(net->d_t, t, n * sizeof(float), hipMemcpyHostToDevice));
    return ALAE_OK;
}

}  // namespace alae

using namespace alae;

extern "C" {

alae_status alae_mlp_create(int device, uint64_t seed, alae_mlp **out) {
    if (!out) {
        set_error("alae_mlp_create: null argument");
        return ALAE_E_ARG;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        set_error("alae_mlp_create: device %d is not available", device);
        return ALAE_E_DEVICE;
    }
    std::unique_ptr<alae_mlp> net(new (std::nothrow) alae_mlp());
    if (!net) {
        set_error("out of host memory");
        return ALAE_E_NOMEM;
    }
    net->device = device;
    MLP_TRY(hipSetDevice(device));
    MLP_TRY(hipMalloc(&net->d_params, kP * sizeof(float)));
    MLP_TRY(hipMalloc(&net->d_grad, kP * sizeof(float)));
    MLP_TRY(hipMalloc(&net->d_m1, kP * sizeof(float)));
    MLP_TRY(hipMalloc(&net->d_m2, kP * sizeof(float)));
    MLP_TRY(hipMalloc(&net->d_loss, sizeof(double)));
    // He-uniform weights, zero biases
    std::vector<float> p(kP, 0.f);
    std::mt19937_64 g(seed);
    auto fill = [&](int off, int fan_out, int fan_in) {
        const float lim = std::sqrt(6.f / (float)fan_in);
        std::uniform_real_distribution<float> u(-lim, lim);
        for (int i = 0; i < fan_out * fan_in; ++i) p[off + i] = u(g);
    };
    fill(oW1, kH, kF);
    fill(oW2, kH, kH);
    fill(oW3, 1, kH);
    MLP_TRY(hipMemcpy(net->d_params, p.data(), kP * sizeof(float), hipMemcpyHostToDevice));
    MLP_TRY(hipMemset(net->d_m1, 0, kP * sizeof(float)));
    MLP_TRY(hipMemset(net->d_m2, 0, kP * sizeof(float)));
    *out = net.release();
    return ALAE_OK;
}

void alae_mlp_free(alae_mlp *net) {
    if (!net) return;
    hipSetDevice(net->device);
    hipFree(net->d_params);
    hipFree(net->d_grad);
    hipFree(net->d_m1);
    hipFree(net->d_m2);
    hipFree(net->d_loss);
    hipFree(net->d_x);
    hipFree(net->d_t);
    hipFree(net->d_idx);
    delete net;
}

alae_status alae_mlp_get_params(const alae_mlp *net, float *params) {
    if (!net || !params) {
        set_error("alae_mlp_get_params: null argument");
        return ALAE_E_ARG;
    }
    MLP_TRY(hipSetDevice(net->device));
    MLP_TRY(hipMemcpy(params, net->d_params, kP * sizeof(float), hipMemcpyDeviceToHost));
    return ALAE_OK;
}

alae_status alae_mlp_set_params(alae_mlp *net, const float *params) {
    if (!net || !params) {
        set_error("alae_mlp_set_params: null argument");
        return ALAE_E_ARG;
    }
    for (int i = 0; i < kP; ++i) {
        if (!std::isfinite(params[i])) {
            set_error("alae_mlp_set_params: parameter %d is not finite", i);
            return ALAE_E_ARG;
        }
    }
    MLP_TRY(hipSetDevice(net->device));
    MLP_TRY(hipMemcpy(net->d_params, params, kP * sizeof(float), hipMemcpyHostToDevice));
    MLP_TRY(hipMemset(net->d_m1, 0, kP * sizeof(float)));
    MLP_TRY(hipMemset(net->d_m2, 0, kP * sizeof(float)));
    net->adam_t = 0;
    return ALAE_OK;
}

alae_status alae_mlp_predict(alae_mlp *net, const float *x, size_t n, float *y) {
    if (!net || (n && (!x || !y))) {
        set_error("alae_mlp_predict: null argument");
        return ALAE_E_ARG;
    }
    if (n == 0) return ALAE_OK;
    if (n >= (1ull << 31)) {
        set_error("alae_mlp_predict: too many samples");
        return ALAE_E_ARG;
    }
    MLP_TRY(hipSetDevice(net->device));
    alae_status st = stage_data(net, x, nullptr, n);
    if (st != ALAE_OK) return st;
    float *d_y = net->d_t;  // predictions overwrite the target buffer
    if ((st = mlp_predict_device(net, net->d_x, (uint32_t)n, d_y, nullptr)) != ALAE_OK) return st;
    MLP_TRY(hipMemcpy(y, d_y, n * sizeof(float), hipMemcpyDeviceToHost));
    return ALAE_OK;
}

alae_status alae_mlp_loss_grad(alae_mlp *net, const float *x, const float *t, size_t n, double *loss, float *grad) {
    if (!net || !x || !t || !loss || !grad || n == 0) {
        set_error("alae_mlp_loss_grad: null argument or no samples");
        return ALAE_E_ARG;
    }
    if (n >= (1ull << 31)) {
        set_error("alae_mlp_loss_grad: too many samples");
        return ALAE_E_ARG;
    }
    MLP_TRY(hipSetDevice(net->device));
    alae_status st = stage_data(net, x, t, n);
    if (st != ALAE_OK) return st;
    k_fill_f32<<<(kP + 255) / 256, 256>>>(net->d_grad, 0.f, kP);
    k_fill_f64<<<1, 64>>>(net->d_loss, 1);
    k_mlp_grad<<<(uint32_t)((n + 255) / 256), 256>>>(net->d_params, net->d_x, net->d_t, nullptr, (uint32_t)n,
                                                      (float)n, net->d_grad, net->d_loss);
    MLP_TRY(hipGetLastError());
    MLP_TRY(hipMemcpy(grad, net->d_grad, kP * sizeof(float), hipMemcpyDeviceToHost));
    MLP_TRY(hipMemcpy(loss, net->d_loss, sizeof(double), hipMemcpyDeviceToHost));
    return ALAE_OK;
}

alae_status alae_mlp_train(alae_mlp *net, const float *x, const float *t, size_t n, uint32_t epochs, uint32_t batch,
                           float lr, uint64_t seed, double *final_loss) {
    if (!net || !x || !t || n == 0 || epochs == 0 || batch == 0 || !(lr > 0.f)) {
        set_error("alae_mlp_train: bad argument");
        return ALAE_E_ARG;
    }
    if (n >= (1ull << 31)) {
        set_error("alae_mlp_train: too many samples");
        return ALAE_E_ARG;
    }
    MLP_TRY(hipSetDevice(net->device));
    alae_status st = stage_data(net, x, t, n);
    if (st != ALAE_OK) return st;
    std::vector<uint32_t> perm(n);
    for (size_t i = 0; i < n; ++i) perm[i] = (uint32_t)i;
    std::mt19937_64 g(seed);
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    for (uint32_t ep = 0; ep < epochs; ++ep) {
        std::shuffle(perm.begin(), perm.end(), g);
        MLP_TRY(hipMemcpy(net->d_idx, perm.data(), n * sizeof(uint32_t), hipMemcpyHostToDevice));
        for (size_t b0 = 0; b0 < n; b0 += batch) {
            const uint32_t nb = (uint32_t)std::min<size_t>(batch, n - b0);
            k_fill_f32<<<(kP + 255) / 256, 256>>>(net->d_grad, 0.f, kP);
            k_mlp_grad<<<(nb + 255) / 256, 256>>>(net->d_params, net->d_x, net->d_t, net->d_idx + b0, nb, (float)nb,
                                                  net->d_grad, net->d_loss);
            ++net->adam_t;
            const float c1 = 1.f - std::pow(b1, (float)net->adam_t);
            const float c2 = 1.f - std::pow(b2, (float)net->adam_t);
            k_mlp_adam<<<(kP + 255) / 256, 256>>>(net->d_params, net->d_grad, net->d_m1, net->d_m2, lr, b1, b2, eps,
                                                  c1, c2);
        }
        MLP_TRY(hipGetLastError());
    }
    MLP_TRY(hipDeviceSynchronize());
    if (final_loss) {
        // loss of the trained parameters over all samples
        std::vector<float> grad(kP);
        double l = 0.0;
        if ((st = alae_mlp_loss_grad(net, x, t, n, &l, grad.data())) != ALAE_OK) return st;
        *final_loss = l;
    }
    return ALAE_OK;
}

}  // extern "C"
