// Training of the order network (3 layers, 64 hidden, ReLU; layout of the
// weight array in sfmm.h): per-sample forward and backward, gradients summed
// per weight in a fixed order (deterministic), Adam.  FP32 master weights;
// inference (k_order_mlp) rounds weights and activations to bfloat16.
//
// Loss per sample: w(r) r^2 with r = y - label and w = kUnder for r < 0:
// predicting too low an order costs accuracy, too high only time.
#include "common.hpp"

namespace sfmm {

static unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b > 0 ? (n + b - 1) / b : 1); }

constexpr float kUnder = 4.0f;
// per-sample record: f [kMlpIn], h1, d1, h2, d2 [kMlpHidden], g, loss
constexpr int kRec = kMlpIn + 4 * kMlpHidden + 2;
constexpr int oW1 = 0, oB1 = oW1 + kMlpHidden * kMlpIn, oW2 = oB1 + kMlpHidden, oB2 = oW2 + kMlpHidden * kMlpHidden,
              oW3 = oB2 + kMlpHidden, oB3 = oW3 + kMlpHidden;
static_assert(oB3 + 1 == kMlpWeights, "weight layout");

__global__ void __launch_bounds__(128) k_mlp_fwd_bwd(const float* __restrict__ w, const float* __restrict__ feat,
                                                     const float* __restrict__ label, int n, float scale,
                                                     float* __restrict__ rec) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const float* f = feat + (size_t)s * kMlpIn;
    float* r = rec + (size_t)s * kRec;
    float h1[kMlpHidden], h2[kMlpHidden];
#pragma unroll
    for (int i = 0; i < kMlpHidden; ++i) {
        float v = w[oB1 + i];
#pragma unroll
        for (int j = 0; j < kMlpIn; ++j) v = fmaf(w[oW1 + i * kMlpIn + j], f[j], v);
        h1[i] = v > 0.0f ? v : 0.0f;
    }
    float y = w[oB3];
    for (int i = 0; i < kMlpHidden; ++i) {
        float v = w[oB2 + i];
#pragma unroll
        for (int j = 0; j < kMlpHidden; ++j) v = fmaf(w[oW2 + i * kMlpHidden + j], h1[j], v);
        h2[i] = v > 0.0f ? v : 0.0f;
        y = fmaf(w[oW3 + i], h2[i], y);
    }
    const float res = y - label[s];
    const float wt = res < 0.0f ? kUnder : 1.0f;
    const float g = 2.0f * wt * res * scale;  // dL/dy with L = scale sum w r^2
    // d2 = g w3 [h2 > 0]; d1 = (W2^T d2) [h1 > 0]
    float d1[kMlpHidden];
#pragma unroll
    for (int j = 0; j < kMlpHidden; ++j) d1[j] = 0.0f;
    for (int i = 0; i < kMlpHidden; ++i) {
        const float d2 = h2[i] > 0.0f ? g * w[oW3 + i] : 0.0f;
        r[kMlpIn + 3 * kMlpHidden + i] = d2;
#pragma unroll
        for (int j = 0; j < kMlpHidden; ++j) d1[j] = fmaf(w[oW2 + i * kMlpHidden + j], d2, d1[j]);
    }
#pragma unroll
    for (int j = 0; j < kMlpIn; ++j) r[j] = f[j];
#pragma unroll
    for (int j = 0; j < kMlpHidden; ++j) {
        r[kMlpIn + j] = h1[j];
        r[kMlpIn + kMlpHidden + j] = h1[j] > 0.0f ? d1[j] : 0.0f;
        r[kMlpIn + 2 * kMlpHidden + j] = h2[j];
    }
    r[kMlpIn + 4 * kMlpHidden] = g;
    r[kMlpIn + 4 * kMlpHidden + 1] = scale * wt * res * res;
}

// FP32 forward only
__global__ void __launch_bounds__(128) k_mlp_fwd(const float* __restrict__ w, const float* __restrict__ feat, int n,
                                                 float* __restrict__ yout) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const float* f = feat + (size_t)s * kMlpIn;
    float h1[kMlpHidden];
#pragma unroll
    for (int i = 0; i < kMlpHidden; ++i) {
        float v = w[oB1 + i];
#pragma unroll
        for (int j = 0; j < kMlpIn; ++j) v = fmaf(w[oW1 + i * kMlpIn + j], f[j], v);
        h1[i] = v > 0.0f ? v : 0.0f;
    }
    float y = w[oB3];
    for (int i = 0; i < kMlpHidden; ++i) {
        float v = w[oB2 + i];
#pragma unroll
        for (int j = 0; j < kMlpHidden; ++j) v = fmaf(w[oW2 + i * kMlpHidden + j], h1[j], v);
        y = fmaf(w[oW3 + i], v > 0.0f ? v : 0.0f, y);
    }
    yout[s] = y;
}

// grad[k] for every weight k, and grad[kMlpWeights] = the loss: sums over
// the n samples in sample order
__global__ void k_mlp_grad(const float* __restrict__ rec, int n, float* __restrict__ grad) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > kMlpWeights) return;
    const int F = 0, H1 = kMlpIn, D1 = H1 + kMlpHidden, H2 = D1 + kMlpHidden, D2 = H2 + kMlpHidden,
              G = D2 + kMlpHidden, L = G + 1;
    int a, b;  // product of record entries a and b (b < 0: entry a alone)
    if (k < oB1) {
        a = D1 + k / kMlpIn;
        b = F + k % kMlpIn;
    } else if (k < oW2) {
        a = D1 + (k - oB1);
        b = -1;
    } else if (k < oB2) {
        a = D2 + (k - oW2) / kMlpHidden;
        b = H1 + (k - oW2) % kMlpHidden;
    } else if (k < oW3) {
        a = D2 + (k - oB2);
        b = -1;
    } else if (k < oB3) {
        a = G;
        b = H2 + (k - oW3);
    } else if (k == oB3) {
        a = G;
        b = -1;
    } else {
        a = L;
        b = -1;
    }
    double acc = 0.0;
    for (int s = 0; s < n; ++s) {
        const float* r = rec + (size_t)s * kRec;
        acc += b < 0 ? (double)r[a] : (double)r[a] * (double)r[b];
    }
    grad[k] = (float)acc;
}

__global__ void k_mlp_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                           const float* __restrict__ grad, float lr, float c1, float c2) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kMlpWeights) return;
    const float b1 = 0.9f, b2 = 0.999f, e = 1e-8f;
    const float g = grad[k];
    const float mk = b1 * m[k] + (1.0f - b1) * g;
    const float vk = b2 * v[k] + (1.0f - b2) * g * g;
    m[k] = mk;
    v[k] = vk;
    w[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + e);
}

void mlp_grad(const float* w, const float* feat, const float* label, int n, float* rec, float* grad, hipStream_t s) {
    if (n <= 0) return;
    k_mlp_fwd_bwd<<<nblk(n, 128), 128, 0, s>>>(w, feat, label, n, 1.0f / (float)n, rec);
    SFMM_LAUNCH_CHECK();
    k_mlp_grad<<<nblk(kMlpWeights + 1, 128), 128, 0, s>>>(rec, n, grad);
    SFMM_LAUNCH_CHECK();
}

void mlp_adam(float* w, float* m, float* v, const float* grad, float lr, int step, hipStream_t s) {
    const float c1 = 1.0f - powf(0.9f, (float)step), c2 = 1.0f - powf(0.999f, (float)step);
    k_mlp_adam<<<nblk(kMlpWeights, 256), 256, 0, s>>>(w, m, v, grad, lr, c1, c2);
    SFMM_LAUNCH_CHECK();
}

void mlp_forward_f32(const float* w, const float* feat, int n, float* y, hipStream_t s) {
    if (n <= 0) return;
    k_mlp_fwd<<<nblk(n, 128), 128, 0, s>>>(w, feat, n, y);
    SFMM_LAUNCH_CHECK();
}

size_t mlp_record_floats() { return kRec; }

}  // namespace sfmm
