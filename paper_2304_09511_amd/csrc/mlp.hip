// The format selector's network: MLP 8-64-64-7 (ReLU, softmax cross-entropy;
// one output per format: COO, CSR, DIA, ELL, SELL-64-1, HYB, HDC) in FP32 with forward,
// backward and Adam kernels.  Parameter layout (row-major, input index
// first): W1[8][64], b1[64], W2[64][64], b2[64], W3[64][7], b3[7].  Reductions over samples run in sample order with FP64
// accumulators, so gradients are deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "common.h"

namespace mxs {

constexpr int NI = 8, NH = 64, NO = MXS_NCLASS;
constexpr int OW1 = 0, OB1 = OW1 + NI * NH, OW2 = OB1 + NH, OB2 = OW2 + NH * NH,
              OW3 = OB2 + NH, OB3 = OW3 + NH * NO, NPAR = OB3 + NO;
static_assert(NPAR == MXS_MLP_NPARAM, "parameter count");

// per-sample scratch of the backward pass: H1, H2, DH1, DH2 [64], DZ [NO], loss
constexpr int kSampleScratch = 4 * NH + NO + 1;

// ---------------------------------------------------------------------------
// Inputs: log1p on count-like features, then z-score
// ---------------------------------------------------------------------------
__global__ void mlp_inputs_kernel(const double *__restrict__ raw, int32_t n,
                                  const float *__restrict__ mu, const float *__restrict__ sd,
                                  float *__restrict__ X)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n * NI) return;
    const int f = (int)(i % NI);
    const double v = raw[i];
    const double t = f < 6 ? log1p(v) : v;
    X[i] = (float)((t - (double)mu[f]) / (double)sd[f]);
}

__global__ void mlp_norm_kernel(const double *__restrict__ raw, int32_t n, float *__restrict__ mu,
                                float *__restrict__ sd)
{
    const int f = threadIdx.x;
    if (f >= NI) return;
    double m = 0.0;
    for (int32_t s = 0; s < n; ++s) {
        const double v = raw[(int64_t)s * NI + f];
        m += f < 6 ? log1p(v) : v;
    }
    m = n ? m / n : 0.0;
    double q = 0.0;
    for (int32_t s = 0; s < n; ++s) {
        const double v = raw[(int64_t)s * NI + f];
        const double d = (f < 6 ? log1p(v) : v) - m;
        q += d * d;
    }
    const double sdev = n ? sqrt(q / n) : 0.0;
    mu[f] = (float)m;
    // a spread below 1e-6 of the mean is a constant feature up to rounding
    // (the two-pass sum need not return the constant exactly): scale 1
    sd[f] = sdev > 1e-6 * fabs(m) && sdev > 0.0 ? (float)sdev : 1.0f;
}

// ---------------------------------------------------------------------------
// Forward (one thread per sample, weights staged in LDS)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void forward_one(const float *w, const float *xin, float z[NO])
{
    float h1[NH];
#pragma unroll 8
    for (int j = 0; j < NH; ++j) {
        float a = w[OB1 + j];
#pragma unroll
        for (int i = 0; i < NI; ++i) a += xin[i] * w[OW1 + i * NH + j];
        h1[j] = a > 0.0f ? a : 0.0f;
    }
    for (int c = 0; c < NO; ++c) z[c] = w[OB3 + c];
    for (int k = 0; k < NH; ++k) {
        float a = w[OB2 + k];
#pragma unroll 8
        for (int j = 0; j < NH; ++j) a += h1[j] * w[OW2 + j * NH + k];
        const float h2 = a > 0.0f ? a : 0.0f;
#pragma unroll
        for (int c = 0; c < NO; ++c) z[c] += h2 * w[OW3 + k * NO + c];
    }
}

template <bool PREDICT>
__global__ __launch_bounds__(256) void mlp_forward_kernel(const float *__restrict__ w,
                                                          const float *__restrict__ X, int32_t n,
                                                          float *__restrict__ logits,
                                                          const uint8_t *__restrict__ feasible,
                                                          int32_t *__restrict__ fmt)
{
    __shared__ float sw[NPAR];
    for (int i = threadIdx.x; i < NPAR; i += blockDim.x) sw[i] = w[i];
    __syncthreads();
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    float xin[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) xin[i] = X[s * NI + i];
    float z[NO];
    forward_one(sw, xin, z);
    if (!PREDICT) {
#pragma unroll
        for (int c = 0; c < NO; ++c) logits[s * NO + c] = z[c];
    } else {
        int best = -1;
        for (int c = 0; c < NO; ++c) {
            if (feasible && !feasible[s * NO + c]) continue;
            if (best < 0 || z[c] > z[best]) best = c;
        }
        fmt[s] = best;
    }
}

// ---------------------------------------------------------------------------
// Backward: one 64-thread workgroup per sample (thread j = hidden unit j)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void mlp_sample_kernel(const float *__restrict__ w,
                                                        const float *__restrict__ X,
                                                        const int32_t *__restrict__ labels,
                                                        int32_t n, float *__restrict__ scratch)
{
    __shared__ float h1[NH], h2[NH], dh2[NH], z[NO], dz[NO];
    const int s = blockIdx.x;
    const int j = threadIdx.x;
    const float *xin = X + (int64_t)s * NI;
    float *o = scratch + (int64_t)s * kSampleScratch;
    float a1 = w[OB1 + j];
    for (int i = 0; i < NI; ++i) a1 += xin[i] * w[OW1 + i * NH + j];
    h1[j] = a1 > 0.0f ? a1 : 0.0f;
    __syncthreads();
    float a2 = w[OB2 + j];
    for (int k = 0; k < NH; ++k) a2 += h1[k] * w[OW2 + k * NH + j];
    h2[j] = a2 > 0.0f ? a2 : 0.0f;
    __syncthreads();
    if (j < NO) {
        float t = w[OB3 + j];
        for (int k = 0; k < NH; ++k) t += h2[k] * w[OW3 + k * NO + j];
        z[j] = t;
    }
    __syncthreads();
    if (j == 0) {
        // shift by the largest logit so that no exponent overflows
        float m = z[0];
        for (int c = 1; c < NO; ++c) m = fmaxf(m, z[c]);
        float e[NO], den = 0.0f;
        for (int c = 0; c < NO; ++c) {
            e[c] = expf(z[c] - m);
            den += e[c];
        }
        const int y = labels[s];
        const bool ok = y >= 0 && y < NO; // a label outside {0, ..., NO-1} gives a NaN loss
        for (int c = 0; c < NO; ++c) {
            dz[c] = (e[c] / den - (c == y ? 1.0f : 0.0f)) / (float)n;
            o[4 * NH + c] = dz[c];
        }
        o[4 * NH + NO] = ok ? -((z[y] - m) - logf(den)) : __builtin_nanf("");
    }
    __syncthreads();
    float g2 = 0.0f;
    for (int c = 0; c < NO; ++c) g2 += w[OW3 + j * NO + c] * dz[c];
    dh2[j] = a2 > 0.0f ? g2 : 0.0f;
    __syncthreads();
    float g1 = 0.0f;
    for (int k = 0; k < NH; ++k) g1 += w[OW2 + j * NH + k] * dh2[k];
    o[j] = h1[j];
    o[NH + j] = h2[j];
    o[2 * NH + j] = a1 > 0.0f ? g1 : 0.0f;
    o[3 * NH + j] = dh2[j];
}

// One thread per parameter (plus one for the mean loss): sums over samples in
// sample order.
__global__ __launch_bounds__(256) void mlp_wgrad_kernel(const float *__restrict__ X, int32_t n,
                                                        const float *__restrict__ scratch,
                                                        float *__restrict__ grad,
                                                        float *__restrict__ loss)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > NPAR) return;
    double acc = 0.0;
    auto S = [&](int s, int off) { return (double)scratch[(int64_t)s * kSampleScratch + off]; };
    if (p == NPAR) {
        for (int s = 0; s < n; ++s) acc += S(s, 4 * NH + NO);
        *loss = (float)(n ? acc / n : 0.0);
        return;
    }
    if (p < OB1) { // W1[i][j] = sum_s x_i dh1_j
        const int i = p / NH, j = p % NH;
        for (int s = 0; s < n; ++s) acc += (double)X[(int64_t)s * NI + i] * S(s, 2 * NH + j);
    } else if (p < OW2) { // b1[j]
        const int j = p - OB1;
        for (int s = 0; s < n; ++s) acc += S(s, 2 * NH + j);
    } else if (p < OB2) { // W2[j][k] = sum_s h1_j dh2_k
        const int j = (p - OW2) / NH, k = (p - OW2) % NH;
        for (int s = 0; s < n; ++s) acc += S(s, j) * S(s, 3 * NH + k);
    } else if (p < OW3) { // b2[k]
        const int k = p - OB2;
        for (int s = 0; s < n; ++s) acc += S(s, 3 * NH + k);
    } else if (p < OB3) { // W3[k][c] = sum_s h2_k dz_c
        const int k = (p - OW3) / NO, c = (p - OW3) % NO;
        for (int s = 0; s < n; ++s) acc += S(s, NH + k) * S(s, 4 * NH + c);
    } else { // b3[c]
        const int c = p - OB3;
        for (int s = 0; s < n; ++s) acc += S(s, 4 * NH + c);
    }
    grad[p] = (float)acc;
}

__global__ void mlp_adam_kernel(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                                const float *__restrict__ g, float lr, float b1, float b2,
                                float eps, float c1, float c2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NPAR) return;
    const float gp = g[p];
    const float mp = b1 * m[p] + (1.0f - b1) * gp;
    const float vp = b2 * v[p] + (1.0f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    w[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
mxs_status mlp_inputs(const double *raw, int32_t n, const float *mu, const float *sd, float *X,
                      hipStream_t s)
{
    if (n <= 0) return MXS_OK;
    const int64_t tot = (int64_t)n * NI;
    mlp_inputs_kernel<<<(uint32_t)((tot + 255) / 256), 256, 0, s>>>(raw, n, mu, sd, X);
    return launch_status();
}

mxs_status mlp_norm_stats(const double *raw, int32_t n, float *mu, float *sd, hipStream_t s)
{
    mlp_norm_kernel<<<1, 64, 0, s>>>(raw, n, mu, sd);
    return launch_status();
}

mxs_status mlp_forward(const float *w, const float *X, int32_t n, float *logits, hipStream_t s)
{
    if (n <= 0) return MXS_OK;
    mlp_forward_kernel<false><<<(uint32_t)((n + 255) / 256), 256, 0, s>>>(w, X, n, logits, nullptr,
                                                                         nullptr);
    return launch_status();
}

mxs_status mlp_predict(const float *w, const float *X, int32_t n, const uint8_t *feasible,
                       int32_t *fmt, hipStream_t s)
{
    if (n <= 0) return MXS_OK;
    mlp_forward_kernel<true><<<(uint32_t)((n + 255) / 256), 256, 0, s>>>(w, X, n, nullptr,
                                                                        feasible, fmt);
    return launch_status();
}

size_t mlp_ws_bytes(int32_t n) { return sizeof(float) * (size_t)std::max(n, 1) * kSampleScratch; }

mxs_status mlp_grad(const float *w, const float *X, const int32_t *labels, int32_t n, float *grad,
                    float *loss, void *ws, hipStream_t s)
{
    if (n > 0) {
        mlp_sample_kernel<<<(uint32_t)n, 64, 0, s>>>(w, X, labels, n, (float *)ws);
        MXS_HIP(hipGetLastError());
    }
    mlp_wgrad_kernel<<<(NPAR + 1 + 255) / 256, 256, 0, s>>>(X, n, (const float *)ws, grad, loss);
    return launch_status();
}

mxs_status mlp_adam(float *w, float *m, float *v, const float *g, float lr, int32_t t, float b1,
                    float b2, float eps, hipStream_t s)
{
    const float c1 = (float)(1.0 - std::pow((double)b1, (double)t));
    const float c2 = (float)(1.0 - std::pow((double)b2, (double)t));
    mlp_adam_kernel<<<(NPAR + 255) / 256, 256, 0, s>>>(w, m, v, g, lr, b1, b2, eps, c1, c2);
    return launch_status();
}

}  // namespace mxs
