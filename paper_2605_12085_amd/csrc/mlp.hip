// Learned initial line-search step: a 5-64-64-1 ReLU perceptron (inference, the gradient
// of its mean-squared training loss, and Adam), all in FP32 with FP64 sums.
//
// Parameters are one FP32 vector in the order W1[64][5], b1[64], W2[64][64], b2[64],
// w3[64], b3.  Training keeps per-sample activations and back-propagated errors in a
// caller-supplied workspace, sample-major ([n][64]), so the gradient kernel's lanes
// (64 consecutive parameters of one weight row) read one contiguous row per sample;
// the per-parameter sums run over sample chunks in FP64 and are added in chunk order,
// so a gradient is reproducible bit for bit.
#include <cmath>

#include "common.h"
#include "device_util.h"

namespace fbl {

namespace {

constexpr int kIn = FBL_MLP_IN;
constexpr int kH = FBL_MLP_HIDDEN;
constexpr int kW1 = 0;
constexpr int kB1 = kW1 + kH * kIn;
constexpr int kW2 = kB1 + kH;
constexpr int kB2 = kW2 + kH * kH;
constexpr int kW3 = kB2 + kH;
constexpr int kB3 = kW3 + kH;
constexpr int kNP = kB3 + 1;
static_assert(kNP == FBL_MLP_NPARAMS, "parameter count");
constexpr int kGradChunks = 32;

struct Work {
    float *h1, *h2, *d1, *d2, *d3;   // [n][64] x 4, [n]
    double *gpart;                   // [kGradChunks][kNP]
    double *lpart;                   // per forward block
};

size_t act_bytes(int64_t n)   // activations and errors, padded to 256 bytes
{
    const size_t b = (size_t)(4 * n * kH + n) * sizeof(float);
    return (b + 255) & ~(size_t)255;
}

Work carve(void *base, int64_t n)
{
    Work w;
    float *f = (float *)base;
    w.h1 = f;
    w.h2 = f + n * kH;
    w.d1 = f + 2 * n * kH;
    w.d2 = f + 3 * n * kH;
    w.d3 = f + 4 * n * kH;
    w.gpart = (double *)((char *)base + act_bytes(n));
    w.lpart = w.gpart + (size_t)kGradChunks * kNP;
    return w;
}

// One thread per sample: y = MLP(x).  With targets, also e = y - t, the FP64 block sum of
// e^2, and the back-propagated errors of the loss L = 1/(2n) sum e^2.
__global__ __launch_bounds__(256) void mlp_fwd_kernel(const float *__restrict__ prm, const float *__restrict__ X,
                                                      const float *__restrict__ tgt, int64_t n, float *__restrict__ out,
                                                      Work w)
{
    __shared__ float P[kNP];
    __shared__ double red[4];
    for (int i = threadIdx.x; i < kNP; i += 256) P[i] = prm[i];
    __syncthreads();
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double l = 0.0;
    if (s < n) {
        float xin[kIn];
#pragma unroll
        for (int k = 0; k < kIn; ++k) xin[k] = X[s * kIn + k];
        float h1[kH], h2[kH];
#pragma unroll
        for (int i = 0; i < kH; ++i) {
            float a = P[kB1 + i];
#pragma unroll
            for (int k = 0; k < kIn; ++k) a = fmaf(P[kW1 + i * kIn + k], xin[k], a);
            h1[i] = fmaxf(a, 0.0f);
        }
#pragma unroll
        for (int j = 0; j < kH; ++j) {
            float a = P[kB2 + j];
#pragma unroll
            for (int i = 0; i < kH; ++i) a = fmaf(P[kW2 + j * kH + i], h1[i], a);
            h2[j] = fmaxf(a, 0.0f);
        }
        float o = P[kB3];
#pragma unroll
        for (int j = 0; j < kH; ++j) o = fmaf(P[kW3 + j], h2[j], o);
        if (out) out[s] = o;
        if (tgt) {
            const float e = o - tgt[s];
            l = (double)e * (double)e;
            const float d3 = e / (float)n;
            w.d3[s] = d3;
#pragma unroll
            for (int j = 0; j < kH; ++j) {
                w.h1[s * kH + j] = h1[j];
                w.h2[s * kH + j] = h2[j];
                h2[j] = h2[j] > 0.0f ? d3 * P[kW3 + j] : 0.0f;   // now the error at layer 2
                w.d2[s * kH + j] = h2[j];
            }
#pragma unroll
            for (int i = 0; i < kH; ++i) {
                float a = 0.0f;
#pragma unroll
                for (int j = 0; j < kH; ++j) a = fmaf(P[kW2 + j * kH + i], h2[j], a);
                w.d1[s * kH + i] = h1[i] > 0.0f ? a : 0.0f;
            }
        }
    }
    if (tgt) {
        const double b = block_sum_256(l, red);
        if (threadIdx.x == 0) w.lpart[blockIdx.x] = b;
    }
}

// Per parameter and sample chunk: the FP64 sum over the chunk's samples of the product
// that parameter's derivative takes (error of its output unit times its input).
__global__ __launch_bounds__(256) void mlp_grad_partial_kernel(const float *__restrict__ X, int64_t n, Work w)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= kNP) return;
    const int64_t per = (n + kGradChunks - 1) / kGradChunks;
    const int64_t s0 = blockIdx.y * per;
    const int64_t s1 = s0 + per < n ? s0 + per : n;
    const float *a;   // error of the output unit, stride sa
    const float *b;   // input of the parameter (nullptr: 1), stride sb
    int64_t sa, sb;
    if (p < kB1) {
        const int i = p / kIn, k = p % kIn;
        a = w.d1 + i; sa = kH; b = X + k; sb = kIn;
    } else if (p < kW2) {
        a = w.d1 + (p - kB1); sa = kH; b = nullptr; sb = 0;
    } else if (p < kB2) {
        const int j = (p - kW2) / kH, i = (p - kW2) % kH;
        a = w.d2 + j; sa = kH; b = w.h1 + i; sb = kH;
    } else if (p < kW3) {
        a = w.d2 + (p - kB2); sa = kH; b = nullptr; sb = 0;
    } else if (p < kB3) {
        a = w.d3; sa = 1; b = w.h2 + (p - kW3); sb = kH;
    } else {
        a = w.d3; sa = 1; b = nullptr; sb = 0;
    }
    double acc = 0.0;
    if (b) {
        for (int64_t s = s0; s < s1; ++s) acc += (double)a[s * sa] * (double)b[s * sb];
    } else {
        for (int64_t s = s0; s < s1; ++s) acc += (double)a[s * sa];
    }
    w.gpart[(int64_t)blockIdx.y * kNP + p] = acc;
}

__global__ __launch_bounds__(256) void mlp_grad_final_kernel(Work w, int n_lblocks, float *__restrict__ grad,
                                                            double *__restrict__ loss)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p < kNP) {
        double acc = 0.0;
        for (int c = 0; c < kGradChunks; ++c) acc += w.gpart[(int64_t)c * kNP + p];
        grad[p] = (float)acc;
    }
    if (loss && blockIdx.x == 0 && threadIdx.x == 0) {
        double l = 0.0;
        for (int b = 0; b < n_lblocks; ++b) l += w.lpart[b];
        *loss = l;
    }
}

// b1, b2 and their complements arrive separately: 1 - b2 formed in FP32 from a rounded
// b2 = 0.999 would carry a 1e-5 relative error.
__global__ __launch_bounds__(256) void mlp_adam_kernel(float *__restrict__ prm, const float *__restrict__ grad,
                                                       float *__restrict__ m, float *__restrict__ v, float lr,
                                                       float b1, float omb1, float b2, float omb2, float eps,
                                                       float c1, float c2)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= kNP) return;
    const float gp = grad[p];
    const float mp = b1 * m[p] + omb1 * gp;
    const float vp = b2 * v[p] + omb2 * gp * gp;
    m[p] = mp;
    v[p] = vp;
    prm[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

}  // namespace

size_t mlp_workspace_bytes(int64_t n)
{
    const int64_t blocks = (n + 255) / 256;
    return act_bytes(n) + ((size_t)kGradChunks * kNP + (size_t)blocks) * sizeof(double);
}

hipError_t launch_mlp_forward(const float *prm, const float *X, int64_t n, float *out, hipStream_t st)
{
    Work w{};
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(mlp_fwd_kernel, dim3(blocks), dim3(256), 0, st, prm, X, (const float *)nullptr, n, out, w);
    return hipGetLastError();
}

hipError_t launch_mlp_loss_grad(const float *prm, const float *X, const float *t, int64_t n, float *grad,
                                double *loss, void *work, hipStream_t st)
{
    Work w = carve(work, n);
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(mlp_fwd_kernel, dim3(blocks), dim3(256), 0, st, prm, X, t, n, (float *)nullptr, w);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned pb = (kNP + 255) / 256;
    hipLaunchKernelGGL(mlp_grad_partial_kernel, dim3(pb, kGradChunks), dim3(256), 0, st, X, n, w);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mlp_grad_final_kernel, dim3(pb), dim3(256), 0, st, w, (int)blocks, grad, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float *prm, const float *grad, float *m, float *v, int64_t step, double lr, double b1,
                           double b2, double eps, hipStream_t st)
{
    const double c1 = 1.0 - std::pow(b1, (double)step);
    const double c2 = 1.0 - std::pow(b2, (double)step);
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((kNP + 255) / 256), dim3(256), 0, st, prm, grad, m, v, (float)lr,
                       (float)b1, (float)(1.0 - b1), (float)b2, (float)(1.0 - b2), (float)eps, (float)c1,
                       (float)c2);
    return hipGetLastError();
}

}  // namespace fbl
