// costmodel.hip -- the learned cost model: an FP32 MLP (24 -> 64 -> 64 -> 1,
// ReLU) that predicts log runtime per sweep of a (stencil, form, launch
// shape) from static features, trained with full-batch Adam on timings this
// library measures.  The paper's own cost model (Sec. Cost Model: constants 0,
// inputs 1, operations 10, memory accesses 100) is one of the features.
//
// Parameter vector (5825 floats): W1 (64 x 24, row = unit), b1 (64),
// W2 (64 x 64), b2 (64), w3 (64), b3 (1).  Activations are kept feature-major
// (unit x row) so every kernel reads rows with consecutive lanes.  Gradient
// sums accumulate in FP64 in a fixed order: training is reproducible.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/stencil.h"
#include "internal.hpp"

namespace stn {

stencil_status fail(stencil_status st, const char *fmt, ...);
stencil_status hip_fail(hipError_t e, const char *what);

namespace {

constexpr int NF = 24, H = 64;
constexpr int OW1 = 0, OB1 = OW1 + H * NF, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H, OB3 = OW3 + H;
constexpr int NP = OB3 + 1;  // 5825

// One thread per row: z1 = W1 x + b1, a1 = relu(z1), z2 = W2 a1 + b2,
// a2 = relu(z2), y = w3 . a2 + b3.  The weights are staged in LDS.
__global__ __launch_bounds__(256) void mlp_fwd(const float *__restrict__ XsT, const float *__restrict__ th, int n,
                                               float *__restrict__ A1T, float *__restrict__ A2T,
                                               float *__restrict__ y) {
    __shared__ float w[NP];
    for (int i = threadIdx.x; i < NP; i += blockDim.x) w[i] = th[i];
    __syncthreads();
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    float x[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) x[f] = XsT[(long long)f * n + r];
    float a1[H];
#pragma unroll
    for (int j = 0; j < H; ++j) {
        float z = w[OB1 + j];
#pragma unroll
        for (int f = 0; f < NF; ++f) z = fmaf(w[OW1 + j * NF + f], x[f], z);
        a1[j] = fmaxf(z, 0.0f);
        if (A1T) A1T[(long long)j * n + r] = a1[j];
    }
    float out = w[OB3];
    for (int j = 0; j < H; ++j) {
        float z = w[OB2 + j];
#pragma unroll
        for (int k = 0; k < H; ++k) z = fmaf(w[OW2 + j * H + k], a1[k], z);
        const float a2 = fmaxf(z, 0.0f);
        if (A2T) A2T[(long long)j * n + r] = a2;
        out = fmaf(w[OW3 + j], a2, out);
    }
    y[r] = out;
}

// One thread per row: dy = 2 (y - t) / n, dZ2 = dy w3 (a2 > 0),
// dZ1 = (W2^T dZ2) (a1 > 0); per-block partial of sum (y - t)^2 (FP64).
__global__ __launch_bounds__(256) void mlp_bwd_rows(const float *__restrict__ th, const float *__restrict__ y,
                                                    const float *__restrict__ t, int n,
                                                    const float *__restrict__ A1T, const float *__restrict__ A2T,
                                                    float *__restrict__ dy, float *__restrict__ dZ2T,
                                                    float *__restrict__ dZ1T, double *__restrict__ loss_part) {
    __shared__ float w[H * H + H];
    __shared__ double red[4];
    for (int i = threadIdx.x; i < H * H; i += blockDim.x) w[i] = th[OW2 + i];
    for (int i = threadIdx.x; i < H; i += blockDim.x) w[H * H + i] = th[OW3 + i];
    __syncthreads();
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    double e2 = 0.0;
    if (r < n) {
        const float e = y[r] - t[r];
        e2 = (double)e * (double)e;
        const float d = 2.0f * e / (float)n;
        dy[r] = d;
        float dz2[H];
#pragma unroll
        for (int j = 0; j < H; ++j) {
            dz2[j] = A2T[(long long)j * n + r] > 0.0f ? d * w[H * H + j] : 0.0f;
            dZ2T[(long long)j * n + r] = dz2[j];
        }
        for (int k = 0; k < H; ++k) {
            float s = 0.0f;
#pragma unroll
            for (int j = 0; j < H; ++j) s = fmaf(w[j * H + k], dz2[j], s);
            dZ1T[(long long)k * n + r] = A1T[(long long)k * n + r] > 0.0f ? s : 0.0f;
        }
    }
    const double s = block_sum_f64(e2, red);
    if (threadIdx.x == 0) loss_part[blockIdx.x] = s;
}

// Block j: gW[j][k] = sum_r dZT[j][r] inT[k][r], gb[j] = sum_r dZT[j][r],
// accumulated in FP64 with a fixed thread stride and block order.
template <int K>
__global__ __launch_bounds__(256) void mlp_grad_layer(const float *__restrict__ dZT, const float *__restrict__ inT,
                                                      int n, float *__restrict__ gW, float *__restrict__ gb) {
    __shared__ double red[4];
    const int j = blockIdx.x;
    double acc[K + 1];
#pragma unroll
    for (int k = 0; k <= K; ++k) acc[k] = 0.0;
    for (int r = threadIdx.x; r < n; r += 256) {
        const double d = dZT[(long long)j * n + r];
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] = fma(d, (double)inT[(long long)k * n + r], acc[k]);
        acc[K] += d;
    }
#pragma unroll
    for (int k = 0; k <= K; ++k) {
        const double s = block_sum_f64(acc[k], red);
        if (threadIdx.x == 0) {
            if (k < K) gW[j * K + k] = (float)s;
            else gb[j] = (float)s;
        }
        __syncthreads();
    }
}

// Sum the loss partials, record the mean loss for this step and advance the
// step counter (read by the following Adam update).
__global__ void mlp_loss_step(const double *__restrict__ part, int nb, int n, float *__restrict__ hist,
                              int *__restrict__ step) {
    __shared__ double red[4];
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) s += part[i];
    s = block_sum_f64(s, red);
    if (threadIdx.x == 0) {
        const int t = *step;
        hist[t] = (float)(s / n);
        *step = t + 1;
    }
}

// Adam (Kingma and Ba 2015), bias-corrected, step = *step (1-based).
__global__ void mlp_adam(float *__restrict__ th, float *__restrict__ m, float *__restrict__ v,
                         const float *__restrict__ g, const int *__restrict__ step, float lr) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NP) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const int t = *step;
    const float mi = b1 * m[i] + (1.0f - b1) * g[i];
    const float vi = b2 * v[i] + (1.0f - b2) * g[i] * g[i];
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / (1.0f - powf(b1, (float)t));
    const float vh = vi / (1.0f - powf(b2, (float)t));
    th[i] -= lr * mh / (sqrtf(vh) + eps);
}

template <typename T>
__global__ void fill_k(T *p, long long n, T v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

struct DevBuf {
    std::vector<void *> ptrs;
    ~DevBuf() {
        for (void *q : ptrs) (void)hipFree(q);
    }
    template <typename T>
    hipError_t get(T **out, size_t count) {
        void *q = nullptr;
        hipError_t e = hipMalloc(&q, count * sizeof(T) + 16);
        if (e == hipSuccess) ptrs.push_back(q);
        *out = (T *)q;
        return e;
    }
};

// Standardize X (n x NF, row-major) with mean/std (std 0 -> 1) into a
// feature-major array.
void standardize_T(const float *X, int n, const float *mean, const float *sd, std::vector<float> &XsT) {
    XsT.resize((size_t)NF * n);
    for (int f = 0; f < NF; ++f)
        for (int r = 0; r < n; ++r) XsT[(size_t)f * n + r] = (X[(size_t)r * NF + f] - mean[f]) / sd[f];
}

}  // namespace

int mlp_param_count() { return NP; }

// Forward pass on the device for n rows of raw features; model = mean (24),
// std (24), parameters (5825).
stencil_status mlp_predict_device(const float *model, const float *X, int n, float *y_out, hipStream_t s) {
    std::vector<float> XsT;
    standardize_T(X, n, model, model + NF, XsT);
    DevBuf b;
    float *dX, *dth, *dy;
    hipError_t e;
    if ((e = b.get(&dX, XsT.size())) != hipSuccess || (e = b.get(&dth, NP)) != hipSuccess ||
        (e = b.get(&dy, (size_t)n)) != hipSuccess)
        return fail(STENCIL_E_NOMEM, "cost model buffers: %s", hipGetErrorString(e));
    if ((e = hipMemcpyAsync(dX, XsT.data(), XsT.size() * 4, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(dth, model + 2 * NF, NP * 4, hipMemcpyHostToDevice, s)) != hipSuccess)
        return hip_fail(e, "cost model upload");
    hipLaunchKernelGGL(mlp_fwd, dim3((n + 255) / 256), dim3(256), 0, s, dX, dth, n, nullptr, nullptr, dy);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "mlp_fwd launch");
    if ((e = hipMemcpyAsync(y_out, dy, (size_t)n * 4, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return hip_fail(e, "cost model download");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return STENCIL_OK;
}

stencil_status mlp_train_device(const float *X, const float *t, int n, const float *init, int epochs, float lr,
                                float *model_out, float *loss_out, int use_graph, hipStream_t s) {
    // standardization statistics of the training rows
    float mean[NF], sd[NF];
    for (int f = 0; f < NF; ++f) {
        double m = 0, q = 0;
        for (int r = 0; r < n; ++r) m += X[(size_t)r * NF + f];
        m /= n;
        for (int r = 0; r < n; ++r) {
            const double d = X[(size_t)r * NF + f] - m;
            q += d * d;
        }
        const double v = std::sqrt(q / n);
        mean[f] = (float)m;
        sd[f] = v > 0 ? (float)v : 1.0f;
    }
    std::vector<float> XsT;
    standardize_T(X, n, mean, sd, XsT);
    DevBuf b;
    float *dX, *dt, *th, *m, *v, *g, *y, *A1T, *A2T, *dy, *dZ2T, *dZ1T, *hist;
    double *lp;
    int *step;
    const int nb = (n + 255) / 256;
    hipError_t e;
    if ((e = b.get(&dX, XsT.size())) != hipSuccess || (e = b.get(&dt, (size_t)n)) != hipSuccess ||
        (e = b.get(&th, NP)) != hipSuccess || (e = b.get(&m, NP)) != hipSuccess || (e = b.get(&v, NP)) != hipSuccess ||
        (e = b.get(&g, NP)) != hipSuccess || (e = b.get(&y, (size_t)n)) != hipSuccess ||
        (e = b.get(&A1T, (size_t)H * n)) != hipSuccess || (e = b.get(&A2T, (size_t)H * n)) != hipSuccess ||
        (e = b.get(&dy, (size_t)n)) != hipSuccess || (e = b.get(&dZ2T, (size_t)H * n)) != hipSuccess ||
        (e = b.get(&dZ1T, (size_t)H * n)) != hipSuccess || (e = b.get(&hist, (size_t)epochs + 1)) != hipSuccess ||
        (e = b.get(&lp, (size_t)nb)) != hipSuccess || (e = b.get(&step, 1)) != hipSuccess)
        return fail(STENCIL_E_NOMEM, "cost model training buffers: %s", hipGetErrorString(e));
    if ((e = hipMemcpyAsync(dX, XsT.data(), XsT.size() * 4, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(dt, t, (size_t)n * 4, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(th, init, NP * 4, hipMemcpyHostToDevice, s)) != hipSuccess)
        return hip_fail(e, "cost model upload");
    hipLaunchKernelGGL(fill_k<float>, dim3(32), dim3(256), 0, s, m, (long long)NP, 0.0f);
    hipLaunchKernelGGL(fill_k<float>, dim3(32), dim3(256), 0, s, v, (long long)NP, 0.0f);
    hipLaunchKernelGGL(fill_k<int>, dim3(1), dim3(64), 0, s, step, 1LL, 0);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "fill launch");

    auto epoch = [&](hipStream_t q) -> hipError_t {
        hipLaunchKernelGGL(mlp_fwd, dim3(nb), dim3(256), 0, q, dX, th, n, A1T, A2T, y);
        hipLaunchKernelGGL(mlp_bwd_rows, dim3(nb), dim3(256), 0, q, th, y, dt, n, A1T, A2T, dy, dZ2T, dZ1T, lp);
        hipLaunchKernelGGL(mlp_loss_step, dim3(1), dim3(256), 0, q, lp, nb, n, hist, step);
        hipLaunchKernelGGL(mlp_grad_layer<NF>, dim3(H), dim3(256), 0, q, dZ1T, dX, n, g + OW1, g + OB1);
        hipLaunchKernelGGL(mlp_grad_layer<H>, dim3(H), dim3(256), 0, q, dZ2T, A1T, n, g + OW2, g + OB2);
        hipLaunchKernelGGL(mlp_grad_layer<H>, dim3(1), dim3(256), 0, q, dy, A2T, n, g + OW3, g + OB3);
        hipLaunchKernelGGL(mlp_adam, dim3((NP + 255) / 256), dim3(256), 0, q, th, m, v, g, step, lr);
        return hipGetLastError();
    };
    if (use_graph && epochs > 0) {
        hipStream_t cap = nullptr;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        if ((e = hipStreamCreate(&cap)) != hipSuccess) return hip_fail(e, "hipStreamCreate");
        if ((e = hipStreamSynchronize(s)) == hipSuccess && (e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal)) == hipSuccess) {
            hipError_t le = epoch(cap);
            e = hipStreamEndCapture(cap, &graph);
            if (le != hipSuccess) e = le;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        for (int ep = 0; ep < epochs && e == hipSuccess; ++ep) e = hipGraphLaunch(exec, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipStreamDestroy(cap);
        if (e != hipSuccess) return hip_fail(e, "training graph");
    } else {
        for (int ep = 0; ep < epochs; ++ep)
            if ((e = epoch(s)) != hipSuccess) return hip_fail(e, "training launch");
    }
    std::memcpy(model_out, mean, sizeof mean);
    std::memcpy(model_out + NF, sd, sizeof sd);
    if ((e = hipMemcpyAsync(model_out + 2 * NF, th, NP * 4, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return hip_fail(e, "parameter download");
    if (loss_out && epochs > 0 &&
        (e = hipMemcpyAsync(loss_out, hist, (size_t)epochs * 4, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return hip_fail(e, "loss download");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return STENCIL_OK;
}

}  // namespace stn
