// Cost model of the variant picker: a 13 -> 64 -> 64 -> 1 ReLU perceptron
// predicting log run time, with its forward, loss, backward, Adam and pick
// kernels.  The paper has the user choose every transformation (sec. 1); the
// model picks records for shapes the exhaustive tuner has not timed.
//
// Flat parameter layout: W1[64][13], b1[64], W2[64][64], b2[64], w3[64], b3.
// All sums run in a fixed order, so results are deterministic.
#include <hip/hip_runtime.h>

#include <cmath>

#include "lpx_internal.h"

namespace lpx {
namespace mlpk {

constexpr int NF = LPX_MLP_FEATURES, NH = LPX_MLP_HIDDEN;
constexpr int OW1 = 0, OB1 = OW1 + NH * NF, OW2 = OB1 + NH, OB2 = OW2 + NH * NH,
              OW3 = OB2 + NH, OB3 = OW3 + NH, NP = OB3 + 1;
static_assert(NP == LPX_MLP_PARAMS, "parameter count");
constexpr int ACT = 2 * NH;  // per row: z1[64], z2[64]

__device__ __forceinline__ float relu(float z) { return z > 0.f ? z : 0.f; }

// Loads the parameters into LDS (all threads of the work-group).
__device__ __forceinline__ void load_params(const float* __restrict__ P, float* sp) {
    for (int i = threadIdx.x; i < NP; i += blockDim.x) sp[i] = P[i];
    __syncthreads();
}

// One row: z1 = W1 x + b1, z2 = W2 relu(z1) + b2, y = w3 . relu(z2) + b3.
__device__ __forceinline__ float row_forward(const float* sp, const float (&x)[NF],
                                             float* __restrict__ act_row) {
    float h1[NH];
#pragma unroll
    for (int j = 0; j < NH; ++j) {
        float z = sp[OB1 + j];
#pragma unroll
        for (int f = 0; f < NF; ++f) z += sp[OW1 + j * NF + f] * x[f];
        if (act_row) act_row[j] = z;
        h1[j] = relu(z);
    }
    float y = sp[OB3];
    for (int k = 0; k < NH; ++k) {
        float z = sp[OB2 + k];
#pragma unroll
        for (int j = 0; j < NH; ++j) z += sp[OW2 + k * NH + j] * h1[j];
        if (act_row) act_row[NH + k] = z;
        y += sp[OW3 + k] * relu(z);
    }
    return y;
}

__global__ __launch_bounds__(256) void forward_kernel(const float* __restrict__ P,
                                                      const float* __restrict__ X, int n,
                                                      float* __restrict__ act,
                                                      float* __restrict__ y) {
    __shared__ float sp[NP];
    load_params(P, sp);
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    float x[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) x[f] = X[(int64_t)b * NF + f];
    y[b] = row_forward(sp, x, act ? act + (int64_t)b * ACT : nullptr);
}

// L = mean((y - t)^2), dy = 2 (y - t) / n; one work-group of 256 threads.
__global__ __launch_bounds__(256) void loss_kernel(const float* __restrict__ y,
                                                   const float* __restrict__ t, int n,
                                                   float* __restrict__ dy,
                                                   float* __restrict__ loss) {
    __shared__ float red[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < n; i += 256) {
        const float d = y[i] - t[i];
        if (dy) dy[i] = 2.f * d / (float)n;
        s += d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss) loss[0] = red[0] / (float)n;
}

// Per-row deltas: dz2 = dy w3 (z2 > 0), dz1 = (W2^T dz2)(z1 > 0).
__global__ __launch_bounds__(256) void delta_kernel(const float* __restrict__ P,
                                                    const float* __restrict__ act,
                                                    const float* __restrict__ dy, int n,
                                                    float* __restrict__ work) {
    __shared__ float sp[NP];
    load_params(P, sp);
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    const float* a = act + (int64_t)b * ACT;
    float* w = work + (int64_t)b * ACT;
    float dz2[NH];
#pragma unroll
    for (int k = 0; k < NH; ++k) {
        dz2[k] = a[NH + k] > 0.f ? dy[b] * sp[OW3 + k] : 0.f;
        w[NH + k] = dz2[k];
    }
    for (int j = 0; j < NH; ++j) {
        float s = 0.f;
#pragma unroll
        for (int k = 0; k < NH; ++k) s += sp[OW2 + k * NH + j] * dz2[k];
        w[j] = a[j] > 0.f ? s : 0.f;
    }
}

// One thread per parameter, summing its gradient over the rows in order.
__global__ __launch_bounds__(256) void grad_kernel(const float* __restrict__ X,
                                                   const float* __restrict__ act,
                                                   const float* __restrict__ dy,
                                                   const float* __restrict__ work, int n,
                                                   float* __restrict__ G) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= NP) return;
    float s = 0.f;
    if (q < OB1) {  // W1[j][f] : dz1[j] x[f]
        const int j = q / NF, f = q % NF;
        for (int b = 0; b < n; ++b) s += work[(int64_t)b * ACT + j] * X[(int64_t)b * NF + f];
    } else if (q < OW2) {  // b1[j]
        const int j = q - OB1;
        for (int b = 0; b < n; ++b) s += work[(int64_t)b * ACT + j];
    } else if (q < OB2) {  // W2[k][j] : dz2[k] h1[j]
        const int k = (q - OW2) / NH, j = (q - OW2) % NH;
        for (int b = 0; b < n; ++b)
            s += work[(int64_t)b * ACT + NH + k] * relu(act[(int64_t)b * ACT + j]);
    } else if (q < OW3) {  // b2[k]
        const int k = q - OB2;
        for (int b = 0; b < n; ++b) s += work[(int64_t)b * ACT + NH + k];
    } else if (q < OB3) {  // w3[k] : dy h2[k]
        const int k = q - OW3;
        for (int b = 0; b < n; ++b) s += dy[b] * relu(act[(int64_t)b * ACT + NH + k]);
    } else {  // b3
        for (int b = 0; b < n; ++b) s += dy[b];
    }
    G[q] = s;
}

__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ P,
                                                   const float* __restrict__ G,
                                                   float* __restrict__ M, float* __restrict__ V,
                                                   int n, float lr, float beta1, float beta2,
                                                   float eps, float c1, float c2) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const float g = G[q];
    const float m = beta1 * M[q] + (1.f - beta1) * g;
    const float v = beta2 * V[q] + (1.f - beta2) * g * g;
    M[q] = m;
    V[q] = v;
    P[q] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// Standardise each candidate's features, predict, and take the argmin (ties:
// lowest index).  One work-group; ncand <= 256.
__global__ __launch_bounds__(256) void pick_kernel(const float* __restrict__ P,
                                                   const float* __restrict__ feats, int ncand,
                                                   const float* __restrict__ mean,
                                                   const float* __restrict__ stdv,
                                                   float* __restrict__ pred,
                                                   int* __restrict__ best) {
    __shared__ float sp[NP];
    __shared__ float sy[256];
    __shared__ int si[256];
    load_params(P, sp);
    const int c = threadIdx.x;
    float y = __builtin_huge_valf();
    if (c < ncand) {
        float x[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const float s = stdv[f] == 0.f ? 1.f : stdv[f];
            x[f] = (feats[c * NF + f] - mean[f]) / s;
        }
        y = row_forward(sp, x, nullptr);
        if (pred) pred[c] = y;
    }
    sy[c] = y;
    si[c] = c;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (c < w) {
            const float yo = sy[c + w];
            const int io = si[c + w];
            if (yo < sy[c] || (yo == sy[c] && io < si[c])) {
                sy[c] = yo;
                si[c] = io;
            }
        }
        __syncthreads();
    }
    if (c == 0) best[0] = si[0];
}

}  // namespace mlpk

lpx_status launch_mlp_pick(const float* P, const float* feats, int ncand, const float* mean,
                           const float* stdv, float* pred, int* best, void* stream) {
    hipLaunchKernelGGL(mlpk::pick_kernel, dim3(1), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), P, feats, ncand, mean, stdv, pred,
                       best);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(LPX_ERR_HIP, "pick launch: %s", hipGetErrorString(e));
    return LPX_OK;
}

}  // namespace lpx

using namespace lpx;

namespace {
lpx_status after_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(LPX_ERR_HIP, "%s launch: %s", what, hipGetErrorString(e));
    return LPX_OK;
}
}  // namespace

extern "C" {

lpx_status lpx_mlp_forward(const float* params, const float* X, int32_t n, float* act, float* y,
                           void* stream) {
    clear_error();
    if (n < 0) return set_error(LPX_ERR_INVALID_ARG, "negative n");
    if (n == 0) return LPX_OK;
    if (!params || !X || !y) return set_error(LPX_ERR_INVALID_ARG, "NULL pointer");
    hipLaunchKernelGGL(mlpk::forward_kernel, dim3((n + 255) / 256), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), params, X, n, act, y);
    return after_launch("mlp forward");
}

lpx_status lpx_mlp_loss(const float* y, const float* t, int32_t n, float* dy, float* loss,
                        void* stream) {
    clear_error();
    if (n <= 0) return set_error(LPX_ERR_INVALID_ARG, "need n > 0");
    if (!y || !t) return set_error(LPX_ERR_INVALID_ARG, "NULL pointer");
    hipLaunchKernelGGL(mlpk::loss_kernel, dim3(1), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), y, t, n, dy, loss);
    return after_launch("mlp loss");
}

lpx_status lpx_mlp_backward(const float* params, const float* X, const float* act,
                            const float* dy, int32_t n, float* work, float* grads, void* stream) {
    clear_error();
    if (n < 0) return set_error(LPX_ERR_INVALID_ARG, "negative n");
    if (!params || !grads || (n > 0 && (!X || !act || !dy || !work)))
        return set_error(LPX_ERR_INVALID_ARG, "NULL pointer");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (n > 0) {
        hipLaunchKernelGGL(mlpk::delta_kernel, dim3((n + 255) / 256), dim3(256), 0, st, params,
                           act, dy, n, work);
        lpx_status s = after_launch("mlp delta");
        if (s != LPX_OK) return s;
    }
    hipLaunchKernelGGL(mlpk::grad_kernel, dim3((mlpk::NP + 255) / 256), dim3(256), 0, st, X, act,
                       dy, work, n, grads);
    return after_launch("mlp gradient");
}

lpx_status lpx_adam_step(float* params, const float* grads, float* m, float* v, int32_t n,
                         int32_t step, float lr, float beta1, float beta2, float eps,
                         void* stream) {
    clear_error();
    if (n < 0 || step < 1) return set_error(LPX_ERR_INVALID_ARG, "need n >= 0 and step >= 1");
    if (n == 0) return LPX_OK;
    if (!params || !grads || !m || !v) return set_error(LPX_ERR_INVALID_ARG, "NULL pointer");
    if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f))
        return set_error(LPX_ERR_INVALID_ARG, "need 0 <= beta < 1 and eps > 0");
    const float c1 = 1.f - (float)std::pow((double)beta1, (double)step);
    const float c2 = 1.f - (float)std::pow((double)beta2, (double)step);
    hipLaunchKernelGGL(mlpk::adam_kernel, dim3((n + 255) / 256), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), params, grads, m, v, n, lr, beta1,
                       beta2, eps, c1, c2);
    return after_launch("adam");
}

lpx_status lpx_mlp_pick(const float* params, const float* feats, int32_t ncand,
                        const float* mean, const float* stdv, float* pred, int32_t* best,
                        void* stream) {
    clear_error();
    if (ncand <= 0 || ncand > 256) return set_error(LPX_ERR_INVALID_ARG, "need 1..256 candidates");
    if (!params || !feats || !mean || !stdv || !best)
        return set_error(LPX_ERR_INVALID_ARG, "NULL pointer");
    return launch_mlp_pick(params, feats, ncand, mean, stdv, pred, best, stream);
}

}  // extern "C"
