// Elementwise kernels: the L2 loss gradient, binary32 -> binary16 copy, and
// the fused Adam step
// that updates the binary32 master tables, refreshes their binary16 image
// (the table the forward gathers from) and optionally clears the gradient.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spx_internal.h"

namespace spx {
namespace {

constexpr int kBlock = 256;

inline unsigned blocks_for(int64_t n, int per_thread) {
    int64_t b = (n + (int64_t)kBlock * per_thread - 1) / ((int64_t)kBlock * per_thread);
    const int64_t cap = 1 << 20;
    return (unsigned)(b < cap ? (b > 0 ? b : 1) : cap);
}

__global__ __launch_bounds__(kBlock) void cast_kernel(int64_t n, const float* __restrict__ src,
                                                      _Float16* __restrict__ dst) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) dst[i] = (_Float16)src[i];
}

__global__ __launch_bounds__(kBlock) void adam_kernel(int64_t n, float* __restrict__ param, float* __restrict__ grad,
                                                      float* __restrict__ m, float* __restrict__ v,
                                                      _Float16* __restrict__ param_f16, float lr, float b1, float b2,
                                                      float eps, float inv_bc1, float inv_bc2, int zero_grad) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        const float g = grad[i];
        const float mi = b1 * m[i] + (1.0f - b1) * g;
        const float vi = b2 * v[i] + (1.0f - b2) * g * g;
        const float p = param[i] - lr * (mi * inv_bc1) / (sqrtf(vi * inv_bc2) + eps);
        m[i] = mi;
        v[i] = vi;
        param[i] = p;
        if (param_f16) param_f16[i] = (_Float16)p;
        if (zero_grad) grad[i] = 0.0f;
    }
}

__global__ __launch_bounds__(kBlock) void mse_grad_kernel(int64_t n, const float* y, const float* target,
                                                          float* d_y, float scale) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
        d_y[i] = scale * (y[i] - target[i]);
}

}  // namespace

hipError_t mse_grad(int64_t n, const float* y, const float* target, float* d_y, float scale, hipStream_t s) {
    trace_begin(s, "mse_grad", 12.0 * (double)n);
    mse_grad_kernel<<<blocks_for(n, 4), kBlock, 0, s>>>(n, y, target, d_y, scale);
    trace_end(s);
    return hipGetLastError();
}

hipError_t cast_f32_f16(int64_t n, const float* src, uint16_t* dst, hipStream_t s) {
    trace_begin(s, "cast_f32_f16", 6.0 * (double)n);
    cast_kernel<<<blocks_for(n, 4), kBlock, 0, s>>>(n, src, (_Float16*)dst);
    trace_end(s);
    return hipGetLastError();
}

hipError_t adam_step(int64_t n, float* param, float* grad, float* m, float* v, uint16_t* param_f16, float lr,
                     float beta1, float beta2, float eps, float bc1, float bc2, int zero_grad, hipStream_t s) {
    trace_begin(s, "adam", (double)n * (28.0 + (zero_grad ? 4.0 : 0.0) + (param_f16 ? 2.0 : 0.0)));
    adam_kernel<<<blocks_for(n, 4), kBlock, 0, s>>>(n, param, grad, m, v, (_Float16*)param_f16, lr, beta1, beta2, eps,
                                                    1.0f / bc1, 1.0f / bc2, zero_grad);
    trace_end(s);
    return hipGetLastError();
}

}  // namespace spx
