// Internal interface between the C ABI layer (api.hip) and the kernel
// translation units.  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spx {

struct SimplexTag { static constexpr bool simplex = true; };
struct GridTag { static constexpr bool simplex = false; };

// Per-call level parameters, passed to the kernels by value.
struct LevelArgs {
    float sigma[32];  // binary32 multiplier of level l
    float Fn;         // skew factor F_n in binary32
    uint32_t mask;    // T - 1
    int32_t L;        // number of levels
};

enum class EncodeOp { Forward, Adjoint, Debug };

struct EncodeCall {
    EncodeOp op;
    int D, F;
    bool table_f16, out_f16, dout_f16;
    int64_t N;
    const float* pts;
    const void* tables;
    void* out;
    const void* d_out;
    float* d_tables;
    uint32_t* idx;
    float* w;
    LevelArgs lv;
    hipStream_t stream;
};

hipError_t encode_simplex(const EncodeCall& c);
hipError_t encode_grid(const EncodeCall& c);

// MLP and elementwise kernels.
struct MlpCall {
    int d_in, hidden, d_out;
    int64_t N;
    const uint16_t* x;
    const uint16_t *W1, *W2, *W3;
    float* y;
    const float* d_y;
    float* d_x;
    float *dW1, *dW2, *dW3;
    void* workspace;
    hipStream_t stream;
};
size_t mlp_bwd_workspace_bytes(int d_in, int hidden, int d_out, int64_t N);
int mlp_bwd_lds_bytes(int d_in);
hipError_t mlp_fwd(const MlpCall& c);
hipError_t mlp_bwd(const MlpCall& c);

hipError_t mse_grad(int64_t n, const float* y, const float* target, float* d_y, float scale, hipStream_t s);
hipError_t cast_f32_f16(int64_t n, const float* src, uint16_t* dst, hipStream_t s);
hipError_t adam_step(int64_t n, float* param, float* grad, float* m, float* v, uint16_t* param_f16, float lr,
                     float beta1, float beta2, float eps, float bc1, float bc2, int zero_grad, hipStream_t s);

}  // namespace spx
