// Matrix-core helpers shared by the MLP kernels and the fused field query:
// the 16x16x32 MFMAs, and the two orders in which a lane's eight k values are
// assigned (see mlp.hip for the layout argument).
#pragma once

#include <hip/hip_runtime.h>

namespace spx {

typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int H = 64;  // hidden width of the network

static __device__ __forceinline__ f4 mma_h(h8 a, h8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}
static __device__ __forceinline__ f4 mma_b(b8 a, b8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

static __device__ __forceinline__ int k_chain(int q, int j) { return j < 4 ? 4 * q + j : 16 + 4 * q + (j - 4); }
static __device__ __forceinline__ int k_load(int q, int j) { return 8 * q + j; }

// ReLU then round to binary16 (the stored activation).
static __device__ __forceinline__ h4 relu_h(f4 c) {
    return h4{(_Float16)fmaxf(c.x, 0.0f), (_Float16)fmaxf(c.y, 0.0f), (_Float16)fmaxf(c.z, 0.0f),
              (_Float16)fmaxf(c.w, 0.0f)};
}
static __device__ __forceinline__ h8 cat_h(h4 a, h4 b) { return h8{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w}; }
static __device__ __forceinline__ b8 cat_b(f4 a, f4 b) {
    return b8{(__bf16)a.x, (__bf16)a.y, (__bf16)a.z, (__bf16)a.w,
              (__bf16)b.x, (__bf16)b.y, (__bf16)b.z, (__bf16)b.w};
}

}  // namespace spx
