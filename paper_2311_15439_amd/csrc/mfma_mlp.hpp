// Matrix-core helpers shared by the MLP kernels, the fused field query and
// the adjoint scatter that computes the network's input gradient itself:
// the 16x16x32 MFMAs, the two orders in which a lane's eight k values are
// assigned (see mlp.hip for the layout argument), and the backward of one
// 16-point tile.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

// ---- the backward for one tile of 16 points (with its forward recompute)
//
// Weight fragments, 16 bytes per lane each, built once per workgroup into
// LDS: W1 and W2 in binary16 for the recomputed forward, W3^T, W2^T and W1^T
// in bfloat16 for the backward products.
template <int DIN>
struct BwdFrags {
    static constexpr int KS1 = DIN / 32;                // k steps of layer 1
    static constexpr int F_W1 = 0;                      // [4][KS1] f16, loaded k order
    static constexpr int F_W2 = F_W1 + 4 * KS1;         // [4][2] f16, chained k order
    static constexpr int F_W3T = F_W2 + 8;              // [4] bf16, loaded k order (outputs padded to 32)
    static constexpr int F_W2T = F_W3T + 4;             // [4][2] bf16, chained
    static constexpr int F_W1T = F_W2T + 8;             // [DIN/16][2] bf16, chained
    static constexpr int NFRAG = F_W1T + 2 * (DIN / 16);
    static constexpr int BYTES = NFRAG * 64 * 16;
};

// Fragments f = first, first + step, ... of the NFRAG, written by one wave
// (every lane of it).
template <int DIN>
__device__ __forceinline__ void stage_bwd_frags(uint4* frag, const _Float16* __restrict__ W1,
                                                const _Float16* __restrict__ W2, const _Float16* __restrict__ W3,
                                                int d_out, int first, int step, int lane) {
    using Fr = BwdFrags<DIN>;
    const int r = lane & 15, q = lane >> 4;
    for (int f = first; f < Fr::NFRAG; f += step) {
        uint4 v;
        if (f < Fr::F_W2) {
            const int t = (f - Fr::F_W1) / Fr::KS1, s = (f - Fr::F_W1) % Fr::KS1;
            h8 a = *reinterpret_cast<const h8*>(W1 + (16 * t + r) * DIN + 32 * s + 8 * q);
            v = *reinterpret_cast<uint4*>(&a);
        } else if (f < Fr::F_W3T) {
            const int t = (f - Fr::F_W2) / 2, s = (f - Fr::F_W2) % 2;
            h8 a;
#pragma unroll
            for (int j = 0; j < 8; ++j) a[j] = W2[(16 * t + r) * H + 32 * s + k_chain(q, j)];
            v = *reinterpret_cast<uint4*>(&a);
        } else if (f < Fr::F_W2T) {
            const int t = f - Fr::F_W3T;
            b8 a;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int o = k_load(q, j);
                a[j] = (__bf16)(o < d_out ? (float)W3[o * H + 16 * t + r] : 0.0f);
            }
            v = *reinterpret_cast<uint4*>(&a);
        } else if (f < Fr::F_W1T) {
            const int t = (f - Fr::F_W2T) / 2, s = (f - Fr::F_W2T) % 2;
            b8 a;
#pragma unroll
            for (int j = 0; j < 8; ++j) a[j] = (__bf16)(float)W2[(32 * s + k_chain(q, j)) * H + 16 * t + r];
            v = *reinterpret_cast<uint4*>(&a);
        } else {
            const int t = (f - Fr::F_W1T) / 2, s = (f - Fr::F_W1T) % 2;
            b8 a;
#pragma unroll
            for (int j = 0; j < 8; ++j) a[j] = (__bf16)(float)W1[(32 * s + k_chain(q, j)) * DIN + 16 * t + r];
            v = *reinterpret_cast<uint4*>(&a);
        }
        frag[f * 64 + lane] = v;
    }
}

// One tile: lane (r, q) holds point r.  run() recomputes the forward
// (binary16 products, activations rounded to binary16) and takes the output
// gradient back to the first hidden layer (bfloat16 operands, the ReLU mask
// on the stored activation); dx(t) is then the input gradient's 16-unit
// tile t, units 16t + 4q .. 16t + 4q + 3 of point r, in binary32.
template <int DIN>
struct BwdTile {
    using Fr = BwdFrags<DIN>;
    h8 xb[Fr::KS1];
    h4 h1[4], h2[4];
    b8 dyb;
    f4 da2[4], da1[4];

    __device__ __forceinline__ static h8 fh(const uint4* frag, int f, int lane) {
        uint4 u = frag[f * 64 + lane];
        return *reinterpret_cast<h8*>(&u);
    }
    __device__ __forceinline__ static b8 fb(const uint4* frag, int f, int lane) {
        uint4 u = frag[f * 64 + lane];
        return *reinterpret_cast<b8*>(&u);
    }

    __device__ __forceinline__ void run(const uint4* frag, int lane, const _Float16* __restrict__ x,
                                        const float* __restrict__ d_y, int d_out, int64_t p, bool valid) {
        load(lane, x, d_y, d_out, p, valid);
        compute(frag, lane);
    }

    // the tile's inputs: features and incoming gradient (dyb in loaded k
    // order, outputs 8q..8q+7), zero for points past the end
    __device__ __forceinline__ void load(int lane, const _Float16* __restrict__ x, const float* __restrict__ d_y,
                                         int d_out, int64_t p, bool valid) {
        const int q = lane >> 4;
#pragma unroll
        for (int s = 0; s < Fr::KS1; ++s)
            xb[s] = valid ? *reinterpret_cast<const h8*>(x + p * DIN + 32 * s + 8 * q) : h8{};
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int o = k_load(q, j);
            dyb[j] = (__bf16)((valid && o < d_out) ? d_y[p * d_out + o] : 0.0f);
        }
    }

    __device__ __forceinline__ void compute(const uint4* frag, int lane) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            f4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < Fr::KS1; ++s) c = mma_h(fh(frag, Fr::F_W1 + t * Fr::KS1 + s, lane), xb[s], c);
            h1[t] = relu_h(c);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            f4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < 2; ++s) c = mma_h(fh(frag, Fr::F_W2 + 2 * t + s, lane), cat_h(h1[2 * s], h1[2 * s + 1]), c);
            h2[t] = relu_h(c);
        }
        // dH2 = W3^T dY, masked by the stored activation
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            f4 c = mma_b(fb(frag, Fr::F_W3T + t, lane), dyb, f4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
            for (int i = 0; i < 4; ++i) c[i] = (float)h2[t][i] > 0.0f ? (float)(__bf16)c[i] : 0.0f;
            da2[t] = c;
        }
        // dH1 = W2^T dA2, masked
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            f4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < 2; ++s)
                c = mma_b(fb(frag, Fr::F_W2T + 2 * t + s, lane), cat_b(da2[2 * s], da2[2 * s + 1]), c);
#pragma unroll
            for (int i = 0; i < 4; ++i) c[i] = (float)h1[t][i] > 0.0f ? (float)(__bf16)c[i] : 0.0f;
            da1[t] = c;
        }
    }

    // dX = W1^T dA1, tile t
    __device__ __forceinline__ f4 dx(const uint4* frag, int lane, int t) const {
        f4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 2; ++s)
            c = mma_b(fb(frag, Fr::F_W1T + 2 * t + s, lane), cat_b(da1[2 * s], da1[2 * s + 1]), c);
        return c;
    }
};

}  // namespace spx
