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
typedef __bf16 b4 __attribute__((ext_vector_type(4)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef uint32_t u2 __attribute__((ext_vector_type(2)));
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

// ReLU then round to binary16 (the stored activation).  Rounded first and
// clamped at zero in binary16, two values per instruction: rounding is
// monotonic and keeps the sign, so the values are those of rounding the
// clamped binary32 (a zero may differ in sign, which no product or mask
// below can see).
static __device__ __forceinline__ h4 relu_h(f4 c) {
    const h4 h = {(_Float16)c.x, (_Float16)c.y, (_Float16)c.z, (_Float16)c.w};
    return __builtin_elementwise_max(h, h4{0, 0, 0, 0});
}
static __device__ __forceinline__ h8 cat_h(h4 a, h4 b) { return __builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7); }
static __device__ __forceinline__ b8 cat_b(b4 a, b4 b) { return __builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7); }

// A hidden unit's gradient as the matrix cores take it: rounded to bfloat16,
// and zero where the stored activation h is not positive.  h comes from
// relu_h, so it is positive exactly where its magnitude bits are not all
// zero; the test runs on the bits, two halves per word (a half's magnitude
// plus 0x7fff sets the half's top bit exactly when the magnitude is not
// zero, and never carries out of the half).
static __device__ __forceinline__ b4 mask_bf(f4 c, h4 h) {
    const b4 r = {(__bf16)c.x, (__bf16)c.y, (__bf16)c.z, (__bf16)c.w};
    u2 rb = __builtin_bit_cast(u2, r);
    const u2 hb = __builtin_bit_cast(u2, h);
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        const uint32_t m = ((hb[w] & 0x7fff7fffu) + 0x7fff7fffu) & 0x80008000u;
        rb[w] &= (m >> 15) * 0xffffu;
    }
    return __builtin_bit_cast(b4, rb);
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

// Copies W1, W2 and W3 (binary16, 16-byte aligned rows) into LDS at raw,
// 16 bytes per access, every thread of the workgroup (tid of NTHREADS) at
// once.  Every thread loads and stores the same number of chunks, with no
// condition (a chunk index past the weights reloads chunk 0 into the spare
// room at the end of raw), so that all of its loads are issued before it
// waits for any: the copy costs one memory latency.  The fragments are then
// built from LDS (stage_bwd_frags with the copies as W1, W2, W3); built from
// global memory, their element loads waited for each other.  raw needs
// raw_copy_bytes<DIN, NTHREADS>() bytes; the caller synchronises the
// workgroup before reading it.
template <int DIN, int NTHREADS>
struct RawCopy {
    static constexpr int C1 = H * DIN / 8, C2 = H * H / 8;  // 16-byte chunks of W1 and W2
    static constexpr int CMAX = C1 + C2 + 16 * H / 8;       // with the widest W3 (16 outputs)
    static constexpr int K = (CMAX + NTHREADS - 1) / NTHREADS;
    static constexpr int BYTES = K * NTHREADS * 16;
};
template <int DIN, int NTHREADS>
__host__ __device__ constexpr int raw_copy_bytes() { return RawCopy<DIN, NTHREADS>::BYTES; }

template <int DIN, int NTHREADS>
__device__ __forceinline__ void copy_weights_lds(uint4* raw, const _Float16* __restrict__ W1,
                                                 const _Float16* __restrict__ W2, const _Float16* __restrict__ W3,
                                                 int d_out, int tid) {
    using Rc = RawCopy<DIN, NTHREADS>;
    const int n = Rc::C1 + Rc::C2 + d_out * H / 8;
    uint4 v[Rc::K];
#pragma unroll
    for (int k = 0; k < Rc::K; ++k) {
        int i = tid + k * NTHREADS;
        i = i < n ? i : 0;
        const uint4* src = i < Rc::C1 ? reinterpret_cast<const uint4*>(W1) + i
                         : i < Rc::C1 + Rc::C2 ? reinterpret_cast<const uint4*>(W2) + (i - Rc::C1)
                                               : reinterpret_cast<const uint4*>(W3) + (i - Rc::C1 - Rc::C2);
        v[k] = *src;
    }
#pragma unroll
    for (int k = 0; k < Rc::K; ++k) raw[tid + k * NTHREADS] = v[k];
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
    b4 da2[4], da1[4];  // masked hidden gradients, bfloat16

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
    // order, outputs 8q..8q+7), zero for points past the end.  The eight
    // gradient loads of a lane are unconditional (an output past d_out reads
    // the row's last one and is then replaced by zero): loads under
    // per-element conditions each waited for their data before the next
    // was issued.
    __device__ __forceinline__ void load(int lane, const _Float16* __restrict__ x, const float* __restrict__ d_y,
                                         int d_out, int64_t p, bool valid) {
        const int q = lane >> 4;
#pragma unroll
        for (int s = 0; s < Fr::KS1; ++s)
            xb[s] = valid ? *reinterpret_cast<const h8*>(x + p * DIN + 32 * s + 8 * q) : h8{};
        float g[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) g[j] = 0.0f;
        if (valid && 8 * q < d_out) {
            const float* row = d_y + p * d_out;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int o = k_load(q, j);
                g[j] = row[o < d_out ? o : d_out - 1];
            }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) dyb[j] = (__bf16)(k_load(q, j) < d_out ? g[j] : 0.0f);
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
            da2[t] = mask_bf(c, h2[t]);
        }
        // dH1 = W2^T dA2, masked
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            f4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < 2; ++s)
                c = mma_b(fb(frag, Fr::F_W2T + 2 * t + s, lane), cat_b(da2[2 * s], da2[2 * s + 1]), c);
            da1[t] = mask_bf(c, h1[t]);
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
