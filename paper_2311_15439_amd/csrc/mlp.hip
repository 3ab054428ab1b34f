// Tiny fully connected network on the matrix cores (Sec. 5 step (e)):
// d_in -> 64 -> 64 -> d_out, ReLU on the hidden layers, linear output.
//
// Layout strategy.  Every product is computed transposed, Out^T = W In^T,
// with the 16x16x32 MFMA: the 16 columns are 16 points, the 16 rows are
// output units.  An MFMA result leaves lane (r, q) = (lane % 16, lane / 16)
// holding point r and units 4q..4q+3 of a 16-unit tile.  Because A and B
// of one MFMA share the same assignment of k to (lane group, item), two
// such 16-unit tiles can feed the next layer's 32-deep k step directly, as
// long as the weight fragments are loaded with the matching k order:
//   chained k order:  item j of group q  ->  unit j<4 ? 4q+j : 16+4q+(j-4)
//   loaded k order:   item j of group q  ->  unit 8q+j   (operands read
//                                            from memory or LDS)
// So activations never leave registers between layers.  The weight
// gradients contract over points, which live one per lane; those operands
// are transposed through LDS.
//
// Precision: forward products in binary16 with binary32 accumulation,
// hidden activations rounded to binary16; backward products in bfloat16
// with binary32 accumulation; the ReLU mask is taken on the stored binary16
// activation.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "mfma_mlp.hpp"
#include "spx_internal.h"

namespace spx {
namespace {

// ------------------------------------------------------------------ forward

template <int DIN>
__global__ __launch_bounds__(256) void mlp_fwd_kernel(int64_t N, const _Float16* __restrict__ x,
                                                      const _Float16* __restrict__ W1,
                                                      const _Float16* __restrict__ W2,
                                                      const _Float16* __restrict__ W3, int d_out,
                                                      float* __restrict__ y) {
    constexpr int KS1 = DIN / 32;  // k steps of layer 1
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    h8 w1[4][KS1], w2[4][2], w3[2];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int s = 0; s < KS1; ++s)
            w1[t][s] = *reinterpret_cast<const h8*>(W1 + (16 * t + r) * DIN + 32 * s + 8 * q);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int j = 0; j < 8; ++j) w2[t][s][j] = W2[(16 * t + r) * H + 32 * s + k_chain(q, j)];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int j = 0; j < 8; ++j) w3[s][j] = r < d_out ? W3[r * H + 32 * s + k_chain(q, j)] : (_Float16)0.0f;

    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    const int64_t ntiles = (N + 15) / 16;
    for (int64_t tile = wave; tile < ntiles; tile += nwaves) {
        const int64_t p = tile * 16 + r;
        const bool valid = p < N;
        h8 xb[KS1];
#pragma unroll
        for (int s = 0; s < KS1; ++s)
            xb[s] = valid ? *reinterpret_cast<const h8*>(x + p * DIN + 32 * s + 8 * q) : h8{};
        h4 h1[4], h2[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            f4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < KS1; ++s) c = mma_h(w1[t][s], xb[s], c);
            h1[t] = relu_h(c);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            f4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < 2; ++s) c = mma_h(w2[t][s], cat_h(h1[2 * s], h1[2 * s + 1]), c);
            h2[t] = relu_h(c);
        }
        f4 o = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 2; ++s) o = mma_h(w3[s], cat_h(h2[2 * s], h2[2 * s + 1]), o);
        if (valid) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (4 * q + i < d_out) y[p * d_out + 4 * q + i] = o[i];
        }
    }
}

// ----------------------------------------------------------------- backward

__device__ __forceinline__ short bf_bits(float v) { return __builtin_bit_cast(short, (__bf16)v); }

constexpr int kBwdWaves = 4;
constexpr int kPts = 16;  // points per wave per iteration
constexpr int kMaxBwdGroups = 512;

template <int DIN>
struct BwdLayout {
    // weight fragments (BwdFrags), then a per-wave transpose area: one row of
    // 16 points (bf16) per unit
    static constexpr int FRAG_BYTES = BwdFrags<DIN>::BYTES;
    static constexpr int R_DY = 0, R_H2 = 16, R_H1 = 80, R_DA2 = 144, R_DA1 = 208, R_X = 272;
    static constexpr int ROWS = R_X + DIN;
    static constexpr int WAVE_BYTES = ROWS * kPts * 2;
    static constexpr int PARTIAL = H * DIN + H * H + 16 * H;  // floats per workgroup
    static constexpr int LDS_BYTES = FRAG_BYTES + kBwdWaves * WAVE_BYTES;
    // weight-gradient tiles (16x16 each): dW3 4, dW2 16, dW1 4 * DIN/16;
    // wave w owns tiles w, w + 4, w + 8, ...
    static constexpr int TILES = 4 + 16 + 4 * (DIN / 16);
    static constexpr int TPW = TILES / kBwdWaves;
};

// d_x (when not NULL) receives units [0, dx_cols) of each point's input
// gradient, in rows of dx_stride floats (dx_cols and dx_stride multiples of
// 4; the full gradient is dx_cols = dx_stride = DIN).
template <int DIN>
__global__ __launch_bounds__(256) void mlp_bwd_kernel(int64_t N, const _Float16* __restrict__ x,
                                                      const _Float16* __restrict__ W1,
                                                      const _Float16* __restrict__ W2,
                                                      const _Float16* __restrict__ W3, int d_out,
                                                      const float* __restrict__ d_y, float* __restrict__ d_x,
                                                      int dx_cols, int dx_stride, float* __restrict__ partial) {
    using Lay = BwdLayout<DIN>;
    constexpr int KS1 = DIN / 32;
    constexpr int TIN = DIN / 16;
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    uint4* frag = reinterpret_cast<uint4*>(lds);
    const int tid = threadIdx.x;
    const int lane = tid & 63, r = lane & 15, q = lane >> 4, wv = tid >> 6;

    short* const S0 = reinterpret_cast<short*>(lds + Lay::FRAG_BYTES);
    // ---- stage the weight fragments (each wave builds a quarter of them)
    // from a copy of the weights in the transpose area, free until the loop
    static_assert(raw_copy_bytes<DIN, 64 * kBwdWaves>() <= kBwdWaves * Lay::WAVE_BYTES, "weights exceed the transpose area");
    {
        uint4* raw = reinterpret_cast<uint4*>(S0);
        copy_weights_lds<DIN, 64 * kBwdWaves>(raw, W1, W2, W3, d_out, tid);
        __syncthreads();
        const _Float16* w = reinterpret_cast<const _Float16*>(raw);
        stage_bwd_frags<DIN>(frag, w, w + H * DIN, w + H * DIN + H * H, d_out, wv, kBwdWaves, lane);
        __syncthreads();
    }
    short* S = S0 + wv * (Lay::WAVE_BYTES / 2);
    static_assert(Lay::TILES % kBwdWaves == 0, "tiles must split evenly over the waves");

    f4 acc[Lay::TPW];
#pragma unroll
    for (int u = 0; u < Lay::TPW; ++u) acc[u] = f4{0.f, 0.f, 0.f, 0.f};

    const int64_t per_iter = (int64_t)kBwdWaves * kPts;
    const int64_t iters = (N + per_iter - 1) / per_iter;
    // Each iteration's inputs are loaded during the previous iteration's
    // products (with two waves per SIMD the loads' latency is otherwise the
    // loop's time).  A point past the end loads zeros.
    BwdTile<DIN> tl;
    {
        const int64_t p = (int64_t)blockIdx.x * per_iter + wv * kPts + r;
        tl.load(lane, x, d_y, d_out, p, p < N);
    }
    for (int64_t it = blockIdx.x; it < iters; it += gridDim.x) {
        const int64_t base = it * per_iter + wv * kPts;
        const int64_t p = base + r;
        const bool valid = p < N;
        BwdTile<DIN> nx;
        {
            const int64_t pn = p + (int64_t)gridDim.x * per_iter;
            nx.load(lane, x, d_y, d_out, pn, pn < N);
        }
        tl.compute(frag, lane);
        if (d_x) {
#pragma unroll
            for (int t = 0; t < TIN; ++t) {
                if (16 * t >= dx_cols) break;  // uniform
                const f4 c = tl.dx(frag, lane, t);
                if (valid && 16 * t + 4 * q < dx_cols) *reinterpret_cast<f4*>(d_x + p * dx_stride + 16 * t + 4 * q) = c;
            }
        }
        // transpose the weight-gradient operands through LDS: row = unit, column = point
        if (q < 2) {
#pragma unroll
            for (int j = 0; j < 8; ++j)
                S[(Lay::R_DY + k_load(q, j)) * kPts + r] = __builtin_bit_cast(short, (__bf16)tl.dyb[j]);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            // the hidden gradients are bfloat16 pairs already: their halves
            // are written as they are (taken from the words with integer
            // shifts; element reads of the bfloat16 vector through a bit
            // cast were compiled to the low half for every element)
            const u2 g2 = __builtin_bit_cast(u2, tl.da2[t]), g1 = __builtin_bit_cast(u2, tl.da1[t]);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int u = 16 * t + 4 * q + i;
                const int sh = 16 * (i & 1);
                S[(Lay::R_H2 + u) * kPts + r] = bf_bits((float)tl.h2[t][i]);
                S[(Lay::R_H1 + u) * kPts + r] = bf_bits((float)tl.h1[t][i]);
                S[(Lay::R_DA2 + u) * kPts + r] = (short)(g2[i >> 1] >> sh);
                S[(Lay::R_DA1 + u) * kPts + r] = (short)(g1[i >> 1] >> sh);
            }
        }
#pragma unroll
        for (int s = 0; s < KS1; ++s)
#pragma unroll
            for (int j = 0; j < 8; ++j)
                S[(Lay::R_X + 32 * s + k_load(q, j)) * kPts + r] = bf_bits((float)tl.xb[s][j]);
        __syncthreads();
        // Weight gradients over the iteration's 64 points: this wave's tiles,
        // k = 32 points per MFMA (lane group q reads 8 points of region
        // 2c + q / 2; A and B use the same assignment).
#pragma unroll
        for (int u = 0; u < Lay::TPW; ++u) {
            const int tile = wv + kBwdWaves * u;
            int ra, rb;
            if (tile < 4) {
                ra = Lay::R_DY + r;
                rb = Lay::R_H2 + 16 * tile + r;
            } else if (tile < 20) {
                ra = Lay::R_DA2 + 16 * ((tile - 4) / 4) + r;
                rb = Lay::R_H1 + 16 * ((tile - 4) % 4) + r;
            } else {
                ra = Lay::R_DA1 + 16 * ((tile - 20) / TIN) + r;
                rb = Lay::R_X + 16 * ((tile - 20) % TIN) + r;
            }
#pragma unroll
            for (int c = 0; c < kBwdWaves / 2; ++c) {
                const short* reg = S0 + (2 * c + (q >> 1)) * (Lay::WAVE_BYTES / 2);
                const b8 a = *reinterpret_cast<const b8*>(reg + ra * kPts + 8 * (q & 1));
                const b8 bb = *reinterpret_cast<const b8*>(reg + rb * kPts + 8 * (q & 1));
                acc[u] = mma_b(a, bb, acc[u]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < KS1; ++s) tl.xb[s] = nx.xb[s];
        tl.dyb = nx.dyb;
    }

    // ---- each wave writes its own tiles of this group's partial
    float* out = partial + (size_t)blockIdx.x * Lay::PARTIAL;
#pragma unroll
    for (int u = 0; u < Lay::TPW; ++u) {
        const int tile = wv + kBwdWaves * u;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = 4 * q + i;  // D layout: lane holds column r, rows 4q..4q+3
            size_t idx;
            if (tile < 4) {
                idx = (size_t)H * DIN + H * H + row * H + 16 * tile + r;  // dW3[out][hidden]
            } else if (tile < 20) {
                const int t = (tile - 4) / 4, s = (tile - 4) % 4;
                idx = (size_t)H * DIN + (16 * t + row) * H + 16 * s + r;  // dW2[out][in]
            } else {
                const int t = (tile - 20) / TIN, s = (tile - 20) % TIN;
                idx = (size_t)(16 * t + row) * DIN + 16 * s + r;  // dW1[hidden][in]
            }
            out[idx] = acc[u][i];
        }
    }
}

// Sum of the per-workgroup weight-gradient partials.  A block owns 32
// outputs; 32 thread rows each add a contiguous segment of the workgroups'
// partials in order, and the segment sums are then added in order, so the
// result does not depend on scheduling.
constexpr int kRedOut = 32, kRedSeg = 32;
template <int DIN>
__global__ __launch_bounds__(kRedOut * kRedSeg) void mlp_reduce_kernel(const float* __restrict__ partial, int groups,
                                                                      int d_out, float* __restrict__ dW1,
                                                                      float* __restrict__ dW2,
                                                                      float* __restrict__ dW3) {
    constexpr int PARTIAL = BwdLayout<DIN>::PARTIAL;
    __shared__ float part[kRedSeg][kRedOut];
    const int o = threadIdx.x % kRedOut, sg = threadIdx.x / kRedOut;
    const int i = blockIdx.x * kRedOut + o;
    const int per = (groups + kRedSeg - 1) / kRedSeg;
    const int g0 = sg * per < groups ? sg * per : groups;
    const int g1 = g0 + per < groups ? g0 + per : groups;
    // the segment's partials loaded all at once (unconditional loads: a
    // slot past the segment reads entry 0 and is not added), then added in
    // workgroup order
    constexpr int kPer = kMaxBwdGroups / kRedSeg;
    float v[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const bool in = i < PARTIAL && g0 + k < g1;
        v[k] = partial[in ? (size_t)(g0 + k) * PARTIAL + i : 0];
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kPer; ++k)
        if (i < PARTIAL && g0 + k < g1) s += v[k];
    part[sg][o] = s;
    __syncthreads();
    if (sg != 0 || i >= PARTIAL) return;
    s = part[0][o];
    for (int k = 1; k < kRedSeg; ++k) s += part[k][o];
    if (i < H * DIN) {
        dW1[i] = s;
    } else if (i < H * DIN + H * H) {
        dW2[i - H * DIN] = s;
    } else {
        const int k = i - H * DIN - H * H;
        if (k / H < d_out) dW3[k] = s;
    }
}

inline int bwd_groups(int64_t N) {
    const int64_t per = (int64_t)kBwdWaves * kPts;
    int64_t g = (N + per - 1) / per;
    return (int)(g < kMaxBwdGroups ? (g > 0 ? g : 1) : kMaxBwdGroups);
}

template <int DIN>
hipError_t fwd_impl(const MlpCall& c) {
    int64_t tiles = (c.N + 15) / 16;
    int64_t blocks = (tiles + 3) / 4;
    const int64_t cap = 4096;
    unsigned g = (unsigned)(blocks < cap ? (blocks > 0 ? blocks : 1) : cap);
    trace_begin(c.stream, "mlp_fwd", (double)c.N * (2.0 * DIN + 4.0 * c.d_out) + 2.0 * (H * DIN + H * H + H * c.d_out));
    mlp_fwd_kernel<DIN><<<g, 256, 0, c.stream>>>(c.N, (const _Float16*)c.x, (const _Float16*)c.W1,
                                                 (const _Float16*)c.W2, (const _Float16*)c.W3, c.d_out, c.y);
    trace_end(c.stream);
    return hipGetLastError();
}

template <int DIN>
hipError_t bwd_impl(const MlpCall& c) {
    using Lay = BwdLayout<DIN>;
    const int g = bwd_groups(c.N);
    float* part = (float*)c.workspace;
    trace_begin(c.stream, "mlp_bwd",
                (double)c.N * (2.0 * DIN + 4.0 * c.d_out + (c.d_x ? 4.0 * (c.dx_cols > 0 ? c.dx_cols : DIN) : 0.0)) + (double)g * Lay::PARTIAL * 4.0);
    const int dx_cols = c.dx_cols > 0 ? c.dx_cols : DIN, dx_stride = c.dx_stride > 0 ? c.dx_stride : DIN;
    mlp_bwd_kernel<DIN><<<g, 256, Lay::LDS_BYTES, c.stream>>>(c.N, (const _Float16*)c.x, (const _Float16*)c.W1,
                                                              (const _Float16*)c.W2, (const _Float16*)c.W3,
                                                              c.d_out, c.d_y, c.d_x, dx_cols, dx_stride, part);
    trace_end(c.stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    trace_begin(c.stream, "mlp_reduce", ((double)g + 1.0) * Lay::PARTIAL * 4.0);
    mlp_reduce_kernel<DIN><<<(Lay::PARTIAL + kRedOut - 1) / kRedOut, kRedOut * kRedSeg, 0, c.stream>>>(
        part, g, c.d_out, c.dW1, c.dW2, c.dW3);
    trace_end(c.stream);
    return hipGetLastError();
}

}  // namespace

// Scratch of the allocation-free backward (spx_mlp_bwd_noalloc): room for the
// per-workgroup weight-gradient partials of the most workgroups the backward
// ever launches (kMaxBwdGroups), 14 MiB per device, held until the process
// ends.  In host code this name is only a stand-in for the symbol: the
// device address comes from hipGetSymbolAddress, once per device.
constexpr size_t kScratchFloats = (size_t)kMaxBwdGroups * BwdLayout<32>::PARTIAL;
static __device__ __align__(256) float scratch[kScratchFloats];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64];

hipError_t mlp_bwd_scratch(void** ptr, size_t* bytes) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    *bytes = kScratchFloats * sizeof(float);
    return hipSuccess;
}

int mlp_bwd_lds_bytes(int d_in) { return d_in == 32 ? BwdLayout<32>::LDS_BYTES : 0; }

size_t mlp_bwd_workspace_bytes(int d_in, int, int, int64_t N) {
    const size_t partial = (size_t)(H * d_in + H * H + 16 * H) * sizeof(float);
    return partial * (size_t)bwd_groups(N);
}

hipError_t mlp_fwd(const MlpCall& c) {
    switch (c.d_in) {
        case 32: return fwd_impl<32>(c);
        default: return hipErrorInvalidValue;
    }
}

hipError_t mlp_bwd(const MlpCall& c) {
    switch (c.d_in) {
        case 32: return bwd_impl<32>(c);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace spx
