// Fused multi-field query for serving: encoding forward and network
// forward in one kernel, over a batch of segments that may each belong to a
// different resident field.
//
// A wave handles 16 points.  Lane (r, q) = (lane % 16, lane / 16) encodes
// levels 4q..4q+3 of point r; with two features per level those are the
// eight binary16 values 8q..8q+7 of the point's feature vector, which is
// exactly the lane's B operand of the network's first 16x16x32 MFMA in the
// "loaded" k order.  The encoded features therefore never leave registers,
// and the result is bit-identical to running the encoding forward (binary16
// output) and the network forward as separate kernels.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "encode_kernels.hpp"
#include "lookup.hpp"
#include "mfma_mlp.hpp"
#include "spx.h"
#include "spx_internal.h"

namespace spx {
namespace {

constexpr int kTilesPerWave = 8;  // contiguous 16-point tiles per wave visit

struct Weights {
    h8 w1[4], w2[4][2], w3[2];
};

__device__ __forceinline__ void load_weights(const spx_field& f, int r, int q, Weights& W) {
    const _Float16* W1 = (const _Float16*)f.W1;
    const _Float16* W2 = (const _Float16*)f.W2;
    const _Float16* W3 = (const _Float16*)f.W3;
#pragma unroll
    for (int t = 0; t < 4; ++t) W.w1[t] = *reinterpret_cast<const h8*>(W1 + (16 * t + r) * 32 + 8 * q);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int j = 0; j < 8; ++j) W.w2[t][s][j] = W2[(16 * t + r) * H + 32 * s + k_chain(q, j)];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int j = 0; j < 8; ++j) W.w3[s][j] = r < f.d_out ? W3[r * H + 32 * s + k_chain(q, j)] : (_Float16)0.0f;
}

// Features 8q..8q+7 (levels 4q..4q+3, two features each) of one point.
template <class Tag, int D>
__device__ __forceinline__ h8 encode_quarter(const spx_field& f, const float* __restrict__ p, bool valid, int q) {
    float x[D], y[D];
#pragma unroll
    for (int i = 0; i < D; ++i) x[i] = valid ? p[i] : 0.0f;
    if constexpr (Tag::simplex) {
        skew<D>(x, f.Fn, y);
    } else {
#pragma unroll
        for (int i = 0; i < D; ++i) y[i] = x[i];
    }
    const f16* tables = (const f16*)f.tables;
    const size_t level_elems = (size_t)(f.mask + 1u) * 2;
    h8 out;
#pragma unroll
    for (int lv = 0; lv < 4; ++lv) {
        const int l = 4 * q + lv;
        const f16* __restrict__ tab = tables + (size_t)l * level_elems;
        float acc[2] = {0.0f, 0.0f};
        visit_level(Tag{}, y, f.sigma[l], SlotRule{f.mask, 0}, [&](const auto& h, const auto& w, int) {
            constexpr int K = sizeof(w) / sizeof(float);
            float v[K][2];
#pragma unroll
            for (int k = 0; k < K; ++k) RowIO<f16, 2>::load(tab + (size_t)h[k] * 2, v[k]);
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[j] = __builtin_fmaf(w[k], v[k][j], acc[j]);
        });
        out[2 * lv] = (_Float16)acc[0];
        out[2 * lv + 1] = (_Float16)acc[1];
    }
    return out;
}

// One tile of 16 points: encode (lane (r, q) holds features 8q..8q+7 of
// point r), optionally store the binary16 features, run the network, store
// the outputs.
template <class Tag, int D>
__device__ __forceinline__ void fwd_tile(const spx_field& f, const Weights& W, const float* __restrict__ pts,
                                         int64_t count, int64_t p, int r, int q, float* __restrict__ out,
                                         _Float16* __restrict__ feats) {
    const bool valid = p >= 0 && p < count;
    const h8 xb = encode_quarter<Tag, D>(f, pts + (valid ? p : 0) * D, valid, q);
    if (feats && valid) *reinterpret_cast<h8*>(feats + p * 32 + 8 * q) = xb;
    h4 h1[4], h2[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) h1[t] = relu_h(mma_h(W.w1[t], xb, f4{0.f, 0.f, 0.f, 0.f}));
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        f4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 2; ++s) c = mma_h(W.w2[t][s], cat_h(h1[2 * s], h1[2 * s + 1]), c);
        h2[t] = relu_h(c);
    }
    f4 o = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 2; ++s) o = mma_h(W.w3[s], cat_h(h2[2 * s], h2[2 * s + 1]), o);
    if (valid) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (4 * q + i < f.d_out) out[p * f.d_out + 4 * q + i] = o[i];
    }
}

template <class Tag, int D>
__device__ __forceinline__ void run_tile(const spx_field& f, const Weights& W, const spx_segment& seg, int64_t p,
                                         int r, int q) {
    fwd_tile<Tag, D>(f, W, seg.pts, seg.count, p, r, q, seg.out, nullptr);
}

// Training forward: one field, N points, tiles of 16 points handed to waves
// in contiguous runs; the binary16 features are kept for the backward.
template <class Tag, int D>
__global__ __launch_bounds__(256) void encode_mlp_fwd_kernel(spx_field f, int64_t N, const float* __restrict__ pts,
                                                             float* __restrict__ out, _Float16* __restrict__ feats) {
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    const int64_t tiles = (N + 15) / 16;
    Weights W;
    load_weights(f, r, q, W);
    for (int64_t t0 = wave * kTilesPerWave; t0 < tiles; t0 += nwaves * kTilesPerWave) {
        const int64_t t1 = t0 + kTilesPerWave < tiles ? t0 + kTilesPerWave : tiles;
        for (int64_t t = t0; t < t1; ++t) fwd_tile<Tag, D>(f, W, pts, N, t * 16 + r, r, q, out, feats);
    }
}

__global__ __launch_bounds__(256) void field_query_kernel(const spx_field* __restrict__ fields, int nfields,
                                                          const spx_segment* __restrict__ segs, int nseg,
                                                          int64_t total_tiles) {
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    int cached = -1;
    Weights W;
    for (int64_t t0 = wave * kTilesPerWave; t0 < total_tiles; t0 += nwaves * kTilesPerWave) {
        const int64_t t1 = t0 + kTilesPerWave < total_tiles ? t0 + kTilesPerWave : total_tiles;
        for (int64_t t = t0; t < t1; ++t) {
            // segment holding tile t: the last one whose first tile is <= t
            int lo = 0, hi = nseg - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (segs[mid].first_tile <= t) lo = mid; else hi = mid - 1;
            }
            const spx_segment seg = segs[lo];
            if (seg.field < 0 || seg.field >= nfields) continue;
            const spx_field& f = fields[seg.field];
            if (seg.field != cached) {
                load_weights(f, r, q, W);
                cached = seg.field;
            }
            const int64_t p = (t - seg.first_tile) * 16 + r;
            if (f.cell == SPX_GRID) {
                if (f.n_dims == 2) run_tile<GridTag, 2>(f, W, seg, p, r, q);
                else run_tile<GridTag, 3>(f, W, seg, p, r, q);
            } else {
                if (f.n_dims == 2) run_tile<SimplexTag, 2>(f, W, seg, p, r, q);
                else run_tile<SimplexTag, 3>(f, W, seg, p, r, q);
            }
        }
    }
}

}  // namespace

hipError_t encode_mlp_fwd(const spx_field& f, int64_t N, const float* pts, float* out, uint16_t* feats,
                          hipStream_t s) {
    const int64_t tiles = (N + 15) / 16;
    const int64_t waves = (tiles + kTilesPerWave - 1) / kTilesPerWave;
    int64_t blocks = (waves + 3) / 4;
    blocks = blocks < 8192 ? (blocks > 0 ? blocks : 1) : 8192;
    const int V = f.cell == SPX_GRID ? (1 << f.n_dims) : f.n_dims + 1;
    trace_begin(s, "encode_mlp_fwd",
                (double)N * (4.0 * f.n_dims + 16.0 * V * 4.0 + 4.0 * f.d_out + (feats ? 64.0 : 0.0)));
    _Float16* fe = (_Float16*)feats;
    if (f.cell == SPX_GRID) {
        if (f.n_dims == 2) encode_mlp_fwd_kernel<GridTag, 2><<<(unsigned)blocks, 256, 0, s>>>(f, N, pts, out, fe);
        else encode_mlp_fwd_kernel<GridTag, 3><<<(unsigned)blocks, 256, 0, s>>>(f, N, pts, out, fe);
    } else {
        if (f.n_dims == 2) encode_mlp_fwd_kernel<SimplexTag, 2><<<(unsigned)blocks, 256, 0, s>>>(f, N, pts, out, fe);
        else encode_mlp_fwd_kernel<SimplexTag, 3><<<(unsigned)blocks, 256, 0, s>>>(f, N, pts, out, fe);
    }
    trace_end(s);
    return hipGetLastError();
}

hipError_t field_query(const spx_field* fields, int nfields, const spx_segment* segs, int nseg, int64_t total_tiles,
                       hipStream_t s) {
    const int64_t waves = (total_tiles + kTilesPerWave - 1) / kTilesPerWave;
    int64_t blocks = (waves + 3) / 4;
    const int64_t cap = 8192;
    blocks = blocks < cap ? (blocks > 0 ? blocks : 1) : cap;
    // nominal bytes for 3-D fields with 4 outputs (the kernel reads the field
    // descriptors on the device): point, 16 levels x 4 vertices x 4 bytes, output
    trace_begin(s, "field_query", (double)total_tiles * 16.0 * (12.0 + 16.0 * 4.0 * 4.0 + 16.0));
    field_query_kernel<<<(unsigned)blocks, 256, 0, s>>>(fields, nfields, segs, nseg, total_tiles);
    trace_end(s);
    return hipGetLastError();
}

}  // namespace spx
