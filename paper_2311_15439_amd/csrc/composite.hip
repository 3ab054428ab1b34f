// Volume rendering of ray samples (Sec. 6, Eq. 5) and its adjoint.
//
// One wave per ray.  Sample k of the ray sits in lane k % 64 of row k / 64,
// so a row's loads are coalesced; the optical depth before each sample is a
// running sum over rows of wave-wide inclusive scans.  The quadrature:
//   sigma = softplus(raw_0), c = sigmoid(raw_1..3), tau = sigma * delta,
//   alpha = 1 - exp(-tau), T_k = exp(-(tau_0 + ... + tau_{k-1})),
//   w_k = T_k alpha_k, rgba = (sum_k w_k c_k, sum_k w_k).
// The adjoint keeps every row's optical depths in registers and walks the
// rows backwards, so the radiance behind a sample is a suffix sum (no
// cancellation against the total).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spx_internal.h"

namespace spx {
namespace {

constexpr int kWaves = 4;  // rays per block

__device__ __forceinline__ float softplus_f(float x) {
    return x > 0.0f ? x + log1pf(expf(-x)) : log1pf(expf(x));
}
__device__ __forceinline__ float sigmoid_f(float x) { return 1.0f / (1.0f + expf(-x)); }

// Inclusive scan over the 64 lanes.
__device__ __forceinline__ float wave_scan(float v, int lane) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const float t = __shfl_up(v, off, 64);
        if (lane >= off) v += t;
    }
    return v;
}
// Suffix scan (inclusive) over the 64 lanes.
__device__ __forceinline__ float wave_suffix(float v, int lane) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const float t = __shfl_down(v, off, 64);
        if (lane + off < 64) v += t;
    }
    return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int ROWS>
__global__ __launch_bounds__(64 * kWaves) void composite_fwd_kernel(int64_t R, int S, const float4* __restrict__ raw,
                                                                     const float* __restrict__ delta,
                                                                     float4* __restrict__ rgba) {
    const int lane = threadIdx.x & 63;
    for (int64_t r = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); r < R; r += (int64_t)gridDim.x * kWaves) {
        const float4* q = raw + r * S;
        const float* d = delta + r * S;
        float carry = 0.0f;  // optical depth before the row
        float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int row = 0; row < ROWS; ++row) {
            const int k = row * 64 + lane;
            const bool ok = k < S;
            const float4 x = ok ? q[k] : float4{-100.0f, 0.0f, 0.0f, 0.0f};
            const float tau = ok ? softplus_f(x.x) * d[k] : 0.0f;
            const float incl = wave_scan(tau, lane);
            const float excl = __shfl_up(incl, 1, 64);
            const float before = carry + (lane > 0 ? excl : 0.0f);
            const float w = expf(-before) * -expm1f(-tau);
            acc[0] += w * sigmoid_f(x.y);
            acc[1] += w * sigmoid_f(x.z);
            acc[2] += w * sigmoid_f(x.w);
            acc[3] += w;
            carry += __shfl(incl, 63, 64);
        }
        float4 o;
        o.x = wave_sum(acc[0]);
        o.y = wave_sum(acc[1]);
        o.z = wave_sum(acc[2]);
        o.w = wave_sum(acc[3]);
        if (lane == 0) rgba[r] = o;
    }
}

template <int ROWS>
__global__ __launch_bounds__(64 * kWaves) void composite_bwd_kernel(int64_t R, int S, const float4* __restrict__ raw,
                                                                     const float* __restrict__ delta,
                                                                     const float4* __restrict__ d_rgba,
                                                                     float4* __restrict__ d_raw) {
    const int lane = threadIdx.x & 63;
    for (int64_t r = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); r < R; r += (int64_t)gridDim.x * kWaves) {
        const float4* q = raw + r * S;
        const float* d = delta + r * S;
        const float4 g = d_rgba[r];
        // forward over the rows: optical depth before every sample
        float before[ROWS], tau[ROWS];
        float carry = 0.0f;
#pragma unroll
        for (int row = 0; row < ROWS; ++row) {
            const int k = row * 64 + lane;
            const bool ok = k < S;
            tau[row] = ok ? softplus_f(q[k].x) * d[k] : 0.0f;
            const float incl = wave_scan(tau[row], lane);
            const float excl = __shfl_up(incl, 1, 64);
            before[row] = carry + (lane > 0 ? excl : 0.0f);
            carry += __shfl(incl, 63, 64);
        }
        // backward over the rows: what lies behind each sample
        float behind = 0.0f;  // sum over later rows of dQ . w q
#pragma unroll
        for (int row = ROWS - 1; row >= 0; --row) {
            const int k = row * 64 + lane;
            const bool ok = k < S;
            const float4 x = ok ? q[k] : float4{0.0f, 0.0f, 0.0f, 0.0f};
            const float T = expf(-before[row]);
            const float alpha = -expm1f(-tau[row]);
            const float w = T * alpha;
            const float c0 = sigmoid_f(x.y), c1 = sigmoid_f(x.z), c2 = sigmoid_f(x.w);
            const float gq = g.x * c0 + g.y * c1 + g.z * c2 + g.w;  // dQ . q_k
            const float mine = ok ? w * gq : 0.0f;
            const float suff = wave_suffix(mine, lane);          // this sample and the later ones in the row
            const float later = __shfl_down(suff, 1, 64);
            const float rest = behind + (lane < 63 ? later : 0.0f);  // strictly later samples
            const float dtau = T * (1.0f - alpha) * gq - rest;   // T_{k+1} = T_k (1 - alpha_k)
            if (ok) {
                float4 o;
                o.x = dtau * d[k] * sigmoid_f(x.x);
                // c (1 - c) with 1 - c = sigmoid(-raw): no cancellation for saturated colours
                o.y = g.x * w * c0 * sigmoid_f(-x.y);
                o.z = g.y * w * c1 * sigmoid_f(-x.z);
                o.w = g.z * w * c2 * sigmoid_f(-x.w);
                d_raw[r * S + k] = o;
            }
            behind += __shfl(suff, 0, 64);
        }
    }
}

}  // namespace

hipError_t composite_fwd(int64_t R, int S, const float* raw, const float* delta, float* rgba, hipStream_t s) {
    trace_begin(s, "composite_fwd", (double)R * S * 20.0 + (double)R * 16.0);
    int64_t blocks = (R + kWaves - 1) / kWaves;
    blocks = blocks < 16384 ? (blocks > 0 ? blocks : 1) : 16384;
    const dim3 g((unsigned)blocks), b(64 * kWaves);
    const int rows = (S + 63) / 64;
    const float4* q = (const float4*)raw;
    float4* o = (float4*)rgba;
    if (rows <= 1) composite_fwd_kernel<1><<<g, b, 0, s>>>(R, S, q, delta, o);
    else if (rows <= 2) composite_fwd_kernel<2><<<g, b, 0, s>>>(R, S, q, delta, o);
    else if (rows <= 4) composite_fwd_kernel<4><<<g, b, 0, s>>>(R, S, q, delta, o);
    else if (rows <= 8) composite_fwd_kernel<8><<<g, b, 0, s>>>(R, S, q, delta, o);
    else composite_fwd_kernel<16><<<g, b, 0, s>>>(R, S, q, delta, o);
    trace_end(s);
    return hipGetLastError();
}

hipError_t composite_bwd(int64_t R, int S, const float* raw, const float* delta, const float* d_rgba, float* d_raw,
                         hipStream_t s) {
    trace_begin(s, "composite_bwd", (double)R * S * 36.0 + (double)R * 16.0);
    int64_t blocks = (R + kWaves - 1) / kWaves;
    blocks = blocks < 16384 ? (blocks > 0 ? blocks : 1) : 16384;
    const dim3 g((unsigned)blocks), b(64 * kWaves);
    const int rows = (S + 63) / 64;
    const float4* q = (const float4*)raw;
    const float4* gi = (const float4*)d_rgba;
    float4* o = (float4*)d_raw;
    if (rows <= 1) composite_bwd_kernel<1><<<g, b, 0, s>>>(R, S, q, delta, gi, o);
    else if (rows <= 2) composite_bwd_kernel<2><<<g, b, 0, s>>>(R, S, q, delta, gi, o);
    else if (rows <= 4) composite_bwd_kernel<4><<<g, b, 0, s>>>(R, S, q, delta, gi, o);
    else if (rows <= 8) composite_bwd_kernel<8><<<g, b, 0, s>>>(R, S, q, delta, gi, o);
    else composite_bwd_kernel<16><<<g, b, 0, s>>>(R, S, q, delta, gi, o);
    trace_end(s);
    return hipGetLastError();
}

}  // namespace spx
