// Device-side lookup of one point at one level: which table slots, with
// which weights.  Shared by the forward, adjoint and debug kernels so that
// the three see exactly the same simplex, slots and binary32 weights.
// A level's slot rule (SlotRule) either hashes the vertex into the level's
// power-of-two table or, for a level stored densely, numbers the vertices
// of its box (coordinates clamped to the box).
//
// Binary32 index path (fixed operation order, no contraction):
//   skew (Eq. 2):   s = x_0 + x_1 + ... (left to right), t = s * F_n,
//                   y_i = x_i + t
//   level (5.1):    p_i = y_i * sigma_l, c_i = floor(p_i), f_i = p_i - c_i
// Simplex (Secs. 4.2-4.3): the fractions ordered largest first, ties to the
// lower axis, give the walk c, c + e_a1, c + e_a1 + e_a2, ...; the weights
// are 1 - f(1), f(1) - f(2), ..., f(n).  The order is found branch-free by
// ranking: r_i = #{j : f_j > f_i, or f_j == f_i and j < i}; vertex k
// includes axis i exactly when r_i < k.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spx_internal.h"

namespace spx {

// Hash multipliers: 1, 2654435761, then the smallest primes not below
// floor(2^32 * frac(sqrt(q))) for q = 2, 3, 5, 7.
__host__ __device__ constexpr uint32_t hash_prime(int i) {
    return i == 0 ? 1u
         : i == 1 ? 2654435761u
         : i == 2 ? 1779033713u
         : i == 3 ? 3144134291u
         : i == 4 ? 1013904263u
                  : 2773480771u;
}

// Skew factor F_n = (sqrt(n+1) - 1) / n in binary32 (Eq. 2), passed in by
// the host.
template <int D>
__device__ __forceinline__ void skew(const float (&x)[D], float Fn, float (&y)[D]) {
#pragma clang fp contract(off)
    float s = x[0];
#pragma unroll
    for (int i = 1; i < D; ++i) s = s + x[i];
    const float t = s * Fn;
#pragma unroll
    for (int i = 0; i < D; ++i) y[i] = x[i] + t;
}

template <int D>
struct SimplexCell {
    static constexpr int V = D + 1;   // vertices per level
    static constexpr int VH = D + 1;  // vertices handled per half (one half)
    static constexpr int HALVES = 1;

    // h[k], w[k] for k = 0..D: the walk's vertices.  cell receives the cell
    // corner and offs[k] the set of axes (bit i = axis i) on which vertex k
    // is one step above it; callers that ignore them pay nothing (inlined).
    __device__ __forceinline__ static void lookup(const float (&y)[D], float sigma, SlotRule rule,
                                                  uint32_t (&h)[V], float (&w)[V], int32_t (&cell)[D],
                                                  uint32_t (&offs)[V]) {
#pragma clang fp contract(off)
        float f[D];
        uint32_t a[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const float p = y[i] * sigma;
            const float fl = floorf(p);
            f[i] = p - fl;
            cell[i] = (int32_t)fl;
            a[i] = (uint32_t)cell[i] * hash_prime(i);
        }
        int r[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            int ri = 0;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                if (j < i) ri += (f[j] >= f[i]) ? 1 : 0;
                if (j > i) ri += (f[j] > f[i]) ? 1 : 0;
            }
            r[i] = ri;
        }
        float fs[D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            float v = 0.0f;
#pragma unroll
            for (int i = 0; i < D; ++i) v = (r[i] == k) ? f[i] : v;
            fs[k] = v;
        }
        w[0] = 1.0f - fs[0];
#pragma unroll
        for (int k = 1; k < D; ++k) w[k] = fs[k - 1] - fs[k];
        w[D] = fs[D - 1];
#pragma unroll
        for (int k = 0; k <= D; ++k) {
            uint32_t hk = 0, ok = 0;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                hk ^= (r[i] < k) ? a[i] + hash_prime(i) : a[i];
                ok |= (r[i] < k) ? (1u << i) : 0u;
            }
            h[k] = hk & rule.mask;
            offs[k] = ok;
        }
        select_rows(cell, rule.dext, offs, h);
    }

    // Rows of a densely stored level (dext > 0): each vertex's coordinates
    // clamped to the box [0, dext - 1] (points outside the unit cube), axis 0
    // fastest.  Computed for every level and selected without a branch, so
    // that the gathers of several levels can stay in flight together; for a
    // hashed level (dext == 0) the hashed rows are kept.
    template <int K>
    __device__ __forceinline__ static void select_rows(const int32_t (&cell)[D], int32_t dext,
                                                       const uint32_t (&offs)[K], uint32_t (&h)[K]) {
        const int32_t top = dext - 1;
        int32_t st[D];
        int32_t stride = 1;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            st[i] = stride;
            stride *= dext;
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            int32_t idx = 0;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                int32_t v = cell[i] + (int32_t)((offs[k] >> i) & 1u);
                v = v < 0 ? 0 : (v > top ? top : v);
                idx += v * st[i];
            }
            h[k] = dext > 0 ? (uint32_t)idx : h[k];
        }
    }
};

// 2^n-corner grid (the multilinear baseline).  Corners are enumerated in
// binary order, bit i for axis i.  Weights are the products
// prod_i (bit_i ? f_i : 1 - f_i) taken in axis order.  To bound register
// use the corners are produced as two halves split on the top axis: the
// low 2^(n-1) partial products over axes 0..n-2 are built by doubling (which
// keeps the axis-order association), then multiplied by the top factor.
template <int D>
struct GridCell {
    static constexpr int V = 1 << D;
    static constexpr int VH = 1 << (D - 1);
    static constexpr int HALVES = 2;

    struct Low {
        uint32_t h[VH];
        float w[VH];
        float ft, gt;       // top-axis factors f, 1 - f
        uint32_t at, bt;    // top-axis hash terms for bit 0 / bit 1
        int32_t cell[D];    // cell corner
    };

    __device__ __forceinline__ static void lookup_low(const float (&x)[D], float sigma, Low& lo) {
#pragma clang fp contract(off)
        float f[D], g[D];
        uint32_t a[D], b[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const float p = x[i] * sigma;
            const float fl = floorf(p);
            f[i] = p - fl;
            g[i] = 1.0f - f[i];
            lo.cell[i] = (int32_t)fl;
            a[i] = (uint32_t)lo.cell[i] * hash_prime(i);
            b[i] = a[i] + hash_prime(i);
        }
        lo.w[0] = 1.0f;
        lo.h[0] = 0u;
#pragma unroll
        for (int i = 0; i < D - 1; ++i) {
#pragma unroll
            for (int c = 0; c < (1 << i); ++c) {
                lo.w[c + (1 << i)] = lo.w[c] * f[i];
                lo.w[c] = lo.w[c] * g[i];
                lo.h[c + (1 << i)] = lo.h[c] ^ b[i];
                lo.h[c] = lo.h[c] ^ a[i];
            }
        }
        lo.ft = f[D - 1];
        lo.gt = g[D - 1];
        lo.at = a[D - 1];
        lo.bt = b[D - 1];
    }

    // Corner c_low + half * 2^(n-1).
    __device__ __forceinline__ static void corners(const Low& lo, int half, SlotRule rule,
                                                   uint32_t (&h)[VH], float (&w)[VH]) {
#pragma clang fp contract(off)
        const float t = half ? lo.ft : lo.gt;
        const uint32_t ht = half ? lo.bt : lo.at;
#pragma unroll
        for (int c = 0; c < VH; ++c) {
            w[c] = lo.w[c] * t;
            h[c] = (lo.h[c] ^ ht) & rule.mask;
        }
        uint32_t offs[VH];
#pragma unroll
        for (int c = 0; c < VH; ++c) offs[c] = (uint32_t)c | ((uint32_t)half << (D - 1));
        SimplexCell<D>::select_rows(lo.cell, rule.dext, offs, h);
    }
};

}  // namespace spx
