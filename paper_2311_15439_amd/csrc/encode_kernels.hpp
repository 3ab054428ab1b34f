// Forward, adjoint and debug kernels of the multiresolution hash encoding,
// generic over the cell (simplex or 2^n-corner grid), the dimension, the
// feature count and the storage types.  One thread handles one point and
// walks all levels: the point is loaded and skewed once, and the L*F
// outputs of a point are produced by the same thread.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lookup.hpp"
#include "spx_internal.h"

namespace spx {

typedef _Float16 f16;
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ---- one table row / one output row of F values -------------------------

template <typename T, int F>
struct RowIO;

template <int F>
struct RowIO<float, F> {
    __device__ __forceinline__ static void load(const float* __restrict__ p, float (&v)[F]) {
        if constexpr (F == 1) {
            v[0] = p[0];
        } else if constexpr (F == 2) {
            f32x2 q = *reinterpret_cast<const f32x2*>(p);
            v[0] = q.x; v[1] = q.y;
        } else {
#pragma unroll
            for (int c = 0; c < F / 4; ++c) {
                f32x4 q = reinterpret_cast<const f32x4*>(p)[c];
                v[4 * c] = q.x; v[4 * c + 1] = q.y; v[4 * c + 2] = q.z; v[4 * c + 3] = q.w;
            }
        }
    }
    __device__ __forceinline__ static void store(float* __restrict__ p, const float (&v)[F]) {
        if constexpr (F == 1) {
            p[0] = v[0];
        } else if constexpr (F == 2) {
            *reinterpret_cast<f32x2*>(p) = f32x2{v[0], v[1]};
        } else {
#pragma unroll
            for (int c = 0; c < F / 4; ++c)
                reinterpret_cast<f32x4*>(p)[c] = f32x4{v[4 * c], v[4 * c + 1], v[4 * c + 2], v[4 * c + 3]};
        }
    }
};

template <int F>
struct RowIO<f16, F> {
    __device__ __forceinline__ static void load(const f16* __restrict__ p, float (&v)[F]) {
        if constexpr (F == 1) {
            v[0] = (float)p[0];
        } else if constexpr (F == 2) {
            f16x2 q = *reinterpret_cast<const f16x2*>(p);
            v[0] = (float)q.x; v[1] = (float)q.y;
        } else if constexpr (F == 4) {
            f16x4 q = *reinterpret_cast<const f16x4*>(p);
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = (float)q[j];
        } else {
            f16x8 q = *reinterpret_cast<const f16x8*>(p);
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = (float)q[j];
        }
    }
    __device__ __forceinline__ static void store(f16* __restrict__ p, const float (&v)[F]) {
        if constexpr (F == 1) {
            p[0] = (f16)v[0];
        } else if constexpr (F == 2) {
            *reinterpret_cast<f16x2*>(p) = f16x2{(f16)v[0], (f16)v[1]};
        } else if constexpr (F == 4) {
            *reinterpret_cast<f16x4*>(p) = f16x4{(f16)v[0], (f16)v[1], (f16)v[2], (f16)v[3]};
        } else {
            f16x8 q;
#pragma unroll
            for (int j = 0; j < 8; ++j) q[j] = (f16)v[j];
            *reinterpret_cast<f16x8*>(p) = q;
        }
    }
};

// ---- visiting the vertices of one level ---------------------------------
// fn(h, w, base) is called with arrays of K slots and weights; base is the
// index of the first of them in the level's vertex list.  visit_level_ex
// also passes the cell corner and, per vertex, the axes on which it is one
// step above the corner.

template <int D, class Fn>
__device__ __forceinline__ void visit_level_ex(SimplexTag, const float (&y)[D], float sigma, SlotRule rule,
                                               Fn&& fn) {
    uint32_t h[D + 1], offs[D + 1];
    float w[D + 1];
    int32_t cell[D];
    SimplexCell<D>::lookup(y, sigma, rule, h, w, cell, offs);
    fn(h, w, 0, cell, offs);
}

template <int D, class Fn>
__device__ __forceinline__ void visit_level_ex(GridTag, const float (&x)[D], float sigma, SlotRule rule,
                                               Fn&& fn) {
    typename GridCell<D>::Low lo;
    GridCell<D>::lookup_low(x, sigma, lo);
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        uint32_t h[GridCell<D>::VH], offs[GridCell<D>::VH];
        float w[GridCell<D>::VH];
        GridCell<D>::corners(lo, half, rule, h, w);
#pragma unroll
        for (int c = 0; c < GridCell<D>::VH; ++c) offs[c] = (uint32_t)(c + half * GridCell<D>::VH);
        fn(h, w, half * GridCell<D>::VH, lo.cell, offs);
    }
}

template <class Tag, int D, class Fn>
__device__ __forceinline__ void visit_level(Tag tag, const float (&y)[D], float sigma, SlotRule rule, Fn&& fn) {
    visit_level_ex(tag, y, sigma, rule,
                   [&](const auto& h, const auto& w, int base, const auto&, const auto&) { fn(h, w, base); });
}

template <class Tag, int D>
__device__ __forceinline__ void load_point(const float* __restrict__ pts, int64_t pt, float Fn, float (&y)[D]) {
    float x[D];
#pragma unroll
    for (int i = 0; i < D; ++i) x[i] = pts[pt * D + i];
    if constexpr (Tag::simplex) {
        skew<D>(x, Fn, y);
    } else {
#pragma unroll
        for (int i = 0; i < D; ++i) y[i] = x[i];
    }
}

constexpr int kBlock = 256;

// ---- forward ------------------------------------------------------------

// Features of one point at one level: the weighted sum of its vertices'
// rows (binary32 accumulation, weights in vertex order).
template <class Tag, int D, int F, typename TT, typename OT>
__device__ __forceinline__ void encode_level(const float (&y)[D], int l, const TT* __restrict__ tables,
                                             OT* __restrict__ orow, const LevelArgs& lv) {
    const TT* __restrict__ tab = tables + lv.off[l] * F;
    float acc[F];
#pragma unroll
    for (int j = 0; j < F; ++j) acc[j] = 0.0f;
    visit_level(Tag{}, y, lv.sigma[l], lv.rule(l), [&](const auto& h, const auto& w, int) {
        constexpr int K = sizeof(w) / sizeof(float);
        float v[K][F];
#pragma unroll
        for (int k = 0; k < K; ++k) RowIO<TT, F>::load(tab + (size_t)h[k] * F, v[k]);
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int j = 0; j < F; ++j) acc[j] = __builtin_fmaf(w[k], v[k][j], acc[j]);
    });
    RowIO<OT, F>::store(orow + l * F, acc);
}

template <class Tag, int D, int F, typename TT, typename OT>
__global__ __launch_bounds__(kBlock) void encode_fwd_kernel(int64_t N, const float* __restrict__ pts,
                                                            const TT* __restrict__ tables, OT* __restrict__ out,
                                                            LevelArgs lv) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t pt = (int64_t)blockIdx.x * kBlock + threadIdx.x; pt < N; pt += stride) {
        float y[D];
        load_point<Tag, D>(pts, pt, lv.Fn, y);
        OT* __restrict__ orow = out + pt * (int64_t)(lv.L * F);
        // unrolled so that several levels' gathers are in flight together
#pragma unroll 4
        for (int l = 0; l < lv.L; ++l) encode_level<Tag, D, F, TT, OT>(y, l, tables, orow, lv);
    }
}

// Level-major forward.  When the levels' tables together exceed an XCD's
// L2 but each group of consecutive levels fits, the grid is ordered group
// by group: blocks [g * chunks, (g + 1) * chunks) encode levels
// [first[g], first[g + 1]) of all points, one point per thread.  Blocks
// start in index order, so the blocks in flight work on one group (two at
// its boundary) and each XCD's L2 holds that group's rows instead of a slice
// of every level's.  Each point is read once per group; the features are
// the same bits as the all-levels kernel's.
template <class Tag, int D, int F, typename TT, typename OT>
__global__ __launch_bounds__(kBlock) void encode_fwd_levels_kernel(int64_t N, const float* __restrict__ pts,
                                                                   const TT* __restrict__ tables,
                                                                   OT* __restrict__ out, LevelArgs lv,
                                                                   LevelGroups lg, uint32_t chunks) {
    const uint32_t g = blockIdx.x / chunks;
    const int64_t pt = (int64_t)(blockIdx.x - g * chunks) * kBlock + threadIdx.x;
    if (pt >= N) return;
    float y[D];
    load_point<Tag, D>(pts, pt, lv.Fn, y);
    OT* __restrict__ orow = out + pt * (int64_t)(lv.L * F);
    const int l1 = lg.first[g + 1];
#pragma unroll 2
    for (int l = lg.first[g]; l < l1; ++l) encode_level<Tag, D, F, TT, OT>(y, l, tables, orow, lv);
}

// ---- gather twin (measurement reference) -------------------------------
// The forward's memory traffic without its arithmetic: the same point stream,
// the same cells and the same number of hashed rows per level (n + 1 for
// the simplex, 2^n for the grid) with the same per-level locality, but the
// simplex walk takes the axes in fixed order (no ranking) and the rows are
// summed without weights.  Binary16 tables with F = 2, binary16 output.
template <int D>
__device__ __forceinline__ void twin_simplex_slots(const float (&y)[D], float sigma, uint32_t mask,
                                                   uint32_t (&h)[D + 1]) {
#pragma clang fp contract(off)
    uint32_t a[D];
#pragma unroll
    for (int i = 0; i < D; ++i) a[i] = (uint32_t)(int32_t)floorf(y[i] * sigma) * hash_prime(i);
#pragma unroll
    for (int k = 0; k <= D; ++k) {
        uint32_t hk = 0;
#pragma unroll
        for (int i = 0; i < D; ++i) hk ^= i < k ? a[i] + hash_prime(i) : a[i];
        h[k] = hk & mask;
    }
}

template <class Tag, int D>
__global__ __launch_bounds__(kBlock) void encode_twin_kernel(int64_t N, const float* __restrict__ pts,
                                                             const f16* __restrict__ tables, f16* __restrict__ out,
                                                             LevelArgs lv) {
    const uint32_t mask = lv.mask;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t pt = (int64_t)blockIdx.x * kBlock + threadIdx.x; pt < N; pt += stride) {
        float y[D];
        load_point<Tag, D>(pts, pt, lv.Fn, y);
        f16* __restrict__ orow = out + pt * (int64_t)(lv.L * 2);
#pragma unroll 4
        for (int l = 0; l < lv.L; ++l) {
            const f16* __restrict__ tab = tables + lv.off[l] * 2;
            float acc[2] = {0.0f, 0.0f};
            auto add = [&](const auto& h) {
                constexpr int K = sizeof(h) / sizeof(uint32_t);
                float v[K][2];
#pragma unroll
                for (int k = 0; k < K; ++k) RowIO<f16, 2>::load(tab + (size_t)h[k] * 2, v[k]);
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    acc[0] += v[k][0];
                    acc[1] += v[k][1];
                }
            };
            if constexpr (Tag::simplex) {
                uint32_t h[D + 1];
                twin_simplex_slots<D>(y, lv.sigma[l], mask, h);
                add(h);
            } else {
                visit_level(Tag{}, y, lv.sigma[l], SlotRule{mask, 0}, [&](const auto& h, const auto&, int) { add(h); });
            }
            RowIO<f16, 2>::store(orow + l * 2, acc);
        }
    }
}

// ---- gradient with respect to the input point ---------------------------
// Inside a simplex the weights are affine in the fractional parts: the
// derivative along the axis stepped between walk vertices k and k+1 is the
// difference of their rows.  The grid differentiates its n-linear weights,
// d w_b / d f_i = (b_i ? 1 : -1) prod_{m != i} (b_m ? f_m : 1 - f_m).  The
// chain to x: d p_i / d x_m = sigma (delta_im + F_n) (skew, Eq. 2) for the
// simplex and sigma delta_im for the grid.
template <class Tag, int D, int F, typename TT, typename GT>
__global__ __launch_bounds__(kBlock) void encode_input_grad_kernel(int64_t N, const float* __restrict__ pts,
                                                                   const TT* __restrict__ tables,
                                                                   const GT* __restrict__ d_out,
                                                                   float* __restrict__ d_pts, LevelArgs lv) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t pt = (int64_t)blockIdx.x * kBlock + threadIdx.x; pt < N; pt += stride) {
        float y[D];
        load_point<Tag, D>(pts, pt, lv.Fn, y);
        const GT* __restrict__ grow = d_out + pt * (int64_t)(lv.L * F);
        float dx[D];
#pragma unroll
        for (int m = 0; m < D; ++m) dx[m] = 0.0f;
        // unrolled so that several levels' gathers are in flight together
#pragma unroll 4
        for (int l = 0; l < lv.L; ++l) {
            const TT* __restrict__ tab = tables + lv.off[l] * F;
            const SlotRule rule = lv.rule(l);
            float d[F], g[D];
            RowIO<GT, F>::load(grow + l * F, d);
#pragma unroll
            for (int m = 0; m < D; ++m) g[m] = 0.0f;
            if constexpr (Tag::simplex) {
                visit_level_ex(Tag{}, y, lv.sigma[l], rule,
                               [&](const auto& h, const auto&, int, const auto&, const auto& offs) {
                    float t[D + 1][F];
#pragma unroll
                    for (int k = 0; k <= D; ++k) RowIO<TT, F>::load(tab + (size_t)h[k] * F, t[k]);
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        const int axis = __builtin_ctz(offs[k + 1] ^ offs[k]);
                        float s = 0.0f;
#pragma unroll
                        for (int j = 0; j < F; ++j) s += (t[k + 1][j] - t[k][j]) * d[j];
#pragma unroll
                        for (int m = 0; m < D; ++m) g[m] += m == axis ? s : 0.0f;
                    }
                });
            } else {
                float f[D];
#pragma unroll
                for (int i = 0; i < D; ++i) {
#pragma clang fp contract(off)
                    const float p = y[i] * lv.sigma[l];
                    f[i] = p - floorf(p);
                }
                visit_level_ex(Tag{}, y, lv.sigma[l], rule,
                               [&](const auto& h, const auto& w, int, const auto&, const auto& offs) {
                    constexpr int K = sizeof(w) / sizeof(float);
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        float t[F];
                        RowIO<TT, F>::load(tab + (size_t)h[k] * F, t);
                        float s = 0.0f;
#pragma unroll
                        for (int j = 0; j < F; ++j) s += t[j] * d[j];
                        const uint32_t b = offs[k];
#pragma unroll
                        for (int i = 0; i < D; ++i) {
                            float c = ((b >> i) & 1u) ? s : -s;
#pragma unroll
                            for (int m = 0; m < D; ++m)
                                if (m != i) c *= ((b >> m) & 1u) ? f[m] : 1.0f - f[m];
                            g[i] += c;
                        }
                    }
                });
            }
            const float sig = lv.sigma[l];
            if constexpr (Tag::simplex) {
                float gs = 0.0f;
#pragma unroll
                for (int m = 0; m < D; ++m) gs += g[m];
#pragma unroll
                for (int m = 0; m < D; ++m) dx[m] += sig * (g[m] + lv.Fn * gs);
            } else {
#pragma unroll
                for (int m = 0; m < D; ++m) dx[m] += sig * g[m];
            }
        }
#pragma unroll
        for (int m = 0; m < D; ++m) d_pts[pt * D + m] = dx[m];
    }
}

// ---- adjoint ------------------------------------------------------------

template <class Tag, int D, int F, typename GT>
__global__ __launch_bounds__(kBlock) void encode_bwd_kernel(int64_t N, const float* __restrict__ pts,
                                                            const GT* __restrict__ d_out,
                                                            float* __restrict__ d_tables, LevelArgs lv) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t pt = (int64_t)blockIdx.x * kBlock + threadIdx.x; pt < N; pt += stride) {
        float y[D];
        load_point<Tag, D>(pts, pt, lv.Fn, y);
        const GT* __restrict__ grow = d_out + pt * (int64_t)(lv.L * F);
        for (int l = 0; l < lv.L; ++l) {
            float g[F];
            RowIO<GT, F>::load(grow + l * F, g);
            float* __restrict__ tab = d_tables + lv.off[l] * F;
            visit_level(Tag{}, y, lv.sigma[l], lv.rule(l), [&](const auto& h, const auto& w, int) {
                constexpr int K = sizeof(w) / sizeof(float);
#pragma unroll
                for (int k = 0; k < K; ++k)
#pragma unroll
                    for (int j = 0; j < F; ++j) unsafeAtomicAdd(tab + (size_t)h[k] * F + j, w[k] * g[j]);
            });
        }
    }
}

// ---- debug --------------------------------------------------------------

template <class Tag, int D>
__global__ __launch_bounds__(kBlock) void encode_debug_kernel(int64_t N, const float* __restrict__ pts,
                                                              uint32_t* __restrict__ idx,
                                                              float* __restrict__ wout, LevelArgs lv) {
    constexpr int V = Tag::simplex ? D + 1 : (1 << D);
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t pt = (int64_t)blockIdx.x * kBlock + threadIdx.x; pt < N; pt += stride) {
        float y[D];
        load_point<Tag, D>(pts, pt, lv.Fn, y);
        for (int l = 0; l < lv.L; ++l) {
            const int64_t base = (pt * lv.L + l) * V;
            visit_level(Tag{}, y, lv.sigma[l], lv.rule(l), [&](const auto& h, const auto& w, int b0) {
                constexpr int K = sizeof(w) / sizeof(float);
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    if (idx) idx[base + b0 + k] = h[k];
                    if (wout) wout[base + b0 + k] = w[k];
                }
            });
        }
    }
}

}  // namespace spx
