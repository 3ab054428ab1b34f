// Internal interface between the C ABI layer (api.hip) and the kernel
// translation units.  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "spx.h"

namespace spx {

// Tracing hooks (no-ops unless a trace is set on the calling thread).
void trace_begin(hipStream_t s, const char* name, double bytes);
void trace_end(hipStream_t s);

struct AuxStream {
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};
// The current device's side stream (nullptr if unavailable); lock is held
// on return and must be kept until the fork/join sequence is issued.
AuxStream* aux_stream(std::unique_lock<std::mutex>& lock);

struct SimplexTag { static constexpr bool simplex = true; };
struct GridTag { static constexpr bool simplex = false; };

// How one level maps a lattice vertex to a row of its table: hashed into
// mask + 1 rows (dext == 0), or stored densely over the box of dext^n
// vertices, vertex v at row sum_i clamp(v_i, 0, dext - 1) dext^i (dext > 0).
struct SlotRule {
    uint32_t mask;
    int32_t dext;
};

// Per-call level parameters, passed to the kernels by value.
struct LevelArgs {
    float sigma[32];  // binary32 multiplier of level l
    float Fn;         // skew factor F_n in binary32
    uint32_t mask;    // T - 1 (rows of the largest level)
    int32_t L;        // number of levels
    uint32_t dense;   // bit l: level l is stored densely
    int32_t ext[32];  // per axis, extent of the vertex box the closed unit cube reaches at level l
    uint32_t rows[32];  // rows of level l's table (a power of two when hashed)
    uint64_t off[32];   // first row of level l
    // Without a branch (a conditional load of ext[l] would split the level
    // loop and keep the gathers of successive levels from overlapping).
    __host__ __device__ SlotRule rule(int l) const {
        const int32_t on = -(int32_t)((dense >> l) & 1u);
        return SlotRule{rows[l] - 1u, ext[l] & on};
    }
    // The same, for kernels instantiated per call on whether any level is
    // dense: without one, the dense rows are never computed.
    template <bool DENSE>
    __host__ __device__ SlotRule rule_if(int l) const {
        if constexpr (DENSE) return rule(l);
        return SlotRule{rows[l] - 1u, 0};
    }
};

// Level groups of the level-major forward: group g holds levels
// [first[g], first[g + 1]); n == 0 selects the all-levels kernel.
struct LevelGroups {
    int32_t n;
    int32_t first[33];
};

constexpr double kXcdL2Bytes = 4.0 * 1024 * 1024;  // L2 of one XCD

// Bytes of level l's table its points can reach: a dense level's rows; for
// a hashed level one 128-byte line per vertex of its box, at most the whole
// table.
inline double level_reach_bytes(const LevelArgs& lv, int l, int D, int row_bytes) {
    const double table = (double)lv.rows[l] * row_bytes;
    if ((lv.dense >> l) & 1u) return table;
    double box = 1.0;
    for (int i = 0; i < D; ++i) box *= (double)lv.ext[l];
    return box * 128.0 < table ? box * 128.0 : table;
}

// Consecutive levels grouped while their reachable rows fit one XCD's L2.
// Level-major order pays when the levels together do not fit but each group
// does, and the batch is large enough (at least 2^18 points) for the blocks
// in flight to cover a fraction of one group.  Measured on MI355X it pays
// from three dimensions up (n = 3..6: 1.3-1.8x); in two dimensions the
// all-levels kernel already gathers faster than the L2's random rate (the
// few vertices of a 2-D cell share lines) and the extra passes over the
// points cost more than they save.
inline LevelGroups fwd_level_groups(const LevelArgs& lv, int D, int row_bytes, int64_t N) {
    LevelGroups g{};
    if (N < (1 << 18) || D < 3) return g;
    double total = 0.0;
    for (int l = 0; l < lv.L; ++l) {
        const double b = level_reach_bytes(lv, l, D, row_bytes);
        if (b > kXcdL2Bytes) return g;
        total += b;
    }
    if (total <= kXcdL2Bytes) return g;
    double used = 0.0;
    for (int l = 0; l < lv.L; ++l) {
        const double b = level_reach_bytes(lv, l, D, row_bytes);
        if (g.n == 0 || used + b > kXcdL2Bytes) {
            g.first[g.n++] = l;
            used = 0.0;
        }
        used += b;
    }
    g.first[g.n] = lv.L;
    const double blocks = (double)((N + 255) / 256) * g.n;
    if (g.n < 2 || blocks > 2147483647.0) g.n = 0;
    return g;
}

// Adam hyper-parameters and state for the fused adjoint + optimizer path
// (param == nullptr: plain adjoint into d_tables).
struct AdamArgs {
    float* param;
    float* m;
    float* v;
    void* param_f16;  // binary16 image of param, or nullptr
    float lr, b1, b2, eps, inv_bc1, inv_bc2;
};

// AdjointPrepare: the binned adjoint's first level group counted and laid
// out in the workspace (it depends only on the points), for a following
// AdjointBinned call with `prepared` set.
enum class EncodeOp { Forward, Adjoint, AdjointBinned, AdjointPrepare, Debug, Twin, InputGrad };

// Binned adjoint: one level group's plan (device pointers into the caller's
// workspace).  Levels [0, P) of group 0 are privatised: their contributions
// from cells inside a dense box of ext[l]^n vertices are summed per
// workgroup in LDS instead of being emitted as records.
struct BinPlan {
    int l0, l1;       // levels [l0, l1) of this group
    int s_log2;       // slots per bucket = 2^s_log2
    int bmax;         // largest bucket count of one level in the group
    int B;            // buckets in this group
    int W;            // workgroups of the count, coarse and scatter passes
    int64_t chunk;    // points per workgroup
    int P;            // privatised levels (all below l1)
    int Dtot;         // dense entries over the privatised levels
    int ext[32];      // dense box extent per privatised level
    int doff[33];     // first dense entry of each privatised level
    int boff[33];     // first bucket of level l in the group (levels l0..l1)
    int ks[32];       // workgroups sharing each bucket of level l (1: not split)
    int voff[33];     // first accumulation workgroup of level l (levels l0..l1)
    int VB;           // accumulation workgroups of the group
    int sboff[33];    // first split bucket of level l (counting split buckets only)
    int nsplit;       // split buckets of the group
    int64_t soff[33]; // first partial slice of level l in `split`
    uint32_t* counts;  // [W][B]
    uint32_t* base;    // [B + 1]
    void* recs;        // records
    float* partial;    // [W][Dtot * F] per-workgroup dense sums
    float* gdense;     // [Dtot * F] their total
    float* split;      // partial slices of split buckets, 2^s * F floats each
};

// Sizes shared by every group; a pure function of the encoding's level
// parameters and N, so the workspace query and the launch agree.
struct BinLayout {
    int L, groups, s_log2, Bmax, W, rec_bytes, V, P, Dtot, lmax;
    int nb[32];       // buckets of level l: ceil(rows / 2^s)
    int gl[33];       // group g holds levels [gl[g], gl[g + 1])
    int ext[32];
    int doff[33];
    int ks[32];       // workgroups sharing each bucket of level l
    int64_t N, chunk;
    size_t off_counts, off_base, off_totals, off_recs, off_partial, off_gdense, off_split, total_bytes;
    bool ok;
};

inline size_t bin_align(size_t x) { return (x + 255) & ~(size_t)255; }

inline BinLayout bin_layout(int D, int F, int64_t N, bool simplex, const LevelArgs& lv) {
    BinLayout b{};
    const int L = lv.L;
    b.L = L;
    b.N = N;
    b.V = simplex ? D + 1 : (1 << D);
    b.rec_bytes = F == 1 ? 8 : F == 2 ? 12 : F == 4 ? 32 : 64;  // sizeof(BinRec<F>)
    const int lf = F == 1 ? 0 : F == 2 ? 1 : F == 4 ? 2 : 3;
    // bucket of 2^s slots: its binary32 accumulator (2^s * F * 4 bytes) is
    // 128 KiB, one accumulation workgroup per CU.  Half the size would let two
    // share a CU, but the scatter's per-bucket runs of records would be half
    // as long, and its record stores are bound by those runs.  At most 16384
    // buckets per level for T <= 2^26.
    int log2T = 31 - __builtin_clz(lv.mask + 1u);
    int s = 15 - lf;
    if (s > log2T) s = log2T;
    b.s_log2 = s;
    b.ok = N >= 0;
    for (int l = 0; l < L; ++l) {
        b.nb[l] = (int)(((uint64_t)lv.rows[l] + (1u << s) - 1) >> s);
        if (b.nb[l] > 16384) b.ok = false;
    }
    // level groups: consecutive levels while the group holds at most 16384
    // buckets, fewer than 2^31 records and at most 2 GiB of records (the
    // count, scan, scatter and accumulation passes repeat per group, so fewer
    // groups are faster; 2 GiB of 288 GB)
    const double per_level = (double)N * b.V;
    if (per_level >= 2147483647.0) b.ok = false;
    b.groups = 0;
    b.Bmax = 0;
    b.lmax = 0;
    int l = 0;
    while (l < L && b.groups < 32) {
        const int g0 = l;
        int nbk = 0;
        while (l < L) {
            const int k = l - g0 + 1;
            const bool fits = nbk + b.nb[l] <= 16384 && per_level * k < 2147483647.0 &&
                              per_level * k * b.rec_bytes <= 2147483648.0;
            if (!fits && l > g0) break;
            nbk += b.nb[l];
            ++l;
        }
        b.gl[b.groups++] = g0;
        if (nbk > b.Bmax) b.Bmax = nbk;
        if (l - g0 > b.lmax) b.lmax = l - g0;
    }
    b.gl[b.groups] = L;
    if (l < L) b.ok = false;
    int64_t W = (N + 255) / 256;
    b.W = (int)(W < 512 ? (W > 0 ? W : 1) : 512);
    b.chunk = (N + b.W - 1) / b.W;
    // privatised coarse levels: the prefix of group 0 whose vertex boxes fit
    // in 96 KiB of binary32 accumulators
    const int dense_max = (96 * 1024) / (4 * F);
    b.P = 0;
    b.Dtot = 0;
    b.doff[0] = 0;
    for (int q = 0; q < b.gl[1] && q < 32; ++q) {
        const double e = (double)lv.ext[q];
        double size = 1.0;
        for (int i = 0; i < D; ++i) size *= e;
        if (size > (double)(dense_max - b.Dtot)) break;
        b.ext[q] = (int)e;
        b.Dtot += (int)size;
        b.P = q + 1;
        b.doff[q + 1] = b.Dtot;
    }
    // Split buckets.  One workgroup sums a bucket, so a level with few
    // buckets and many contributions (a small table: a coarse level stored
    // densely or sized to its share) puts all of them on a few CUs while the
    // rest idle.  A bucket expected to hold more than a CU's share of all
    // records (N V per level, before merging; none for privatised levels) is
    // split over ks workgroups, each summing a contiguous part of its records
    // into its own partial slice; a second pass adds the partials in order.
    {
        double total = 0.0;
        for (int q = 0; q < L; ++q) total += q < b.P ? 0.0 : per_level;
        const double per_cu = total / 256.0;
        for (int q = 0; q < L; ++q) {
            const double e = q < b.P ? 0.0 : per_level / (double)b.nb[q];
            int k = 1;
            if (e > 65536.0 && e > per_cu) {
                const double want = e / per_cu;
                k = want > 256.0 ? 256 : (int)want + 1;
            }
            b.ks[q] = k;
        }
    }
    size_t split_floats = 0;  // the largest group's partial slices
    for (int g = 0; g < b.groups; ++g) {
        size_t n = 0;
        for (int q = b.gl[g]; q < b.gl[g + 1]; ++q)
            if (b.ks[q] > 1) n += (size_t)b.nb[q] * b.ks[q] * ((size_t)F << s);
        if (n > split_floats) split_floats = n;
    }
    size_t off = 0;
    b.off_counts = off;
    off = bin_align(off + (size_t)b.W * b.Bmax * 4);
    b.off_base = off;
    off = bin_align(off + ((size_t)b.Bmax + 1) * 4);
    b.off_totals = off;
    off = bin_align(off + (size_t)b.Bmax * 4);
    b.off_partial = off;
    off = bin_align(off + (size_t)b.W * b.Dtot * F * 4);
    b.off_gdense = off;
    off = bin_align(off + (size_t)b.Dtot * F * 4);
    b.off_split = off;
    off = bin_align(off + split_floats * 4);
    b.off_recs = off;
    off = bin_align(off + (size_t)N * b.lmax * b.V * b.rec_bytes);
    b.total_bytes = off;
    return b;
}

inline BinPlan bin_plan(const BinLayout& lay, int g, char* ws) {
    BinPlan p;
    p.l0 = lay.gl[g];
    p.l1 = lay.gl[g + 1];
    p.s_log2 = lay.s_log2;
    p.W = lay.W;
    p.chunk = lay.chunk;
    p.P = g == 0 ? lay.P : 0;
    p.Dtot = g == 0 ? lay.Dtot : 0;
    for (int l = 0; l < 32; ++l) p.ext[l] = lay.ext[l];
    for (int l = 0; l < 33; ++l) p.doff[l] = lay.doff[l];
    for (int l = 0; l < 33; ++l) p.boff[l] = 0;
    int acc = 0;
    p.bmax = 0;
    for (int l = p.l0; l < p.l1; ++l) {
        p.boff[l] = acc;
        acc += lay.nb[l];
        if (lay.nb[l] > p.bmax) p.bmax = lay.nb[l];
    }
    p.boff[p.l1] = acc;
    p.B = acc;
    int vacc = 0, sacc = 0;
    int64_t sl = 0;
    for (int l = 0; l < 32; ++l) p.ks[l] = lay.ks[l];
    for (int l = 0; l < 33; ++l) p.voff[l] = p.sboff[l] = 0, p.soff[l] = 0;
    for (int l = p.l0; l < p.l1; ++l) {
        p.voff[l] = vacc;
        p.sboff[l] = sacc;
        p.soff[l] = sl;
        vacc += lay.nb[l] * lay.ks[l];
        if (lay.ks[l] > 1) {
            sacc += lay.nb[l];
            sl += (int64_t)lay.nb[l] * lay.ks[l];
        }
    }
    p.voff[p.l1] = vacc;
    p.sboff[p.l1] = sacc;
    p.soff[p.l1] = sl;
    p.VB = vacc;
    p.nsplit = sacc;
    p.counts = (uint32_t*)(ws + lay.off_counts);
    p.base = (uint32_t*)(ws + lay.off_base);
    p.recs = ws + lay.off_recs;
    p.partial = (float*)(ws + lay.off_partial);
    p.gdense = (float*)(ws + lay.off_gdense);
    p.split = (float*)(ws + lay.off_split);
    return p;
}

// The network (d_in -> 64 -> 64 -> d_out) whose input gradient the fused
// adjoint computes itself: binary16 features x [N][d_in] and weights, the
// binary32 output gradient d_y [N][d_out].
struct NetArgs {
    const _Float16* x;
    const _Float16 *W1, *W2, *W3;
    const float* d_y;
    int d_out;
    int coarse_stride;
    int check_only;  // only check that the fused path covers the configuration
};

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
    void* workspace;  // binned adjoint only
    bool prepared;    // binned adjoint only: group 0 counted by a preceding AdjointPrepare call
    AdamArgs adam;    // binned adjoint only
    // binned adjoint only: when net.x is set, the output gradient is the
    // network's input gradient, computed in the scatter from the features
    // and the network's output gradient (d_out then holds only the
    // privatised coarse levels' units, rows of net.coarse_stride floats)
    NetArgs net;
    LevelArgs lv;
    hipStream_t stream;
};

// Kernels of one (cell, dimension, feature count), one translation unit
// each (encode_unit.hip); encode_cell() picks the triple.
template <bool Grid, int D, int F>
hipError_t encode_unit(const EncodeCall& c);
#define SPX_DECLARE_UNIT(G, D) \
    template <> hipError_t encode_unit<G, D, 1>(const EncodeCall& c); \
    template <> hipError_t encode_unit<G, D, 2>(const EncodeCall& c); \
    template <> hipError_t encode_unit<G, D, 4>(const EncodeCall& c); \
    template <> hipError_t encode_unit<G, D, 8>(const EncodeCall& c);
SPX_DECLARE_UNIT(false, 1) SPX_DECLARE_UNIT(false, 2) SPX_DECLARE_UNIT(false, 3)
SPX_DECLARE_UNIT(false, 4) SPX_DECLARE_UNIT(false, 5) SPX_DECLARE_UNIT(false, 6)
SPX_DECLARE_UNIT(true, 1) SPX_DECLARE_UNIT(true, 2) SPX_DECLARE_UNIT(true, 3)
SPX_DECLARE_UNIT(true, 4) SPX_DECLARE_UNIT(true, 5) SPX_DECLARE_UNIT(true, 6)
#undef SPX_DECLARE_UNIT

template <bool Grid, int D>
inline hipError_t encode_dim(const EncodeCall& c) {
    switch (c.F) {
        case 1: return encode_unit<Grid, D, 1>(c);
        case 2: return encode_unit<Grid, D, 2>(c);
        case 4: return encode_unit<Grid, D, 4>(c);
        case 8: return encode_unit<Grid, D, 8>(c);
        default: return hipErrorInvalidValue;
    }
}

template <bool Grid>
inline hipError_t encode_cell(const EncodeCall& c) {
    switch (c.D) {
        case 1: return encode_dim<Grid, 1>(c);
        case 2: return encode_dim<Grid, 2>(c);
        case 3: return encode_dim<Grid, 3>(c);
        case 4: return encode_dim<Grid, 4>(c);
        case 5: return encode_dim<Grid, 5>(c);
        case 6: return encode_dim<Grid, 6>(c);
        default: return hipErrorInvalidValue;
    }
}

// MLP and elementwise kernels.
struct MlpCall {
    int d_in, hidden, d_out;
    int64_t N;
    const uint16_t* x;
    const uint16_t *W1, *W2, *W3;
    float* y;
    const float* d_y;
    float* d_x;
    int dx_cols, dx_stride;  // units of d_x written per point and its row stride (0: all d_in)
    float *dW1, *dW2, *dW3;
    void* workspace;
    hipStream_t stream;
};
size_t mlp_bwd_workspace_bytes(int d_in, int hidden, int d_out, int64_t N);
int mlp_bwd_lds_bytes(int d_in);
// Device address and size of the current device's scratch for the
// allocation-free backward (looked up on first use per device).
hipError_t mlp_bwd_scratch(void** ptr, size_t* bytes);
hipError_t mlp_fwd(const MlpCall& c);
hipError_t mlp_bwd(const MlpCall& c);

hipError_t field_query(const spx_field* fields, int nfields, const spx_segment* segs, int nseg, int64_t total_tiles,
                       hipStream_t s);
hipError_t mse_grad(int64_t n, const float* y, const float* target, float* d_y, float scale, hipStream_t s);
hipError_t cast_f32_f16(int64_t n, const float* src, uint16_t* dst, hipStream_t s);
hipError_t encode_mlp_fwd(const spx_field& f, int64_t N, const float* pts, float* out, uint16_t* feats,
                          hipStream_t s);
hipError_t composite_fwd(int64_t R, int S, const float* raw, const float* delta, float* rgba, hipStream_t s);
hipError_t composite_bwd(int64_t R, int S, const float* raw, const float* delta, const float* d_rgba, float* d_raw,
                         hipStream_t s);
hipError_t gather_probe(const void* table, int64_t n_words, int64_t n_threads, int per_thread, uint32_t seed,
                        uint32_t* out, hipStream_t s);
hipError_t adam_step(int64_t n, float* param, float* grad, float* m, float* v, uint16_t* param_f16, float lr,
                     float beta1, float beta2, float eps, float bc1, float bc2, int zero_grad, hipStream_t s);

}  // namespace spx
