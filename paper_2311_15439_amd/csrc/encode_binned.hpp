// Binned adjoint of the encoding: the gradient scatter without global
// atomics.
//
// On MI355X a scattered binary32 atomic costs one L2 request per lane (about
// four times a scattered store), and atomics that pile onto one line
// serialise; the coarse levels of a multiresolution table send thousands of
// updates to each slot.  This path therefore sorts the contributions by slot
// range first and sums them in LDS:
//   count    every (point, level, vertex) contribution is assigned a bucket
//            (level, slot >> s); each workgroup counts its contributions per
//            bucket in LDS and writes its row of counts;
//   colscan  per bucket, exclusive prefix over workgroups, plus the bucket
//            total;
//   scan     exclusive prefix over bucket totals: where each bucket's
//            records start;
//   scatter  each workgroup recomputes its points' lookups and writes one
//            record {slot within the bucket, w * d_out[F]} per contribution
//            into its reserved range of the bucket: staged in LDS in bucket
//            order so that each bucket's records leave as a contiguous run
//            (the direct kernel, for shapes the staging does not fit, keeps
//            one LDS cursor per bucket);
//   coarse   levels whose whole vertex box fits in LDS are summed densely
//            per workgroup instead (no records, no hot buckets), on a side
//            stream beside the three kernels above;
//   accum    one workgroup per bucket adds its records into an LDS copy of
//            the bucket's 2^s slots, then adds that slice to d_tables with
//            coalesced read-modify-write (each slot is owned by exactly one
//            workgroup) -- or, in the fused variant, applies the Adam step
//            to the slice directly, so no gradient table is stored at all
//            (binned_accum.hpp).
// Levels are processed in groups when the bucket count or the record count
// of all levels together would not fit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "binned_accum.hpp"
#include "encode_kernels.hpp"
#include "mfma_mlp.hpp"

namespace spx {

constexpr int kBinBlock = 256;

// Record store that bypasses the caches' write-back: records are read only
// by the next kernel, and dirty lines left behind in L2 would be written back
// while that kernel streams the table state.  Only the staged scatter uses it,
// where a wave's stores form contiguous runs (scattered non-temporal stores
// would reach HBM as partial lines).
typedef float f32x3_a4 __attribute__((ext_vector_type(3), aligned(4)));
template <int F>
__device__ __forceinline__ void store_rec_nt(BinRec<F>* p, const BinRec<F>& r) {
    constexpr int W = sizeof(BinRec<F>) / 4;  // 32-bit words: 2, 3 or a power of two >= 4
    float w[W];
    w[0] = __builtin_bit_cast(float, r.slot);
#pragma unroll
    for (int j = 0; j < F; ++j) w[1 + j] = r.v[j];
#pragma unroll
    for (int j = F + 1; j < W; ++j) w[j] = 0.0f;
    if constexpr (W == 2) {
        __builtin_nontemporal_store(f32x2{w[0], w[1]}, reinterpret_cast<f32x2*>(p));
    } else if constexpr (W == 3) {
        __builtin_nontemporal_store(f32x3_a4{w[0], w[1], w[2]}, reinterpret_cast<f32x3_a4*>(p));
    } else {
#pragma unroll
        for (int c = 0; c < W / 4; ++c)
            __builtin_nontemporal_store(f32x4{w[4 * c], w[4 * c + 1], w[4 * c + 2], w[4 * c + 3]},
                                        reinterpret_cast<f32x4*>(p) + c);
    }
}

// Per-workgroup contiguous range of points.
__device__ __forceinline__ void bin_chunk(int64_t N, int64_t chunk, int64_t& lo, int64_t& hi) {
    lo = (int64_t)blockIdx.x * chunk;
    hi = lo + chunk < N ? lo + chunk : N;
}

// Is the cell (corner c, all vertices c + {0,1}^n) inside level l's dense
// box?  If so, write the dense index of its corner and the per-axis strides.
template <int D>
__device__ __forceinline__ bool dense_cell(const BinPlan& plan, int l, const int32_t (&c)[D], int32_t& e0,
                                           int32_t (&stride)[D]) {
    const int ext = plan.ext[l];
    bool in = true;
    int32_t e = plan.doff[l], st = 1;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        in = in && c[i] >= 0 && c[i] <= ext - 2;
        e += c[i] * st;
        stride[i] = st;
        st *= ext;
    }
    e0 = e;
    return in;
}

template <int D>
__device__ __forceinline__ int32_t dense_vertex(int32_t e0, const int32_t (&stride)[D], uint32_t offs) {
    int32_t e = e0;
#pragma unroll
    for (int i = 0; i < D; ++i) e += ((offs >> i) & 1u) ? stride[i] : 0;
    return e;
}

template <class Tag, int D>
__global__ __launch_bounds__(kBinBlock) void bin_count_kernel(int64_t N, const float* __restrict__ pts, LevelArgs lv,
                                                              BinPlan plan) {
    extern __shared__ uint32_t hist[];
    for (int b = threadIdx.x; b < plan.B; b += kBinBlock) hist[b] = 0;
    __syncthreads();
    int64_t lo, hi;
    bin_chunk(N, plan.chunk, lo, hi);
    for (int64_t pt = lo + threadIdx.x; pt < hi; pt += kBinBlock) {
        float y[D];
        load_point<Tag, D>(pts, pt, lv.Fn, y);
        for (int l = plan.l0; l < plan.l1; ++l) {
            const uint32_t bl = (uint32_t)plan.boff[l];
            visit_level_ex(Tag{}, y, lv.sigma[l], lv.rule(l),
                           [&](const auto& h, const auto& w, int, const auto& cell, const auto&) {
                constexpr int K = sizeof(w) / sizeof(float);
                int32_t e0, stride[D];
                if (l < plan.P && dense_cell<D>(plan, l, cell, e0, stride)) return;  // summed in LDS instead
#pragma unroll
                for (int k = 0; k < K; ++k) atomicAdd(&hist[bl + (h[k] >> plan.s_log2)], 1u);
            });
        }
    }
    __syncthreads();
    uint32_t* row = plan.counts + (size_t)blockIdx.x * plan.B;
    for (int b = threadIdx.x; b < plan.B; b += kBinBlock) row[b] = hist[b];
}

// Per bucket: exclusive prefix of the counts over workgroups, and the total.
// A block handles 64 buckets; 16 threads per bucket each take a contiguous
// segment of workgroups (at most 32: W <= 512), the 16 segment sums are
// scanned in LDS, and each thread then rewrites its segment as an exclusive
// prefix.  A thread's counts are loaded once, all at once (unconditional
// loads: a slot past its segment or a bucket past B reads entry 0 and is
// then taken as zero), and kept in registers between the two passes.
constexpr int kColBuckets = 64, kColSegs = 16;
constexpr int kColPer = 512 / kColSegs;  // workgroups per segment at most
static __global__ __launch_bounds__(kColBuckets * kColSegs) void bin_colscan_kernel(BinPlan plan,
                                                                                  uint32_t* __restrict__ totals) {
    __shared__ uint32_t seg[kColSegs][kColBuckets];
    const int lb = threadIdx.x % kColBuckets, sg = threadIdx.x / kColBuckets;
    const int b = blockIdx.x * kColBuckets + lb;
    const int per = (plan.W + kColSegs - 1) / kColSegs;
    const int w0 = sg * per, w1 = w0 + per < plan.W ? w0 + per : plan.W;
    uint32_t v[kColPer];
#pragma unroll
    for (int k = 0; k < kColPer; ++k) {
        const bool in = b < plan.B && w0 + k < w1;
        v[k] = plan.counts[in ? (size_t)(w0 + k) * plan.B + b : 0];
        v[k] = in ? v[k] : 0u;
    }
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kColPer; ++k) s += v[k];
    seg[sg][lb] = s;
    __syncthreads();
    uint32_t run = 0;
    for (int k = 0; k < sg; ++k) run += seg[k][lb];
    if (b < plan.B) {
#pragma unroll
        for (int k = 0; k < kColPer; ++k) {
            if (w0 + k < w1) plan.counts[(size_t)(w0 + k) * plan.B + b] = run;
            run += v[k];
        }
        if (sg == kColSegs - 1) totals[b] = run;
    }
}

// Exclusive scan of the bucket totals by one workgroup: base[b], base[B].
static __global__ __launch_bounds__(1024) void bin_scan_kernel(int B, const uint32_t* __restrict__ totals,
                                                        uint32_t* __restrict__ base) {
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    const int per = (B + 1023) / 1024;
    const int b0 = t * per, b1 = b0 + per < B ? b0 + per : B;
    uint32_t s = 0;
    for (int b = b0; b < b1; ++b) s += totals[b];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {  // inclusive Hillis-Steele scan of the 1024 partial sums
        const uint32_t v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = t > 0 ? part[t - 1] : 0u;
    for (int b = b0; b < b1; ++b) {
        base[b] = run;
        run += totals[b];
    }
    if (t == 1023) base[B] = part[1023];
}

template <class Tag, int D, int F, typename GT>
__global__ __launch_bounds__(kBinBlock) void bin_scatter_kernel(int64_t N, const float* __restrict__ pts,
                                                                const GT* __restrict__ d_out, LevelArgs lv,
                                                                BinPlan plan) {
    extern __shared__ uint32_t cursor[];
    const uint32_t* row = plan.counts + (size_t)blockIdx.x * plan.B;
    for (int b = threadIdx.x; b < plan.B; b += kBinBlock) cursor[b] = plan.base[b] + row[b];
    __syncthreads();
    BinRec<F>* __restrict__ recs = reinterpret_cast<BinRec<F>*>(plan.recs);
    const uint32_t smask = (1u << plan.s_log2) - 1u;
    int64_t lo, hi;
    bin_chunk(N, plan.chunk, lo, hi);
    for (int64_t pt = lo + threadIdx.x; pt < hi; pt += kBinBlock) {
        float y[D];
        load_point<Tag, D>(pts, pt, lv.Fn, y);
        const GT* __restrict__ grow = d_out + pt * (int64_t)(lv.L * F);
        for (int l = plan.l0; l < plan.l1; ++l) {
            float g[F];
            RowIO<GT, F>::load(grow + l * F, g);
            const uint32_t bl = (uint32_t)plan.boff[l];
            visit_level_ex(Tag{}, y, lv.sigma[l], lv.rule(l),
                           [&](const auto& h, const auto& w, int, const auto& cell, const auto&) {
                constexpr int K = sizeof(w) / sizeof(float);
                int32_t e0, stride[D];
                if (l < plan.P && dense_cell<D>(plan, l, cell, e0, stride)) return;  // summed in LDS instead
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const uint32_t pos = atomicAdd(&cursor[bl + (h[k] >> plan.s_log2)], 1u);
                    BinRec<F> r;
                    r.slot = h[k] & smask;
#pragma unroll
                    for (int j = 0; j < F; ++j) r.v[j] = w[k] * g[j];
                    recs[pos] = r;
                }
            });
        }
    }
}

// Staged scatter.  Written straight from the lookup, consecutive lanes send
// their records to unrelated buckets, so every record is a lone 16-byte store
// and the L2 fills and writes back partial lines.  Here a workgroup takes
// its points in rounds of kStageBlock * PPT; per round and level it counts its
// contributions per bucket in LDS (the atomic's return value is the
// record's rank within its bucket), scans the counts, places the records in
// LDS in bucket order, and then writes them out with consecutive threads on
// consecutive records: each bucket's records of the round form one
// contiguous run that continues where the workgroup's previous run ended.
// The records and their positions are the same as the direct kernel's, up to
// the order within a bucket (which the sums do not depend on beyond
// rounding).
//
// Two shapes, chosen per call.  Levels of many buckets (the image
// workload's 256 per level) need long rounds for their per-bucket runs to be
// long: 12 contributions per thread per round and eight levels of output
// gradient held per point, one workgroup per CU (154 registers).  Levels of
// few buckets (at most kStageFewBuckets: the volume workload's 32) have long
// runs anyway; there 10 contributions per thread and four levels of
// gradient fit two workgroups per CU (at most 128 registers), which hides
// more latency where cells have four or more vertices (volume step 2.22 ->
// 2.05 ms; with three vertices it was slower: image workload 1.65 -> 1.78
// ms, the n = 2 sweep's adjoint by 5 %).  The count pass takes the same
// shape, as it must see the same rounds.
constexpr int kStageBlock = 512;  // threads of the staged scatter (longer runs than kStageBlock)
constexpr int kStageFewBuckets = 64;
__host__ __device__ constexpr int stage_slots(bool few) { return few ? 10 : 12; }  // contributions per thread per round
__host__ __device__ constexpr int stage_gl(bool few) { return few ? 4 : 8; }       // levels of output gradient held per point
__host__ __device__ constexpr int stage_waves(bool few) { return few ? 4 : 1; }    // minimum waves per SIMD
// LDS budget of the staged kernel; configurations that need more use the
// direct kernel.
constexpr size_t kStageLdsMax = 150 * 1024;

template <int V, bool FEW>
constexpr int stage_ppt() { return V > stage_slots(FEW) ? 0 : stage_slots(FEW) / V; }

// LDS layout of the staged scatter (in 32-bit words): cursors [B], local
// counts/offsets [bmax + 1] (bmax: the most buckets of one level), staged
// keys [CAP], staged values [CAP * F].
struct StageLds {
    size_t cursor, loff, key, val, words;
};
__host__ __device__ inline size_t stage_round4(size_t w) { return (w + 3) & ~(size_t)3; }
template <int V, int F, bool FEW>
__host__ __device__ inline StageLds stage_lds(int B, int bpl) {
    constexpr size_t CAP = (size_t)kStageBlock * stage_ppt<V, FEW>() * V;
    StageLds s;
    s.cursor = 0;
    s.loff = stage_round4((size_t)B);
    s.key = s.loff + stage_round4((size_t)bpl + 1);
    s.val = s.key + CAP;
    s.words = s.val + CAP * F;
    return s;
}

// Staged record key: the slot within its bucket in the low 16 bits, the
// bucket within the level above (buckets hold 2^s <= 2^15 slots, and a level
// has at most 16384 buckets).
__device__ __forceinline__ uint32_t stage_key(uint32_t h, int s_log2, uint32_t smask) {
    return (h & smask) | ((h >> s_log2) << 16);
}

// Sums each run of equal keys across consecutive lanes into the run's last
// lane and drops the others' records (key = kNoKey).  Every lane of the
// wave must call it; a wave without runs (random points) returns after one
// ballot.
template <int F>
__device__ __forceinline__ void merge_run_wave(uint32_t& key, float (&v)[F]) {
    const uint64_t heads = __ballot(!joins_prev(key));
    if (heads == ~0ull) return;
    run_sums<F>(heads, v);
    if (!run_last(heads)) key = kNoKey;
}

// Count pass for the staged scatter: the same rounds, lanes and merged runs,
// so each workgroup reserves exactly the records it will write per bucket.
template <class Tag, int D, bool FEW, bool DENSE>
__global__ __launch_bounds__(kStageBlock) void bin_count_staged_kernel(int64_t N, const float* __restrict__ pts,
                                                                      LevelArgs lv, BinPlan plan) {
    constexpr int V = Tag::simplex ? D + 1 : (1 << D);
    constexpr int PPT = stage_ppt<V, FEW>();
    extern __shared__ uint32_t hist[];
    const int tid = threadIdx.x;
    for (int b = tid; b < plan.B; b += kStageBlock) hist[b] = 0;
    __syncthreads();
    const uint32_t smask = (1u << plan.s_log2) - 1u;
    int64_t lo, hi;
    bin_chunk(N, plan.chunk, lo, hi);
    for (int64_t r0 = lo; r0 < hi; r0 += (int64_t)kStageBlock * PPT) {
        float y[PPT][D];
        bool ok[PPT];
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int64_t pt = r0 + tid + (int64_t)j * kStageBlock;
            ok[j] = pt < hi;
            load_point<Tag, D>(pts, ok[j] ? pt : lo, lv.Fn, y[j]);
        }
        for (int l = plan.l0; l < plan.l1; ++l) {
            const uint32_t bl = (uint32_t)plan.boff[l];
            uint32_t key[PPT][V];
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
#pragma unroll
                for (int k = 0; k < V; ++k) key[j][k] = kNoKey;
                if (!ok[j]) continue;
                visit_level_ex(Tag{}, y[j], lv.sigma[l], lv.template rule_if<DENSE>(l),
                               [&](const auto& h, const auto& w, int base, const auto& cell, const auto&) {
                    constexpr int K = sizeof(w) / sizeof(float);
                    int32_t e0, stride[D];
                    if (l < plan.P && dense_cell<D>(plan, l, cell, e0, stride)) return;  // summed in LDS instead
#pragma unroll
                    for (int k = 0; k < K; ++k) key[j][base + k] = stage_key(h[k], plan.s_log2, smask);
                });
            }
#pragma unroll
            for (int j = 0; j < PPT; ++j)
#pragma unroll
                for (int k = 0; k < V; ++k) {
                    // every lane takes part in the shuffle, whether it holds a record or not
                    const bool joins = joins_prev(key[j][k]);
                    if (key[j][k] != kNoKey && !joins) atomicAdd(&hist[bl + (key[j][k] >> 16)], 1u);
                }
        }
    }
    __syncthreads();
    uint32_t* row = plan.counts + (size_t)blockIdx.x * plan.B;
    for (int b = tid; b < plan.B; b += kStageBlock) row[b] = hist[b];
}

// The network's input gradient (NET below): all kNetUnits units of a
// point, 16 levels of 2 features; transposed through LDS in rows of
// kNetRow floats (16 units, padded against bank conflicts).
constexpr int kNetUnits = 32;
constexpr int kNetRow = 20;

// LDS accesses of one wave to rows that other lanes of the same wave wrote:
// a wave's LDS instructions execute in order, so only the compiler's
// reordering has to be fenced.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// NET: the output gradient is not read from d_out but computed here, as the
// input gradient of the network (Sec. 5 steps (d)-(e)) that maps the
// encoding to the field: once per round, on the matrix cores, from the
// stored binary16 features and the network's output gradient.  Each wave
// takes its own points 16 at a time (lane (r, q) of a tile holds point r
// and units 4q..4q+3 of each 16-unit half), and a per-wave transpose through
// LDS hands every lane its point's 32 units, held in registers for the
// round.  The products are the ones the separate network backward makes
// (shared code), so the gradients are the same bits.  NET requires F = 2,
// 16 levels and a single level group (l0 = 0, l1 = 16).
template <class Tag, int D, int F, typename GT, bool FEW, bool DENSE, bool NET = false>
__global__ __launch_bounds__(kStageBlock, NET ? 2 : stage_waves(FEW)) void bin_scatter_staged_kernel(
    int64_t N, const float* __restrict__ pts, const GT* __restrict__ d_out, LevelArgs lv, BinPlan plan,
    NetArgs net) {
    constexpr int V = Tag::simplex ? D + 1 : (1 << D);
    constexpr int PPT = stage_ppt<V, FEW>();
    constexpr int GL = stage_gl(FEW);
    constexpr uint32_t kNone = kNoKey;
    static_assert(!NET || (F == 2 && kNetUnits % (GL * F) == 0), "the network covers 16 levels of 2 features");
    // the transpose rows of the 8 waves fit in the staging area (free between level passes)
    static_assert(!NET || (kStageBlock / 64) * 64 * kNetRow <= kStageBlock * PPT * V * (1 + F),
                  "transpose area exceeds the staging area");
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    __shared__ uint32_t wave_sum[kStageBlock / 64];
    const StageLds lay = stage_lds<V, F, FEW>(plan.B, plan.bmax);
    uint32_t* cursor = lds + lay.cursor;
    uint32_t* loff = lds + lay.loff;
    uint32_t* skey = lds + lay.key;
    float* sval = reinterpret_cast<float*>(lds + lay.val);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    const uint32_t* row = plan.counts + (size_t)blockIdx.x * plan.B;
    for (int b = tid; b < plan.B; b += kStageBlock) cursor[b] = plan.base[b] + row[b];
    // NET: the network's weight fragments, after the staging layout
    const uint4* frag = reinterpret_cast<const uint4*>(lds + lay.words);
    if constexpr (NET) {
        // from a copy of the weights in the staging area (free until the first level pass)
        static_assert(raw_copy_bytes<kNetUnits, kStageBlock>() <= kStageBlock * PPT * V * (1 + F) * 4,
                      "weights exceed the staging area");
        uint4* raw = reinterpret_cast<uint4*>(lds + lay.key);
        copy_weights_lds<kNetUnits, kStageBlock>(raw, net.W1, net.W2, net.W3, net.d_out, tid);
        __syncthreads();
        const _Float16* w = reinterpret_cast<const _Float16*>(raw);
        stage_bwd_frags<kNetUnits>(reinterpret_cast<uint4*>(lds + lay.words), w, w + H * kNetUnits,
                                   w + H * kNetUnits + H * H, net.d_out, wave, kStageBlock / 64, lane);
        __syncthreads();
    }
    BinRec<F>* __restrict__ recs = reinterpret_cast<BinRec<F>*>(plan.recs);
    const uint32_t smask = (1u << plan.s_log2) - 1u;
    int64_t lo, hi;
    bin_chunk(N, plan.chunk, lo, hi);
    for (int64_t r0 = lo; r0 < hi; r0 += (int64_t)kStageBlock * PPT) {
        float y[PPT][D];
        bool ok[PPT];
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const int64_t pt = r0 + tid + (int64_t)j * kStageBlock;
            ok[j] = pt < hi;
            load_point<Tag, D>(pts, ok[j] ? pt : lo, lv.Fn, y[j]);
        }
        float gall[NET ? PPT : 1][NET ? kNetUnits : 1];
        if constexpr (NET) {
            // the staging area is free here: the previous round's last
            // level pass ended with a barrier after its records left
            float* tr = reinterpret_cast<float*>(lds + lay.key) + wave * (64 * kNetRow);
            const int r = lane & 15, q = lane >> 4;
            // Tiles one after another (the scheduling barriers keep the
            // chains from being interleaved, which would hold several tiles'
            // activations at once), each tile's inputs loaded while the
            // previous tile computes: units 0..15 go to the transpose rows
            // at once, units 16..31 wait in registers.
            BwdTile<kNetUnits> tl;
            {
                const int64_t p = r0 + wave * 64 + r;
                tl.load(lane, net.x, net.d_y, net.d_out, p, p < hi);
            }
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
                f4 hi16[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    BwdTile<kNetUnits> nx;  // the next tile's inputs (this round's)
                    const int jn = k == 3 ? j + 1 : j, kn = k == 3 ? 0 : k + 1;
                    if (jn < PPT) {
                        const int64_t p = r0 + (int64_t)jn * kStageBlock + wave * 64 + 16 * kn + r;
                        nx.load(lane, net.x, net.d_y, net.d_out, p, p < hi);
                    }
                    tl.compute(frag, lane);
                    *reinterpret_cast<f4*>(tr + (16 * k + r) * kNetRow + 4 * q) = tl.dx(frag, lane, 0);
                    hi16[k] = tl.dx(frag, lane, 1);
                    __builtin_amdgcn_sched_barrier(0);
                    if (jn < PPT) {
#pragma unroll
                        for (int s2 = 0; s2 < BwdFrags<kNetUnits>::KS1; ++s2) tl.xb[s2] = nx.xb[s2];
                        tl.dyb = nx.dyb;
                    }
                }
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    if (h == 1) {
#pragma unroll
                        for (int k = 0; k < 4; ++k)
                            *reinterpret_cast<f4*>(tr + (16 * k + r) * kNetRow + 4 * q) = hi16[k];
                    }
                    wave_lds_sync();
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const f4 v = *reinterpret_cast<const f4*>(tr + lane * kNetRow + 4 * i);
#pragma unroll
                        for (int e = 0; e < 4; ++e) gall[j][16 * h + 4 * i + e] = v[e];
                    }
                    wave_lds_sync();
                }
            }
        }
        // The points' output gradients are read GL levels at a time
        // into registers: between two levels of the same point a whole round
        // passes, long enough for its row to leave L2, so reading one level
        // per visit would fetch each row's lines once per level.
        float gch[NET ? 1 : PPT][NET ? 1 : GL][F];
        for (int l = plan.l0; l < plan.l1; ++l) {
            const int li = (l - plan.l0) % GL;
            if (!NET && li == 0) {
#pragma unroll
                for (int j = 0; j < PPT; ++j) {
                    const int64_t pt = r0 + tid + (int64_t)j * kStageBlock;
                    const GT* __restrict__ grow = d_out + (ok[j] ? pt : lo) * (int64_t)(lv.L * F);
#pragma unroll
                    for (int q = 0; q < GL; ++q)
                        if (l + q < plan.l1) RowIO<GT, F>::load(grow + (l + q) * F, gch[j][q]);
                }
            }
            const uint32_t bl = (uint32_t)plan.boff[l];
            const int bpl = plan.boff[l + 1] - plan.boff[l];  // buckets of this level
            __syncthreads();  // the previous level's offsets are no longer read
            for (int b = tid; b <= bpl; b += kStageBlock) loff[b] = 0;
            __syncthreads();
            uint32_t key[PPT][V], rank[PPT][V];
            float val[PPT][V][F];
#pragma unroll
            for (int j = 0; j < PPT; ++j) {
#pragma unroll
                for (int k = 0; k < V; ++k) key[j][k] = kNone;
                if (!ok[j]) continue;
                float g[F];
                if constexpr (NET) {
                    // level l's units, selected from the round's registers
                    // (a copy per level group would double them)
#pragma unroll
                    for (int f = 0; f < F; ++f) g[f] = gall[j][f];
#pragma unroll
                    for (int q = 1; q < kNetUnits / F; ++q)
                        if (l == q)
#pragma unroll
                            for (int f = 0; f < F; ++f) g[f] = gall[j][q * F + f];
                } else {
#pragma unroll
                    for (int f = 0; f < F; ++f) g[f] = gch[j][0][f];
#pragma unroll
                    for (int q = 1; q < GL; ++q)
                        if (li == q)
#pragma unroll
                            for (int f = 0; f < F; ++f) g[f] = gch[j][q][f];
                }
                visit_level_ex(Tag{}, y[j], lv.sigma[l], lv.template rule_if<DENSE>(l),
                               [&](const auto& h, const auto& w, int base, const auto& cell, const auto&) {
                    constexpr int K = sizeof(w) / sizeof(float);
                    int32_t e0, stride[D];
                    if (l < plan.P && dense_cell<D>(plan, l, cell, e0, stride)) return;  // summed in LDS instead
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        key[j][base + k] = stage_key(h[k], plan.s_log2, smask);
#pragma unroll
                        for (int f = 0; f < F; ++f) val[j][base + k][f] = w[k] * g[f];
                    }
                });
            }
            // Consecutive lanes hold consecutive points: where they put the
            // same vertex at the same list position (samples along a ray in
            // one cell), the run is summed across lanes and leaves as one
            // record (the count kernel counted runs the same way); then each
            // kept record takes its rank within its bucket.
#pragma unroll
            for (int j = 0; j < PPT; ++j)
#pragma unroll
                for (int k = 0; k < V; ++k) {
                    merge_run_wave<F>(key[j][k], val[j][k]);
                    if (key[j][k] != kNone) rank[j][k] = atomicAdd(&loff[key[j][k] >> 16], 1u);
                }
            __syncthreads();
            // exclusive scan of the per-bucket counts; loff[bpl] = round total
            {
                const int per = (bpl + kStageBlock - 1) / kStageBlock;
                const int b0 = tid * per < bpl ? tid * per : bpl;
                const int b1 = b0 + per < bpl ? b0 + per : bpl;
                uint32_t sum = 0;
                for (int b = b0; b < b1; ++b) sum += loff[b];
                uint32_t inc = sum;
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) {
                    const uint32_t t = __shfl_up(inc, off, 64);
                    if (lane >= off) inc += t;
                }
                if (lane == 63) wave_sum[wave] = inc;
                __syncthreads();
                uint32_t run = inc - sum;
                for (int w = 0; w < wave; ++w) run += wave_sum[w];
                for (int b = b0; b < b1; ++b) {
                    const uint32_t c = loff[b];
                    loff[b] = run;
                    run += c;
                }
                if (tid == kStageBlock - 1) loff[bpl] = run;
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < PPT; ++j)
#pragma unroll
                for (int k = 0; k < V; ++k) {
                    if (key[j][k] == kNone) continue;
                    const uint32_t i = loff[key[j][k] >> 16] + rank[j][k];
                    skey[i] = key[j][k];
#pragma unroll
                    for (int f = 0; f < F; ++f) sval[i * F + f] = val[j][k][f];
                }
            __syncthreads();
            const uint32_t total = loff[bpl];
            for (uint32_t i = tid; i < total; i += kStageBlock) {
                const uint32_t kk = skey[i], b = kk >> 16;
                BinRec<F> r;
                r.slot = kk & smask;
#pragma unroll
                for (int f = 0; f < F; ++f) r.v[f] = sval[i * F + f];
                store_rec_nt<F>(&recs[cursor[bl + b] + (i - loff[b])], r);
            }
            __syncthreads();
            for (int b = tid; b < bpl; b += kStageBlock) cursor[bl + b] += loff[b + 1] - loff[b];
        }
    }
}

// Privatised coarse levels: each workgroup sums its points' contributions
// from in-box cells into a dense LDS array, then stores it as its partial.
// The point loop's bounds are uniform over the workgroup (lanes past the
// chunk idle) because the wave-level adds need every lane.
template <class Tag, int D, int F, typename GT>
__global__ __launch_bounds__(kBinBlock) void bin_coarse_kernel(int64_t N, const float* __restrict__ pts,
                                                               const GT* __restrict__ d_out, int64_t gstride,
                                                               LevelArgs lv, BinPlan plan) {
    extern __shared__ __attribute__((aligned(16))) float dacc[];
    const int n = plan.Dtot * F;
    for (int i = threadIdx.x; i < n; i += kBinBlock) dacc[i] = 0.0f;
    __syncthreads();
    int64_t lo, hi;
    bin_chunk(N, plan.chunk, lo, hi);
    for (int64_t p0 = lo; p0 < hi; p0 += kBinBlock) {
        const bool in = p0 + threadIdx.x < hi;
        const int64_t pt = in ? p0 + threadIdx.x : lo;
        float y[D];
        load_point<Tag, D>(pts, pt, lv.Fn, y);
        const GT* __restrict__ grow = d_out + pt * gstride;
        for (int l = 0; l < plan.P; ++l) {
            float g[F];
            RowIO<GT, F>::load(grow + l * F, g);
            visit_level_ex(Tag{}, y, lv.sigma[l], lv.rule(l),
                           [&](const auto& h, const auto& w, int, const auto& cell, const auto& offs) {
                constexpr int K = sizeof(w) / sizeof(float);
                int32_t e0, stride[D];
                // cells outside the box are emitted as records instead
                const bool ok = dense_cell<D>(plan, l, cell, e0, stride) && in;
                // Lanes in different cells almost never share a vertex at the
                // same list position.  The run merging costs about as much as
                // a few retried adds, so it is used when at least 8 lanes share
                // their cell with the lane before them (a wave-uniform test):
                // coherent points, not the odd pair of random ones.
                const uint32_t ck = ok ? (uint32_t)e0 : 0xFFFFFFFFu;
                const bool coherent =
                    __popcll(__ballot(ok && joins_prev(ck))) >= 8;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    float v[F];
#pragma unroll
                    for (int j = 0; j < F; ++j) v[j] = w[k] * g[j];
                    const uint32_t e = (uint32_t)dense_vertex<D>(e0, stride, offs[k]);
                    if (coherent) {
                        lds_add_wave<F>(dacc, ok, e, v);
                    } else if (ok) {
                        lds_add_row<F>(&dacc[e * F], v);
                    }
                }
            });
        }
    }
    __syncthreads();
    float* __restrict__ out = plan.partial + (size_t)blockIdx.x * n;
    for (int i = threadIdx.x; i < n; i += kBinBlock) out[i] = dacc[i];
}

// Sum of the workgroups' dense partials.  A block owns 64 entries; 16
// thread rows each add a contiguous segment of workgroups (at most 32), and
// the segment sums are added in order (the result does not depend on
// scheduling).  A thread's partials are loaded all at once (unconditional
// loads, as in the column scan) and then added in workgroup order.
static __global__ __launch_bounds__(kColBuckets * kColSegs) void bin_coarse_reduce_kernel(BinPlan plan, int n) {
    __shared__ float seg[kColSegs][kColBuckets];
    const int li = threadIdx.x % kColBuckets, sg = threadIdx.x / kColBuckets;
    const int i = blockIdx.x * kColBuckets + li;
    const int per = (plan.W + kColSegs - 1) / kColSegs;
    const int w0 = sg * per, w1 = w0 + per < plan.W ? w0 + per : plan.W;
    float v[kColPer];
#pragma unroll
    for (int k = 0; k < kColPer; ++k) {
        const bool in = i < n && w0 + k < w1;
        v[k] = plan.partial[in ? (size_t)(w0 + k) * n + i : 0];
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kColPer; ++k)
        if (i < n && w0 + k < w1) s += v[k];
    seg[sg][li] = s;
    __syncthreads();
    if (sg != 0 || i >= n) return;
    float t = 0.0f;
    for (int k = 0; k < kColSegs; ++k) t += seg[k][li];
    plan.gdense[i] = t;
}

// The fused network backward covers 16 levels of 2 features in 1 to 3
// dimensions, one level group and a staged scatter whose LDS (with the
// network's weight fragments) fits the CU.
constexpr size_t kNetLdsMax = 160 * 1024 - 256;  // beside the kernel's static LDS

template <int V, int F>
inline size_t staged_lds_bytes(int B, int bmax, bool few) {
    return (few ? stage_lds<V, F, true>(B, bmax) : stage_lds<V, F, false>(B, bmax)).words * sizeof(uint32_t);
}

// The fused scatter runs in the shape with more points per thread whatever
// the bucket count: its registers hold the round's network gradients, so it
// runs one workgroup per CU either way, and the longer rounds give longer
// runs of records.  (The count pass's shape does not change what it counts:
// the runs it merges are those of aligned 64-point rows in either shape.)
template <int V, int F>
inline size_t net_lds_bytes(int B, int bmax) {
    return staged_lds_bytes<V, F>(B, bmax, false) + BwdFrags<kNetUnits>::BYTES;
}

// Shape of a group's count pass and scatter: the staged scatter (when its
// LDS fits) merges runs of one slot across lanes, and its count pass counts
// the merged records the same way, in the same shape (few buckets per level
// or many).
template <int V, int F>
struct ScatterShape {
    bool few, staged;
    size_t staged_lds;
    explicit ScatterShape(const BinPlan& p) : few(p.bmax <= kStageFewBuckets && V >= 4), staged(false), staged_lds(0) {
        if constexpr (stage_ppt<V, false>() >= 1 && stage_ppt<V, true>() >= 1) {
            staged_lds = staged_lds_bytes<V, F>(p.B, p.bmax, few);
            staged = staged_lds <= kStageLdsMax;
        }
    }
};

// The part of a group's adjoint that depends only on the points: records
// counted per (workgroup, bucket), the column scan and the scan of the
// bucket totals, which lay out every record's place in the workspace.
template <class Tag, int D, int F>
hipError_t bin_prepare_group(const EncodeCall& c, const BinPlan& p, uint32_t* totals) {
    constexpr int V = Tag::simplex ? D + 1 : (1 << D);
    const ScatterShape<V, F> sh(p);
    const double N = (double)c.N, counts = (double)p.W * p.B * 4.0;
    trace_begin(c.stream, "bin_count", N * 4.0 * D + counts);
    // Without a densely stored level the staged kernels never compute dense
    // rows (they are bound by vector instructions where runs are merged).
    const bool dense = c.lv.dense != 0;
    const bool few = sh.few;
    if (sh.staged) {
        if constexpr (stage_ppt<V, false>() >= 1 && stage_ppt<V, true>() >= 1) {
            const size_t lds = p.B * sizeof(uint32_t);
            if (few && dense)
                bin_count_staged_kernel<Tag, D, true, true><<<p.W, kStageBlock, lds, c.stream>>>(c.N, c.pts, c.lv, p);
            else if (few)
                bin_count_staged_kernel<Tag, D, true, false><<<p.W, kStageBlock, lds, c.stream>>>(c.N, c.pts, c.lv, p);
            else if (dense)
                bin_count_staged_kernel<Tag, D, false, true><<<p.W, kStageBlock, lds, c.stream>>>(c.N, c.pts, c.lv, p);
            else
                bin_count_staged_kernel<Tag, D, false, false><<<p.W, kStageBlock, lds, c.stream>>>(c.N, c.pts, c.lv, p);
        }
    } else {
        bin_count_kernel<Tag, D><<<p.W, kBinBlock, p.B * sizeof(uint32_t), c.stream>>>(c.N, c.pts, c.lv, p);
    }
    trace_end(c.stream);
    trace_begin(c.stream, "bin_colscan", 2.0 * counts + 4.0 * p.B);
    bin_colscan_kernel<<<(p.B + kColBuckets - 1) / kColBuckets, kColBuckets * kColSegs, 0, c.stream>>>(p, totals);
    trace_end(c.stream);
    trace_begin(c.stream, "bin_scan", 8.0 * p.B + 4.0);
    bin_scan_kernel<<<1, 1024, 0, c.stream>>>(p.B, totals, p.base);
    trace_end(c.stream);
    return hipGetLastError();
}

// One level group of the adjoint; `prepared`: its count and scans were run
// by a preceding prepare call on the same points and workspace.
template <class Tag, int D, int F, typename GT>
hipError_t binned_adjoint_group(const EncodeCall& c, const BinPlan& p, uint32_t* totals, bool prepared) {
    const GT* d_out = (const GT*)c.d_out;
    constexpr int V = Tag::simplex ? D + 1 : (1 << D);
    constexpr bool kNetOk = F == 2 && D <= 3;
    const bool net = c.net.x != nullptr;
    const double N = (double)c.N, gs = sizeof(GT);
    const double counts = (double)p.W * p.B * 4.0;
    // the method's scatter payload: one binary32 value per point, level,
    // vertex and feature (however many records carry it)
    const double payload = N * (p.l1 - p.l0) * V * F * 4.0;
    const ScatterShape<V, F> sh(p);
    const bool few = sh.few, staged = sh.staged;
    const size_t staged_lds = sh.staged_lds;
    if (net && (!kNetOk || !staged || net_lds_bytes<V, F>(p.B, p.bmax) > kNetLdsMax))
        return hipErrorNotSupported;  // checked by the caller before any launch
    if (!prepared) {
        const hipError_t e = bin_prepare_group<Tag, D, F>(c, p, totals);
        if (e != hipSuccess) return e;
    }
    const bool dense = c.lv.dense != 0;
    // The privatised coarse levels depend only on the points and the output
    // gradient, and their sums are needed only by the accumulation: they run
    // on a side stream beside the scatter (LDS-atomic bound beside store
    // bound) and are joined before the accumulation.  They are forked after
    // the scan: forked earlier, their workgroups hold every CU and the
    // one-workgroup scan waits for them to drain.
    std::unique_lock<std::mutex> aux_lock;
    AuxStream* aux = nullptr;
    if (p.P > 0) {
        aux = aux_stream(aux_lock);
        hipStream_t cs = c.stream;
        if (aux && (hipEventRecord(aux->fork, c.stream) != hipSuccess ||
                    hipStreamWaitEvent(aux->s, aux->fork, 0) != hipSuccess))
            aux = nullptr;  // run the coarse levels in order on the caller's stream
        if (aux) cs = aux->s;
        const int n = p.Dtot * F;
        const int64_t gstride = net ? c.net.coarse_stride : (int64_t)c.lv.L * F;
        trace_begin(cs, "bin_coarse", N * (4.0 * D + p.P * F * gs) + (double)p.W * n * 4.0);
        bin_coarse_kernel<Tag, D, F, GT><<<p.W, kBinBlock, (size_t)n * sizeof(float), cs>>>(c.N, c.pts, d_out, gstride,
                                                                                            c.lv, p);
        trace_end(cs);
        trace_begin(cs, "bin_coarse_reduce", ((double)p.W + 1.0) * n * 4.0);
        bin_coarse_reduce_kernel<<<(n + kColBuckets - 1) / kColBuckets, kColBuckets * kColSegs, 0, cs>>>(p, n);
        trace_end(cs);
        if (aux) {
            const hipError_t e = hipEventRecord(aux->join, aux->s);
            if (e != hipSuccess) return e;
        }
    }
    if (net) {
        // features and network output gradient in, instead of the output gradient
        trace_begin(c.stream, "bin_scatter_net",
                    N * (4.0 * D + 2.0 * kNetUnits + 4.0 * c.net.d_out) + counts + payload);
        if constexpr (kNetOk && std::is_same<GT, float>::value && stage_ppt<V, false>() >= 1 &&
                      stage_ppt<V, true>() >= 1) {
            const size_t lds = net_lds_bytes<V, F>(p.B, p.bmax);
            if (dense)
                bin_scatter_staged_kernel<Tag, D, F, GT, false, true, true><<<p.W, kStageBlock, lds, c.stream>>>(
                    c.N, c.pts, d_out, c.lv, p, c.net);
            else
                bin_scatter_staged_kernel<Tag, D, F, GT, false, false, true><<<p.W, kStageBlock, lds, c.stream>>>(
                    c.N, c.pts, d_out, c.lv, p, c.net);
        }
    } else {
        trace_begin(c.stream, "bin_scatter", N * (4.0 * D + (p.l1 - p.l0) * F * gs) + counts + payload);
        if (staged) {
            if constexpr (stage_ppt<V, false>() >= 1 && stage_ppt<V, true>() >= 1) {
                if (few && dense)
                    bin_scatter_staged_kernel<Tag, D, F, GT, true, true><<<p.W, kStageBlock, staged_lds, c.stream>>>(
                        c.N, c.pts, d_out, c.lv, p, c.net);
                else if (few)
                    bin_scatter_staged_kernel<Tag, D, F, GT, true, false><<<p.W, kStageBlock, staged_lds, c.stream>>>(
                        c.N, c.pts, d_out, c.lv, p, c.net);
                else if (dense)
                    bin_scatter_staged_kernel<Tag, D, F, GT, false, true><<<p.W, kStageBlock, staged_lds, c.stream>>>(
                        c.N, c.pts, d_out, c.lv, p, c.net);
                else
                    bin_scatter_staged_kernel<Tag, D, F, GT, false, false><<<p.W, kStageBlock, staged_lds, c.stream>>>(
                        c.N, c.pts, d_out, c.lv, p, c.net);
            }
        } else
            bin_scatter_kernel<Tag, D, F, GT><<<p.W, kBinBlock, p.B * sizeof(uint32_t), c.stream>>>(c.N, c.pts, d_out,
                                                                                                    c.lv, p);
    }
    trace_end(c.stream);
    if (aux) {
        const hipError_t e = hipStreamWaitEvent(c.stream, aux->join, 0);
        if (e != hipSuccess) return e;
    }
    return launch_accum<D, F>(c, p, payload);
}

template <class Tag, int D, int F>
hipError_t binned_adjoint(const EncodeCall& c) {
    BinLayout lay = bin_layout(c.D, c.F, c.N, Tag::simplex, c.lv);
    char* ws = (char*)c.workspace;
    if (c.net.x || c.net.check_only) {
        // the fused network backward: checked before anything is launched
        constexpr int V = Tag::simplex ? D + 1 : (1 << D);
        if constexpr (F != 2 || D > 3 || stage_ppt<V, false>() < 1 || stage_ppt<V, true>() < 1) {
            return hipErrorNotSupported;
        } else {
            if (!lay.ok || lay.groups != 1 || c.lv.L * F != kNetUnits || c.dout_f16) return hipErrorNotSupported;
            int B = 0, bmax = 0;  // the one group's buckets, as its plan counts them
            for (int l = 0; l < lay.L; ++l) {
                B += lay.nb[l];
                bmax = lay.nb[l] > bmax ? lay.nb[l] : bmax;
            }
            const bool few = bmax <= kStageFewBuckets && V >= 4;
            if (staged_lds_bytes<V, F>(B, bmax, few) > kStageLdsMax || net_lds_bytes<V, F>(B, bmax) > kNetLdsMax)
                return hipErrorNotSupported;
        }
        if (c.net.check_only) return hipSuccess;
    }
    if (c.op == EncodeOp::AdjointPrepare) {
        if (!lay.ok || c.net.x) return hipErrorInvalidValue;
        BinPlan p = bin_plan(lay, 0, ws);
        return bin_prepare_group<Tag, D, F>(c, p, (uint32_t*)(ws + lay.off_totals));
    }
    for (int g = 0; g < lay.groups; ++g) {
        BinPlan p = bin_plan(lay, g, ws);
        uint32_t* totals = (uint32_t*)(ws + lay.off_totals);
        const bool prepared = c.prepared && g == 0;
        hipError_t e = c.dout_f16 ? binned_adjoint_group<Tag, D, F, f16>(c, p, totals, prepared)
                                  : binned_adjoint_group<Tag, D, F, float>(c, p, totals, prepared);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace spx
