// Accumulation step of the binned adjoint: one workgroup per bucket sums
// the bucket's records into an LDS copy of its 2^s slots, then either adds
// the slice to the gradient table or applies the Adam step to it (each slot
// is owned by exactly one workgroup, so both are plain coalesced
// read-modify-writes).  Also defines the record format the scatter writes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "encode_kernels.hpp"
#include "wave_runs.hpp"

namespace spx {

// One record per contribution: slot within the bucket and the F values.
// F = 1 and F = 2 records are unpadded (8 and 12 bytes: one 64- or 96-bit
// access, and a wave's run of records is contiguous); wider ones are padded
// to a power of two.
template <int F>
struct alignas(F == 1 ? 8 : F == 2 ? 4 : F == 4 ? 32 : 64) BinRec {
    uint32_t slot;
    float v[F];
};

// Float add into LDS.  On this chip the LDS float-add instruction keeps the
// LDS busy for about 200 cycles per wave, a 32-bit compare-and-swap for a
// small fraction of that, so the add is a compare-and-swap loop: one pass
// unless another lane changed the word in between, in which case the lane
// retries with the value it saw.
__device__ __forceinline__ void lds_add(float* p, float v) {
    uint32_t* q = reinterpret_cast<uint32_t*>(p);
    uint32_t seen = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    uint32_t want;
    do {
        want = __float_as_uint(__uint_as_float(seen) + v);
    } while (!__hip_atomic_compare_exchange_strong(q, &seen, want, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP));
}

// Adds a row of F floats.  Pairs of floats go through one 64-bit
// compare-and-swap (the LDS takes about as long for it as for a 32-bit one,
// so a two-feature row costs one retry loop instead of two); each float
// is still the plain binary32 sum of the old value and the addend.
template <int F>
__device__ __forceinline__ void lds_add_row(float* row, const float (&v)[F]) {
    if constexpr (F == 1) {
        lds_add(row, v[0]);
    } else {
#pragma unroll
        for (int j = 0; j < F; j += 2) {
            uint64_t* q = reinterpret_cast<uint64_t*>(row + j);
            uint64_t seen = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            uint64_t want;
            do {
                const float lo = __uint_as_float((uint32_t)seen) + v[j];
                const float hi = __uint_as_float((uint32_t)(seen >> 32)) + v[j + 1];
                want = (uint64_t)__float_as_uint(lo) | ((uint64_t)__float_as_uint(hi) << 32);
            } while (!__hip_atomic_compare_exchange_strong(q, &seen, want, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_WORKGROUP));
        }
    }
}

constexpr int kAccBlock = 1024;  // one workgroup per CU (128 KiB accumulator)
// Records loaded per thread before their LDS adds.  With the fused Adam
// step one: the preloaded state holds 96 registers through the record
// phase, and two records were no faster and spilled.  Without it (the
// gradient-table variant) the registers are free and four loads per thread
// are in flight at once: a bucket's record phase is a loop of dependent
// load-then-add steps, paced by the loads' latency.
template <bool ADAM>
constexpr int acc_unroll() { return ADAM ? 1 : 4; }

// Adam update of four parameters with their summed gradients (the same
// binary32 operation sequence as the standalone Adam kernel).
__device__ __forceinline__ void adam4(const AdamArgs& a, f32x4 g, f32x4& p, f32x4& m, f32x4& v, f16x4& h) {
#pragma clang fp contract(off)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        m[q] = a.b1 * m[q] + (1.0f - a.b1) * g[q];
        v[q] = a.b2 * v[q] + (1.0f - a.b2) * g[q] * g[q];
        p[q] = p[q] - a.lr * (m[q] * a.inv_bc1) / (sqrtf(v[q] * a.inv_bc2) + a.eps);
        h[q] = (f16)p[q];
    }
}

// Adds one value per lane (F floats at acc[slot * F]) to an LDS
// accumulator.  Spatially coherent points (samples along a ray) put runs of
// lanes on the same slot, and a compare-and-swap add retries once per lane
// that got in first.  So when any lane holds the same slot as the lane
// before it, the wave first sums each run of equal slots across lanes (a
// segmented scan) and only the run's last lane adds the sum.  The sums group
// the same terms in a different order.  Every lane of the wave must call it.
template <int F>
__device__ __forceinline__ void lds_add_wave(float* acc, bool ok, uint32_t slot, const float (&val)[F]) {
    const uint32_t key = ok ? slot : kNoKey;
    const bool joins = joins_prev(key);
    const uint64_t heads = __ballot(!joins);
    if (heads == ~0ull) {
        if (ok) lds_add_row<F>(&acc[slot * F], val);
        return;
    }
    float v[F];
#pragma unroll
    for (int j = 0; j < F; ++j) v[j] = val[j];
    run_sums<F>(heads, v);
    if (ok && run_last(heads)) lds_add_row<F>(&acc[slot * F], v);
}

// The same update of one entry, in place (binary32 state, optional binary16
// copy of the parameter).
__device__ __forceinline__ void adam1(const AdamArgs& a, float g, size_t i) {
#pragma clang fp contract(off)
    const float m = a.b1 * a.m[i] + (1.0f - a.b1) * g;
    const float v = a.b2 * a.v[i] + (1.0f - a.b2) * g * g;
    const float p = a.param[i] - a.lr * (m * a.inv_bc1) / (sqrtf(v * a.inv_bc2) + a.eps);
    a.m[i] = m;
    a.v[i] = v;
    a.param[i] = p;
    if (a.param_f16) ((f16*)a.param_f16)[i] = (f16)p;
}

// A bucket's records are stored in point order, so runs of records for one
// slot come from coherent points.
template <int F>
__device__ __forceinline__ void add_record_wave(float* acc, bool ok, const BinRec<F>& rec) {
    lds_add_wave<F>(acc, ok, rec.slot, rec.v);
}

// U records per thread in flight before their LDS adds; the loop bounds
// are uniform over the workgroup (lanes past the end idle).  The loads are
// unconditional (a lane past the end rereads record rb, which exists) so
// that all of them are issued before the first wait.
template <int F, int U>
__device__ __forceinline__ void accum_records(float* acc, const BinRec<F>* __restrict__ recs, uint32_t r0,
                                              uint32_t r1) {
    for (uint32_t rb = r0; rb < r1; rb += U * kAccBlock) {
        BinRec<F> rec[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t r = rb + threadIdx.x + u * kAccBlock;
            ok[u] = r < r1;
            rec[u] = recs[ok[u] ? r : rb];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) add_record_wave<F>(acc, ok[u], rec[u]);
    }
}

constexpr int kAccPre = 8;  // float4 chunks of the slice a thread preloads

template <int D, int F, bool ADAM>
__global__ __launch_bounds__(kAccBlock) void bin_accum_kernel(BinPlan plan, LevelArgs lv, float* __restrict__ d_tables,
                                                              AdamArgs adam) {
    extern __shared__ __attribute__((aligned(16))) float acc[];
    const int S = 1 << plan.s_log2;
    int l = plan.l0;  // the level this workgroup works on (uniform over the workgroup)
    while (l + 1 < plan.l1 && (int)blockIdx.x >= plan.voff[l + 1]) ++l;
    // bucket `slice` of level l; a split bucket's workgroups take parts of it
    const int K = plan.ks[l];
    const int local = (int)blockIdx.x - plan.voff[l];
    const int slice = local / K, part = local - slice * K;
    const int b = plan.boff[l] + slice;
    // slots of this bucket: a whole 2^s slice, or the rest of a level whose
    // rows are not a multiple of it (a densely stored level)
    const int64_t left = (int64_t)lv.rows[l] - (int64_t)slice * S;
    const int cnt = left < S ? (int)left : S;
    const size_t off = ((size_t)lv.off[l] + (size_t)slice * S) * F;
    const int n4 = cnt * F / 4;
    const float* base_ptr = ADAM ? adam.param : d_tables;
    const bool vec = K == 1 && n4 * 4 == cnt * F && ((uintptr_t)(base_ptr + off) & 15) == 0 &&
                     n4 <= kAccPre * kAccBlock;
    // The slice's state does not depend on the records: issue its loads first
    // so they overlap the record phase.
    f32x4 P[kAccPre], M[kAccPre], Vv[kAccPre];
    if (vec) {
#pragma unroll
        for (int c = 0; c < kAccPre; ++c) {
            const int i = threadIdx.x + c * kAccBlock;
            if (i < n4) {
                // read once per step: non-temporal, so they do not displace the records
                P[c] = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(base_ptr + off) + i);
                if constexpr (ADAM) {
                    M[c] = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(adam.m + off) + i);
                    Vv[c] = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(adam.v + off) + i);
                }
            }
        }
    }
    for (int i = threadIdx.x; i < S * F; i += kAccBlock) acc[i] = 0.0f;
    __syncthreads();
    // privatised level: pick up the dense sums whose slot falls in this bucket
    // (a densely stored level numbers its rows over the same box)
    if (l < plan.P && part == 0) {
        const int ext = plan.ext[l];
        const SlotRule rule = lv.rule(l);
        const uint32_t want = (uint32_t)slice, smask = (uint32_t)S - 1u;
        for (int e = plan.doff[l] + threadIdx.x; e < plan.doff[l + 1]; e += kAccBlock) {
            int32_t rem = e - plan.doff[l];
            uint32_t h = (uint32_t)rem;
            if (rule.dext == 0) {
                h = 0;
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    h ^= (uint32_t)(rem % ext) * hash_prime(i);
                    rem /= ext;
                }
                h &= rule.mask;
            }
            if ((h >> plan.s_log2) != want) continue;
#pragma unroll
            for (int j = 0; j < F; ++j) {
                const float g = plan.gdense[(size_t)e * F + j];
                if (g != 0.0f) lds_add(&acc[(h & smask) * F + j], g);
            }
        }
    }
    const BinRec<F>* __restrict__ recs = reinterpret_cast<const BinRec<F>*>(plan.recs);
    uint32_t r0 = plan.base[b], r1 = plan.base[b + 1];
    if (K > 1) {  // part `part` of K equal parts of the bucket's records
        const uint64_t n = r1 - r0;
        r1 = r0 + (uint32_t)(n * (uint64_t)(part + 1) / (uint64_t)K);
        r0 = r0 + (uint32_t)(n * (uint64_t)part / (uint64_t)K);
    }
    // A bucket of many records (64 or more per thread: the volume
    // workload's fine levels) is bound by its record phase; there four
    // records per thread are in flight even beside the preloaded state
    // (128 registers, no spill).
    if (ADAM && r1 - r0 >= 64u * kAccBlock)
        accum_records<F, 4>(acc, recs, r0, r1);
    else
        accum_records<F, acc_unroll<ADAM>()>(acc, recs, r0, r1);
    __syncthreads();
    if (K > 1) {  // a part of a split bucket: its sums go to its partial slice
        float* __restrict__ dst = plan.split + (size_t)(plan.soff[l] + (int64_t)slice * K + part) * ((size_t)F << plan.s_log2);
        for (int i = threadIdx.x; i < cnt * F; i += kAccBlock) dst[i] = acc[i];
        return;
    }
    if (vec) {
#pragma unroll
        for (int c = 0; c < kAccPre; ++c) {
            const int i = threadIdx.x + c * kAccBlock;
            if (i >= n4) break;
            const f32x4 g = reinterpret_cast<const f32x4*>(acc)[i];
            if constexpr (!ADAM) {
                reinterpret_cast<f32x4*>(d_tables + off)[i] = P[c] + g;
            } else {
                f16x4 h;
                adam4(adam, g, P[c], M[c], Vv[c], h);
                reinterpret_cast<f32x4*>(adam.param + off)[i] = P[c];
                reinterpret_cast<f32x4*>(adam.m + off)[i] = M[c];
                reinterpret_cast<f32x4*>(adam.v + off)[i] = Vv[c];
                if (adam.param_f16) reinterpret_cast<f16x4*>((f16*)adam.param_f16 + off)[i] = h;
            }
        }
    } else {
        for (int i = threadIdx.x; i < cnt * F; i += kAccBlock) {
            const float g = acc[i];
            if constexpr (!ADAM)
                d_tables[off + i] += g;
            else
                adam1(adam, g, off + i);
        }
    }
}

// Second pass over the split buckets: each entry's partial sums added in
// part order (the result does not depend on scheduling), then the same
// update as an unsplit bucket's.  kSplitChunks workgroups per bucket.
constexpr int kSplitBlock = 256, kSplitChunks = 32;
template <int F, bool ADAM>
__global__ __launch_bounds__(kSplitBlock) void bin_split_finish_kernel(BinPlan plan, LevelArgs lv,
                                                                      float* __restrict__ d_tables, AdamArgs adam) {
    const int S = 1 << plan.s_log2;
    const int sb = (int)blockIdx.x / kSplitChunks, c = (int)blockIdx.x - sb * kSplitChunks;
    int l = plan.l0;  // levels without split buckets have sboff[l + 1] == sboff[l]
    while (l + 1 < plan.l1 && sb >= plan.sboff[l + 1]) ++l;
    const int K = plan.ks[l];
    const int slice = sb - plan.sboff[l];
    const int64_t left = (int64_t)lv.rows[l] - (int64_t)slice * S;
    const int cnt = left < S ? (int)left : S;
    const size_t off = ((size_t)lv.off[l] + (size_t)slice * S) * F;
    const size_t stride = (size_t)F << plan.s_log2;
    const float* __restrict__ src = plan.split + (size_t)(plan.soff[l] + (int64_t)slice * K) * stride;
    for (int i = c * kSplitBlock + threadIdx.x; i < cnt * F; i += kSplitChunks * kSplitBlock) {
        float g = src[i];
        for (int k = 1; k < K; ++k) g += src[(size_t)k * stride + i];
        if constexpr (!ADAM)
            d_tables[off + i] += g;
        else
            adam1(adam, g, off + i);
    }
}

// Launch of the accumulation for one level group.  Its algorithmic bytes
// (for the trace) are the method's scatter payload (4 bytes per point,
// level, vertex and feature) plus the update of every table entry.
template <int D, int F>
hipError_t launch_accum(const EncodeCall& c, const BinPlan& p, double payload) {
    double slots = 0.0;  // table entries of the group's levels
    for (int l = p.l0; l < p.l1; ++l) slots += (double)c.lv.rows[l] * F;
    const size_t lds = (size_t)(F << p.s_log2) * sizeof(float);
    if (c.adam.param) {
        trace_begin(c.stream, "bin_accum_adam", payload + slots * (c.adam.param_f16 ? 26.0 : 24.0));
        bin_accum_kernel<D, F, true><<<p.VB, kAccBlock, lds, c.stream>>>(p, c.lv, nullptr, c.adam);
        if (p.nsplit > 0)
            bin_split_finish_kernel<F, true><<<p.nsplit * kSplitChunks, kSplitBlock, 0, c.stream>>>(p, c.lv, nullptr,
                                                                                                  c.adam);
    } else {
        trace_begin(c.stream, "bin_accum", payload + slots * 8.0);
        bin_accum_kernel<D, F, false><<<p.VB, kAccBlock, lds, c.stream>>>(p, c.lv, c.d_tables, c.adam);
        if (p.nsplit > 0)
            bin_split_finish_kernel<F, false><<<p.nsplit * kSplitChunks, kSplitBlock, 0, c.stream>>>(p, c.lv,
                                                                                                   c.d_tables, c.adam);
    }
    trace_end(c.stream);
    return hipGetLastError();
}

}  // namespace spx
