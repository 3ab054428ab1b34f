// Measurement reference (not part of the method): uniformly random 4-byte
// gathers from a buffer of a given size.  Its rate at a table level's
// footprint is the memory system's random-access gather rate there, the
// ceiling against which the encoding's gathers are reported.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spx_internal.h"

namespace spx {
namespace {

constexpr int kProbeBlock = 256;
constexpr int kInFlight = 16;  // independent loads issued before their sum

// Counter-based 32-bit mixer (the finaliser of MurmurHash3): a well-mixed
// word per (seed, thread, k) with no state between threads.
__device__ inline uint32_t mix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

__global__ __launch_bounds__(kProbeBlock) void gather_probe_kernel(const uint32_t* __restrict__ table,
                                                                   uint32_t mask, int64_t n_threads, int rounds,
                                                                   uint32_t seed, uint32_t* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * kProbeBlock + threadIdx.x;
    if (t >= n_threads) return;
    uint32_t key = mix32(seed ^ mix32((uint32_t)t ^ (uint32_t)(t >> 32) * 0x9e3779b1u));
    uint32_t acc = 0;
    for (int r = 0; r < rounds; ++r) {
        uint32_t v[kInFlight];
#pragma unroll
        for (int k = 0; k < kInFlight; ++k) {
            key = mix32(key + 0x632be5abu);
            v[k] = table[key & mask];
        }
#pragma unroll
        for (int k = 0; k < kInFlight; ++k) acc += v[k];
    }
    out[t] = acc;
}

}  // namespace

hipError_t gather_probe(const void* table, int64_t n_words, int64_t n_threads, int per_thread, uint32_t seed,
                        uint32_t* out, hipStream_t s) {
    const int rounds = per_thread / kInFlight;
    const int64_t blocks = (n_threads + kProbeBlock - 1) / kProbeBlock;
    trace_begin(s, "gather_probe", 4.0 * (double)n_threads * (double)(rounds * kInFlight + 1));
    gather_probe_kernel<<<(unsigned)blocks, kProbeBlock, 0, s>>>((const uint32_t*)table, (uint32_t)(n_words - 1),
                                                                 n_threads, rounds, seed, out);
    trace_end(s);
    return hipGetLastError();
}

}  // namespace spx
