// Runs of equal keys across the lanes of a 64-wide wave, summed without
// going through the LDS.
//
// Coherent points (samples along a ray, neighbouring pixels) put runs of
// consecutive lanes on the same table slot.  Summing each run across lanes
// before it is added or written out turns many updates of one address into
// one.  The lane moves here are DPP operand modifiers (a VALU instruction
// reads another lane's register directly), not ds_bpermute, which goes
// through the LDS and competes with the LDS traffic of the kernels that use
// these helpers.  The run structure itself is one ballot: the bit mask of
// the lanes that begin a run.
//
// Every lane of the wave must call these functions (full exec mask).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spx {

// DPP controls of GFX9 (wave64): shift right by n lanes within each row of
// 16; broadcast lane 15 of each row to the next row; broadcast lane 31 to
// rows 2 and 3; shift right by one lane across the whole wave.
constexpr int kDppRowShr = 0x110;
constexpr int kDppRowBcast15 = 0x142;
constexpr int kDppRowBcast31 = 0x143;
constexpr int kDppWaveShr1 = 0x138;

// The value of `v` in the lane before this one; lane 0 receives `first`.
__device__ __forceinline__ uint32_t lane_before(uint32_t v, uint32_t first) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)first, (int)v, kDppWaveShr1, 0xf, 0xf, false);
}

constexpr uint32_t kNoKey = 0xFFFFFFFFu;

// Does this lane continue the run of the lane before it (same key, both
// holding one; kNoKey marks a lane without a record)?
__device__ __forceinline__ bool joins_prev(uint32_t key) {
    const uint32_t prev = lane_before(key, kNoKey);  // read by every lane, whatever its key
    return (key != kNoKey) & (prev == key);
}

// value from the lane `CTRL` names (0 where the control gives no source or
// masks the row out)
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_take(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xf, false));
}

// Each step is skipped when no lane of the wave adds in it (runs shorter
// than the step's reach, or not crossing the rows it joins): one scalar
// test against several vector instructions per value.
template <int OFF, int F>
__device__ __forceinline__ void run_row_step(float (&v)[F], int lane, int start) {
    const bool add = (lane & 15) >= OFF && lane - OFF >= start;
    if (__ballot(add) == 0) return;
#pragma unroll
    for (int j = 0; j < F; ++j) {
        const float t = dpp_take<kDppRowShr + OFF, 0xf>(v[j]);
        if (add) v[j] += t;
    }
}

// Inclusive sums of v over each run, given `heads` (bit i set when lane i
// begins a run; bit 0 always set).  Afterwards the last lane of a run holds
// the run's sum.  Steps of a Hillis-Steele scan: shifts by 1, 2, 4, 8
// within rows of 16 lanes, then lane 15 of rows 0 and 2 into rows 1 and 3,
// then lane 31 into rows 2 and 3; a lane adds only values from its own run.
template <int F>
__device__ __forceinline__ void run_sums(uint64_t heads, float (&v)[F]) {
    const int lane = threadIdx.x & 63;
    const int start = 63 - __clzll(heads & (~0ull >> (63 - lane)));  // first lane of this lane's run
    run_row_step<1>(v, lane, start);
    run_row_step<2>(v, lane, start);
    run_row_step<4>(v, lane, start);
    run_row_step<8>(v, lane, start);
    const bool add15 = (lane & 16) != 0 && start < (lane & ~15);
    if (__ballot(add15) != 0) {
#pragma unroll
        for (int j = 0; j < F; ++j) {
            const float t = dpp_take<kDppRowBcast15, 0xa>(v[j]);
            if (add15) v[j] += t;
        }
    }
    const bool add31 = lane >= 32 && start < 32;
    if (__ballot(add31) != 0) {
#pragma unroll
        for (int j = 0; j < F; ++j) {
            const float t = dpp_take<kDppRowBcast31, 0xc>(v[j]);
            if (add31) v[j] += t;
        }
    }
}

// Is this lane the last of its run?
__device__ __forceinline__ bool run_last(uint64_t heads) {
    const int lane = threadIdx.x & 63;
    return lane == 63 || ((heads >> (lane + 1)) & 1ull) != 0;
}

}  // namespace spx
