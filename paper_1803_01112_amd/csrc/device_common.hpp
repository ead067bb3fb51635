// device_common.hpp -- device helpers shared by the DROP kernels of the
// single-image and batched sweeps.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstdint>
#include <type_traits>

#include "tvs_internal.hpp"

namespace tvs {
namespace dev {

constexpr uint32_t kNoRow = 0xffffffffu;

// Row (within its block) of an entry tag.
__device__ inline uint32_t row_of(const TileBlock &t, uint32_t m)
{
    return (m >> kTileShift) & t.rowmask;
}

// Chord of entry e (index into the block's arrays) with tag m: float32,
// float16, or fixed point (the low 16 bits of the code in chq, the high bits
// in the tag above the row field) in units of qunit mm.
template <typename CH>
__device__ inline float entry_chord(const TileBlock &t, int64_t e, uint32_t m)
{
    if constexpr (sizeof(CH) == 4) {
        return t.ch32[e];
    } else if constexpr (std::is_same<CH, uint16_t>::value) {
        const uint32_t code = ((m >> t.qshift) << 16) | (uint32_t)t.chq[e];
        return (float)((double)code * t.qunit);
    } else {
        return __half2float(t.ch16[e]);
    }
}

// Wavefront bookkeeping for sums over runs of equal keys: lanes holding the
// same key in consecutive lanes form a run (the entries of one row inside
// one tile are consecutive in its list).
struct Runs {
    int start;     // first lane of this lane's run
    bool tail;     // this lane ends its run
};

__device__ inline Runs wave_runs(uint32_t key)
{
    const int lane = threadIdx.x & 63;
    const uint32_t prev = __shfl_up(key, 1, 64);
    const uint32_t next = __shfl_down(key, 1, 64);
    const bool head = (lane == 0) || (prev != key);
    const unsigned long long heads = __ballot(head);
    const unsigned long long upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
    Runs r;
    r.start = 63 - __clzll((long long)(heads & upto));
    r.tail = (lane == 63) || (next != key);
    return r;
}

// Inclusive sum of v over the lanes of this lane's run up to this lane
// (integers: exact, so the total does not depend on how runs are cut).
__device__ inline long long run_sum(long long v, const Runs &r)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const long long o = __shfl_up(v, d, 64);
        if (lane - d >= r.start) v += o;
    }
    return v;
}

}  // namespace dev
}  // namespace tvs
