// device_common.hpp -- device helpers shared by the DROP sweep kernels:
// cross-lane sums, the wavefront-aggregated touched-list append and the
// bounded device-wide barrier of the persistent sweeps.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstdint>

namespace tvs {
namespace dev {

// Spin bound of one barrier wait (about 4 s); on expiry the barrier raises
// its error flag so that every workgroup leaves and the host reports it.
constexpr uint32_t kSpinLimit = 1u << 22;

template <typename CH>
__device__ inline float chord_at(const CH *p, int64_t e)
{
    if constexpr (sizeof(CH) == 4) return p[e];
    else return __half2float(p[e]);
}

// Sum over groups of LPR consecutive lanes (LPR a power of two <= 64).
template <int LPR>
__device__ inline double group_sum(double v)
{
#pragma unroll
    for (int o = LPR / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Appends j to the touched list when `first`; one atomic per wavefront.
__device__ inline void append_touched(bool first, int32_t j, int32_t *touched, uint32_t *cnt)
{
    unsigned long long m = __ballot(first);
    if (m == 0) return;
    int lane = threadIdx.x & 63;
    int leader = __ffsll((long long)m) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(cnt, (uint32_t)__popcll(m));
    base = __shfl(base, leader, 64);
    if (first) {
        unsigned long long below = m & ((1ull << lane) - 1ull);
        touched[base + (uint32_t)__popcll(below)] = j;
    }
}

// Device-wide barrier of a persistent launch whose workgroups are all
// resident: bar[0] = arrivals, bar[1] = generation, bar[2] = error flag.
// The last arriving workgroup resets the arrival count and bumps the
// generation; the others wait (relaxed polling, one acquire fence after)
// for the generation to change.  Returns false once the error flag is up.
__device__ inline bool grid_barrier(uint32_t *bar)
{
    __shared__ uint32_t ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t good = 1;
        __threadfence();
        uint32_t gen = __hip_atomic_load(bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t arrived =
            __hip_atomic_fetch_add(bar, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1u;
        if (arrived == gridDim.x) {
            __hip_atomic_store(bar, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(bar + 1, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            uint32_t spins = 0;
            while (__hip_atomic_load(bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                if (__hip_atomic_load(bar + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                    good = 0;
                    break;
                }
                if (++spins > kSpinLimit) {
                    __hip_atomic_store(bar + 2, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    good = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __threadfence();
        ok = good;
    }
    __syncthreads();
    return ok != 0u;
}

}  // namespace dev
}  // namespace tvs
