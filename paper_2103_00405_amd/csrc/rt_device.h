// rt_device.h -- device-side wrappers of the numeric core for the kernels.
#pragma once
#define RT_HD __device__ __forceinline__
#define RT_LOG_CONST __constant__
#include <hip/hip_runtime.h>

#include "rt_math.h"

// Read-only launch data (network tables, item descriptors, prefix sums, the
// sample grid) read through the constant address space: the compiler may
// then treat the loads as invariant and, where the address is uniform, issue
// them as scalar loads into SGPRs.  Only for memory that no kernel of the
// launch writes.  (The host pass of this single-source file only parses the
// kernels; it sees plain pointers.)
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using rt_cptr = const __attribute__((address_space(4))) T*;
#else
template <typename T>
using rt_cptr = const T*;
#endif

template <typename T>
__device__ __forceinline__ rt_cptr<T> rt_const(const T* p)
{
    return (rt_cptr<T>)p;
}

// RN(-ln u) for the wave's active lanes.  The fast phase runs in every lane;
// lanes whose rounding it cannot certify (about one draw in 2^17) take turns
// on the wave's LDS slice sc (RT_LOG_SCRATCH words) for the accurate phase
// and add one to the device counter *slow.
__device__ __forceinline__ double rt_neglog_wave(uint64_t m, bool force_accurate,
                                                 unsigned long long* slow, uint32_t* sc)
{
    int e, i;
    double z;
    rt_neglog_reduce(m, e, i, z);
    double y = 0.0;
    bool need = m != 0x1FFFFFFFFFFFFFull;                     // u = 1 gives +0
    if (need && !force_accurate) {
        double yh, yl;
        rt_neglog_fast(e, i, z, yh, yl);
        y = yh;
        need = !rt_rounding_certain(yh, yl);
    }
    unsigned long long pending = __ballot(need);
    if (__builtin_expect(pending != 0ull, 0)) {
        const int me = (int)(threadIdx.x & 63u);
        while (pending) {
            const int lane = __ffsll((long long)pending) - 1;
            if (lane == me) {
                y = rt_neglog_accurate(e, i, z, sc);
                atomicAdd(slow, 1ull);
            }
            pending &= pending - 1ull;
        }
    }
    return y;
}

// RN(-ln u) when every active lane holds the same m (a draw computed by a
// whole wavefront for one channel): the accurate phase, when needed, runs
// once in the first active lane and its result is broadcast; *slow counts
// one per draw.
__device__ __forceinline__ double rt_neglog_uniform(uint64_t m, unsigned long long* slow,
                                                    uint32_t* sc)
{
    int e, i;
    double z;
    rt_neglog_reduce(m, e, i, z);
    double y = 0.0;
    bool need = m != 0x1FFFFFFFFFFFFFull;                     // u = 1 gives +0
    if (need) {
        double yh, yl;
        rt_neglog_fast(e, i, z, yh, yl);
        y = yh;
        need = !rt_rounding_certain(yh, yl);
    }
    if (__builtin_expect(__ballot(need) != 0ull, 0)) {
        const unsigned long long active = __ballot(true);
        const int first = __ffsll((long long)active) - 1;
        if ((int)(threadIdx.x & 63u) == first) {
            y = rt_neglog_accurate(e, i, z, sc);
            atomicAdd(slow, 1ull);
        }
        y = __shfl(y, first, 64);
    }
    return y;
}

__device__ __forceinline__ double rt_exp1_wave(uint32_t k0, uint32_t k1, uint32_t traj,
                                               uint32_t net, uint32_t k, uint32_t n,
                                               unsigned long long* slow, uint32_t* sc)
{
    return rt_neglog_wave(rt_draw_m53(k0, k1, traj, net, k, n), false, slow, sc);
}

// E for channel k at firing index n, computed by every active lane alike.
__device__ __forceinline__ double rt_exp1_uniform(uint32_t k0, uint32_t k1, uint32_t traj,
                                                  uint32_t net, uint32_t k, uint32_t n,
                                                  unsigned long long* slow, uint32_t* sc)
{
    return rt_neglog_uniform(rt_draw_m53(k0, k1, traj, net, k, n), slow, sc);
}
