// rt_device.h -- device-side wrappers of the numeric core for the kernels.
#pragma once
#define RT_HD __device__ __forceinline__
#define RT_LOG_CONST __constant__
#include <hip/hip_runtime.h>

#include "internal.h"
#include "rt_math.h"

constexpr uint32_t kTieNone = 0xFFFFFFFFu;                 // tie_step of a path without near-ties
constexpr unsigned long long kFnvOffset = 0xcbf29ce484222325ull;   // seq_hash start
constexpr unsigned long long kFnvPrime = 0x100000001b3ull;         // seq_hash multiplier

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

// ---------------------------------------------------------------------
// Arithmetic of one channel and of the selection, shared by every kernel.

// RN((double)h) for h < 2^64: both halves convert exactly, one rounding.
__device__ __forceinline__ double rt_u64_to_f64(uint64_t h)
{
    return fma((double)(uint32_t)(h >> 32), 0x1p32, (double)(uint32_t)h);
}

// a_k = RN(c_k RN(h_k(X))) of Eq. 1-2 with h_k = prod_j C(X_j, sigma_jk)
// exact in 64-bit integers (C(X, 2) = X(X - 1) / 2); kind, s0 and s1 come
// from the reactant table (RT_H_*), x(j) reads species j.  One-species h is
// below 2^32 and converts exactly without the two-part form.
template <class XGet>
__device__ __forceinline__ double rt_propensity(int kind, int s0, int s1, double c, XGet x)
{
    uint64_t h;
    if (kind == RT_H_ZERO) {
        h = 1;
    } else if (kind == RT_H_ONE) {
        return c * (double)(uint32_t)x(s0);
    } else if (kind == RT_H_PAIR) {
        const uint32_t v = (uint32_t)x(s0);
        h = ((uint64_t)v * (uint32_t)(v - 1u)) >> 1;   // v = 0 gives 0
    } else {
        h = (uint64_t)(uint32_t)x(s0) * (uint32_t)x(s1);
    }
    return c * rt_u64_to_f64(h);
}

// The same from the reactant counts v0 = X_s0 and v1 = X_s1 (read only as
// the kind needs them), as selects rather than branches: lanes of one
// wavefront holding channels of different kinds take one path.  One-species h
// converts exactly either way, so the value is the one above.
__device__ __forceinline__ double rt_propensity_counts(int kind, uint32_t v0, uint32_t v1, double c)
{
    const uint64_t pair = ((uint64_t)v0 * (uint32_t)(v0 - 1u)) >> 1;
    const uint64_t two = (uint64_t)v0 * v1;
    const uint64_t h = kind == RT_H_ZERO ? 1ull
                     : kind == RT_H_ONE ? (uint64_t)v0
                     : kind == RT_H_PAIR ? pair : two;
    return c * rt_u64_to_f64(h);
}

// The same with X in memory (LDS) and the packed reactant-table entry
// rr = (s0 | kind << 29, s1), in the select form.
__device__ __forceinline__ double rt_propensity_mem(int2 rr, double c, const int32_t* X)
{
    const int kind = (int)((uint32_t)rr.x >> 29);
    int32_t v0 = 0, v1 = 0;
    if (kind != RT_H_ZERO) v0 = X[rr.x & RT_SPECIES_MASK];
    if (kind == RT_H_TWO) v1 = X[rr.y];
    return rt_propensity_counts(kind, (uint32_t)v0, (uint32_t)v1, c);
}

// The near-tie rule (Eq. 4 gives ties probability zero; in binary64 the two
// smallest gaps d1 <= d2 can still round within reach of each other):
// RN(d2 - d1) <= RN(1e-12 d1).
__device__ __forceinline__ bool rt_near_tie(double d1, double d2)
{
    return d2 - d1 <= 1e-12 * d1;
}

// Orders the wavefront's LDS accesses (the hardware completes them in order
// for one wavefront; this keeps the compiler from reordering them).
__device__ __forceinline__ void rt_wave_lds_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Index of the item owning global unit u: unit_start[i] <= u < unit_start[i+1].
__device__ __forceinline__ int rt_find_item(rt_cptr<int64_t> unit_start, int count, int64_t u)
{
    int lo = 0, hi = count;   // unit_start[lo] <= u < unit_start[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (unit_start[mid] <= u) lo = mid; else hi = mid;
    }
    return lo;
}

// RN(-ln u) for the wave's active lanes.  The fast phase runs in every lane;
// lanes whose rounding it cannot certify (about one draw in 2^17) take turns
// on the wave's LDS slice sc (RT_LOG_SCRATCH words) for the accurate phase;
// each such lane adds one to the device counter *slow, or, with slow = NULL,
// sets *took_slow instead (for a draw that may be discarded and counted only
// once it is used).
__device__ __forceinline__ double rt_neglog_wave(uint64_t m, bool force_accurate,
                                                 unsigned long long* slow, uint32_t* sc,
                                                 bool* took_slow = nullptr)
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
    if (took_slow) *took_slow = need;
    unsigned long long pending = __ballot(need);
    if (__builtin_expect(pending != 0ull, 0)) {
        const int me = (int)(threadIdx.x & 63u);
        while (pending) {
            const int lane = __ffsll((long long)pending) - 1;
            if (lane == me) {
                y = rt_neglog_accurate(e, i, z, sc);
                if (slow) atomicAdd(slow, 1ull);
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
