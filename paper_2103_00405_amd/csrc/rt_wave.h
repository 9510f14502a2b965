// rt_wave.h -- argmin with second minimum across the lanes of a wavefront,
// by VALU lane exchanges only (no LDS crossbar).
//
// The selection of Eq. 25 (smallest internal-time gap, lowest channel on
// ties) runs as an all-reduce over groups of W = 2..64 aligned lanes:
//   W >= 2   DPP quad_perm [1,0,3,2]     (partner lane ^ 1)
//   W >= 4   DPP quad_perm [2,3,0,1]     (partner lane ^ 2)
//   W >= 8   DPP row_half_mirror         (lane i <-> 7 - i in each half row)
//   W >= 16  DPP row_mirror              (lane i <-> 15 - i in each row)
//   W >= 32  v_permlane16_swap           (rows 0 <-> 1 and 2 <-> 3)
//   W == 64  v_permlane32_swap           (lanes 0..31 <-> 32..63)
// After the first two steps a quad holds one value, after the mirrors a row;
// the swaps leave every lane with one value from each side of the pair.  The
// merge is commutative, so every lane of the group ends with the same
// result.  Every lane of a group must be active.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// (d1, d2, k): smallest gap, second smallest gap (order statistic with
// multiplicity) and the channel k of the smallest gap (lowest k on ties).
// Gaps are never NaN.
struct rt_min2 {
    double d1, d2;
    int32_t k;
};

__device__ __forceinline__ rt_min2 rt_min2_empty()
{
    return rt_min2{__builtin_inf(), __builtin_inf(), 0x7FFFFFFF};
}

// Adds channel k with gap d to a lane-local minimum; channels must come in
// increasing k so that the first of equal gaps is kept.
__device__ __forceinline__ void rt_min2_push(rt_min2& v, double d, int k)
{
    const bool lt = d < v.d1;
    v.d2 = fmin(v.d2, fmax(v.d1, d));
    v.d1 = fmin(v.d1, d);
    v.k = lt ? k : v.k;
}

// The two smallest gaps of the union of two disjoint channel sets.
__device__ __forceinline__ rt_min2 rt_min2_merge(const rt_min2& a, const rt_min2& b)
{
    rt_min2 r;
    r.d1 = fmin(a.d1, b.d1);
    r.d2 = fmin(fmin(a.d2, b.d2), fmax(a.d1, b.d1));
    r.k = a.d1 < b.d1 ? a.k : (b.d1 < a.d1 ? b.k : min(a.k, b.k));
    return r;
}

template <int CTRL>
__device__ __forceinline__ int32_t rt_dpp(int32_t x)
{
    return __builtin_amdgcn_mov_dpp(x, CTRL, 0xF, 0xF, false);
}

template <int CTRL>
__device__ __forceinline__ double rt_dpp_f64(double x)
{
    const int32_t lo = rt_dpp<CTRL>(__double2loint(x));
    const int32_t hi = rt_dpp<CTRL>(__double2hiint(x));
    return __hiloint2double(hi, lo);
}

template <int CTRL>
__device__ __forceinline__ rt_min2 rt_min2_dpp_step(const rt_min2& v)
{
    rt_min2 o;
    o.d1 = rt_dpp_f64<CTRL>(v.d1);
    o.d2 = rt_dpp_f64<CTRL>(v.d2);
    o.k = rt_dpp<CTRL>(v.k);
    return rt_min2_merge(v, o);
}

// One swap step: x from both sides of the lane pair.
template <int ROWS>
__device__ __forceinline__ void rt_swap(uint32_t x, uint32_t& p, uint32_t& q)
{
    if (ROWS == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
        p = r[0];
        q = r[1];
    } else {
        const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
        p = r[0];
        q = r[1];
    }
}

template <int ROWS>
__device__ __forceinline__ double rt_swap_f64(double x, double& other)
{
    uint32_t plo, qlo, phi, qhi;
    rt_swap<ROWS>((uint32_t)__double2loint(x), plo, qlo);
    rt_swap<ROWS>((uint32_t)__double2hiint(x), phi, qhi);
    other = __hiloint2double((int)qhi, (int)qlo);
    return __hiloint2double((int)phi, (int)plo);
}

template <int ROWS>
__device__ __forceinline__ rt_min2 rt_min2_swap_step(const rt_min2& v)
{
    rt_min2 p, q;
    p.d1 = rt_swap_f64<ROWS>(v.d1, q.d1);
    p.d2 = rt_swap_f64<ROWS>(v.d2, q.d2);
    uint32_t pk, qk;
    rt_swap<ROWS>((uint32_t)v.k, pk, qk);
    p.k = (int32_t)pk;
    q.k = (int32_t)qk;
    return rt_min2_merge(p, q);
}

// All-reduce over aligned groups of W lanes (W a power of two, 1..64).
template <int W>
__device__ __forceinline__ rt_min2 rt_min2_allreduce(rt_min2 v)
{
    if (W >= 2) v = rt_min2_dpp_step<0xB1>(v);     // quad_perm [1,0,3,2]
    if (W >= 4) v = rt_min2_dpp_step<0x4E>(v);     // quad_perm [2,3,0,1]
    if (W >= 8) v = rt_min2_dpp_step<0x141>(v);    // row_half_mirror
    if (W >= 16) v = rt_min2_dpp_step<0x140>(v);   // row_mirror
    if (W >= 32) v = rt_min2_swap_step<16>(v);
    if (W >= 64) v = rt_min2_swap_step<32>(v);
    return v;
}

// A lane that pushed its slots s (channel lane + s L) in increasing order
// names its channel: slot -> lane + slot L (empty stays empty).
__device__ __forceinline__ rt_min2 rt_min2_slot_to_channel(rt_min2 v, int lane, int log2L)
{
    v.k = v.k == 0x7FFFFFFF ? v.k : lane + (v.k << log2L);
    return v;
}

// All-reduce over a workgroup of L = 64 W threads: the wavefront all-reduce,
// then the W wavefront results through LDS (wave_min[W]) behind one
// workgroup barrier, which every thread of the group must reach; every lane
// reads partial (lane mod W), so the groups of W lanes all reduce the same W
// values and every thread returns the same result.
template <int L>
__device__ __forceinline__ rt_min2 rt_min2_group_allreduce(rt_min2 v, rt_min2* wave_min)
{
    constexpr int W = L / 64;
    v = rt_min2_allreduce<64>(v);
    if constexpr (W > 1) {
        if ((threadIdx.x & 63u) == 0) wave_min[threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if constexpr (W > 1) v = rt_min2_allreduce<W>(wave_min[threadIdx.x & (W - 1)]);
    return v;
}

// ---------------------------------------------------------------------
// Selection in two single-value reductions, for a workgroup whose lanes hold
// lane-local (d1, d2, channel): d1 <= d2 the two smallest gaps of the lane
// (>= 0 or +inf, never NaN), channel the lowest one holding d1.  The
// smallest gap and its channel are exact; the second smallest is carried
// only where it can decide the near-tie rule: a part's d2 is exact when it
// lies within reach of the part's d1 (d2 <= d1 + 2 RN(1e-12 d1)), else +inf.
// The returned d2 is then exact whenever the near-tie test can hold, and
// otherwise no smaller than the true second minimum and out of reach, so
// rt_near_tie(d1, d2) decides exactly as on the true values.

__device__ __forceinline__ double rt_min_sel(double a, double b) { return b < a ? b : a; }

// A 64-bit value of the wavefront's first active lane, known to the compiler
// as the same in every lane (so that what depends on it stays scalar).
__device__ __forceinline__ unsigned long long rt_first_lane_u64(unsigned long long v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

// Smallest value over the wavefront, in every lane.
__device__ __forceinline__ double rt_wave_min_f64(double v)
{
    v = rt_min_sel(v, rt_dpp_f64<0xB1>(v));              // quad_perm [1,0,3,2]
    v = rt_min_sel(v, rt_dpp_f64<0x4E>(v));              // quad_perm [2,3,0,1]
    v = rt_min_sel(v, rt_dpp_f64<0x141>(v));             // row_half_mirror
    v = rt_min_sel(v, rt_dpp_f64<0x140>(v));             // row_mirror
    double q;
    double p = rt_swap_f64<16>(v, q);
    v = rt_min_sel(p, q);
    p = rt_swap_f64<32>(v, q);
    return rt_min_sel(p, q);
}

struct rt_sel_part {
    double d1, d2;
    int32_t k, pad;
};

// The wavefront's part (every lane of the wavefront active).
__device__ __forceinline__ rt_sel_part rt_select_wave(double d1, double d2, int32_t ch)
{
    const int lane = (int)(threadIdx.x & 63u);
    rt_sel_part p;
    p.d1 = rt_wave_min_f64(d1);
    p.pad = 0;
    const unsigned long long own = __ballot(d1 == p.d1);
    if (__builtin_expect(__popcll(own) == 1, 1)) {
        const int ol = __ffsll((long long)own) - 1;
        p.k = __builtin_amdgcn_readlane(ch, ol);
        // candidates for the second smallest: the owner's second, every
        // other lane's smallest; reduced only when one is within reach
        const double cand = lane == ol ? d2 : d1;
        const double reach = p.d1 + 2.0 * (1e-12 * p.d1);
        p.d2 = __builtin_inf();
        if (p.d1 != __builtin_inf() && __ballot(cand <= reach) != 0ull)
            p.d2 = rt_wave_min_f64(cand);
    } else {
        // several lanes hold the smallest value (or every value is +inf): the
        // lowest channel among them; the second smallest equals the smallest
        unsigned long long m = own;
        int32_t k = 0x7FFFFFFF;
        while (m) {
            const int l = __ffsll((long long)m) - 1;
            k = min(k, (int32_t)__builtin_amdgcn_readlane(ch, l));
            m &= m - 1ull;
        }
        p.k = k;
        p.d2 = p.d1;
    }
    return p;
}

// The union of two parts: b wins on a smaller d1 or an equal one with a
// lower channel; the loser's d1 joins the candidates for the second smallest.
__device__ __forceinline__ rt_sel_part rt_sel_merge(const rt_sel_part& a, const rt_sel_part& b)
{
    const bool bw = (b.d1 < a.d1) | ((b.d1 == a.d1) & (b.k < a.k));
    rt_sel_part r;
    r.d1 = bw ? b.d1 : a.d1;
    r.k = bw ? b.k : a.k;
    r.d2 = rt_min_sel(bw ? b.d2 : a.d2, bw ? a.d1 : b.d1);
    r.pad = 0;
    return r;
}

// The workgroup's selection (L = 64 W threads, all reaching the one barrier
// inside; part: W entries of LDS, not read by another selection until every
// thread has passed this one's barrier).  Every thread returns the same.
template <int L>
__device__ __forceinline__ rt_min2 rt_select_group(double d1, double d2, int32_t ch,
                                                   rt_sel_part* part)
{
    constexpr int W = L / 64;
    const rt_sel_part p = rt_select_wave(d1, d2, ch);
    if constexpr (W == 1) {
        __syncthreads();
        return rt_min2{p.d1, p.d2, p.k};
    } else {
        if ((threadIdx.x & 63u) == 0) part[threadIdx.x >> 6] = p;
        __syncthreads();
        // every part at once, merged as a tree (the merge is commutative)
        rt_sel_part q[W];
#pragma unroll
        for (int w = 0; w < W; ++w) q[w] = part[w];
#pragma unroll
        for (int h = 1; h < W; h <<= 1)
#pragma unroll
            for (int w = 0; w + h < W; w += 2 * h) q[w] = rt_sel_merge(q[w], q[w + h]);
        return rt_min2{q[0].d1, q[0].d2, q[0].k};
    }
}
