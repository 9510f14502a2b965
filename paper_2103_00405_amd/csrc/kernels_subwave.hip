// kernels_subwave.hip -- L lanes per trajectory (L = 4 .. 64), 64 / L
// trajectories per wavefront, for mid-size networks.
//
// Channel k of a trajectory belongs to lane k mod L of its group, slot k / L;
// T_k, P_k, a_k and 1/a_k live in that lane's VGPRs (slots past the
// network's M are frozen channels that never win).  Each group has its own
// species counts X, firing counts n_k and one stale word per lane (bit s:
// slot s must recompute its propensity) in LDS.  The groups of a
// wavefront advance in lockstep, one firing per pass, but each group runs its
// own trajectory: the expensive per-firing tail (one Philox block and one
// correctly rounded logarithm for the fired channel, Eq. 26) runs in one lane
// per group, so a wavefront pays it once for 64 / L firings, and it runs
// while the fired channel's fixed-stride rows (its jump and the channels of
// D(mu), the lazy form's rows) load in one round trip.  There are no
// workgroup barriers: a group lives inside one wavefront, whose LDS accesses
// complete in program order.
//
// Work units are trajectories of the class's items, taken from a device
// counter by one lane per group; every rare event (start or end of a
// trajectory, a sample point, a near-tie, a clamped gap, an overflow, the
// firing cap) is handled in a branch entered only when some group needs it.
// With piecewise-constant rates (SCHED, Eq. 28), a rate breakpoint passed by
// a group's next firing is one more such event: the group's clocks run to the
// breakpoint at the old rates (a pending event with no fired channel) and
// every slot turns stale, so the next pass takes the new rates.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "rt_device.h"
#include "rt_wave.h"

namespace {

constexpr int kBlock = 256;

// Waves per SIMD the register allocation must allow: 2.  With 8 slots of
// channel state, the fired channel's rows and its early draw, 3 waves would
// spill to scratch (40-80 bytes per lane); at 2 the classes of 9-64 and
// 65-128 channels of a 4096-network batch ran 20 and 15 % faster alone, the
// 129-256 class 5 % slower.
constexpr int subwave_min_waves(int, bool) { return 2; }

template <int L, int S, bool SCHED>
__global__ __launch_bounds__(kBlock, subwave_min_waves(S, SCHED)) void rt_subwave_kernel(rt_class_dev C)
{
    constexpr unsigned long long kGroupBits = L == 64 ? ~0ull : ((1ull << L) - 1ull);
    rt_ws* const ws = C.ws;
    // Issue priority over other kernels' wavefronts sharing a CU (batches):
    // below the thread mapping's, above the lazy and workgroup kernels'.
    __builtin_amdgcn_s_setprio(2);
    const uint32_t key0 = ws->key0, key1 = ws->key1;
    const int tid = threadIdx.x, li = tid % L, lane = tid & 63;
    const unsigned long long gmask = kGroupBits << (lane - li);
    extern __shared__ int32_t dyn_lds[];
    __shared__ uint32_t log_scratch[kBlock / 64][RT_LOG_SCRATCH];
    uint32_t* sc = log_scratch[tid >> 6];
    constexpr int LOG2L = __builtin_ctz(L);
    const int NP = (C.max_N + 3) & ~3, MP = (C.max_M + 3) & ~3;
    int32_t* X = dyn_lds + (tid / L) * (NP + L + MP);   // [N] species counts
    uint32_t* stale_w = (uint32_t*)(X + NP);            // [L] stale words
    uint32_t* nk = stale_w + L;                         // [M] firing counts
    const rt_cptr<int64_t> unit_start = rt_const(C.unit_start);
    const int64_t total = unit_start[C.count];

    // channel state of this lane's slots
    double T[S], Pk[S], a[S], inv[S];
#pragma unroll
    for (int s = 0; s < S; ++s) { T[s] = 0.0; Pk[s] = 0.0; a[s] = 0.0; inv[s] = __builtin_inf(); }
    // trajectory context (identical in every lane of the group)
    rt_cptr<rt_item_dev> it = rt_const(C.items);
    int M = 0, N = 0, mu = 0;
    int64_t r = 0;
    uint32_t traj = 0, net_id = 0, fired = 0, tie = kTieNone;
    double t = 0.0, t_end = 0.0, s_next = 0.0, delta = 0.0, E = 0.0;
    int32_t g = 0;
    unsigned long long hash = kFnvOffset;
    bool active = true, fresh = true, capped = false, pending = false;
    // rate schedule: breakpoints passed, and the next one
    int32_t piece = 0;
    double b_next = __builtin_inf();

    while (__ballot(active) != 0ull) {
        if (!active) continue;
        const rt_cptr<rt_net_dev> net = &it->net;
        // ---- pass over own channels: apply the pending event, refresh, gap
        if (pending) {
            // every internal clock advances by a_k delta (Eq. 15) ...
#pragma unroll
            for (int s = 0; s < S; ++s) T[s] = fma(a[s], delta, T[s]);
            // ... except the fired one: its firing time, then the next (Eq. 26);
            // mu < 0 after a rate breakpoint
            if ((!SCHED || mu >= 0) && li == (mu & (L - 1))) {
                const int sm = mu >> LOG2L;
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    const bool f = s == sm;
                    T[s] = f ? Pk[s] : T[s];
                    Pk[s] = f ? Pk[s] + E : Pk[s];
                }
            }
            // the pending event's stale bits for this lane (read and cleared;
            // the pass then runs with pending = false if it is repeated)
            unsigned int stale = stale_w[li];
            stale_w[li] = 0u;
            pending = false;
            // rates in force: c before the first breakpoint, row i of the
            // schedule from breakpoint i on
            const rt_cptr<double> crate =
                SCHED && piece > 0 ? rt_const(net->sched_c) + (size_t)(piece - 1) * M
                                   : rt_const(net->c);
            // refresh one stale slot at a time (rare; keeps the code and the
            // register footprint of the propensity out of the unrolled pass)
            while (stale) {
                const int s1 = __builtin_ctz(stale);
                stale &= stale - 1u;
                const int k = li + s1 * L;
                const double an = rt_propensity_mem(rt_const(net->react)[k], crate[k], X);
                const double in = 1.0 / an;
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    a[s] = s == s1 ? an : a[s];
                    inv[s] = s == s1 ? in : inv[s];
                }
            }
        }
        rt_min2 loc = rt_min2_empty();
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const double raw = (Pk[s] - T[s]) * inv[s];
            const double d = a[s] == 0.0 ? __builtin_inf() : fmax(raw, 0.0);
            rt_min2_push(loc, d, s);                       // slot now, channel below
        }
        loc = rt_min2_slot_to_channel(loc, li, LOG2L);
        // ---- argmin across the group's lanes (lowest k wins ties)
        loc = rt_min2_allreduce<L>(loc);
        const double d1 = loc.d1, d2 = loc.d2;
        const int kmin = loc.k;
        const double t_new = t + d1;
        const bool absorbed = d1 == __builtin_inf();
        const bool live = !fresh && !capped;
        // the next firing would come after a rate breakpoint (Eq. 28)
        const bool brk = SCHED && live && b_next < t_end && t_new > b_next;
        const bool term = !brk && (absorbed || t_new > t_end);
        const bool event = live && !term && !brk;
        // ---- the fired channel's fixed-stride rows, one round trip: its jump
        // (lane li < nu_stride: entry li) and its touch row (lane li: the 64 / L
        // consecutive entries from li 64 / L; entry 0 counts the channels of
        // D(kmin) other than kmin, entries 1..63 name them, -1 past the end)
        constexpr int kTE = 64 / L;                         // touch entries per lane
        const int kr = event ? kmin : 0;                    // row 0 exists (M >= 1)
        const int nu_stride = net->nu_stride;
        const int2 nv = rt_const(net->nu_fixed)[kr * nu_stride + min(li, nu_stride - 1)];
        int32_t tch[kTE];
        {
            const rt_cptr<int32_t> row = rt_const(net->touch) + (size_t)kr * 64 + li * kTE;
#pragma unroll
            for (int e = 0; e < kTE; ++e) tch[e] = row[e];
        }
        // the fired channel's next Exp(1) (Eq. 26) in its owner lane, while
        // the rows load (discarded if the event is not applied in this pass)
        uint32_t nm_new = 0;
        double E_new = 0.0;
        bool slow_new = false;                              // counted when applied
        if (event && li == (kmin & (L - 1))) {
            nm_new = nk[kmin] + 1u;
            E_new = rt_neglog_wave(rt_draw_m53(key0, key1, traj, net_id, (uint32_t)kmin, nm_new),
                                   false, nullptr, sc, &slow_new);
        }
        // ---- the jump v_mu, checked against [0, 2^31 - 1] by lanes < |v_mu|
        int32_t xv = 0, xs = 0;
        bool okl = true;
        const bool has_nu = event && li < nu_stride && nv.x >= 0;
        if (has_nu) {
            xs = nv.x;
            const int64_t v = (int64_t)X[xs] + nv.y;
            okl = v >= 0 && v <= 0x7FFFFFFF;
            xv = (int32_t)v;
        }
        const bool ok = (__ballot(!okl) & gmask) == 0ull;
        const bool near_tie = event && rt_near_tie(d1, d2);
        // a zero gap may have been clamped from a negative raw gap
        const bool rare =
            !live || term || near_tie || d1 == 0.0 || !ok || s_next < t_new || brk;
        if (__builtin_expect(__ballot(rare) != 0ull, 0)) {
            // Counted once per event: when another group of the wavefront
            // stops or meets a breakpoint, this group repeats its pass below
            // without applying its event, so the counters are bumped only once
            // the event is known to be applied (or, for a near-tie, when the
            // event ends the trajectory by an overflow, as the oracle counts
            // it); tie and the samples are idempotent.
            bool clamped = false;
            if (event) {
                if (near_tie) tie = tie == kTieNone ? fired : tie;
                while (s_next < t_new) {
                    if (it->samples) {
                        int32_t* dst = it->samples + r * it->ss_r + (int64_t)g * it->ss_g;
                        for (int j = li; j < N; j += L) dst[j * it->ss_n] = X[j];
                    }
                    ++g;
                    s_next = g < it->G ? rt_const(it->s)[g] : __builtin_inf();
                }
                if (ok && d1 == 0.0 && li == (kmin & (L - 1))) {
                    const int sm = kmin >> LOG2L;
#pragma unroll
                    for (int s = 0; s < S; ++s)
                        clamped = s == sm ? (Pk[s] - T[s]) * inv[s] < 0.0 : clamped;
                }
            }
            const bool stop = !live || term || !ok;
            if (near_tie && stop && li == 0) atomicAdd(&ws->near_ties, 1ull);   // event && !ok
            if (stop && !fresh) {
                // ---- end of the trajectory
                const int st = capped ? RTSSA_TRAJ_MAX_FIRINGS
                                      : (absorbed ? RTSSA_TRAJ_ABSORBED
                                                  : (term ? RTSSA_TRAJ_OK : RTSSA_TRAJ_OVERFLOW));
                const bool good = st == RTSSA_TRAJ_OK || st == RTSSA_TRAJ_ABSORBED;
                if (it->samples) {
                    for (; g < it->G; ++g) {
                        int32_t* dst = it->samples + r * it->ss_r + (int64_t)g * it->ss_g;
                        for (int j = li; j < N; j += L) dst[j * it->ss_n] = good ? X[j] : -1;
                    }
                }
                const double dt = t_end - t;
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    const int k = li + s * L;
                    if (k < M) {
                        if (good) T[s] = fma(a[s], dt, T[s]);
                        if (it->n_out) it->n_out[r * M + k] = nk[k];
                        if (it->T_out) it->T_out[r * M + k] = T[s];
                    }
                }
                if (it->x_final)
                    for (int j = li; j < N; j += L) it->x_final[r * N + j] = X[j];
                if (li == 0) {
                    if (it->t_last) it->t_last[r] = t;
                    if (it->status) it->status[r] = (uint8_t)st;
                    if (it->seq_hash) it->seq_hash[r] = hash;
                    if (it->tie_step) it->tie_step[r] = tie;
                    atomicAdd(&ws->firings, (unsigned long long)fired);
                    atomicAdd(&ws->status_count[st], 1ull);
                }
            }
            if (stop) {
                // ---- take the next trajectory unit
                unsigned long long u = 0;
                if (li == 0) u = atomicAdd(&ws->next_unit, 1ull);
                u = __shfl(u, lane - li, 64);
                rt_wave_lds_fence();                          // X and flags are reused
                fresh = false;
                capped = false;
                pending = false;
                active = (int64_t)u < total;
                if (active) {
                    const int item = rt_find_item(unit_start, C.count, (int64_t)u);
                    it = rt_const(C.items) + item;
                    r = (int64_t)u - unit_start[item];
                    M = it->net.M;
                    N = it->net.N;
                    t_end = it->t_end;
                    net_id = it->net_id;
                    traj = it->traj_offset + (uint32_t)r;
                    const int32_t* x0 = it->x0 + (it->x0_per_traj ? r * N : 0);
                    for (int j = li; j < N; j += L) X[j] = x0[j];
                    for (int k = li; k < M; k += L) nk[k] = 0u;
                    stale_w[li] = 0u;
                    t = 0.0;
                    g = 0;
                    s_next = it->G > 0 ? rt_const(it->s)[0] : __builtin_inf();
                    piece = 0;
                    b_next = SCHED && it->net.sched_B > 0 ? rt_const(it->net.sched_t)[0]
                                                          : __builtin_inf();
                    fired = 0;
                    tie = kTieNone;
                    hash = kFnvOffset;
                    rt_wave_lds_fence();
#pragma unroll
                    for (int s = 0; s < S; ++s) {
                        T[s] = 0.0;
                        Pk[s] = 0.0;
                        a[s] = 0.0;
                        inv[s] = __builtin_inf();
                    }
                    // first internal firing times and propensities, one slot at a time
#pragma unroll 1
                    for (int s1 = 0; s1 < S; ++s1) {
                        const int k = li + s1 * L;
                        if (k < M) {
                            const double p0 = rt_exp1_wave(key0, key1, traj, net_id, (uint32_t)k,
                                                           0u, &ws->slow_logs, sc);
                            const double an = rt_propensity_mem(rt_const(it->net.react)[k],
                                                            rt_const(it->net.c)[k], X);
                            const double in = 1.0 / an;
#pragma unroll
                            for (int s = 0; s < S; ++s) {
                                Pk[s] = s == s1 ? p0 : Pk[s];
                                a[s] = s == s1 ? an : a[s];
                                inv[s] = s == s1 ? in : inv[s];
                            }
                        }
                    }
                }
            }
            if (SCHED && brk) {
                // the clocks run to the breakpoint at the old rates, then
                // every propensity takes the new ones
                delta = b_next - t;
                t = b_next;
                ++piece;
                b_next = piece < net->sched_B ? rt_const(net->sched_t)[piece]
                                              : __builtin_inf();
                uint32_t all = 0u;
#pragma unroll
                for (int s = 0; s < S; ++s) all |= li + s * L < M ? 1u << s : 0u;
                stale_w[li] = all;
                mu = -1;
                pending = true;
            }
            // started groups compute first gaps, groups past a breakpoint
            // solve again; the others repeat their (idempotent) pass
            if (__ballot(stop || brk) != 0ull) continue;
            // the event is applied below
            if (near_tie && li == 0) atomicAdd(&ws->near_ties, 1ull);
            if (clamped) atomicAdd(&ws->clamps, 1ull);
        }
        // ---- the event: jump, dependency flags, fresh draw by the owner lane
        mu = kmin;
        if (has_nu) X[xs] = xv;
        // stale bits: mu itself (its propensity may read a species it
        // changes) and the channels of its touch row
        if (li == 0) atomicOr(&stale_w[mu & (L - 1)], 1u << (mu >> LOG2L));
#pragma unroll
        for (int e = 0; e < kTE; ++e) {
            const int kk = tch[e];
            if (li * kTE + e > 0 && kk >= 0) atomicOr(&stale_w[kk & (L - 1)], 1u << (kk >> LOG2L));
        }
        {
            // more than 63 others: the rest of the CSR list D(mu) (rare)
            const int n_other = __shfl(tch[0], lane - li, 64);
            if (n_other > 63) {
                const int de = rt_const(net->dep_ptr)[mu + 1];
                for (int q = rt_const(net->touch_more)[mu] + li; q < de; q += L) {
                    const int kk = rt_const(net->dep_idx)[q];
                    atomicOr(&stale_w[kk & (L - 1)], 1u << (kk >> LOG2L));
                }
            }
        }
        if (li == (mu & (L - 1))) {
            nk[mu] = nm_new;
            E = E_new;
            if (slow_new) atomicAdd(&ws->slow_logs, 1ull);
        }
        rt_wave_lds_fence();
        t = t_new;
        delta = d1;
        ++fired;
        hash = (hash ^ (unsigned long long)(uint32_t)mu) * kFnvPrime;
        pending = true;
        capped = fired >= C.max_firings;
    }
}

typedef void (*subwave_kernel_t)(rt_class_dev);

template <int L, int S>
subwave_kernel_t sw_pick(bool sched)
{
    return sched ? rt_subwave_kernel<L, S, true> : rt_subwave_kernel<L, S, false>;
}

subwave_kernel_t select_subwave(int L, int S, bool sched)
{
#define RT_CASE(l, s) if (L == l && S == s) return sw_pick<l, s>(sched);
    RT_CASE(4, 2) RT_CASE(4, 4) RT_CASE(4, 8)
    RT_CASE(8, 4) RT_CASE(8, 8)
    RT_CASE(16, 4) RT_CASE(16, 8)
    RT_CASE(32, 4) RT_CASE(32, 8)
    RT_CASE(64, 4) RT_CASE(64, 8)
#undef RT_CASE
    return nullptr;
}

}  // namespace

// Lanes per trajectory for an M-channel network: the fewest lanes that keep
// at most 8 channels per lane (at least 4 lanes).
int rt_subwave_lanes(int M)
{
    int L = 4;
    while (L < 64 && L * 8 < M) L <<= 1;
    return L;
}

int rt_subwave_slots(int M, int L)
{
    int s = (M + L - 1) / L;
    int p = 2;
    while (p < s) p <<= 1;
    if (L > 4 && p < 4) p = 4;
    return p;
}

int rt_launch_subwave(int max_M, const rt_class_dev& C, int L, int grid, hipStream_t stream,
                      int* grid_used)
{
    const int S = rt_subwave_slots(max_M, L);
    subwave_kernel_t kfn = select_subwave(L, S, C.has_schedule != 0);
    if (!kfn) return rt_fail(RTSSA_E_UNSUPPORTED, "no sub-wave kernel for this size");
    const int NP = (C.max_N + 3) & ~3, MP = (C.max_M + 3) & ~3;
    const size_t lds = (size_t)(kBlock / L) * (NP + L + MP) * 4;
    if (lds > 64 * 1024) return rt_fail(RTSSA_E_UNSUPPORTED, "sub-wave LDS too large");
    if (grid <= 0) {
        int dev = 0, cus = 0, per_cu = 0;
        hipGetDevice(&dev);
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, kBlock, lds) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        grid = cus * per_cu;
    }
    if (grid_used) *grid_used = grid;
    hipLaunchKernelGGL(kfn, dim3(grid), dim3(kBlock), lds, stream, C);
    return hipGetLastError() == hipSuccess ? RTSSA_OK
                                           : rt_fail(RTSSA_E_HIP, "sub-wave kernel launch failed");
}
