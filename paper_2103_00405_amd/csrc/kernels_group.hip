// kernels_group.hip -- wavefront- and workgroup-per-trajectory mappings.
//
// One workgroup of L threads (L = 64: one wavefront; L = 128..1024: several)
// simulates one trajectory at a time; the grid is persistent and takes
// trajectory indices from a device work queue.  Channel k belongs to thread
// k mod L, slot k / L; each thread keeps its channels' T_k, P_k, a_k and
// 1/a_k in registers (slots past M are frozen channels that never win).  The
// species counts X, the firing counts n_k and one stale word per thread (bit
// s: slot s must recompute its propensity) live in LDS.
//
// One firing (section 4, Table 2, in the internal-time form of Eq. 14-16):
//   pass   every thread: T_k += a_k Delta for all its channels (Eq. 15); the
//          owner of the previous event's channel sets T_mu = P_mu and adds
//          the fresh Exp(1) to P_mu (Eq. 26); stale slots recompute a_k and
//          1/a_k; then the gaps (P_k - T_k)/a_k and a local argmin with
//          second minimum, branch-free;
//   argmin across the wavefront by DPP and permlane exchanges, across
//          wavefronts through LDS (barrier 1); lowest k wins ties (Eq. 25);
//   event  wavefront 0 applies the jump v_mu to X; the threads of the
//          dependency list D(mu) (the channels reading a changed species,
//          Gibson & Bruck's dependency graph cited in section 5) set stale
//          bits; the owner of mu draws the fresh Exp(1) (barrier 2) and
//          counts the firing in n_mu.
// With piecewise-constant rates (Eq. 28), a next firing that would fall past
// the next rate breakpoint b instead runs every clock to b at the old rates
// (a pending event with no fired channel) and marks every slot stale, so the
// next pass takes the new rates; the branch is uniform over the workgroup.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "rt_device.h"
#include "rt_wave.h"

namespace {

struct rt_group_shared {
    rt_min2 wave_min[16];
    unsigned long long next_traj;
    int ok;
    uint32_t log_scratch[16][RT_LOG_SCRATCH];
};

// Waves per SIMD the register allocation aims at: 16 slots of channel state
// fit 2, 8 fit 3 (2 with a rate schedule's state), fewer fit 4.
constexpr int group_min_waves(int S, bool SCHED)
{
    return S >= 16 || (SCHED && S >= 8) ? 2 : (S >= 8 ? 3 : 4);
}

template <int L, int S, bool SCHED>
__global__ __launch_bounds__(L, group_min_waves(S, SCHED)) void rt_group_kernel(rt_class_dev C)
{
    constexpr int W = L / 64;
    constexpr int LOG2L = __builtin_ctz(L);
    extern __shared__ int32_t dyn_lds[];
    __shared__ rt_group_shared sh;
    rt_ws* const ws = C.ws;
    const uint32_t key0 = ws->key0, key1 = ws->key1;
    const rt_cptr<int64_t> unit_start = rt_const(C.unit_start);
    const int64_t total = unit_start[C.count];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int32_t* X = dyn_lds;                                            // [N] species counts
    uint32_t* nk = (uint32_t*)(dyn_lds + ((C.max_N + 3) & ~3));      // [M] firing counts n_k
    // stale words: bit s of word t marks channel t + s L, so each thread
    // reads (and clears) its whole stale set at once.  The event of one firing
    // sets bits between barriers 1 and 2; every thread reads and clears its
    // own word in the next pass, before the next barrier 1.
    uint32_t* stale_w = nk + ((C.max_M + 3) & ~3);                   // [L]
    uint32_t* sc = sh.log_scratch[wave];

    // channel state: slot s of thread tid is channel tid + s L; slots past M
    // are frozen channels (a = 0) and never win
    double T[S], Pk[S], a[S], inv[S];
#pragma unroll
    for (int s = 0; s < S; ++s) { T[s] = 0.0; Pk[s] = 0.0; a[s] = 0.0; inv[s] = __builtin_inf(); }

    for (;;) {
        // ---- next trajectory unit
        if (tid == 0) sh.next_traj = atomicAdd(&ws->next_unit, 1ull);
        __syncthreads();
        // the unit is the same for the whole workgroup: keep it (and with it
        // the item descriptor and the network's table pointers) in SGPRs
        const unsigned long long u_lds = sh.next_traj;
        const int64_t u = (int64_t)(((unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane(
                                         (int)(u_lds >> 32)) << 32) |
                                     (uint32_t)__builtin_amdgcn_readfirstlane((int)u_lds));
        if (u >= total) break;
        const int item = __builtin_amdgcn_readfirstlane(rt_find_item(unit_start, C.count, u));
        const rt_cptr<rt_item_dev> it = rt_const(C.items) + item;
        const rt_net_dev net = it->net;
        const int N = net.N, M = net.M;
        const rt_cptr<int2> react = rt_const(net.react);
        const rt_cptr<double> cc = rt_const(net.c);
        const rt_cptr<int32_t> nu_ptr = rt_const(net.nu_ptr), nu_sp = rt_const(net.nu_sp);
        const rt_cptr<int32_t> nu_dl = rt_const(net.nu_dl), dep_ptr = rt_const(net.dep_ptr);
        const rt_cptr<int32_t> dep_idx = rt_const(net.dep_idx);
        const rt_cptr<double> grid_s = rt_const(it->s);
        const int64_t r = u - unit_start[item];
        const uint32_t traj = it->traj_offset + (uint32_t)r;
        const uint32_t net_id = it->net_id;
        const double t_end = it->t_end;
        // rates in force: the network's c before the first breakpoint, row
        // i of the schedule from breakpoint i on
        const int32_t sB = SCHED ? net.sched_B : 0;
        rt_cptr<double> crate = cc;
        int32_t piece = 0;
        double b_next = sB > 0 ? rt_const(net.sched_t)[0] : __builtin_inf();
        const int32_t* x0 = it->x0 + (it->x0_per_traj ? r * N : 0);
        for (int j = tid; j < N; j += L) X[j] = x0[j];
        for (int k = tid; k < M; k += L) nk[k] = 0u;
        stale_w[tid] = 0u;
        __syncthreads();
#pragma unroll
        for (int s = 0; s < S; ++s) { T[s] = 0.0; Pk[s] = 0.0; a[s] = 0.0; inv[s] = __builtin_inf(); }
        // first internal firing times and propensities, one slot at a time
#pragma unroll 1
        for (int s1 = 0; s1 < S; ++s1) {
            const int k = tid + s1 * L;
            if (k < M) {
                const double p0 = rt_exp1_wave(key0, key1, traj, net_id, (uint32_t)k, 0u,
                                               &ws->slow_logs, sc);
                const double an = rt_propensity_mem(react[k], cc[k], X);
                const double in = 1.0 / an;
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    Pk[s] = s == s1 ? p0 : Pk[s];
                    a[s] = s == s1 ? an : a[s];
                    inv[s] = s == s1 ? in : inv[s];
                }
            }
        }
        double t = 0.0, s_next = it->G > 0 ? grid_s[0] : __builtin_inf();
        int32_t g = 0;
        uint32_t fired = 0, tie = kTieNone;
        unsigned long long hash = kFnvOffset;
        int st = -1;
        // pending event (applied at the start of the next pass)
        bool pending = false;
        int mu = -1;
        double delta = 0.0, E = 0.0;

        for (;;) {
            // ---- pass over own channels: apply the pending event, refresh, gap
            if (pending) {
                // every internal clock advances by a_k delta (Eq. 15) ...
#pragma unroll
                for (int s = 0; s < S; ++s) T[s] = fma(a[s], delta, T[s]);
                // ... except the fired one, which is set to its firing time and
                // gets its next one (Eq. 26); mu < 0 after a rate breakpoint
                if ((!SCHED || mu >= 0) && tid == (mu & (L - 1))) {
                    const int sm = mu >> LOG2L;
#pragma unroll
                    for (int s = 0; s < S; ++s) {
                        if (s == sm) {
                            T[s] = Pk[s];
                            Pk[s] = Pk[s] + E;
                        }
                    }
                }
                // refresh the slots whose propensity reads a changed species,
                // one at a time (keeps the propensity code out of the
                // unrolled pass)
                unsigned int stale = stale_w[tid];
                stale_w[tid] = 0u;
                while (stale) {
                    const int s1 = __builtin_ctz(stale);
                    stale &= stale - 1u;
                    const int k = tid + s1 * L;
                    const double an = rt_propensity_mem(react[k], crate[k], X);
                    const double in = 1.0 / an;
#pragma unroll
                    for (int s = 0; s < S; ++s) {
                        a[s] = s == s1 ? an : a[s];
                        inv[s] = s == s1 ? in : inv[s];
                    }
                }
            }
            if (st == RTSSA_TRAJ_MAX_FIRINGS) break;       // the capped event is now applied
            rt_min2 loc = rt_min2_empty();
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const double raw = (Pk[s] - T[s]) * inv[s];
                const double d = a[s] == 0.0 ? __builtin_inf() : fmax(raw, 0.0);
                rt_min2_push(loc, d, s);                   // slot now, channel below
            }
            loc = rt_min2_slot_to_channel(loc, tid, LOG2L);
            // ---- argmin over the workgroup (barrier 1 inside)
            loc = rt_min2_group_allreduce<L>(loc, sh.wave_min);
            const double d1 = loc.d1, d2 = loc.d2;
            mu = __builtin_amdgcn_readfirstlane(loc.k);
            const double t_new = t + d1;
            // (the test is uniform; readfirstlane keeps the schedule state scalar)
            if (SCHED && __builtin_amdgcn_readfirstlane(b_next < t_end && t_new > b_next)) {
                // the next firing would come after a rate breakpoint: the
                // clocks run to it at the old rates, then every propensity
                // takes the new ones and the gaps are solved again (Eq. 28)
                delta = b_next - t;
                t = b_next;
                crate = rt_const(net.sched_c) + (size_t)piece * M;
                ++piece;
                b_next = piece < sB ? rt_const(net.sched_t)[piece] : __builtin_inf();
                uint32_t all = 0u;
#pragma unroll
                for (int s = 0; s < S; ++s) all |= tid + s * L < M ? 1u << s : 0u;
                stale_w[tid] = all;
                mu = -1;
                pending = true;
                __syncthreads();                           // wave_min is rewritten next
                continue;
            }
            if (d1 == __builtin_inf()) { st = RTSSA_TRAJ_ABSORBED; break; }
            if (t_new > t_end) { st = RTSSA_TRAJ_OK; break; }
            if (rt_near_tie(d1, d2)) {
                if (tid == 0) atomicAdd(&ws->near_ties, 1ull);
                tie = tie == kTieNone ? fired : tie;
            }
            if (s_next < t_new) {
                // sample points before the event see the current X
                while (s_next < t_new) {
                    if (it->samples) {
                        int32_t* dst = it->samples + r * it->ss_r + (int64_t)g * it->ss_g;
                        for (int j = tid; j < N; j += L) dst[j * it->ss_n] = X[j];
                    }
                    ++g;
                    s_next = g < it->G ? grid_s[g] : __builtin_inf();
                }
                __syncthreads();
            }
            // ---- the event: wavefront 0 applies the jump and sets the stale
            // bits of D(mu); the owner's wavefront draws the fresh Exp(1), all
            // its lanes alike (a uniform branch, not a one-lane one)
            const int nb = nu_ptr[mu], ne = nu_ptr[mu + 1];
            const int db = dep_ptr[mu], de = dep_ptr[mu + 1];
            const int owner_lane = mu & (L - 1);
            if (wave == 0) {
                const int cnt = ne - nb, dcnt = de - db;
                // every lane loads a valid entry (lists have a padding entry),
                // so all loads issue before the first use
                const int qs = nb + max(0, min(lane, cnt - 1));
                const int qd = db + max(0, min(lane, dcnt - 1));
                const int sp = nu_sp[qs], dl = nu_dl[qs], kk = dep_idx[qd];
                const int64_t nv = (int64_t)X[sp] + dl;
                const bool okl = lane >= cnt || (nv >= 0 && nv <= 0x7FFFFFFF);
                const bool ok = __ballot(!okl) == 0ull;
                if (ok && lane < cnt) X[sp] = (int32_t)nv;
                if (lane < dcnt) atomicOr(&stale_w[kk & (L - 1)], 1u << (kk >> LOG2L));
                for (int q = db + 64 + lane; q < de; q += 64) {   // beyond 64 dependents
                    const int k2 = dep_idx[q];
                    atomicOr(&stale_w[k2 & (L - 1)], 1u << (k2 >> LOG2L));
                }
                if (lane == 0) sh.ok = ok;
            }
            uint32_t nm = 0;
            bool clamped = false;
            if (wave == (owner_lane >> 6)) {
                nm = nk[mu];
                E = rt_exp1_uniform(key0, key1, traj, net_id, (uint32_t)mu, nm + 1u,
                                    &ws->slow_logs, sc);
                if (d1 == 0.0 && tid == owner_lane) {
                    // a zero gap: was it clamped from a negative raw gap?
                    const int sm = mu >> LOG2L;
#pragma unroll
                    for (int s = 0; s < S; ++s)
                        if (s == sm) clamped = (Pk[s] - T[s]) * inv[s] < 0.0;
                }
            }
            __syncthreads();                               // barrier 2
            if (!sh.ok) { st = RTSSA_TRAJ_OVERFLOW; break; }
            if (tid == owner_lane) {
                nk[mu] = nm + 1u;
                if (clamped) atomicAdd(&ws->clamps, 1ull);
            }
            t = t_new;
            delta = d1;
            ++fired;
            hash = (hash ^ (unsigned long long)(uint32_t)mu) * kFnvPrime;
            pending = true;
            if (fired >= C.max_firings) st = RTSSA_TRAJ_MAX_FIRINGS;   // apply, then stop
        }

        // ---- end of the trajectory
        const bool good = st == RTSSA_TRAJ_OK || st == RTSSA_TRAJ_ABSORBED;
        if (it->samples) {
            for (; g < it->G; ++g) {
                int32_t* dst = it->samples + r * it->ss_r + (int64_t)g * it->ss_g;
                for (int j = tid; j < N; j += L) dst[j * it->ss_n] = good ? X[j] : -1;
            }
        }
        const double dt = t_end - t;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int k = tid + s * L;
            if (k < M) {
                if (good) T[s] = fma(a[s], dt, T[s]);
                if (it->n_out) it->n_out[r * M + k] = nk[k];
                if (it->T_out) it->T_out[r * M + k] = T[s];
            }
        }
        if (it->x_final)
            for (int j = tid; j < N; j += L) it->x_final[r * N + j] = X[j];
        if (tid == 0) {
            if (it->t_last) it->t_last[r] = t;
            if (it->status) it->status[r] = (uint8_t)st;
            if (it->seq_hash) it->seq_hash[r] = hash;
            if (it->tie_step) it->tie_step[r] = tie;
            atomicAdd(&ws->firings, (unsigned long long)fired);
            atomicAdd(&ws->status_count[st], 1ull);
        }
        __syncthreads();                                   // X and nk are reused next
    }
}

typedef void (*group_kernel_t)(rt_class_dev);

template <int L, int S>
group_kernel_t pick_kernel(bool sched)
{
    return sched ? rt_group_kernel<L, S, true> : rt_group_kernel<L, S, false>;
}

group_kernel_t select_group(int L, int S, bool sched)
{
#define RT_CASE(l, s) if (L == l && S == s) return pick_kernel<l, s>(sched);
    RT_CASE(64, 1) RT_CASE(64, 2) RT_CASE(64, 4) RT_CASE(64, 8) RT_CASE(64, 16)
    RT_CASE(256, 1) RT_CASE(256, 2) RT_CASE(256, 4) RT_CASE(256, 8) RT_CASE(256, 16)
    RT_CASE(128, 4) RT_CASE(128, 8) RT_CASE(128, 16)
    RT_CASE(512, 1) RT_CASE(512, 2) RT_CASE(512, 4) RT_CASE(512, 8)
    RT_CASE(1024, 1) RT_CASE(1024, 2) RT_CASE(1024, 4) RT_CASE(1024, 8)
#undef RT_CASE
    return nullptr;
}

}  // namespace

size_t rt_group_lds_bytes(int N, int M, int L)
{
    return (size_t)((N + 3) & ~3) * 4 + (size_t)((M + 3) & ~3) * 4 + (size_t)L * 4;
}

int rt_group_slots(int M, int L)
{
    int s = (M + L - 1) / L;
    int p = 1;
    while (p < s) p <<= 1;
    return p < 1 ? 1 : p;
}

bool rt_group_supported(int M, int L)
{
    return M >= 1 && select_group(L, rt_group_slots(M, L), false) != nullptr;
}

int rt_launch_group(int M, int max_N, int max_M, const rt_class_dev& C, int L, int grid,
                    hipStream_t stream, int* grid_used)
{
    const int S = rt_group_slots(M, L);
    group_kernel_t kfn = select_group(L, S, C.has_schedule != 0);
    if (!kfn) return rt_fail(RTSSA_E_UNSUPPORTED, "no group kernel for this network size and L");
    const size_t lds = rt_group_lds_bytes(max_N, max_M, L);
    if (lds > 96 * 1024) return rt_fail(RTSSA_E_UNSUPPORTED, "network too large for LDS");
    if (lds > 48 * 1024 &&
        hipFuncSetAttribute((const void*)kfn, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds) != hipSuccess)
        return rt_fail(RTSSA_E_HIP, "cannot raise the LDS limit");
    if (grid <= 0) {
        int dev = 0, cus = 0, per_cu = 0;
        hipGetDevice(&dev);
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, L, lds) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        grid = cus * per_cu;
    }
    if (grid_used) *grid_used = grid;
    hipLaunchKernelGGL(kfn, dim3(grid), dim3(L), lds, stream, C);
    return hipGetLastError() == hipSuccess ? RTSSA_OK
                                           : rt_fail(RTSSA_E_HIP, "group kernel launch failed");
}
