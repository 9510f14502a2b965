// kernels_group.hip -- wavefront- and workgroup-per-trajectory mappings.
//
// One workgroup of L threads (L = 64: one wavefront; L = 256..1024: several)
// simulates one trajectory at a time; the grid is persistent and takes
// trajectory indices from a device work queue.  Channel k belongs to thread
// k mod L, slot k / L; each thread keeps its channels' T_k, P_k, a_k, 1/a_k
// and n_k in registers.  The species counts X and a bitmap of channels whose
// propensity must be recomputed live in LDS.
//
// One firing (section 4, Table 2, in the internal-time form of Eq. 14-16):
//   pass   every thread, for its channels: apply the previous event
//          (T_k += a_k Delta, or T_mu = P_mu and P_mu += E for the fired
//          channel), recompute a_k and 1/a_k if the channel reads a species
//          the previous event changed, then the gap (P_k - T_k)/a_k and a
//          local argmin with second minimum;
//   argmin across the wavefront by shuffles, across wavefronts through LDS
//          (barrier 1); lowest k wins ties (Eq. 25);
//   event  wavefront 0 applies the jump v_mu to X; the threads of the
//          dependency list D(mu) (the channels reading a changed species,
//          Gibson & Bruck's dependency graph cited in section 5) flag their
//          channels; the owner of mu draws the fresh Exp(1) (Eq. 26)
//          (barrier 2).
#include <hip/hip_runtime.h>

#include "internal.h"
#include "rt_device.h"

namespace {

constexpr uint32_t kTieNone = 0xFFFFFFFFu;
constexpr unsigned long long kFnvOffset = 0xcbf29ce484222325ull;
constexpr unsigned long long kFnvPrime = 0x100000001b3ull;

__device__ __forceinline__ double u64_to_f64(uint64_t h)
{
    return fma((double)(uint32_t)(h >> 32), 0x1p32, (double)(uint32_t)h);
}

// a_k = RN(c_k RN(h_k(X))) with X in LDS (Eq. 1-2).
__device__ __forceinline__ double group_propensity(int2 rr, double c, const int32_t* X)
{
    const int kind = (int)((uint32_t)rr.x >> 29);
    const int s0 = rr.x & RT_SPECIES_MASK;
    uint64_t h;
    if (kind == RT_H_ZERO) {
        h = 1;
    } else if (kind == RT_H_ONE) {
        h = (uint32_t)X[s0];
    } else if (kind == RT_H_PAIR) {
        const uint32_t x = (uint32_t)X[s0];
        h = ((uint64_t)x * (uint32_t)(x - 1u)) >> 1;
    } else {
        h = (uint64_t)(uint32_t)X[s0] * (uint32_t)X[rr.y];
    }
    return c * u64_to_f64(h);
}

// (d1, d2, k, clamped): smallest gap, second smallest gap (order statistic
// with multiplicity), its channel, and whether its raw gap was negative.
struct rt_min2 {
    double d1, d2;
    int k;
    int clamped;
};

__device__ __forceinline__ void min2_merge(rt_min2& a, const rt_min2& b)
{
    const bool bw = b.d1 < a.d1 || (b.d1 == a.d1 && b.k < a.k);
    const double d2 = bw ? fmin(b.d2, a.d1) : fmin(a.d2, b.d1);
    a.d1 = bw ? b.d1 : a.d1;
    a.k = bw ? b.k : a.k;
    a.clamped = bw ? b.clamped : a.clamped;
    a.d2 = d2;
}

__device__ __forceinline__ rt_min2 min2_shfl_xor(const rt_min2& v, int off)
{
    rt_min2 o;
    o.d1 = __shfl_xor(v.d1, off, 64);
    o.d2 = __shfl_xor(v.d2, off, 64);
    o.k = __shfl_xor(v.k, off, 64);
    o.clamped = __shfl_xor(v.clamped, off, 64);
    return o;
}

__device__ __forceinline__ void min2_wave(rt_min2& v, int width)
{
    for (int off = width >> 1; off > 0; off >>= 1) min2_merge(v, min2_shfl_xor(v, off));
}

struct rt_group_shared {
    rt_min2 wave_min[16];
    unsigned long long next_traj;
    int ok;
    uint32_t log_scratch[16][RT_LOG_SCRATCH];
};

// Index of the item owning global unit u: unit_start[i] <= u < unit_start[i+1].
__device__ __forceinline__ int group_find_item(const int64_t* unit_start, int count, int64_t u)
{
    int lo = 0, hi = count;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (unit_start[mid] <= u) lo = mid; else hi = mid;
    }
    return lo;
}

template <int L, int S>
__global__ __launch_bounds__(L) void rt_group_kernel(rt_class_dev C)
{
    constexpr int W = L / 64;
    extern __shared__ int32_t dyn_lds[];
    __shared__ rt_group_shared sh;
    rt_ws* const ws = C.ws;
    const uint32_t key0 = ws->key0, key1 = ws->key1;
    const int64_t total = C.unit_start[C.count];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int32_t* X = dyn_lds;                                   // [N]
    // two bitmaps of channels to refresh, alternating by event parity: one is
    // read (and then cleared) while the next event sets the other
    const int nflag = (C.max_M + 31) >> 5;
    uint32_t* flag_buf = (uint32_t*)(dyn_lds + ((C.max_N + 3) & ~3));   // [2][nflag]
    uint32_t* sc = sh.log_scratch[wave];

    double T[S], Pk[S], a[S], inv[S];
    uint32_t n[S];
#pragma unroll
    for (int s = 0; s < S; ++s) { T[s] = 0.0; Pk[s] = 0.0; a[s] = 0.0; inv[s] = 0.0; n[s] = 0; }

    for (;;) {
        // ---- next trajectory unit
        if (tid == 0) sh.next_traj = atomicAdd(&ws->next_unit, 1ull);
        __syncthreads();
        const int64_t u = (int64_t)sh.next_traj;
        if (u >= total) break;
        const int item = group_find_item(C.unit_start, C.count, u);
        const rt_item_dev* it = C.items + item;
        const rt_net_dev net = it->net;
        const int N = net.N, M = net.M;
        const int64_t r = u - C.unit_start[item];
        const uint32_t traj = it->traj_offset + (uint32_t)r;
        const uint32_t net_id = it->net_id;
        const double t_end = it->t_end;
        const int32_t* x0 = it->x0 + (it->x0_per_traj ? r * N : 0);
        for (int j = tid; j < N; j += L) X[j] = x0[j];
        for (int q = tid; q < 2 * nflag; q += L) flag_buf[q] = 0u;
        __syncthreads();
        uint32_t* flags_rd = flag_buf;            // set by the pending event
        uint32_t* flags_wr = flag_buf + nflag;    // set by the next event
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int k = tid + s * L;
            T[s] = 0.0;
            n[s] = 0;
            if (k < M) {
                Pk[s] = rt_exp1_wave(key0, key1, traj, net_id, (uint32_t)k, 0u,
                                     &ws->slow_logs, sc);
                a[s] = group_propensity(net.react[k], net.c[k], X);
                inv[s] = 1.0 / a[s];
            }
        }
        double t = 0.0, s_next = it->G > 0 ? it->s[0] : __builtin_inf();
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
            rt_min2 loc = {__builtin_inf(), __builtin_inf(), 0x7FFFFFFF, 0};
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int k = tid + s * L;
                if (k < M) {
                    if (pending) {
                        if (k == mu) {
                            T[s] = Pk[s];
                            Pk[s] = Pk[s] + E;
                            n[s] += 1u;
                        } else {
                            T[s] = fma(a[s], delta, T[s]);
                        }
                        const uint32_t bit = 1u << (k & 31);
                        if (flags_rd[k >> 5] & bit) {
                            a[s] = group_propensity(net.react[k], net.c[k], X);
                            inv[s] = 1.0 / a[s];
                        }
                    }
                    const double raw = (Pk[s] - T[s]) * inv[s];
                    double d = raw < 0.0 ? 0.0 : raw;
                    d = a[s] == 0.0 ? __builtin_inf() : d;
                    const bool lt = d < loc.d1;
                    loc.d2 = lt ? loc.d1 : (d < loc.d2 ? d : loc.d2);
                    loc.d1 = lt ? d : loc.d1;
                    loc.k = lt ? k : loc.k;
                    loc.clamped = lt ? (raw < 0.0) : loc.clamped;
                }
            }
            if (st == RTSSA_TRAJ_MAX_FIRINGS) break;       // the capped event is now applied
            // ---- argmin over the workgroup
            min2_wave(loc, 64);
            if (W > 1) {
                if (lane == 0) sh.wave_min[wave] = loc;
            }
            __syncthreads();                               // barrier 1
            if (pending) {
                // every thread has read the pending event's flags: clear them
                for (int q = tid; q < nflag; q += L) flags_rd[q] = 0u;
            }
            if (W > 1) {
                rt_min2 v = lane < W ? sh.wave_min[lane] : rt_min2{__builtin_inf(), __builtin_inf(), 0x7FFFFFFF, 0};
                min2_wave(v, W < 2 ? 2 : W);
                loc = v;
            }
            const double d1 = __shfl(loc.d1, 0, 64), d2 = __shfl(loc.d2, 0, 64);
            mu = __builtin_amdgcn_readfirstlane(__shfl(loc.k, 0, 64));
            const int clamped = __builtin_amdgcn_readfirstlane(__shfl(loc.clamped, 0, 64));
            const double t_new = t + d1;
            if (d1 == __builtin_inf()) { st = RTSSA_TRAJ_ABSORBED; break; }
            if (t_new > t_end) { st = RTSSA_TRAJ_OK; break; }
            if (d2 - d1 <= 1e-12 * d1) {
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
                    s_next = g < it->G ? it->s[g] : __builtin_inf();
                }
                __syncthreads();
            }
            // ---- the event: jump (wave 0), dependency flags, fresh draw (owner)
            const int nb = net.nu_ptr[mu], ne = net.nu_ptr[mu + 1];
            if (wave == 0) {
                int32_t v = 0;
                bool okl = true;
                if (lane < ne - nb) {
                    const int64_t nv = (int64_t)X[net.nu_sp[nb + lane]] + net.nu_dl[nb + lane];
                    okl = nv >= 0 && nv <= 0x7FFFFFFF;
                    v = (int32_t)nv;
                }
                const bool ok = __ballot(!okl) == 0ull;
                if (ok && lane < ne - nb) X[net.nu_sp[nb + lane]] = v;
                if (lane == 0) sh.ok = ok;
            }
            const int db = net.dep_ptr[mu], de = net.dep_ptr[mu + 1];
            for (int q = db + tid; q < de; q += L) {
                const int kk = net.dep_idx[q];
                atomicOr(&flags_wr[kk >> 5], 1u << (kk & 31));
            }
            if (tid == (mu % L)) {
                const int slot = mu / L;
                uint32_t nm = n[0];
#pragma unroll
                for (int s = 1; s < S; ++s) nm = slot == s ? n[s] : nm;
                E = rt_exp1_wave(key0, key1, traj, net_id, (uint32_t)mu, nm + 1u,
                                 &ws->slow_logs, sc);
            }
            __syncthreads();                               // barrier 2
            if (!sh.ok) { st = RTSSA_TRAJ_OVERFLOW; break; }
            if (clamped && tid == 0) atomicAdd(&ws->clamps, 1ull);
            t = t_new;
            delta = d1;
            ++fired;
            hash = (hash ^ (unsigned long long)(uint32_t)mu) * kFnvPrime;
            pending = true;
            uint32_t* tmp = flags_rd;
            flags_rd = flags_wr;
            flags_wr = tmp;
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
                if (it->n_out) it->n_out[r * M + k] = n[s];
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
        __syncthreads();                                   // X is reused next
    }
}

typedef void (*group_kernel_t)(rt_class_dev);

template <int L, int S>
group_kernel_t pick_kernel() { return rt_group_kernel<L, S>; }

group_kernel_t select_group(int L, int S)
{
#define RT_CASE(l, s) if (L == l && S == s) return pick_kernel<l, s>();
    RT_CASE(64, 1) RT_CASE(64, 2) RT_CASE(64, 4) RT_CASE(64, 8) RT_CASE(64, 16)
    RT_CASE(256, 1) RT_CASE(256, 2) RT_CASE(256, 4) RT_CASE(256, 8) RT_CASE(256, 16)
    RT_CASE(128, 16) RT_CASE(128, 32)
    RT_CASE(512, 1) RT_CASE(512, 2) RT_CASE(512, 4) RT_CASE(512, 8)
    RT_CASE(1024, 1) RT_CASE(1024, 2) RT_CASE(1024, 4) RT_CASE(1024, 8)
#undef RT_CASE
    return nullptr;
}

}  // namespace

size_t rt_group_lds_bytes(int N, int M)
{
    return (size_t)((N + 3) & ~3) * 4 + (size_t)((M + 31) >> 5) * 8 + 16;
}

int rt_group_slots(int M, int L)
{
    int s = (M + L - 1) / L;
    int p = 1;
    while (p < s) p <<= 1;
    return p < 1 ? 1 : p;
}

int rt_launch_group(int M, int max_N, int max_M, const rt_class_dev& C, int L, int grid,
                    hipStream_t stream, int* grid_used)
{
    const int S = rt_group_slots(M, L);
    group_kernel_t kfn = select_group(L, S);
    if (!kfn) return rt_fail(RTSSA_E_UNSUPPORTED, "no group kernel for this network size and L");
    const size_t lds = rt_group_lds_bytes(max_N, max_M);
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
