// kernels_thread.hip -- thread-per-trajectory mapping for small networks.
//
// One lane owns one trajectory at a time; its whole state (t, X, and per
// channel T_k, P_k, a_k, 1/a_k, n_k) lives in VGPRs, the network constants of
// the wavefront's current item in SGPRs.  The grid is persistent: a lane that
// finishes a trajectory takes the next trajectory of the same item from a
// device counter, so lanes stay busy despite uneven trajectory lengths; a
// wavefront moves to another item only when all of its lanes are idle.
//
// The step is the next reaction random time algorithm (section 4, Table 2)
// in the internal-time form of Eq. 14-16: gaps (P_k - T_k)/a_k, argmin
// (Eq. 25), internal-time advance, jump, and one fresh Exp(1) (Eq. 26).
// The same kernel also runs Gillespie's direct method (section 3, Eq.
// 17-22), the method the paper compares against: total rate a_0 = sum a_k,
// waiting time Exp(1)/a_0 and a search of the running sums for the first to
// reach u a_0, both numbers from one Philox block per firing at counter
// (firing index, 0xFFFFFFFF, trajectory, net).
#include <hip/hip_runtime.h>

#include "internal.h"
#include "rt_device.h"
#include "rt_wave.h"

namespace {

// X[j] for a wave-uniform j (a species index of the network): a switch
// becomes scalar branches, so X stays in registers instead of being copied
// to scratch memory for an indexed load.
template <int NT>
__device__ __forceinline__ int32_t pick(const int32_t (&X)[NT], int j)
{
    switch (j) {
        case 1: if constexpr (NT > 1) return X[1]; break;
        case 2: if constexpr (NT > 2) return X[2]; break;
        case 3: if constexpr (NT > 3) return X[3]; break;
        case 4: if constexpr (NT > 4) return X[4]; break;
        case 5: if constexpr (NT > 5) return X[5]; break;
        case 6: if constexpr (NT > 6) return X[6]; break;
        case 7: if constexpr (NT > 7) return X[7]; break;
        default: break;
    }
    return X[0];
}

// a_k of Eq. 1-2 with the reaction kind fixed per channel (uniform branch)
// and X in registers.
template <int NT>
__device__ __forceinline__ double propensity(int kind, int s0, int s1, double c,
                                             const int32_t (&X)[NT])
{
    return rt_propensity(kind, s0, s1, c, [&](int j) { return pick<NT>(X, j); });
}

// Collects one lane's writes to one 64-byte line in its LDS buffer and
// stores them together when the next write falls in another line (or on
// flush); only the words the lane wrote are stored.
struct rt_line_writer {
    int32_t* buf;       // 16 words of LDS
    uint64_t line;      // address >> 6 of the buffered line (~0: none)
    uint32_t mask;      // words written

    __device__ __forceinline__ void flush()
    {
        if (mask) {
            int32_t* const base = (int32_t*)(line << 6);
#pragma unroll
            for (int w = 0; w < 16; ++w)
                if (mask & (1u << w)) base[w] = buf[w];
            mask = 0u;
        }
    }

    __device__ __forceinline__ void put(int32_t* p, int32_t v)
    {
        const uint64_t addr = (uint64_t)p;
        if ((addr >> 6) != line) {
            flush();
            line = addr >> 6;
        }
        const int w = (int)((addr >> 2) & 15u);
        buf[w] = v;
        mask |= 1u << w;
    }
};

// Waves per SIMD each instantiation is compiled for: the most at which its
// state (X, n, a and, for the random-time method, T, P and 1/a, in registers;
// the network in SGPRs; with a rate schedule, the lane's rates too) fits
// without spilling to scratch.
constexpr int thread_min_waves(int MT, int NT, int METHOD, bool SCHED)
{
    if (METHOD == RTSSA_METHOD_DIRECT) return 4;
    // 5 waves fit without scratch up to 3 channels and 2 species (and 2 x 4);
    // on the Lotka-Volterra ensemble they measured 2.7 % faster than 4
    if (!SCHED && ((MT <= 2 && NT <= 4) || (MT == 3 && NT <= 2))) return 5;
    if (!SCHED) return MT <= 4 ? 4 : (MT == 8 && NT == 8 ? 2 : 3);
    // with a schedule each lane also holds its rates in force
    if (MT <= 2 || (MT <= 4 && NT <= 4)) return 4;
    if (MT <= 4 || (MT == 6 && NT <= 4)) return 3;
    return 2;
}

template <int MT, int NT, int METHOD, bool SCHED>
__global__ __launch_bounds__(256, thread_min_waves(MT, NT, METHOD, SCHED)) void rt_thread_kernel(rt_class_dev C)
{
    rt_ws* const ws = C.ws;
    // Issue priority of this kernel's wavefronts over other kernels' sharing a
    // CU (a batch runs class kernels side by side): a small network's class is
    // bound by its longest trajectories, one lane each, so its wavefronts go
    // first; alone on the device every wavefront has the same priority.
    __builtin_amdgcn_s_setprio(3);
    const uint32_t key0 = ws->key0, key1 = ws->key1;
    __shared__ uint32_t log_scratch[4][RT_LOG_SCRATCH];     // one slice per wave
    uint32_t* sc = log_scratch[threadIdx.x >> 6];
    // per-lane buffer of one 64-byte line of sample output: a lane's sample
    // row is written a few bytes at a time, at its own event times; collecting
    // the words of a line and storing them together lets the L2 write each
    // line back once instead of once per sample point
    __shared__ int32_t line_buf[256][16];
    int32_t* const lb = line_buf[threadIdx.x];

    int item = C.exclusive ? -1 : 0;
    bool first = true;
    for (;;) {
        // ---- the wavefront's next item (uniform)
        if (C.exclusive) {
            unsigned int v = 0;
            if ((threadIdx.x & 63) == 0) v = (unsigned int)atomicAdd(&ws->next_unit, 1ull);
            item = (int)__builtin_amdgcn_readfirstlane((int)__shfl((int)v, 0, 64));
        } else if (!first) {
            item = C.count;
        }
        first = false;
        if (item >= C.count) break;
        // read-only descriptor and network through the constant address space:
        // with a uniform item the loads are scalar and the constants SGPRs
        const rt_cptr<rt_item_dev> it = rt_const(C.items) + item;
        const rt_net_dev net = it->net;
        unsigned long long* const traj_ctr = C.item_next + item;

        // ---- network constants (uniform)
        int kind[MT], s0[MT], s1[MT], nu[MT][NT];
        double c[MT];
#pragma unroll
        for (int k = 0; k < MT; ++k) {
            if (k < net.M) {
                int2 rr = rt_const(net.react)[k];
                kind[k] = (int)((uint32_t)rr.x >> 29);
                s0[k] = rr.x & RT_SPECIES_MASK;
                s1[k] = rr.y;
                c[k] = rt_const(net.c)[k];
            } else {
                kind[k] = RT_H_ZERO; s0[k] = 0; s1[k] = 0; c[k] = 0.0;   // dead padding channel
            }
#pragma unroll
            for (int j = 0; j < NT; ++j)
                nu[k][j] = (k < net.M && j < net.N) ? rt_const(net.nu_dense)[k * net.N + j] : 0;
        }
        const int N = net.N, M = net.M;
        // rate schedule of the item (SCHED builds only): breakpoints and rows
        const int32_t sB = SCHED ? net.sched_B : 0;
        const rt_cptr<double> sched_t = rt_const(net.sched_t);
        const rt_cptr<double> sched_c = rt_const(net.sched_c);
        const double t_end = it->t_end;
        const uint32_t net_id = it->net_id, traj_offset = it->traj_offset;
        const bool want_hash = it->seq_hash != nullptr;

        // ---- trajectory state
        int32_t X[NT];
        double T[MT], Pk[MT], a[MT], inv[MT];
        uint32_t n[MT];
#pragma unroll
        for (int j = 0; j < NT; ++j) X[j] = 0;
#pragma unroll
        for (int k = 0; k < MT; ++k) { T[k] = 0.0; Pk[k] = 0.0; a[k] = 0.0; inv[k] = 0.0; n[k] = 0; }
        double t = 0.0, s_next = 0.0;
        // SCHED: the rates in force for this lane's trajectory, the index of
        // the next breakpoint and its time
        double cl[MT];
        int32_t piece = 0;
        double b_next = __builtin_inf();
#pragma unroll
        for (int k = 0; k < MT; ++k) cl[k] = c[k];
        int32_t g = 0;
        uint32_t fired = 0, tie = kTieNone, traj = 0;
        unsigned long long hash = kFnvOffset;
        int64_t r = 0;

        rt_line_writer lw{lb, ~0ull, 0u};
        auto write_sample = [&](int32_t gg, bool invalid) {
            int32_t* dst = it->samples + r * it->ss_r + (int64_t)gg * it->ss_g;
#pragma unroll
            for (int j = 0; j < NT; ++j)
                if (j < N) lw.put(dst + j * it->ss_n, invalid ? -1 : X[j]);
        };

        // Each pass is one firing of every active lane.  The common path is
        // straight-line; every rare event (start or end of a trajectory, a
        // sample point, a near-tie, a clamped gap, an overflow, the firing
        // cap) is handled in one branch entered only when some lane of the
        // wave needs it.
        bool active = true, fresh = true, capped = false;
        while (__ballot(active) != 0ull) {
            if (!active) continue;
            // gaps and argmin (lowest k wins ties; d2 = second smallest gap)
            double d1 = __builtin_inf(), d2 = __builtin_inf();
            int mu = 0;
            if constexpr (METHOD == RTSSA_METHOD_RANDOM_TIME) {
                // A frozen channel (a_k = 0, 1/a_k = +inf) gives +inf while
                // P_k > T_k, so the raw gaps are the gaps unless one is negative
                // (clamped to 0) or a frozen channel has P_k <= T_k (NaN, -inf):
                // then, rarely, the wavefront takes the exact form.
                rt_min2 sel{__builtin_inf(), __builtin_inf(), 0};
                bool bad = false;
#pragma unroll
                for (int k = 0; k < MT; ++k) {
                    const double raw = (Pk[k] - T[k]) * inv[k];
                    bad = bad || !(raw >= 0.0);
                    rt_min2_push(sel, raw, k);
                }
                if (__builtin_expect(__ballot(bad) != 0ull, 0)) {
                    sel = rt_min2{__builtin_inf(), __builtin_inf(), 0};
#pragma unroll
                    for (int k = 0; k < MT; ++k) {
                        const double raw = (Pk[k] - T[k]) * inv[k];
                        const double d = a[k] == 0.0 ? __builtin_inf() : fmax(raw, 0.0);
                        rt_min2_push(sel, d, k);
                    }
                }
                d1 = sel.d1;
                d2 = sel.d2;
                mu = sel.k;
            } else {
                // direct method: total rate, one block for the waiting time and
                // the search (padding channels add +0 and are never reached)
                double a0 = 0.0;
#pragma unroll
                for (int k = 0; k < MT; ++k) a0 += a[k];
                const rt_u4 w = rt_philox4x32_10(rt_u4{fired, 0xFFFFFFFFu, traj, net_id}, key0, key1);
                const uint64_t m1 = (((uint64_t)w.y << 32) | w.x) >> 11;
                const uint64_t m2 = (((uint64_t)w.w << 32) | w.z) >> 11;
                const double E1 = rt_neglog_wave(m1, false, &ws->slow_logs, sc);
                d1 = a0 == 0.0 ? __builtin_inf() : E1 / a0;
                const double target = (double)(m2 + 1) * 0x1p-53 * a0;
                double run = 0.0;
                bool found = false;
                mu = MT - 1;
#pragma unroll
                for (int k = 0; k < MT; ++k) {
                    run += a[k];
                    const bool hit = !found && run >= target;
                    mu = hit ? k : mu;
                    found = found || hit;
                }
            }
            const double t_new = t + d1;
            const bool live = !fresh && !capped;          // a trajectory is in progress
            // a rate breakpoint before the next firing (and before t_end):
            // Eq. 28 is solved again from there
            const bool brk = SCHED && live && b_next < t_end && t_new > b_next;
            const bool absorbed = !brk && d1 == __builtin_inf();
            const bool term = !brk && (absorbed || t_new > t_end);
            // jump v_mu, checked against [0, 2^31 - 1]
            int32_t Xn[NT];
            bool ok = true;
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                int32_t dl = nu[0][j];
#pragma unroll
                for (int k = 1; k < MT; ++k) dl = (mu == k) ? nu[k][j] : dl;
                // X_j in [0, 2^31 - 1] and an int32 change: the exact sum is
                // outside that range exactly when its 32-bit wrap is negative
                const int32_t v = (int32_t)((uint32_t)X[j] + (uint32_t)dl);
                ok = ok && v >= 0;
                Xn[j] = v;
            }
            const bool event = live && !term && !brk;     // this pass may apply an event
            const bool near_tie = METHOD == RTSSA_METHOD_RANDOM_TIME && event &&
                                  rt_near_tie(d1, d2);
            // a zero gap may have been clamped from a negative raw gap
            const bool rare = !live || term || brk || near_tie ||
                              (METHOD == RTSSA_METHOD_RANDOM_TIME && d1 == 0.0) || !ok ||
                              s_next < t_new;
            if (__builtin_expect(__ballot(rare) != 0ull, 0)) {
                // Counted once per event: when another lane of the wave stops or
                // meets a breakpoint, this lane repeats its pass below without
                // applying its event, so the counters are bumped only once the
                // event is known to be applied (or, for a near-tie, when the
                // event ends the trajectory by an overflow, as the oracle counts
                // it); tie and the samples are idempotent.
                bool clamped = false;
                if (event) {
                    if (near_tie) tie = tie == kTieNone ? fired : tie;
                    while (s_next < t_new) {
                        if (it->samples) write_sample(g, false);
                        ++g;
                        s_next = g < it->G ? it->s[g] : __builtin_inf();
                    }
                    if (METHOD == RTSSA_METHOD_RANDOM_TIME && ok && d1 == 0.0) {
#pragma unroll
                        for (int k = 0; k < MT; ++k)
                            clamped = mu == k ? (Pk[k] - T[k]) * inv[k] < 0.0 : clamped;
                    }
                }
                if (SCHED && brk) {
                    // every internal clock runs to the breakpoint at the old
                    // rates; the propensities take the next piece's rates
                    const double db = b_next - t;
#pragma unroll
                    for (int k = 0; k < MT; ++k) T[k] = fma(a[k], db, T[k]);
                    t = b_next;
#pragma unroll
                    for (int k = 0; k < MT; ++k) cl[k] = k < M ? sched_c[piece * M + k] : 0.0;
                    ++piece;
                    b_next = piece < sB ? sched_t[piece] : __builtin_inf();
#pragma unroll
                    for (int k = 0; k < MT; ++k) {
                        a[k] = propensity<NT>(kind[k], s0[k], s1[k], cl[k], X);
                        inv[k] = 1.0 / a[k];
                    }
                }
                const bool stop = !live || term || (!ok && !brk);
                if (near_tie && stop) atomicAdd(&ws->near_ties, 1ull);   // event && !ok
                if (stop && !fresh) {
                    // end of the trajectory
                    const int st = capped ? RTSSA_TRAJ_MAX_FIRINGS
                                          : (absorbed ? RTSSA_TRAJ_ABSORBED
                                                      : (term ? RTSSA_TRAJ_OK : RTSSA_TRAJ_OVERFLOW));
                    const bool good = st == RTSSA_TRAJ_OK || st == RTSSA_TRAJ_ABSORBED;
                    if (it->samples) {
                        for (int32_t gg = g; gg < it->G; ++gg) write_sample(gg, !good);
                        lw.flush();
                    }
                    if (METHOD == RTSSA_METHOD_RANDOM_TIME && good) {
                        const double dt = t_end - t;
#pragma unroll
                        for (int k = 0; k < MT; ++k) T[k] = fma(a[k], dt, T[k]);
                    }
                    if (it->n_out) {
#pragma unroll
                        for (int k = 0; k < MT; ++k) if (k < M) it->n_out[r * M + k] = n[k];
                    }
                    if (METHOD == RTSSA_METHOD_RANDOM_TIME && it->T_out) {
#pragma unroll
                        for (int k = 0; k < MT; ++k) if (k < M) it->T_out[r * M + k] = T[k];
                    }
                    if (it->x_final) {
#pragma unroll
                        for (int j = 0; j < NT; ++j) if (j < N) it->x_final[r * N + j] = X[j];
                    }
                    if (it->t_last) it->t_last[r] = t;
                    if (it->status) it->status[r] = (uint8_t)st;
                    if (it->seq_hash) it->seq_hash[r] = hash;
                    if (METHOD == RTSSA_METHOD_RANDOM_TIME && it->tie_step) it->tie_step[r] = tie;
                    atomicAdd(&ws->firings, (unsigned long long)fired);
                    atomicAdd(&ws->status_count[st], 1ull);
                }
                if (stop) {
                    // take the next trajectory of this item
                    const int64_t rr = (int64_t)atomicAdd(traj_ctr, 1ull);
                    fresh = false;
                    capped = false;
                    active = rr < it->R;
                    if (active) {
                        r = rr;
                        traj = traj_offset + (uint32_t)rr;
                        const int32_t* x0 = it->x0 + (it->x0_per_traj ? rr * N : 0);
#pragma unroll
                        for (int j = 0; j < NT; ++j) X[j] = j < N ? x0[j] : 0;
                        t = 0.0;
                        g = 0;
                        s_next = it->G > 0 ? it->s[0] : __builtin_inf();
                        fired = 0;
                        tie = kTieNone;
                        hash = kFnvOffset;
                        if constexpr (SCHED) {
                            piece = 0;
                            b_next = sB > 0 ? sched_t[0] : __builtin_inf();
#pragma unroll
                            for (int k = 0; k < MT; ++k) cl[k] = c[k];
                        }
#pragma unroll
                        for (int k = 0; k < MT; ++k) {
                            n[k] = 0;
                            a[k] = propensity<NT>(kind[k], s0[k], s1[k], SCHED ? cl[k] : c[k], X);
                        }
                        if constexpr (METHOD == RTSSA_METHOD_RANDOM_TIME) {
#pragma unroll
                            for (int k = 0; k < MT; ++k) {
                                T[k] = 0.0;
                                inv[k] = 1.0 / a[k];
                            }
                            // first internal firing times, one draw at a time
#pragma unroll 1
                            for (int k = 0; k < MT; ++k) {
                                const double E0 = rt_exp1_wave(key0, key1, traj, net_id,
                                                               (uint32_t)k, 0u, &ws->slow_logs, sc);
#pragma unroll
                                for (int q = 0; q < MT; ++q) Pk[q] = q == k ? E0 : Pk[q];
                            }
                        }
                    }
                }
                // started lanes (and lanes past a breakpoint) compute their gaps
                if (__ballot(stop || brk) != 0ull) continue;
                // the event is applied below
                if (near_tie) atomicAdd(&ws->near_ties, 1ull);
                if (clamped) atomicAdd(&ws->clamps, 1ull);
            }
            if constexpr (METHOD == RTSSA_METHOD_DIRECT) {
#pragma unroll
                for (int k = 0; k < MT; ++k) n[k] += mu == k ? 1u : 0u;
#pragma unroll
                for (int j = 0; j < NT; ++j) X[j] = Xn[j];
                t = t_new;
                ++fired;
                if (want_hash) hash = (hash ^ (unsigned long long)(uint32_t)mu) * kFnvPrime;
#pragma unroll
                for (int k = 0; k < MT; ++k) a[k] = propensity<NT>(kind[k], s0[k], s1[k], SCHED ? cl[k] : c[k], X);
                capped = fired >= C.max_firings;
                continue;
            }
            // internal times advance by a_k Delta (Eq. 15); the fired channel
            // lands exactly on its firing internal time
            uint32_t n_mu = 0;
            double p_mu = 0.0;
#pragma unroll
            for (int k = 0; k < MT; ++k) {
                const bool f = mu == k;
                T[k] = f ? Pk[k] : fma(a[k], d1, T[k]);
                n[k] += f ? 1u : 0u;
                n_mu = f ? n[k] : n_mu;
                p_mu = f ? Pk[k] : p_mu;
            }
#pragma unroll
            for (int j = 0; j < NT; ++j) X[j] = Xn[j];
            t = t_new;
            ++fired;
            if (want_hash) hash = (hash ^ (unsigned long long)(uint32_t)mu) * kFnvPrime;
            p_mu = p_mu + rt_exp1_wave(key0, key1, traj, net_id, (uint32_t)mu, n_mu,
                                       &ws->slow_logs, sc);
            // a_k is a pure function of X; inv_k = RN(1 / a_k) (+inf for a dead
            // channel, whose gap is +inf by the a_k = 0 test and never reads it)
#pragma unroll
            for (int k = 0; k < MT; ++k) {
                Pk[k] = (mu == k) ? p_mu : Pk[k];
                a[k] = propensity<NT>(kind[k], s0[k], s1[k], SCHED ? cl[k] : c[k], X);
                inv[k] = 1.0 / a[k];
            }
            capped = fired >= C.max_firings;
        }
    }
}

// Prepares one launch: clears the counters of ws and `extra` (item counters),
// sets the Philox key (from key_src when given, so that a captured graph can
// be replayed with new seeds), and for a single run checks its sample grid
// and stores its item descriptor and unit range.  A grid that is not
// non-decreasing within [0, t_end] leaves the run with no work (R = 0 in the
// stored descriptor), marks every trajectory RTSSA_TRAJ_NOT_RUN and sets
// ws->bad_input, so the simulation kernels that follow exit at once and the
// host learns of it without reading the grid itself.
__global__ void rt_setup_kernel(rt_ws* ws, unsigned long long* extra, int64_t n_extra,
                                uint32_t key0, uint32_t key1, const uint32_t* key_src,
                                rt_item_dev item, rt_item_dev* item_dst, int64_t* unit_start,
                                int64_t R)
{
    const int64_t i0 = threadIdx.x + (int64_t)blockIdx.x * blockDim.x;
    const int64_t stride = (int64_t)blockDim.x * gridDim.x;
    for (int64_t i = i0; i < n_extra; i += stride) extra[i] = 0ull;
    bool bad = false;
    if (item_dst && blockIdx.x == 0) {             // uniform over the block
        for (int g = threadIdx.x; g < item.G; g += blockDim.x) {
            const double s = item.s[g];
            bad = bad || !(s >= 0.0 && s <= item.t_end) || (g > 0 && s < item.s[g - 1]);
        }
        bad = __syncthreads_or(bad);
        if (bad && item.status)
            for (int64_t r = threadIdx.x; r < R; r += blockDim.x)
                item.status[r] = (uint8_t)RTSSA_TRAJ_NOT_RUN;
    }
    if (i0 == 0) {
        ws->firings = ws->near_ties = ws->clamps = ws->slow_logs = 0ull;
        for (int q = 0; q < 4; ++q) ws->status_count[q] = 0ull;
        ws->next_unit = 0ull;
        ws->bad_input = bad ? 1ull : 0ull;
        ws->key0 = key_src ? key_src[0] : key0;
        ws->key1 = key_src ? key_src[1] : key1;
        if (item_dst) {
            rt_item_dev it = item;
            if (bad) it.R = 0;
            *item_dst = it;
            unit_start[0] = 0;
            unit_start[1] = bad ? 0 : R;
        }
    }
}

typedef void (*thread_kernel_t)(rt_class_dev);

template <int MT, int NT>
int launch_mn(const rt_class_dev& C, int block, int grid, hipStream_t stream, int* grid_used,
              int64_t lanes_wanted, int method, bool sched)
{
    thread_kernel_t kfn = method == RTSSA_METHOD_DIRECT
                              ? rt_thread_kernel<MT, NT, RTSSA_METHOD_DIRECT, false>
                              : (sched ? rt_thread_kernel<MT, NT, RTSSA_METHOD_RANDOM_TIME, true>
                                       : rt_thread_kernel<MT, NT, RTSSA_METHOD_RANDOM_TIME, false>);
    if (grid <= 0) {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return rt_fail(RTSSA_E_HIP, "device query failed");
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, block, 0) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        int64_t need = (lanes_wanted + block - 1) / block;
        int64_t full = (int64_t)cus * per_cu;
        grid = (int)std::max<int64_t>(1, std::min<int64_t>(need, full));
    }
    if (grid_used) *grid_used = grid;
    hipLaunchKernelGGL(kfn, dim3(grid), dim3(block), 0, stream, C);
    return hipGetLastError() == hipSuccess ? RTSSA_OK : rt_fail(RTSSA_E_HIP, "thread kernel launch failed");
}

template <int MT>
int launch_m(int N, const rt_class_dev& C, int block, int grid, hipStream_t stream, int* gu,
             int64_t lanes, int method, bool sched)
{
    if (N <= 1) return launch_mn<MT, 1>(C, block, grid, stream, gu, lanes, method, sched);
    if (N <= 2) return launch_mn<MT, 2>(C, block, grid, stream, gu, lanes, method, sched);
    if (N <= 4) return launch_mn<MT, 4>(C, block, grid, stream, gu, lanes, method, sched);
    return launch_mn<MT, 8>(C, block, grid, stream, gu, lanes, method, sched);
}

}  // namespace

int rt_thread_supported(int M, int N)
{
    return M >= 0 && N >= 0 && M <= RT_THREAD_MAX_M && N <= RT_THREAD_MAX_N;
}

// M and N are the largest of the class (the kernel pads with dead channels
// and absent species); lanes = trajectories wanted in flight.
int rt_launch_thread(int M, int N, const rt_class_dev& C, int block, int grid,
                     hipStream_t stream, int* grid_used, int64_t lanes, int method)
{
    const bool sched = C.has_schedule != 0;
    if (sched && method != RTSSA_METHOD_RANDOM_TIME)
        return rt_fail(RTSSA_E_UNSUPPORTED, "rate schedules run with the random-time method");
    if (!rt_thread_supported(M, N))
        return rt_fail(RTSSA_E_UNSUPPORTED, "network too large for the thread mapping");
    if (block <= 0) block = 256;
    if (block > 256 || block % 64)
        return rt_fail(RTSSA_E_INVALID, "thread mapping block must be a multiple of 64, <= 256");
    switch (M) {
        case 0:
        case 1: return launch_m<1>(N, C, block, grid, stream, grid_used, lanes, method, sched);
        case 2: return launch_m<2>(N, C, block, grid, stream, grid_used, lanes, method, sched);
        case 3: return launch_m<3>(N, C, block, grid, stream, grid_used, lanes, method, sched);
        case 4: return launch_m<4>(N, C, block, grid, stream, grid_used, lanes, method, sched);
        case 5:
        case 6: return launch_m<6>(N, C, block, grid, stream, grid_used, lanes, method, sched);
        default: return launch_m<8>(N, C, block, grid, stream, grid_used, lanes, method, sched);
    }
}

int rt_launch_setup(rt_ws* ws, unsigned long long* extra, int64_t n_extra, uint32_t key0,
                    uint32_t key1, const uint32_t* key_src, const rt_item_dev* item,
                    rt_item_dev* item_dst, int64_t* unit_start, hipStream_t stream)
{
    rt_item_dev it{};
    if (item) it = *item;
    const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(64, (n_extra + 255) / 256));
    hipLaunchKernelGGL(rt_setup_kernel, dim3(nb), dim3(256), 0, stream, ws, extra, n_extra, key0,
                       key1, key_src, it, item ? item_dst : nullptr, unit_start,
                       item ? item->R : (int64_t)0);
    return hipGetLastError() == hipSuccess ? RTSSA_OK : rt_fail(RTSSA_E_HIP, "setup launch failed");
}
