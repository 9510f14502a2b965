// kernels_group_lds.hip -- workgroup-per-trajectory mapping with the
// propensities in LDS and one workgroup barrier per firing.
//
// One workgroup of L threads (W = L / 64 wavefronts) simulates one trajectory
// at a time from a device work queue (persistent grid).  Channel k belongs to
// thread k mod L, slot k / L (slots past M are frozen channels).  Per thread,
// registers hold each slot's T_k, P_k, the channel's next unit-exponential
// draw E(k, n_k + 1) (computed ahead, off the firing's critical path) and
// n_k.  LDS holds (a_k, 1/a_k) of every
// channel and two buffers of the species counts X.
//
// One firing (section 4, Table 2, in the internal-time form of Eq. 14-16):
//   pass    every thread reads (a_k, 1/a_k) of its slots, forms the gaps
//           (P_k - T_k)/a_k and a local argmin with second minimum;
//   argmin  across the wavefront by DPP and permlane exchanges, across
//           wavefronts through LDS -- the firing's only barrier; lowest k wins
//           ties (Eq. 25);
//   event   every wavefront loads mu's fixed-stride rows (its jump v_mu and
//           the records of the channels D(mu) reading a changed species --
//           Gibson & Bruck's dependency graph, cited in section 5 -- with
//           their reactants, rates and the reactants' changes under v_mu:
//           one round trip), checks the jump, advances
//           its own internal clocks (Eq. 15: T_k += a_k Delta; T_mu = P_mu and
//           P_mu += E, Eq. 26), and recomputes (a_k, 1/a_k) of the channels
//           of D(mu) it owns, from X + v_mu; wavefront 0 writes X + v_mu into
//           the other X buffer.
// A wavefront writes only its own channels' LDS entries, and the X buffer
// written at firing f is read only after the next firing's barrier, so the
// event needs no second barrier.  The draws E(k, n + 1) a channel will need
// are kept per slot; after a firing the slot's next draw is refilled later,
// for many slots of a wavefront at once (one Philox4x32-10 block and one
// logarithm per lane), at once when the channel fires again before its
// refill.  Refills run between issuing mu's row loads and using them.  Every
// value is the one of the contract: the schedule of the refills changes no
// result.
//
// With piecewise-constant rates (Eq. 28), a next firing past the next rate
// breakpoint b instead runs every clock to b at the old rates and recomputes
// every propensity with the new ones; nothing fires at b.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "rt_device.h"
#include "rt_wave.h"

namespace {

struct g2_shared {
    rt_sel_part part[2][16];             // per selection parity, per wavefront
    unsigned long long next_traj;
    uint32_t log_scratch[16][RT_LOG_SCRATCH];
};

// Refills are made once this many lanes of a wavefront have one pending.
constexpr int kRefillLanes = 16;

// Waves per SIMD the register allocation aims at (per slot: T, P and the next
// draw, 6 registers, plus n_k).
constexpr int g2_min_waves(int S) { return S >= 16 ? 2 : (S >= 8 ? 3 : 4); }

template <int L, int S, bool SCHED>
__global__ __launch_bounds__(L, g2_min_waves(S)) void rt_group_lds_kernel(rt_class_dev C)
{
    constexpr int W = L / 64;
    constexpr int LOG2L = __builtin_ctz(L);
    extern __shared__ __align__(16) double g2_lds[];
    __shared__ g2_shared sh;
    rt_ws* const ws = C.ws;
    const uint32_t key0 = ws->key0, key1 = ws->key1;
    const rt_cptr<int64_t> unit_start = rt_const(C.unit_start);
    const int64_t total = unit_start[C.count];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // a_k and 1/a_k as two arrays, so that a wavefront reading either for its
    // slots touches consecutive 8-byte words (no bank conflicts)
    double* const pa = g2_lds;                                    // [L S] a_k
    double* const pinv = g2_lds + L * S;                          // [L S] 1/a_k
    const int Npad = (C.max_N + 3) & ~3;
    int32_t* const Xb = (int32_t*)(g2_lds + 2 * L * S);           // [2][Npad]
    uint32_t* sc = sh.log_scratch[wave];

    double T[S], P[S], En[S];
    uint32_t nk[S];
#pragma unroll
    for (int s = 0; s < S; ++s) { T[s] = 0.0; P[s] = 0.0; En[s] = 0.0; nk[s] = 0u; }

    for (;;) {
        // ---- next trajectory unit (uniform over the workgroup)
        if (tid == 0) sh.next_traj = atomicAdd(&ws->next_unit, 1ull);
        __syncthreads();
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
        const rt_cptr<int32_t> dep_ptr = rt_const(net.dep_ptr), dep_idx = rt_const(net.dep_idx);
        const rt_cptr<int4> grow = rt_const(net.grow);
        const rt_cptr<double> growc = rt_const(net.growc);
        const rt_cptr<int2> gdel = rt_const(net.gdel);
        const rt_cptr<int2> nu_fixed = rt_const(net.nu_fixed);
        const int nu_stride = net.nu_stride;
        const rt_cptr<double> grid_s = rt_const(it->s);
        const int64_t r = u - unit_start[item];
        const uint32_t traj = it->traj_offset + (uint32_t)r;
        const uint32_t net_id = it->net_id;
        const double t_end = it->t_end;
        const int32_t sB = SCHED ? net.sched_B : 0;
        rt_cptr<double> crate = cc;
        int32_t piece = 0;
        double b_next = sB > 0 ? rt_const(net.sched_t)[0] : __builtin_inf();

        // ---- initial state: both X buffers = x0; per channel a, 1/a, P = E(k, 0)
        // and the next draw E(k, 1) (the two words of one Philox block)
        const int32_t* x0 = it->x0 + (it->x0_per_traj ? r * N : 0);
        for (int j = tid; j < N; j += L) {
            const int32_t v = x0[j];
            Xb[j] = v;
            Xb[Npad + j] = v;
        }
        __syncthreads();
#pragma unroll 1
        for (int s1 = 0; s1 < S; ++s1) {
            const int k = tid + s1 * L;
            const bool live = k < M;
            double an = 0.0, in = __builtin_inf();
            uint64_t m0 = 0x1FFFFFFFFFFFFFull, m1 = 0x1FFFFFFFFFFFFFull;   // u = 1: no work
            if (live) {
                an = rt_propensity_mem(react[k], crate[k], Xb);
                in = 1.0 / an;
                const rt_u4 w =
                    rt_philox4x32_10<false>(rt_u4{0u, (uint32_t)k, traj, net_id}, key0, key1);
                m0 = (((uint64_t)w.y << 32) | w.x) >> 11;
                m1 = (((uint64_t)w.w << 32) | w.z) >> 11;
            }
            // a padding slot (k >= M) keeps P = +inf: its gap is +inf in the pass
            const double e0 = rt_neglog_wave(m0, false, &ws->slow_logs, sc);
            const double p1 = rt_neglog_wave(m1, false, &ws->slow_logs, sc);
            const double p0 = live ? e0 : __builtin_inf();
            pa[k] = an;
            pinv[k] = in;
#pragma unroll
            for (int s = 0; s < S; ++s) {
                P[s] = s == s1 ? p0 : P[s];
                En[s] = s == s1 ? p1 : En[s];
            }
        }
#pragma unroll
        for (int s = 0; s < S; ++s) { T[s] = 0.0; nk[s] = 0u; }
        uint32_t pending = 0u;       // slots whose next draw is not computed yet
        int prev_sp = -1;            // this lane's jump entry of the previous firing
        double t = 0.0, s_next = it->G > 0 ? grid_s[0] : __builtin_inf();
        int32_t g = 0;
        uint32_t fired = 0, tie = kTieNone;
        unsigned long long hash = kFnvOffset;
        int st = RTSSA_TRAJ_OK;
        uint32_t reduces = 0;        // parity picks the argmin's LDS buffer

        for (;;) {
            // ---- pass: gaps (P_k - T_k) / a_k and the lane's two smallest.
            // A frozen channel (a_k = 0, 1/a_k = +inf) gives +inf while
            // P_k > T_k; a negative raw gap (clamped to 0) or a frozen channel
            // with P_k <= T_k (NaN, -inf) is rare and sends the wavefront
            // through the exact form below.
            double d1 = __builtin_inf(), d2 = __builtin_inf();
            int ks = 0;
            bool bad = false;
            // every slot's 1/a_k read at once (the scheduling barrier keeps the
            // compiler from interleaving the reads with the arithmetic and
            // waiting on each in turn)
            double iv[S];
#pragma unroll
            for (int s = 0; s < S; ++s) iv[s] = pinv[tid + s * L];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const double raw = (P[s] - T[s]) * iv[s];
                bad = bad || !(raw >= 0.0);
                const bool lt = raw < d1;          // the lower slot wins equal values
                d2 = fmin(d2, fmax(d1, raw));
                d1 = fmin(d1, raw);
                ks = lt ? s : ks;
            }
            if (__builtin_expect(__ballot(bad) != 0ull, 0)) {
                d1 = __builtin_inf();
                d2 = __builtin_inf();
                ks = 0;
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    const double raw = (P[s] - T[s]) * pinv[tid + s * L];
                    const double d = pa[tid + s * L] == 0.0 ? __builtin_inf() : fmax(raw, 0.0);
                    const bool lt = d < d1;
                    d2 = fmin(d2, fmax(d1, d));
                    d1 = fmin(d1, d);
                    ks = lt ? s : ks;
                }
            }
            // ---- selection over the workgroup: the firing's barrier
            const rt_min2 sel = rt_select_group<L>(d1, d2, tid + (ks << LOG2L),
                                                   sh.part[reduces & 1u]);
            ++reduces;
            d1 = sel.d1;
            d2 = sel.d2;
            const int mu = __builtin_amdgcn_readfirstlane(sel.k);
            const double t_new = t + d1;
            const int32_t* const Xc = Xb + (fired & 1u) * Npad;      // X after `fired` firings
            int32_t* const Xn = Xb + ((fired + 1u) & 1u) * Npad;     // the other buffer
            // ---- mu's rows, one round trip: the jump (lane q: entry q) and
            // the dependency records (lane 0: mu itself, whose propensity may
            // read a species it changes; lane q >= 1: the q-th other channel
            // of D(mu) or k = -1), each with its reactants, rate and the
            // change of those reactants under v_mu.  Without a rate schedule
            // they are issued before the end tests (row 0 when nothing can
            // fire), which then run while they load.
            const int mr = d1 == __builtin_inf() ? 0 : mu;
            int4 gr;
            double gc;
            int2 dd, nv;
            auto load_rows = [&]() {
                gr = grow[mr * 64 + lane];
                gc = growc[mr * 64 + lane];
                dd = gdel[mr * 64 + lane];
                nv = nu_fixed[mr * nu_stride + min(lane, nu_stride - 1)];
            };
            if constexpr (!SCHED) load_rows();
            if (SCHED && __builtin_amdgcn_readfirstlane(b_next < t_end && t_new > b_next)) {
                // every clock runs to the breakpoint at the old rates; every
                // propensity takes the next piece's rates (Eq. 28 again)
                const double db = b_next - t;
#pragma unroll
                for (int s = 0; s < S; ++s) T[s] = fma(pa[tid + s * L], db, T[s]);
                t = b_next;
                crate = rt_const(net.sched_c) + (size_t)piece * M;
                ++piece;
                b_next = piece < sB ? rt_const(net.sched_t)[piece] : __builtin_inf();
#pragma unroll 1
                for (int s1 = 0; s1 < S; ++s1) {
                    const int k = tid + s1 * L;
                    if (k < M) {
                        const double an = rt_propensity_mem(react[k], crate[k], Xc);
                        pa[k] = an;
                        pinv[k] = 1.0 / an;
                    }
                }
                continue;
            }
            if (d1 == __builtin_inf()) { st = RTSSA_TRAJ_ABSORBED; break; }
            if (t_new > t_end) { st = RTSSA_TRAJ_OK; break; }
            if constexpr (SCHED) load_rows();
            // ---- draws, while the rows load: a wavefront refills one waiting
            // slot per lane once enough lanes have one, and at once when it
            // owns mu and mu's next draw E(mu, n_mu + 1) is still waiting (the
            // owner lane then takes that slot)
            const int owner = mu & (L - 1);
            const int sm = mu >> LOG2L;                     // uniform slot of mu
            const bool need = wave == (owner >> 6) &&
                              __builtin_amdgcn_readlane((int)((pending >> sm) & 1u), owner & 63);
            if (need || __popcll(__ballot(pending != 0u)) >= kRefillLanes) {
                const bool has = pending != 0u;
                const int s1 = (need && tid == owner) ? sm : (has ? __builtin_ctz(pending) : 0);
                uint32_t n1 = 0u;
#pragma unroll
                for (int s = 0; s < S; ++s) n1 = s == s1 ? nk[s] : n1;
                const uint64_t m = has ? rt_draw_m53<false>(key0, key1, traj, net_id,
                                                            (uint32_t)(tid + s1 * L), n1 + 1u)
                                       : 0x1FFFFFFFFFFFFFull;
                const double E = rt_neglog_wave(m, false, &ws->slow_logs, sc);
#pragma unroll
                for (int s = 0; s < S; ++s) En[s] = (has && s == s1) ? E : En[s];
                pending &= ~(has ? 1u << s1 : 0u);
            }
            const int n_other = __builtin_amdgcn_readlane(gr.w, 0);
            const int kd = gr.x;
            const bool mine = kd >= 0 && ((kd & (L - 1)) >> 6) == wave;
            const int2 rr = make_int2(gr.y, gr.z);
            // (with a rate schedule the rates in force come from the piece)
            const double cr = SCHED ? crate[mine ? kd : mu] : gc;
            if (rt_near_tie(d1, d2)) {
                if (tid == 0) atomicAdd(&ws->near_ties, 1ull);
                tie = tie == kTieNone ? fired : tie;
            }
            while (s_next < t_new) {                        // samples before the event
                if (it->samples) {
                    int32_t* dst = it->samples + r * it->ss_r + (int64_t)g * it->ss_g;
                    for (int j = tid; j < N; j += L) dst[j * it->ss_n] = Xc[j];
                }
                ++g;
                s_next = g < it->G ? grid_s[g] : __builtin_inf();
            }
            // ---- the jump v_mu, checked against [0, 2^31 - 1] (every
            // wavefront takes the same decision)
            const bool has_nu = lane < nu_stride && nv.x >= 0;
            const int sp = max(nv.x, 0), dl = nv.y;
            const int64_t xv = (int64_t)Xc[sp] + dl;
            const bool okl = !has_nu || (xv >= 0 && xv <= 0x7FFFFFFF);
            if (__ballot(!okl) != 0ull) { st = RTSSA_TRAJ_OVERFLOW; break; }
            // ---- internal clocks (Eq. 15), the fired channel's firing time and
            // next draw (Eq. 26)
            bool clamped = false;
            if (d1 == 0.0 && tid == owner) {
                // a zero gap: was it clamped from a negative raw gap?
#pragma unroll
                for (int s = 0; s < S; ++s)
                    if (s == sm) clamped = (P[s] - T[s]) * pinv[mu] < 0.0;
            }
            // (a_k as read by the pass: this wavefront writes its channels'
            // entries only below)
            {
                double av[S];
#pragma unroll
                for (int s = 0; s < S; ++s) av[s] = pa[tid + s * L];
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int s = 0; s < S; ++s) T[s] = fma(av[s], d1, T[s]);
            }
            if (tid == owner) {
                if constexpr (!SCHED) {
                    // (sm is uniform: the compiler indexes the register arrays
                    // directly rather than selecting over every slot)
                    const double pm = P[sm];
                    T[sm] = pm;
                    P[sm] = pm + En[sm];
                    ++nk[sm];
                } else {
                    // (with the schedule's registers the indexed form would
                    // move the arrays to scratch memory)
#pragma unroll
                    for (int s = 0; s < S; ++s)
                        if (s == sm) {
                            T[s] = P[s];
                            P[s] = P[s] + En[s];
                            ++nk[s];
                        }
                }
                pending |= 1u << sm;
                if (clamped) atomicAdd(&ws->clamps, 1ull);
            }
            // ---- X + v_mu into the other buffer (wavefront 0): that buffer
            // holds X before the previous firing, so the previous firing's
            // species are copied first, then this firing's written
            if (wave == 0) {
                if (prev_sp >= 0) Xn[prev_sp] = Xc[prev_sp];
                if (has_nu) Xn[sp] = (int32_t)xv;
            }
            prev_sp = has_nu ? sp : -1;
            // ---- new propensities of the channels of D(mu) this wavefront owns
            {
                auto xnew = [&](int j) {
                    int32_t v = Xc[j];
                    for (int q = 0; q < nu_stride; ++q) {
                        const int sq = __builtin_amdgcn_readlane(nv.x, q);
                        const int dq = __builtin_amdgcn_readlane(nv.y, q);
                        v += sq == j ? dq : 0;
                    }
                    return v;
                };
                if (mine) {
                    // both reactant counts after the jump: X before it plus
                    // the record's precomputed changes; h without branching
                    // on the lanes' kinds
                    const int kind = (int)((uint32_t)rr.x >> 29);
                    const int s0 = rr.x & RT_SPECIES_MASK, s1 = rr.y;
                    int32_t v0 = 0, v1 = 0;
                    if (kind != RT_H_ZERO) v0 = Xc[s0] + dd.x;
                    if (kind == RT_H_TWO) v1 = Xc[s1] + dd.y;
                    const double an = rt_propensity_counts(kind, (uint32_t)v0, (uint32_t)v1, cr);
                    pa[kd] = an;
                    pinv[kd] = 1.0 / an;
                }
                if (n_other > 63) {
                    // the rest of D(mu) from its 64th other channel on
                    const int de = dep_ptr[mu + 1];
                    for (int q0 = __builtin_amdgcn_readlane(gr.w, 1); q0 < de; q0 += 64) {
                        const int q = q0 + lane;
                        const int k2 = q < de ? dep_idx[q] : -1;
                        if (k2 >= 0 && k2 != mu && ((k2 & (L - 1)) >> 6) == wave) {
                            const int2 r2 = react[k2];
                            const double an = rt_propensity((int)((uint32_t)r2.x >> 29),
                                                            r2.x & RT_SPECIES_MASK, r2.y,
                                                            crate[k2], xnew);
                            pa[k2] = an;
                            pinv[k2] = 1.0 / an;
                        }
                    }
                }
            }
            ++fired;
            t = t_new;
            hash = (hash ^ (unsigned long long)(uint32_t)mu) * kFnvPrime;
            if (fired >= C.max_firings) { st = RTSSA_TRAJ_MAX_FIRINGS; break; }
        }

        // ---- end of the trajectory (after a capped firing wavefront 0's
        // X writes must be visible first)
        __syncthreads();
        const int32_t* const Xf = Xb + (fired & 1u) * Npad;
        const bool good = st == RTSSA_TRAJ_OK || st == RTSSA_TRAJ_ABSORBED;
        if (it->samples) {
            for (; g < it->G; ++g) {
                int32_t* dst = it->samples + r * it->ss_r + (int64_t)g * it->ss_g;
                for (int j = tid; j < N; j += L) dst[j * it->ss_n] = good ? Xf[j] : -1;
            }
        }
        const double dt = t_end - t;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int k = tid + s * L;
            if (k < M) {
                // OK / ABSORBED: the propensities in force since the last event
                if (good) T[s] = fma(pa[k], dt, T[s]);
                if (it->n_out) it->n_out[r * M + k] = nk[s];
                if (it->T_out) it->T_out[r * M + k] = T[s];
            }
        }
        if (it->x_final)
            for (int j = tid; j < N; j += L) it->x_final[r * N + j] = Xf[j];
        if (tid == 0) {
            if (it->t_last) it->t_last[r] = t;
            if (it->status) it->status[r] = (uint8_t)st;
            if (it->seq_hash) it->seq_hash[r] = hash;
            if (it->tie_step) it->tie_step[r] = tie;
            atomicAdd(&ws->firings, (unsigned long long)fired);
            atomicAdd(&ws->status_count[st], 1ull);
        }
        __syncthreads();                                   // LDS is reused next
    }
}

typedef void (*g2_kernel_t)(rt_class_dev);

template <int L, int S>
g2_kernel_t pick(bool sched)
{
    return sched ? rt_group_lds_kernel<L, S, true> : rt_group_lds_kernel<L, S, false>;
}

g2_kernel_t select_g2(int L, int S, bool sched)
{
#define RT_CASE(l, s) if (L == l && S == s) return pick<l, s>(sched);
    RT_CASE(64, 1) RT_CASE(64, 2) RT_CASE(64, 4) RT_CASE(64, 8) RT_CASE(64, 16)
    RT_CASE(128, 4) RT_CASE(128, 8) RT_CASE(128, 16)
    RT_CASE(256, 1) RT_CASE(256, 2) RT_CASE(256, 4) RT_CASE(256, 8) RT_CASE(256, 16)
    RT_CASE(512, 1) RT_CASE(512, 2) RT_CASE(512, 4) RT_CASE(512, 8)
    RT_CASE(1024, 1) RT_CASE(1024, 2) RT_CASE(1024, 4) RT_CASE(1024, 8)
#undef RT_CASE
    return nullptr;
}

}  // namespace

size_t rt_group_lds2_bytes(int N, int L, int S)
{
    return (size_t)L * S * 16 + (size_t)2 * ((N + 3) & ~3) * 4;
}

// The LDS-propensity kernel for this class, or nullptr when it does not
// exist or its LDS (dynamic and static) exceeds the device's per-workgroup
// limit.
const void* rt_group_lds_kernel_for(int M, int max_N, int L, bool sched)
{
    const int S = rt_group_slots(M, L);
    const g2_kernel_t k = select_g2(L, S, sched);
    if (!k) return nullptr;
    int dev = 0, lds_max = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
            hipSuccess)
        return nullptr;
    if (rt_group_lds2_bytes(max_N, L, S) + sizeof(g2_shared) > (size_t)lds_max) return nullptr;
    return (const void*)k;
}

int rt_launch_group_lds(int M, int max_N, const rt_class_dev& C, int L, int grid,
                        hipStream_t stream, int* grid_used)
{
    const int S = rt_group_slots(M, L);
    const void* kfn = rt_group_lds_kernel_for(M, max_N, L, C.has_schedule != 0);
    if (!kfn) return rt_fail(RTSSA_E_UNSUPPORTED, "no LDS-propensity group kernel for this size");
    const size_t lds = rt_group_lds2_bytes(max_N, L, S);
    if (lds > 48 * 1024 &&
        hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
            hipSuccess)
        return rt_fail(RTSSA_E_HIP, "cannot raise the LDS limit");
    if (grid <= 0) {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return rt_fail(RTSSA_E_HIP, "device query failed");
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, L, lds) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        grid = cus * per_cu;
    }
    if (grid_used) *grid_used = grid;
    hipLaunchKernelGGL((g2_kernel_t)kfn, dim3(grid), dim3(L), lds, stream, C);
    return hipGetLastError() == hipSuccess
               ? RTSSA_OK
               : rt_fail(RTSSA_E_HIP, "LDS-propensity group kernel launch failed");
}
