// kernels_lazy.hip -- the lazy form for large networks: one wavefront per
// trajectory, a minimum tree of fan-out 8 in LDS.
//
// The lazy form follows section 5's dependency graph in internal times
// (Eq. 14-16): after a firing of mu only the channels of D(mu) (those whose
// propensity reads a species mu changed) and mu itself are touched.  Each
// such channel k runs its internal time from its last update s_k to now at
// its old propensity, T_k = fma(a_k, t - s_k, T_k) (mu instead lands on its
// firing internal time, T_mu = P_mu, and draws the next one, Eq. 26), takes
// its new propensity and gets the absolute next firing time
// tau_k = t + max(0, (P_k - T_k) / a_k).  The next event is the smallest
// tau_k, lowest k on ties (Eq. 25).  Work per firing is O(|D(mu)| log M)
// rather than the eager form's O(M).
//
// Layout.  The wavefront's LDS region holds the species counts X and a
// minimum tree over the tau_k: the leaves are tau_k (M doubles); a node of
// level l >= 1 holds the smallest tau over its kFan children of level l - 1
// and that tau's channel.  Levels are built up to the first with at most 512
// entries (the leaves themselves when M <= 512); each lane scans its entries
// of that top level (up to 8, only the 64-entry chunks that exist) and one
// wavefront min reduction plus a ballot gives the next event, which every
// lane keeps in registers.  Each level is stored as two arrays (tau, channel)
// padded to a multiple of kFan entries with empty values, so that a node's
// children are read with a few 16-byte loads and no bounds tests; merges use
// selects, not branches.  Fan-out 8 measured faster than 16.  The near-tie
// test (a count only) needs the second smallest tau, the smallest over the
// siblings of mu's leaf and of its ancestors below the top level and over the
// top level's other entries; it is decided by one ballot while the firing's
// global loads are in flight.  The channels' T_k, s_k, P_k, a_k (32 bytes),
// n_k and the spare word of their last Philox block live in a global
// workspace, one slice per wavefront of the grid.
//
// A firing: the argmin gives mu; the wavefront loads mu's firing count and
// kept word first, then mu's fixed-stride rows (its jump and the channels it
// touches, so that one load round trip suffices before the records); mu's
// next Exp(1) is drawn from wave-uniform values (without a rate schedule its
// Philox rounds run on the scalar unit) while the records are on their way;
// the jump is checked and applied, then one lane per touched channel updates
// it and writes its leaf; the touched leaves' ancestors are recomputed level
// by level, one lane per touched channel (lanes that share an ancestor
// compute the same node), and the top level is reduced again.  No workgroup
// barrier is used: a wavefront's LDS accesses complete in program order.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "rt_device.h"
#include "rt_wave.h"

namespace {

constexpr int kFanLog = 3;               // children per node: 2^kFanLog
constexpr int kFan = 1 << kFanLog;
constexpr int kMaxLevels = 64 / kFan;    // the sum tree's levels above the leaves, at most
constexpr int kTopPer = 8;               // top-level entries per lane
constexpr int kTopMax = 64 * kTopPer;    // the tree stops at a level this small
// the lazy form's levels above the leaves: 2 reach 512 x 8^2 = 32768 channels,
// more than a wavefront's LDS holds
constexpr int kLazyLevels = 2;

struct rt_lazy_rec {                     // a channel's state in the workspace
    double T, s, P, a;
};

// A refreshed channel's next firing time: +inf when a = 0, else
// t + max(0, RN(RN(P - T) * RN(1 / a))); *clamped when the raw gap is negative.
__device__ __forceinline__ double lazy_tau(double t, double T, double P, double a, bool* clamped)
{
    const double raw = (P - T) * (1.0 / a);
    *clamped = a != 0.0 && raw < 0.0;
    return a == 0.0 ? __builtin_inf() : t + fmax(raw, 0.0);
}

// The tree of one trajectory: level 0 holds the leaves (tau; channel =
// index), levels 1 .. top the nodes; cnt = entries in use, every array padded
// to a multiple of kFan entries (+inf, INT_MAX).  Times are never -0 (t starts
// at +0 and only grows), so selects on '<' order them exactly.
struct lazy_tree {
    double* d[kMaxLevels + 1];
    int32_t* kk[kMaxLevels + 1];
    int cnt[kMaxLevels + 1];
    int top;
};

struct lazy_min {                        // smallest tau of a subtree and its channel
    double d;
    int32_t k;
};

__device__ __forceinline__ int padf(int n) { return (n + kFan - 1) & ~(kFan - 1); }

// The smaller of two entries, a covering lower channels than b (siblings in
// channel order): on equal values a, and so the lower channel, wins.
__device__ __forceinline__ lazy_min lazy_merge(const lazy_min& a, const lazy_min& b)
{
    const bool blt = b.d < a.d;
    return lazy_min{blt ? b.d : a.d, blt ? b.k : a.k};
}

// Node j of level l (1 <= l) from its kFan children, loaded together (the padded
// arrays make every child present) and merged pairwise, always left with
// right, so that ties go to the lower channel.
__device__ __forceinline__ lazy_min lazy_node(const lazy_tree& tr, int l, int j)
{
    const int c0 = j << kFanLog;
    lazy_min v[kFan];
    const double2* vd = (const double2*)(tr.d[l - 1] + c0);
#pragma unroll
    for (int i = 0; i < kFan / 2; ++i) {
        const double2 x = vd[i];
        v[2 * i].d = x.x;
        v[2 * i + 1].d = x.y;
    }
    if (l == 1) {
#pragma unroll
        for (int i = 0; i < kFan; ++i) v[i].k = c0 + i;
    } else {
        const int4* vk = (const int4*)(tr.kk[l - 1] + c0);
#pragma unroll
        for (int i = 0; i < kFan / 4; ++i) {
            const int4 x = vk[i];
            v[4 * i].k = x.x;
            v[4 * i + 1].k = x.y;
            v[4 * i + 2].k = x.z;
            v[4 * i + 3].k = x.w;
        }
    }
#pragma unroll
    for (int w = kFan / 2; w >= 1; w >>= 1)
#pragma unroll
        for (int i = 0; i < w; ++i) v[i] = lazy_merge(v[2 * i], v[2 * i + 1]);
    return v[0];
}

__device__ __forceinline__ void lazy_store(const lazy_tree& tr, int l, int j, const lazy_min& v)
{
    tr.d[l][j] = v.d;
    tr.kk[l][j] = v.k;
}

// The smallest entry (and its channel) over the wavefront, in every lane: the
// smallest value by a min reduction, then the channel of the one lane holding
// it; when several lanes hold it (or every value is +inf) the lowest of their
// channels (the order of lanes is not channel order).
__device__ __forceinline__ lazy_min lazy_wave_argmin(const lazy_min& v)
{
    const double m = rt_wave_min_f64(v.d);
    unsigned long long own = __ballot(v.d == m);
    int32_t k;
    if (__builtin_expect(__popcll(own) == 1, 1)) {
        k = __builtin_amdgcn_readlane(v.k, __ffsll((long long)own) - 1);
    } else {
        k = 0x7FFFFFFF;
        while (own) {
            k = min(k, (int32_t)__builtin_amdgcn_readlane(v.k, __ffsll((long long)own) - 1));
            own &= own - 1ull;
        }
    }
    return lazy_min{m, k};
}

// The top level (at most kTopMax entries; lane l holds entries l + 64 i) as
// the lane's smallest entry (channel order wins ties: a lane's entries come in
// channel order), the lane's second smallest and the index of its smallest;
// the wavefront argmin of the lanes' smallest is the next event.
struct lazy_top {
    lazy_min m;
    double d2;
    int e1;
};

__device__ __forceinline__ lazy_top lazy_top_scan(const double* top_d, const int32_t* top_k,
                                                  int top_cnt, bool leaves_on_top, int lane)
{
    double dv[kTopPer];
    int32_t kv[kTopPer];
#pragma unroll
    for (int i = 0; i < kTopPer; ++i) {
        const int e = lane + 64 * i;
        dv[i] = __builtin_inf();
        kv[i] = 0x7FFFFFFF;
        if (64 * i < top_cnt && e < top_cnt) {           // the first test: every lane alike
            dv[i] = top_d[e];
            kv[i] = leaves_on_top ? e : top_k[e];
        }
    }
    lazy_top r{lazy_min{__builtin_inf(), 0x7FFFFFFF}, __builtin_inf(), -1};
    // chunks past the level's entries (the same in every lane) are skipped
#pragma unroll
    for (int i = 0; i < kTopPer; ++i) {
        if (64 * i >= top_cnt) break;
        const bool lt = dv[i] < r.m.d;
        r.d2 = rt_min_sel(r.d2, lt ? r.m.d : dv[i]);
        r.m.d = lt ? dv[i] : r.m.d;
        r.m.k = lt ? kv[i] : r.m.k;
        r.e1 = lt ? lane + 64 * i : r.e1;
    }
    return r;
}

// The near-tie test of a firing (d1 = tau_mu - t).  The second smallest tau
// over all leaves is the smallest of the candidates: every leaf but mu lies in
// the group of mu's leaf, below a sibling of one of mu's ancestors under the
// top level, or below another entry of the top level.  The test is monotone in
// the second smallest (a larger value gives a larger rounded gap), so it holds
// for it exactly when it holds for one of the candidates: each lane tests its
// own and one ballot decides, with no reduction.  Lane kFan l + i reads
// sibling i at level l < top (level_off holds each level's tau array as a
// byte offset into the LDS region, a table in LDS so that the per-lane level
// index does not turn into a private-memory array); every lane also takes its
// own top-level minimum, or its second when it holds mu's ancestor.
__device__ __forceinline__ bool lazy_near_tie(const char* region, const uint32_t* level_off,
                                              int top, int mu, const lazy_top& tp, int lane,
                                              double t, double d1)
{
    double sib = __builtin_inf();
    if (top > 0) {
        const int lev = min(lane >> kFanLog, top - 1), i = lane & (kFan - 1);
        const int jl = mu >> (kFanLog * lev);
        const double x = ((const double*)(region + level_off[lev]))[(jl & ~(kFan - 1)) + i];
        sib = (lane >> kFanLog) < top && i != (jl & (kFan - 1)) ? x : __builtin_inf();
    }
    const int anc = mu >> (kFanLog * top);
    const double own = lane == (anc & 63) && tp.e1 == anc ? tp.d2 : tp.m.d;
    return __ballot(rt_near_tie(d1, rt_min_sel(sib, own) - t)) != 0ull;
}

// A touched channel's update (mu: fresh = true, T_mu = P_mu, P_mu += E;
// otherwise its clock runs from s to t at its old propensity), its new
// propensity and its leaf; returns the record to store.
__device__ __forceinline__ rt_lazy_rec lazy_touch(rt_lazy_rec rc, bool fresh, double E,
                                                  double t, int2 rr, double c, const int32_t* X,
                                                  double* leaf, unsigned long long* clamps)
{
    if (fresh) {
        rc.T = rc.P;
        rc.P = rc.P + E;
    } else {
        rc.T = fma(rc.a, t - rc.s, rc.T);
    }
    rc.s = t;
    rc.a = rt_propensity_mem(rr, c, X);
    bool cl;
    *leaf = lazy_tau(t, rc.T, rc.P, rc.a, &cl);
    if (cl) atomicAdd(clamps, 1ull);
    return rc;
}

// SCHED: some network of the class has piecewise-constant rates.  When the
// next event lies past the next breakpoint b (b < t_end), every channel runs
// its clock to b at its old propensity, takes the next piece's rates and a new
// next firing time from b, the tree is rebuilt, and nothing fires at b.
template <bool SCHED>
__global__ __launch_bounds__(64) void rt_lazy_kernel(rt_class_dev C, rt_lazy_rec* rec_ws,
                                                     unsigned long long* w_ws, uint32_t* n_ws,
                                                     int64_t m_stride)
{
    extern __shared__ int32_t dyn_lds[];
    __shared__ uint32_t log_scratch[RT_LOG_SCRATCH];
    __shared__ uint32_t level_off[kLazyLevels + 1];
    rt_ws* const ws = C.ws;
    const uint32_t key0 = ws->key0, key1 = ws->key1;
    const int lane = threadIdx.x;
    const rt_cptr<int64_t> unit_start = rt_const(C.unit_start);
    const int64_t total = unit_start[C.count];
    rt_lazy_rec* const recs = rec_ws + (int64_t)blockIdx.x * m_stride;
    uint32_t* const nks = n_ws + (int64_t)blockIdx.x * m_stride;
    // a channel's Philox block holds the words of two consecutive draws (n
    // even: words 1:0, n odd: words 3:2); the odd one is kept here until the
    // channel's next firing uses it
    unsigned long long* const wnext = w_ws + (int64_t)blockIdx.x * m_stride;

    for (;;) {
        unsigned long long u = 0;
        if (lane == 0) u = atomicAdd(&ws->next_unit, 1ull);
        // lane 0's unit; broadcast by readfirstlane the compiler keeps what
        // depends on it (the trajectory index, the fired channel's Philox
        // block) on the scalar unit, which measured faster without a rate
        // schedule and slower with one (whose loop holds more scalar state)
        u = SCHED ? __shfl(u, 0, 64) : rt_first_lane_u64(u);
        if ((int64_t)u >= total) break;
        const int item = __builtin_amdgcn_readfirstlane(rt_find_item(unit_start, C.count, (int64_t)u));
        const rt_cptr<rt_item_dev> it = rt_const(C.items) + item;
        const rt_net_dev net = it->net;
        const int N = net.N, M = net.M;
        const rt_cptr<int2> react = rt_const(net.react);
        rt_cptr<double> cc = rt_const(net.c);             // the rates of the current piece
        const rt_cptr<int32_t> dep_ptr = rt_const(net.dep_ptr), dep_idx = rt_const(net.dep_idx);
        const rt_cptr<int32_t> touch = rt_const(net.touch), touch_more = rt_const(net.touch_more);
        const rt_cptr<int2> nu_fixed = rt_const(net.nu_fixed);
        const int nu_stride = net.nu_stride;
        const int64_t r = (int64_t)u - unit_start[item];
        const uint32_t traj = it->traj_offset + (uint32_t)r;
        const uint32_t net_id = it->net_id;
        const double t_end = it->t_end;

        // LDS: X [N, padded to 4], the leaves, then the node levels 1 .. top
        // (sizes ceil(previous / 8)); the top level is the first with at
        // most kTopMax entries (the leaves themselves when M <= kTopMax),
        // scanned kTopPer entries per lane and reduced to the next event by
        // one wavefront argmin.  Every level index below is
        // a compile-time constant after unrolling.
        lazy_tree tr;
        int32_t* X = dyn_lds;
        {
            char* p = (char*)(dyn_lds + ((N + 3) & ~3));
            tr.cnt[0] = M > 0 ? M : 1;
            tr.d[0] = (double*)p;
            tr.kk[0] = (int32_t*)p;                      // unused (leaves carry no channel)
            p += 8 * padf(tr.cnt[0]);
            int top_l = tr.cnt[0] <= kTopMax ? 0 : -1;
#pragma unroll
            for (int l = 1; l <= kLazyLevels; ++l) {
                tr.cnt[l] = (tr.cnt[l - 1] + kFan - 1) >> kFanLog;
                const int P = top_l < 0 ? padf(tr.cnt[l]) : 0;
                tr.d[l] = (double*)p;
                tr.kk[l] = (int32_t*)(p + 8 * P);
                p += 12 * P;
                if (top_l < 0 && tr.cnt[l] <= kTopMax) top_l = l;
            }
            tr.top = top_l;
        }
        const int top = tr.top;
        double* const leaves = tr.d[0];
#pragma unroll
        for (int l = 0; l <= kLazyLevels; ++l)
            if (lane == l) level_off[l] = (uint32_t)((char*)tr.d[l] - (char*)dyn_lds);
        const double* top_d = tr.d[0];
        const int32_t* top_k = tr.kk[0];
        int top_cnt = tr.cnt[0];
#pragma unroll
        for (int l = 1; l <= kLazyLevels; ++l) {
            top_d = l == top ? tr.d[l] : top_d;
            top_k = l == top ? tr.kk[l] : top_k;
            top_cnt = l == top ? tr.cnt[l] : top_cnt;
        }

        // ---- initial state: X, every channel's record and leaf, the tree
        const int32_t* x0 = it->x0 + (it->x0_per_traj ? r * N : 0);
        for (int j = lane; j < N; j += 64) X[j] = x0[j];
        // padding entries (and the single leaf of an empty network) are empty
        for (int k = M + lane; k < padf(tr.cnt[0]); k += 64) leaves[k] = __builtin_inf();
#pragma unroll
        for (int l = 1; l <= kLazyLevels; ++l) {
            if (l > top) break;
            for (int j = tr.cnt[l] + lane; j < padf(tr.cnt[l]); j += 64)
                lazy_store(tr, l, j, lazy_min{__builtin_inf(), 0x7FFFFFFF});
        }
        rt_wave_lds_fence();
        for (int k = lane; k < M; k += 64) {
            const rt_u4 w = rt_philox4x32_10(rt_u4{0u, (uint32_t)k, traj, net_id}, key0, key1);
            wnext[k] = ((unsigned long long)w.w << 32) | w.z;
            const double P = rt_neglog_wave((((uint64_t)w.y << 32) | w.x) >> 11, false,
                                            &ws->slow_logs, log_scratch);
            const double a = rt_propensity_mem(react[k], cc[k], X);
            bool cl;
            leaves[k] = lazy_tau(0.0, 0.0, P, a, &cl);
            recs[k] = rt_lazy_rec{0.0, 0.0, P, a};
            nks[k] = 0u;
        }
        rt_wave_lds_fence();
#pragma unroll
        for (int l = 1; l <= kLazyLevels; ++l) {
            if (l > top) break;
            for (int j = lane; j < tr.cnt[l]; j += 64) lazy_store(tr, l, j, lazy_node(tr, l, j));
            rt_wave_lds_fence();
        }

        // the next event: the top level's argmin, kept in registers (every
        // lane holds it) and recomputed at the end of each tree update
        lazy_top top_e = lazy_top_scan(top_d, top_k, top_cnt, top == 0, lane);
        lazy_min root = lazy_wave_argmin(top_e.m);
        double root_tau = root.d;
        int root_ch = root.k;
        double t = 0.0, s_next = it->G > 0 ? rt_const(it->s)[0] : __builtin_inf();
        int32_t g = 0;
        uint32_t fired = 0, tie = kTieNone;
        unsigned long long hash = kFnvOffset;
        int st = RTSSA_TRAJ_OK;
        int32_t piece = 0;
        double b_next = SCHED && net.sched_B > 0 ? rt_const(net.sched_t)[0] : __builtin_inf();
        // the count and kept word of the channel that fired last (last_mu)
        // come from registers, not from a load of what this wavefront stored
        // at that firing: when the same channel fires again its draw starts
        // without a round trip to the workspace.
        int last_mu = -1;
        uint32_t last_nm = 0;
        unsigned long long last_w = 0;

        for (;;) {
            // ---- the next event: the root of the tree
            const double tau1 = root_tau;
            const int mu = __builtin_amdgcn_readfirstlane(root_ch);
            const double t_new = tau1;
            if (SCHED && b_next < t_end && t_new > b_next) {
                // ---- a rate breakpoint comes first (every value tested here
                // is the same in every lane): all clocks run to it at their old
                // propensities, then new rates, new leaves, the whole tree
                t = b_next;
                cc = rt_const(net.sched_c + (int64_t)piece * M);
                ++piece;
                b_next = piece < net.sched_B ? rt_const(net.sched_t)[piece] : __builtin_inf();
                for (int k = lane; k < M; k += 64)
                    recs[k] = lazy_touch(recs[k], false, 0.0, t, react[k], cc[k], X, &leaves[k],
                                         &ws->clamps);
                rt_wave_lds_fence();
#pragma unroll
                for (int l = 1; l <= kLazyLevels; ++l) {
                    if (l > top) break;
                    for (int j = lane; j < tr.cnt[l]; j += 64)
                        lazy_store(tr, l, j, lazy_node(tr, l, j));
                    rt_wave_lds_fence();
                }
                top_e = lazy_top_scan(top_d, top_k, top_cnt, top == 0, lane);
                root = lazy_wave_argmin(top_e.m);
                root_tau = root.d;
                root_ch = root.k;
                continue;
            }
            if (tau1 == __builtin_inf()) { st = RTSSA_TRAJ_ABSORBED; break; }
            if (t_new > t_end) break;
            while (s_next < t_new) {
                if (it->samples) {
                    int32_t* dst = it->samples + r * it->ss_r + (int64_t)g * it->ss_g;
                    for (int j = lane; j < N; j += 64) dst[j * it->ss_n] = X[j];
                }
                ++g;
                s_next = g < it->G ? rt_const(it->s)[g] : __builtin_inf();
            }
            // ---- every load of the firing is issued before any is used:
            // mu's firing count and kept word, mu's fixed-stride rows (the
            // jump; the touched channels of the first round: lane 0 takes mu,
            // lane q the q-th other channel of D(mu)), then their records and
            // reaction data; lanes without a channel load mu's (valid, unused)
            const uint32_t nm_ld = nks[mu];
            const unsigned long long w_ld = wnext[mu];
            const int n_other = touch[mu * 64];
            const int tv = touch[mu * 64 + lane];
            const int2 nv = nu_fixed[mu * nu_stride + min(lane, nu_stride - 1)];
            const bool has_nu = lane < nu_stride && nv.x >= 0;
            const int sp = max(nv.x, 0), dl = nv.y;
            const bool act = lane == 0 || tv >= 0;
            const int k = lane == 0 || !act ? mu : tv;
            const rt_lazy_rec rc0 = recs[k];
            const int2 rr0 = react[k];
            const double c0 = cc[k];
            // the same in every lane (without a schedule the draw below then
            // runs on the scalar unit)
            const uint32_t nm_v = mu == last_mu ? last_nm : nm_ld;
            const unsigned long long w_v = mu == last_mu ? last_w : w_ld;
            const uint32_t nm = SCHED ? nm_v : __builtin_amdgcn_readfirstlane(nm_v);
            const unsigned long long w_odd = SCHED ? w_v : rt_first_lane_u64(w_v);
            // near-tie test (statistics only) while the loads are in flight
            if (lazy_near_tie((const char*)dyn_lds, level_off, top, mu, top_e, lane, t,
                              t_new - t)) {
                if (lane == 0) atomicAdd(&ws->near_ties, 1ull);
                tie = tie == kTieNone ? fired : tie;
            }
            // the fired channel's next Exp(1) (Eq. 26) while the records are
            // on their way: draw n = nm + 1 takes the kept word when n is
            // odd, else a new block whose odd word is kept
            const uint32_t nd = nm + 1u;
            uint64_t word = w_odd;
            unsigned long long w_keep = w_odd;              // wnext[mu] after this firing
            if ((nd & 1u) == 0u) {
                const rt_u4 w = rt_philox4x32_10<SCHED>(
                    rt_u4{nd >> 1, (uint32_t)mu, traj, net_id}, key0, key1);
                word = ((uint64_t)w.y << 32) | w.x;
                w_keep = ((unsigned long long)w.w << 32) | w.z;
                if (lane == 0) wnext[mu] = w_keep;
            }
            const double E = rt_neglog_uniform(word >> 11, &ws->slow_logs, log_scratch);
            // ---- the jump v_mu, checked against [0, 2^31 - 1]
            const int64_t xv = (int64_t)X[sp] + dl;
            const bool okl = !has_nu || (xv >= 0 && xv <= 0x7FFFFFFF);
            if (__ballot(!okl) != 0ull) { st = RTSSA_TRAJ_OVERFLOW; break; }
            if (has_nu) X[sp] = (int32_t)xv;
            rt_wave_lds_fence();
            // ---- first round of touched channels, then their ancestors
            if (act) recs[k] = lazy_touch(rc0, lane == 0, E, t_new, rr0, c0, X, &leaves[k],
                                          &ws->clamps);
            rt_wave_lds_fence();
            // (lanes without a touched channel follow mu's path: they compute
            // and store the same values as lane 0)
#pragma unroll
            for (int l = 1; l <= kLazyLevels; ++l) {
                if (l > top) break;
                const int j = k >> (kFanLog * l);
                lazy_store(tr, l, j, lazy_node(tr, l, j));
                rt_wave_lds_fence();
            }
            // ---- more than 63 other dependents: the rest of the CSR list
            // D(mu) from the 64th on, 64 per round (mu itself skipped)
            if (n_other > 63) {
                const int de = dep_ptr[mu + 1];
                for (int q0 = touch_more[mu]; q0 < de; q0 += 64) {
                    const int q = q0 + lane;
                    int k2 = q < de ? dep_idx[q] : -1;
                    if (k2 == mu) k2 = -1;
                    if (k2 >= 0)
                        recs[k2] = lazy_touch(recs[k2], false, E, t_new, react[k2], cc[k2], X,
                                              &leaves[k2], &ws->clamps);
                    rt_wave_lds_fence();
#pragma unroll
                    for (int l = 1; l <= kLazyLevels; ++l) {
                        if (l > top) break;
                        const int j = (k2 >= 0 ? k2 : mu) >> (kFanLog * l);
                        lazy_store(tr, l, j, lazy_node(tr, l, j));
                        rt_wave_lds_fence();
                    }
                }
            }
            top_e = lazy_top_scan(top_d, top_k, top_cnt, top == 0, lane);
            root = lazy_wave_argmin(top_e.m);
            root_tau = root.d;
            root_ch = root.k;
            if (lane == 0) nks[mu] = nm + 1u;
            last_mu = mu;
            last_nm = nm + 1u;
            last_w = w_keep;
            t = t_new;
            ++fired;
            hash = (hash ^ (unsigned long long)(uint32_t)mu) * kFnvPrime;
            if (fired >= C.max_firings) { st = RTSSA_TRAJ_MAX_FIRINGS; break; }
        }

        // ---- end of the trajectory: every clock runs to t_end (or stops at
        // the last event after an overflow or the firing cap)
        const bool good = st == RTSSA_TRAJ_OK || st == RTSSA_TRAJ_ABSORBED;
        if (it->samples) {
            for (; g < it->G; ++g) {
                int32_t* dst = it->samples + r * it->ss_r + (int64_t)g * it->ss_g;
                for (int j = lane; j < N; j += 64) dst[j * it->ss_n] = good ? X[j] : -1;
            }
        }
        const double t_stop = good ? t_end : t;
        for (int k = lane; k < M; k += 64) {
            const rt_lazy_rec rc = recs[k];
            if (it->T_out) it->T_out[r * M + k] = fma(rc.a, t_stop - rc.s, rc.T);
            if (it->n_out) it->n_out[r * M + k] = nks[k];
        }
        if (it->x_final)
            for (int j = lane; j < N; j += 64) it->x_final[r * N + j] = X[j];
        if (lane == 0) {
            if (it->t_last) it->t_last[r] = t;
            if (it->status) it->status[r] = (uint8_t)st;
            if (it->seq_hash) it->seq_hash[r] = hash;
            if (it->tie_step) it->tie_step[r] = tie;
            atomicAdd(&ws->firings, (unsigned long long)fired);
            atomicAdd(&ws->status_count[st], 1ull);
        }
        rt_wave_lds_fence();                                  // X and the tree are reused
    }
}

// ---------------------------------------------------------------------------
// The direct method on a sum tree (Gillespie's method, section 3, Eq. 17-22,
// with a_0 and the channel search on a fixed tree of fan-out 8), in the same
// mapping as the lazy form: one wavefront per trajectory, the tree in LDS
// (leaves a_k, padding 0; a node adds its 8 children pairwise,
// ((v0 + v1) + (v2 + v3)) + ((v4 + v5) + (v6 + v7)); the root is a_0).  A
// firing: tau = RN(E / a_0) from the firing's Philox block (counter (firing
// index, 0xFFFFFFFF, trajectory, net_id)); the search walks down from the
// root with r = RN(u2 a_0), taking at each node the first positive child with
// r <= v_i (the last positive child if r passes them all) and subtracting the
// children it passes; then mu's jump, the new propensities of mu and D(mu),
// and their ancestors' sums.  A firing's draws do not depend on the state, so
// the next firing's block and logarithm are computed while this firing's
// loads are in flight.

static_assert(kFan == 8, "the sum tree adds 8 children pairwise");

__device__ __forceinline__ double dt_sum_node(const lazy_tree& tr, int l, int j)
{
    const double2* v = (const double2*)(tr.d[l - 1] + (j << 3));
    const double2 a = v[0], b = v[1], c = v[2], d = v[3];
    return ((a.x + a.y) + (b.x + b.y)) + ((c.x + c.y) + (d.x + d.y));
}

// E = RN(-ln u1) and the search's 53 bits of firing `fired`, every lane alike.
__device__ __forceinline__ double dt_draw(uint32_t key0, uint32_t key1, uint32_t traj,
                                          uint32_t net_id, uint32_t fired, uint64_t* m2,
                                          unsigned long long* slow, uint32_t* sc)
{
    const rt_u4 w =
        rt_philox4x32_10<false>(rt_u4{fired, 0xFFFFFFFFu, traj, net_id}, key0, key1);
    *m2 = (((uint64_t)w.w << 32) | w.z) >> 11;
    return rt_neglog_uniform((((uint64_t)w.y << 32) | w.x) >> 11, slow, sc);
}

__global__ __launch_bounds__(64) void rt_dmtree_kernel(rt_class_dev C)
{
    extern __shared__ int32_t dyn_lds[];
    __shared__ uint32_t log_scratch[RT_LOG_SCRATCH];
    rt_ws* const ws = C.ws;
    const uint32_t key0 = ws->key0, key1 = ws->key1;
    const int lane = threadIdx.x;
    const rt_cptr<int64_t> unit_start = rt_const(C.unit_start);
    const int64_t total = unit_start[C.count];

    for (;;) {
        unsigned long long u = 0;
        if (lane == 0) u = atomicAdd(&ws->next_unit, 1ull);
        u = __shfl(u, 0, 64);
        if ((int64_t)u >= total) break;
        const int item = __builtin_amdgcn_readfirstlane(rt_find_item(unit_start, C.count, (int64_t)u));
        const rt_cptr<rt_item_dev> it = rt_const(C.items) + item;
        const rt_net_dev net = it->net;
        const int N = net.N, M = net.M;
        const rt_cptr<int2> react = rt_const(net.react);
        const rt_cptr<double> cc = rt_const(net.c);
        const rt_cptr<int32_t> dep_ptr = rt_const(net.dep_ptr), dep_idx = rt_const(net.dep_idx);
        const rt_cptr<int32_t> touch = rt_const(net.touch), touch_more = rt_const(net.touch_more);
        const rt_cptr<int2> nu_fixed = rt_const(net.nu_fixed);
        const int nu_stride = net.nu_stride;
        const int64_t r = (int64_t)u - unit_start[item];
        const uint32_t traj = it->traj_offset + (uint32_t)r;
        const uint32_t net_id = it->net_id;
        const double t_end = it->t_end;
        uint32_t* const n_row = it->n_out ? it->n_out + r * M : nullptr;

        // LDS: X, the leaves a_k, the node levels (the lazy form's layout;
        // the channel arrays are unused)
        lazy_tree tr;
        int32_t* X = dyn_lds;
        {
            char* p = (char*)(dyn_lds + ((N + 3) & ~3));
            tr.cnt[0] = M > 0 ? M : 1;
            tr.d[0] = (double*)p;
            tr.kk[0] = nullptr;
            p += 8 * padf(tr.cnt[0]);
            tr.top = 0;
#pragma unroll
            for (int l = 1; l <= kMaxLevels; ++l) {
                tr.cnt[l] = (tr.cnt[l - 1] + kFan - 1) >> kFanLog;
                const int P = tr.top == 0 ? padf(tr.cnt[l]) : 0;
                tr.d[l] = (double*)p;
                tr.kk[l] = (int32_t*)(p + 8 * P);
                p += 12 * P;
                if (tr.top == 0 && tr.cnt[l] == 1) tr.top = l;
            }
        }
        const int top = tr.top;
        double* const leaves = tr.d[0];
        double* root_d = tr.d[1];
#pragma unroll
        for (int l = 2; l <= kMaxLevels; ++l) root_d = l == top ? tr.d[l] : root_d;

        // ---- initial state: X, the propensities, every node, zero counts
        const int32_t* x0 = it->x0 + (it->x0_per_traj ? r * N : 0);
        for (int j = lane; j < N; j += 64) X[j] = x0[j];
        rt_wave_lds_fence();
        for (int k = lane; k < padf(tr.cnt[0]); k += 64)
            leaves[k] = k < M ? rt_propensity_mem(react[k], cc[k], X) : 0.0;
#pragma unroll
        for (int l = 1; l <= kMaxLevels; ++l) {
            if (l > top) break;
            for (int j = tr.cnt[l] + lane; j < padf(tr.cnt[l]); j += 64) tr.d[l][j] = 0.0;
        }
        rt_wave_lds_fence();
#pragma unroll
        for (int l = 1; l <= kMaxLevels; ++l) {
            if (l > top) break;
            for (int j = lane; j < tr.cnt[l]; j += 64) tr.d[l][j] = dt_sum_node(tr, l, j);
            rt_wave_lds_fence();
        }
        if (n_row) {
            for (int k = lane; k < M; k += 64) n_row[k] = 0u;
            __threadfence();                               // before the counts' atomics
        }
        double a0 = *root_d;
        uint64_t m2 = 0;
        double E1 = dt_draw(key0, key1, traj, net_id, 0u, &m2, &ws->slow_logs, log_scratch);

        double t = 0.0, s_next = it->G > 0 ? rt_const(it->s)[0] : __builtin_inf();
        int32_t g = 0;
        uint32_t fired = 0;
        unsigned long long hash = kFnvOffset;
        int st = RTSSA_TRAJ_OK;

        for (;;) {
            if (a0 == 0.0) { st = RTSSA_TRAJ_ABSORBED; break; }
            const double t_new = t + E1 / a0;
            if (t_new > t_end) break;
            while (s_next < t_new) {
                if (it->samples) {
                    int32_t* dst = it->samples + r * it->ss_r + (int64_t)g * it->ss_g;
                    for (int j = lane; j < N; j += 64) dst[j * it->ss_n] = X[j];
                }
                ++g;
                s_next = g < it->G ? rt_const(it->s)[g] : __builtin_inf();
            }
            // ---- the search, from the root down (every lane alike)
            double rem = (double)(m2 + 1) * 0x1p-53 * a0;
            int j = 0;
#pragma unroll
            for (int l = kMaxLevels; l >= 1; --l) {
                if (l > top) continue;
                const double2* vd = (const double2*)(tr.d[l - 1] + (j << 3));
                double v[8];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const double2 x = vd[i];
                    v[2 * i] = x.x;
                    v[2 * i + 1] = x.y;
                }
                int last = 0;
#pragma unroll
                for (int i = 0; i < 8; ++i) last = v[i] > 0.0 ? i : last;
                int take = last;
                bool found = false;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const bool hit = !found && v[i] > 0.0 && (rem <= v[i] || i == last);
                    take = hit ? i : take;
                    rem = found || hit ? rem : rem - v[i];
                    found = found || hit;
                }
                j = __builtin_amdgcn_readfirstlane((j << 3) + take);
            }
            const int mu = j;
            // ---- mu's fixed-stride rows, then the touched channels' data
            const int n_other = touch[mu * 64];
            const int tv = touch[mu * 64 + lane];
            const int2 nv = nu_fixed[mu * nu_stride + min(lane, nu_stride - 1)];
            const bool has_nu = lane < nu_stride && nv.x >= 0;
            const int sp = max(nv.x, 0), dl = nv.y;
            const bool act = lane == 0 || tv >= 0;
            const int k = lane == 0 || !act ? mu : tv;
            const int2 rr0 = react[k];
            const double c0 = cc[k];
            // the next firing's draws while the loads are in flight
            uint64_t m2n;
            const double E1n = dt_draw(key0, key1, traj, net_id, fired + 1u, &m2n,
                                       &ws->slow_logs, log_scratch);
            // ---- the jump v_mu, checked against [0, 2^31 - 1]
            const int64_t xv = (int64_t)X[sp] + dl;
            const bool okl = !has_nu || (xv >= 0 && xv <= 0x7FFFFFFF);
            if (__ballot(!okl) != 0ull) { st = RTSSA_TRAJ_OVERFLOW; break; }
            if (has_nu) X[sp] = (int32_t)xv;
            rt_wave_lds_fence();
            // ---- new propensities (mu and D(mu)) and their ancestors' sums
            if (act) leaves[k] = rt_propensity_mem(rr0, c0, X);
            rt_wave_lds_fence();
#pragma unroll
            for (int l = 1; l <= kMaxLevels; ++l) {
                if (l > top) break;
                const int jn = k >> (kFanLog * l);
                const double v = dt_sum_node(tr, l, jn);
                tr.d[l][jn] = v;
                a0 = l == top ? v : a0;
                rt_wave_lds_fence();
            }
            if (n_other > 63) {
                const int de = dep_ptr[mu + 1];
                for (int q0 = touch_more[mu]; q0 < de; q0 += 64) {
                    const int q = q0 + lane;
                    int k2 = q < de ? dep_idx[q] : -1;
                    if (k2 == mu) k2 = -1;
                    if (k2 >= 0) leaves[k2] = rt_propensity_mem(react[k2], cc[k2], X);
                    rt_wave_lds_fence();
#pragma unroll
                    for (int l = 1; l <= kMaxLevels; ++l) {
                        if (l > top) break;
                        const int jn = (k2 >= 0 ? k2 : mu) >> (kFanLog * l);
                        const double v = dt_sum_node(tr, l, jn);
                        tr.d[l][jn] = v;
                        a0 = l == top ? v : a0;
                        rt_wave_lds_fence();
                    }
                }
            }
            if (n_row && lane == 0) atomicAdd(&n_row[mu], 1u);
            t = t_new;
            ++fired;
            hash = (hash ^ (unsigned long long)(uint32_t)mu) * kFnvPrime;
            E1 = E1n;
            m2 = m2n;
            if (fired >= C.max_firings) { st = RTSSA_TRAJ_MAX_FIRINGS; break; }
        }

        const bool good = st == RTSSA_TRAJ_OK || st == RTSSA_TRAJ_ABSORBED;
        if (it->samples) {
            for (; g < it->G; ++g) {
                int32_t* dst = it->samples + r * it->ss_r + (int64_t)g * it->ss_g;
                for (int j = lane; j < N; j += 64) dst[j * it->ss_n] = good ? X[j] : -1;
            }
        }
        if (it->x_final)
            for (int j = lane; j < N; j += 64) it->x_final[r * N + j] = X[j];
        if (lane == 0) {
            if (it->t_last) it->t_last[r] = t;
            if (it->status) it->status[r] = (uint8_t)st;
            if (it->seq_hash) it->seq_hash[r] = hash;
            atomicAdd(&ws->firings, (unsigned long long)fired);
            atomicAdd(&ws->status_count[st], 1ull);
        }
        rt_wave_lds_fence();                                  // X and the tree are reused
    }
}

}  // namespace

// LDS bytes of one trajectory: X, the leaves and the node levels up to the
// first with at most top_max entries (arrays padded to kFan entries; the
// leaves count as that level when top_max > 1, while the sum tree always has
// a root level above them); 0 when that takes more than max_levels levels.
static size_t tree_lds_bytes(int N, int M, int top_max, int max_levels)
{
    size_t n = (size_t)((N + 3) & ~3) * 4;
    int c = M > 0 ? M : 1;
    n += (size_t)((c + kFan - 1) & ~(kFan - 1)) * 8;
    if (top_max > 1 && c <= top_max) return n;
    for (int l = 1; l <= max_levels; ++l) {
        c = (c + kFan - 1) >> kFanLog;
        n += (size_t)((c + kFan - 1) & ~(kFan - 1)) * 12;
        if (c <= top_max) return n;
    }
    return 0;
}

// the lazy form's tree stops at a top level of at most kTopMax entries
size_t rt_lazy_lds_bytes(int N, int M) { return tree_lds_bytes(N, M, kTopMax, kLazyLevels); }

// the sum tree goes up to its single root
static size_t dmtree_lds_bytes(int N, int M) { return tree_lds_bytes(N, M, 1, kMaxLevels); }

// The lazy kernel's grid: the requested one, or the resident wavefronts
// (LDS-limited) of the device, never more than the trajectories.
int rt_lazy_grid(int max_N, int max_M, int grid, int64_t units, bool sched, int* grid_out,
                 int max_per_cu)
{
    const void* fn = sched ? (const void*)rt_lazy_kernel<true> : (const void*)rt_lazy_kernel<false>;
    const size_t lds = rt_lazy_lds_bytes(max_N, max_M);
    if (lds == 0) return rt_fail(RTSSA_E_UNSUPPORTED, "network too large for the lazy form");
    int dev = 0, lds_max = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
            hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return rt_fail(RTSSA_E_HIP, "device query failed");
    if (lds + RT_LOG_SCRATCH * 4 > (size_t)lds_max)
        return rt_fail(RTSSA_E_UNSUPPORTED, "network too large for the lazy form's LDS tree");
    if (lds > 48 * 1024 &&
        hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
            hipSuccess)
        return rt_fail(RTSSA_E_HIP, "cannot raise the LDS limit");
    if (grid <= 0) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64, lds) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        if (max_per_cu > 0) per_cu = std::min(per_cu, max_per_cu);
        grid = cus * per_cu;
    }
    if ((int64_t)grid > units) grid = (int)std::max<int64_t>(units, 1);
    *grid_out = grid;
    return RTSSA_OK;
}

// one slice of channel records, kept draw words and counts per wavefront
size_t rt_lazy_workspace_bytes(int grid, int max_M)
{
    const size_t m = (size_t)std::max(max_M, 1);
    return (size_t)grid * m * (sizeof(rt_lazy_rec) + sizeof(unsigned long long) + sizeof(uint32_t));
}

int rt_launch_lazy(const rt_class_dev& C, int max_N, int max_M, int grid, int64_t units,
                   hipStream_t stream, int* grid_used, void* workspace)
{
    const bool sched = C.has_schedule != 0;
    int rc = rt_lazy_grid(max_N, max_M, grid, units, sched, &grid);
    if (rc) return rc;
    if (grid_used) *grid_used = grid;
    const size_t lds = rt_lazy_lds_bytes(max_N, max_M);
    const int64_t m_stride = std::max(max_M, 1);
    void* wsp = workspace;
    if (!wsp) {
        rc = check_hip(hipMallocAsync(&wsp, rt_lazy_workspace_bytes(grid, max_M), stream),
                       "lazy workspace");
        if (rc) return rc;
    }
    const size_t rec_bytes = (size_t)grid * m_stride * sizeof(rt_lazy_rec);
    const size_t word_bytes = (size_t)grid * m_stride * sizeof(unsigned long long);
    auto* kern = sched ? rt_lazy_kernel<true> : rt_lazy_kernel<false>;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(64), lds, stream, C, (rt_lazy_rec*)wsp,
                       (unsigned long long*)((char*)wsp + rec_bytes),
                       (uint32_t*)((char*)wsp + rec_bytes + word_bytes), m_stride);
    rc = hipGetLastError() == hipSuccess ? RTSSA_OK
                                         : rt_fail(RTSSA_E_HIP, "lazy kernel launch failed");
    if (!workspace && hipFreeAsync(wsp, stream) != hipSuccess && !rc)
        rc = rt_fail(RTSSA_E_HIP, "freeing the lazy workspace failed");
    return rc;
}

int rt_launch_dmtree(const rt_class_dev& C, int max_N, int max_M, int grid, int64_t units,
                     hipStream_t stream, int* grid_used)
{
    const size_t lds = dmtree_lds_bytes(max_N, max_M);
    if (lds == 0) return rt_fail(RTSSA_E_UNSUPPORTED, "network too large for the sum tree");
    int dev = 0, lds_max = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
            hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return rt_fail(RTSSA_E_HIP, "device query failed");
    if (lds + RT_LOG_SCRATCH * 4 > (size_t)lds_max)
        return rt_fail(RTSSA_E_UNSUPPORTED, "network too large for the sum tree in LDS");
    if (lds > 48 * 1024 &&
        hipFuncSetAttribute((const void*)rt_dmtree_kernel,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return rt_fail(RTSSA_E_HIP, "cannot raise the LDS limit");
    if (grid <= 0) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, rt_dmtree_kernel, 64, lds) !=
                hipSuccess || per_cu < 1)
            per_cu = 1;
        grid = cus * per_cu;
    }
    if ((int64_t)grid > units) grid = (int)std::max<int64_t>(units, 1);
    if (grid_used) *grid_used = grid;
    hipLaunchKernelGGL(rt_dmtree_kernel, dim3(grid), dim3(64), lds, stream, C);
    return hipGetLastError() == hipSuccess ? RTSSA_OK
                                           : rt_fail(RTSSA_E_HIP, "sum-tree kernel launch failed");
}
