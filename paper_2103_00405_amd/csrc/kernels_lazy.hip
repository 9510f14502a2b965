// kernels_lazy.hip -- the lazy form for large networks: one wavefront per
// trajectory, an 8-ary minimum tree in LDS.
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
// Layout.  The wavefront's LDS region holds the species counts X and the
// tree: the leaves are tau_k (M doubles); a node of level l >= 1 holds the
// smallest and second smallest tau and the smallest's channel over its 8
// children of level l - 1; the last level is the root.  Each level is stored
// as separate arrays (smallest, second smallest, channel) padded to a multiple
// of 8 entries with empty values, so that a node's 8 children are read with a
// few 16-byte loads and no bounds tests; merges use selects, not branches.  The channels' T_k,
// s_k, P_k, a_k (32 bytes) and n_k live in a global workspace, one slice per
// wavefront of the grid.  A firing: the root gives mu; wavefront loads mu's
// jump and dependency lists, checks and applies the jump, draws mu's next
// Exp(1) with all lanes, then one lane per touched channel updates it and
// writes its leaf; the touched leaves' ancestors are recomputed level by
// level, one lane per touched channel (lanes that share an ancestor compute
// the same node).  No workgroup barrier is used: a wavefront's LDS accesses
// complete in program order.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "rt_device.h"
#include "rt_wave.h"

namespace {

constexpr uint32_t kTieNone = 0xFFFFFFFFu;
constexpr unsigned long long kFnvOffset = 0xcbf29ce484222325ull;
constexpr unsigned long long kFnvPrime = 0x100000001b3ull;
constexpr int kMaxLevels = 6;            // 8^6 leaves would need 2 MB of LDS

struct rt_lazy_rec {                     // a channel's state in the workspace
    double T, s, P, a;
};

__device__ __forceinline__ double u64_to_f64(uint64_t h)
{
    return fma((double)(uint32_t)(h >> 32), 0x1p32, (double)(uint32_t)h);
}

// a_k = RN(c_k RN(h_k(X))) with X in LDS (Eq. 1-2).
__device__ __forceinline__ double lazy_propensity(int2 rr, double c, const int32_t* X)
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

__device__ __forceinline__ void wave_lds_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int find_item(rt_cptr<int64_t> unit_start, int count, int64_t u)
{
    int lo = 0, hi = count;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (unit_start[mid] <= u) lo = mid; else hi = mid;
    }
    return lo;
}

// A refreshed channel's next firing time: +inf when a = 0, else
// t + max(0, RN(RN(P - T) * RN(1 / a))); *clamped when the raw gap is negative.
__device__ __forceinline__ double lazy_tau(double t, double T, double P, double a, bool* clamped)
{
    const double raw = (P - T) * (1.0 / a);
    *clamped = a != 0.0 && raw < 0.0;
    return a == 0.0 ? __builtin_inf() : t + fmax(raw, 0.0);
}

// The tree of one trajectory: level 0 holds the leaves (d1 = tau, channel =
// index), levels 1 .. top the nodes; cnt = entries in use, every array padded
// to a multiple of 8 entries (+inf, +inf, INT_MAX).  Times are never -0 (t
// starts at +0 and only grows), so selects on '<' order them exactly.
struct lazy_tree {
    double* d1[kMaxLevels + 1];
    double* d2[kMaxLevels + 1];
    int32_t* kk[kMaxLevels + 1];
    int cnt[kMaxLevels + 1];
    int top;
};

__device__ __forceinline__ int pad8(int n) { return (n + 7) & ~7; }

// Smallest, second smallest and the smallest's channel of two entries; on
// equal smallest values the lower channel wins.
__device__ __forceinline__ rt_min2 lazy_merge(const rt_min2& a, const rt_min2& b)
{
    const bool blt = b.d1 < a.d1, alt = a.d1 < b.d1;
    const double hi = blt ? a.d1 : b.d1;                 // the larger of the two minima
    const double m2 = b.d2 < a.d2 ? b.d2 : a.d2;
    rt_min2 r;
    r.d1 = blt ? b.d1 : a.d1;
    r.d2 = m2 < hi ? m2 : hi;
    // blt: b.k; a.d1 < b.d1: a.k; equal: the lower channel.  Written so that
    // both channels feed both selects (no branch, no load sunk into one)
    r.k = min(blt ? b.k : a.k, alt ? a.k : b.k);
    return r;
}

// Two leaves a (channel ka) and b (channel kb > ka).
__device__ __forceinline__ rt_min2 lazy_pair(double a, int ka, double b, int kb)
{
    const bool blt = b < a;
    rt_min2 r;
    r.d1 = blt ? b : a;
    r.d2 = blt ? a : b;
    r.k = blt ? kb : ka;
    return r;
}

// Node j of level l (1 <= l) from its 8 children, loaded together (the padded
// arrays make every child present) and merged pairwise; minimum, second
// minimum and the lowest-channel tie-break do not depend on the merge order.
__device__ __forceinline__ rt_min2 lazy_node(const lazy_tree& tr, int l, int j)
{
    const int c0 = j << 3;
    const double2* v1 = (const double2*)(tr.d1[l - 1] + c0);
    const double2 a01 = v1[0], a23 = v1[1], a45 = v1[2], a67 = v1[3];
    if (l == 1) {
        const rt_min2 a = lazy_merge(lazy_pair(a01.x, c0, a01.y, c0 + 1),
                                     lazy_pair(a23.x, c0 + 2, a23.y, c0 + 3));
        const rt_min2 b = lazy_merge(lazy_pair(a45.x, c0 + 4, a45.y, c0 + 5),
                                     lazy_pair(a67.x, c0 + 6, a67.y, c0 + 7));
        return lazy_merge(a, b);
    }
    const double2* v2 = (const double2*)(tr.d2[l - 1] + c0);
    const double2 b01 = v2[0], b23 = v2[1], b45 = v2[2], b67 = v2[3];
    const int4* vk = (const int4*)(tr.kk[l - 1] + c0);
    const int4 k03 = vk[0], k47 = vk[1];
    const rt_min2 n0{a01.x, b01.x, k03.x}, n1{a01.y, b01.y, k03.y};
    const rt_min2 n2{a23.x, b23.x, k03.z}, n3{a23.y, b23.y, k03.w};
    const rt_min2 n4{a45.x, b45.x, k47.x}, n5{a45.y, b45.y, k47.y};
    const rt_min2 n6{a67.x, b67.x, k47.z}, n7{a67.y, b67.y, k47.w};
    const rt_min2 a = lazy_merge(lazy_merge(n0, n1), lazy_merge(n2, n3));
    const rt_min2 b = lazy_merge(lazy_merge(n4, n5), lazy_merge(n6, n7));
    return lazy_merge(a, b);
}

__device__ __forceinline__ void lazy_store(const lazy_tree& tr, int l, int j, const rt_min2& v)
{
    tr.d1[l][j] = v.d1;
    tr.d2[l][j] = v.d2;
    tr.kk[l][j] = v.k;
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
    rc.a = lazy_propensity(rr, c, X);
    bool cl;
    *leaf = lazy_tau(t, rc.T, rc.P, rc.a, &cl);
    if (cl) atomicAdd(clamps, 1ull);
    return rc;
}

__global__ __launch_bounds__(64) void rt_lazy_kernel(rt_class_dev C, rt_lazy_rec* rec_ws,
                                                     uint32_t* n_ws, int64_t m_stride)
{
    extern __shared__ int32_t dyn_lds[];
    __shared__ uint32_t log_scratch[RT_LOG_SCRATCH];
    rt_ws* const ws = C.ws;
    const uint32_t key0 = ws->key0, key1 = ws->key1;
    const int lane = threadIdx.x;
    const rt_cptr<int64_t> unit_start = rt_const(C.unit_start);
    const int64_t total = unit_start[C.count];
    rt_lazy_rec* const recs = rec_ws + (int64_t)blockIdx.x * m_stride;
    uint32_t* const nks = n_ws + (int64_t)blockIdx.x * m_stride;

    for (;;) {
        unsigned long long u = 0;
        if (lane == 0) u = atomicAdd(&ws->next_unit, 1ull);
        u = __shfl(u, 0, 64);
        if ((int64_t)u >= total) break;
        const int item = __builtin_amdgcn_readfirstlane(find_item(unit_start, C.count, (int64_t)u));
        const rt_cptr<rt_item_dev> it = rt_const(C.items) + item;
        const rt_net_dev net = it->net;
        const int N = net.N, M = net.M;
        const rt_cptr<int2> react = rt_const(net.react);
        const rt_cptr<double> cc = rt_const(net.c);
        const rt_cptr<int32_t> nu_ptr = rt_const(net.nu_ptr), nu_sp = rt_const(net.nu_sp);
        const rt_cptr<int32_t> nu_dl = rt_const(net.nu_dl), dep_ptr = rt_const(net.dep_ptr);
        const rt_cptr<int32_t> dep_idx = rt_const(net.dep_idx);
        const int64_t r = (int64_t)u - unit_start[item];
        const uint32_t traj = it->traj_offset + (uint32_t)r;
        const uint32_t net_id = it->net_id;
        const double t_end = it->t_end;

        // LDS: X [N, padded to 4], the leaves, then the node levels 1 .. top
        // (sizes ceil(previous / 8), the root alone on top); every level
        // index below is a compile-time constant after unrolling
        lazy_tree tr;
        int32_t* X = dyn_lds;
        {
            char* p = (char*)(dyn_lds + ((N + 3) & ~3));
            tr.cnt[0] = M > 0 ? M : 1;
            tr.d1[0] = (double*)p;
            tr.d2[0] = nullptr;
            tr.kk[0] = nullptr;
            p += 8 * pad8(tr.cnt[0]);
            tr.top = 0;
#pragma unroll
            for (int l = 1; l <= kMaxLevels; ++l) {
                tr.cnt[l] = (tr.cnt[l - 1] + 7) >> 3;
                const int P = tr.top == 0 ? pad8(tr.cnt[l]) : 0;
                tr.d1[l] = (double*)p;
                tr.d2[l] = (double*)(p + 8 * P);
                tr.kk[l] = (int32_t*)(p + 16 * P);
                p += 20 * P;
                if (tr.top == 0 && tr.cnt[l] == 1) tr.top = l;
            }
        }
        const int top = tr.top;
        double* const leaves = tr.d1[0];
        double* root_d1 = tr.d1[1];
        double* root_d2 = tr.d2[1];
        int32_t* root_k = tr.kk[1];
#pragma unroll
        for (int l = 2; l <= kMaxLevels; ++l) {
            root_d1 = l == top ? tr.d1[l] : root_d1;
            root_d2 = l == top ? tr.d2[l] : root_d2;
            root_k = l == top ? tr.kk[l] : root_k;
        }

        // ---- initial state: X, every channel's record and leaf, the tree
        const int32_t* x0 = it->x0 + (it->x0_per_traj ? r * N : 0);
        for (int j = lane; j < N; j += 64) X[j] = x0[j];
        // padding entries (and the single leaf of an empty network) are empty
        for (int k = M + lane; k < pad8(tr.cnt[0]); k += 64) leaves[k] = __builtin_inf();
#pragma unroll
        for (int l = 1; l <= kMaxLevels; ++l) {
            if (l > top) break;
            for (int j = tr.cnt[l] + lane; j < pad8(tr.cnt[l]); j += 64)
                lazy_store(tr, l, j, rt_min2_empty());
        }
        wave_lds_fence();
        for (int k = lane; k < M; k += 64) {
            const double P = rt_exp1_wave(key0, key1, traj, net_id, (uint32_t)k, 0u,
                                          &ws->slow_logs, log_scratch);
            const double a = lazy_propensity(react[k], cc[k], X);
            bool cl;
            leaves[k] = lazy_tau(0.0, 0.0, P, a, &cl);
            recs[k] = rt_lazy_rec{0.0, 0.0, P, a};
            nks[k] = 0u;
        }
        wave_lds_fence();
#pragma unroll
        for (int l = 1; l <= kMaxLevels; ++l) {
            if (l > top) break;
            for (int j = lane; j < tr.cnt[l]; j += 64) lazy_store(tr, l, j, lazy_node(tr, l, j));
            wave_lds_fence();
        }

        double t = 0.0, s_next = it->G > 0 ? rt_const(it->s)[0] : __builtin_inf();
        int32_t g = 0;
        uint32_t fired = 0, tie = kTieNone;
        unsigned long long hash = kFnvOffset;
        int st = RTSSA_TRAJ_OK;

        for (;;) {
            // ---- the next event: the root of the tree
            const double tau1 = *root_d1, tau2 = *root_d2;
            const int mu = __builtin_amdgcn_readfirstlane(*root_k);
            if (tau1 == __builtin_inf()) { st = RTSSA_TRAJ_ABSORBED; break; }
            const double t_new = tau1;
            if (t_new > t_end) break;
            const double d1 = t_new - t, d2 = tau2 - t;
            if (d2 - d1 <= 1e-12 * d1) {
                if (lane == 0) atomicAdd(&ws->near_ties, 1ull);
                tie = tie == kTieNone ? fired : tie;
            }
            while (s_next < t_new) {
                if (it->samples) {
                    int32_t* dst = it->samples + r * it->ss_r + (int64_t)g * it->ss_g;
                    for (int j = lane; j < N; j += 64) dst[j * it->ss_n] = X[j];
                }
                ++g;
                s_next = g < it->G ? rt_const(it->s)[g] : __builtin_inf();
            }
            // ---- every load of the firing is issued before any is used:
            // mu's jump, the touched channels of the first round (lane 0: mu,
            // lane q: entry q - 1 of D(mu), mu itself skipped there), their
            // records and reaction data, and mu's firing count.  Indices are
            // clamped so that every lane loads a valid entry (the lists end
            // with a padding entry); unused loads are discarded.
            const int nb = nu_ptr[mu], ne = nu_ptr[mu + 1];
            const int db = dep_ptr[mu], de = dep_ptr[mu + 1];
            const int n_nu = ne - nb, n_dep = de - db;
            const int qs = nb + max(0, min(lane, n_nu - 1));
            const int sp = nu_sp[qs], dl = nu_dl[qs];
            const int kq = dep_idx[db + max(0, min(lane - 1, n_dep - 1))];
            const bool act = lane == 0 || (lane <= n_dep && kq != mu);
            const int k = lane == 0 || !act ? mu : kq;
            const rt_lazy_rec rc0 = recs[k];
            const int2 rr0 = react[k];
            const double c0 = cc[k];
            const uint32_t nm = nks[mu];
            // the fired channel's next Exp(1) (Eq. 26), drawn by every lane
            // while the loads are in flight
            const double E = rt_exp1_uniform(key0, key1, traj, net_id, (uint32_t)mu, nm + 1u,
                                             &ws->slow_logs, log_scratch);
            // ---- the jump v_mu, checked against [0, 2^31 - 1]
            const int64_t xv = (int64_t)X[sp] + dl;
            const bool okl = lane >= n_nu || (xv >= 0 && xv <= 0x7FFFFFFF);
            if (__ballot(!okl) != 0ull) { st = RTSSA_TRAJ_OVERFLOW; break; }
            if (lane < n_nu) X[sp] = (int32_t)xv;
            wave_lds_fence();
            // ---- first round of touched channels, then their ancestors
            if (act) recs[k] = lazy_touch(rc0, lane == 0, E, t_new, rr0, c0, X, &leaves[k],
                                          &ws->clamps);
            wave_lds_fence();
            // (lanes without a touched channel follow mu's path: they compute
            // and store the same values as lane 0)
#pragma unroll
            for (int l = 1; l <= kMaxLevels; ++l) {
                if (l > top) break;
                const int j = k >> (3 * l);
                lazy_store(tr, l, j, lazy_node(tr, l, j));
                wave_lds_fence();
            }
            // ---- more than 63 dependents: further rounds of 64
            for (int q0 = 63; q0 < n_dep; q0 += 64) {
                const int q = q0 + lane;
                int k2 = q < n_dep ? dep_idx[db + q] : -1;
                if (k2 == mu) k2 = -1;
                if (k2 >= 0)
                    recs[k2] = lazy_touch(recs[k2], false, E, t_new, react[k2], cc[k2], X,
                                          &leaves[k2], &ws->clamps);
                wave_lds_fence();
#pragma unroll
                for (int l = 1; l <= kMaxLevels; ++l) {
                    if (l > top) break;
                    const int j = (k2 >= 0 ? k2 : mu) >> (3 * l);
                    lazy_store(tr, l, j, lazy_node(tr, l, j));
                    wave_lds_fence();
                }
            }
            if (lane == 0) nks[mu] = nm + 1u;
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
        wave_lds_fence();                                  // X and the tree are reused
    }
}

}  // namespace

// LDS bytes of one trajectory: X, the leaves and every node level (arrays
// padded to 8 entries); 0 when the tree would need more than kMaxLevels levels.
size_t rt_lazy_lds_bytes(int N, int M)
{
    size_t n = (size_t)((N + 3) & ~3) * 4;
    int c = M > 0 ? M : 1;
    n += (size_t)((c + 7) & ~7) * 8;
    for (int l = 1; l <= kMaxLevels; ++l) {
        c = (c + 7) >> 3;
        n += (size_t)((c + 7) & ~7) * 20;
        if (c == 1) return n;
    }
    return 0;
}

int rt_launch_lazy(const rt_class_dev& C, int max_N, int max_M, int grid, int64_t units,
                   hipStream_t stream, int* grid_used)
{
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
        hipFuncSetAttribute((const void*)rt_lazy_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds) != hipSuccess)
        return rt_fail(RTSSA_E_HIP, "cannot raise the LDS limit");
    if (grid <= 0) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, rt_lazy_kernel, 64, lds) !=
                hipSuccess || per_cu < 1)
            per_cu = 1;
        grid = cus * per_cu;
    }
    if ((int64_t)grid > units) grid = (int)std::max<int64_t>(units, 1);
    if (grid_used) *grid_used = grid;
    // one workspace slice of channel records and counts per wavefront
    const int64_t m_stride = std::max(max_M, 1);
    void* wsp = nullptr;
    const size_t rec_bytes = (size_t)grid * m_stride * sizeof(rt_lazy_rec);
    const size_t n_bytes = (size_t)grid * m_stride * sizeof(uint32_t);
    int rc = check_hip(hipMallocAsync(&wsp, rec_bytes + n_bytes, stream), "lazy workspace");
    if (rc) return rc;
    hipLaunchKernelGGL(rt_lazy_kernel, dim3(grid), dim3(64), lds, stream, C, (rt_lazy_rec*)wsp,
                       (uint32_t*)((char*)wsp + rec_bytes), m_stride);
    rc = hipGetLastError() == hipSuccess ? RTSSA_OK
                                         : rt_fail(RTSSA_E_HIP, "lazy kernel launch failed");
    if (hipFreeAsync(wsp, stream) != hipSuccess && !rc)
        rc = rt_fail(RTSSA_E_HIP, "freeing the lazy workspace failed");
    return rc;
}
