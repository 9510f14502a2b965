// batch.cpp -- many independent networks in one captured launch, and the
// autotuner that picks each size class's mapping parameters.
//
// rtssa_batch_create sorts the items into classes -- one per kernel
// instantiation (thread mapping by padded (M, N); sub-wavefront mapping by
// lanes per trajectory; workgroup mapping by group size) -- and uploads, per
// class, the item descriptors, the prefix sums of trajectory counts and a
// workspace.  The first rtssa_batch_run captures a hipGraph: one setup kernel
// per class, then one persistent kernel per class on its own stream (parallel
// branches of the graph, joined at the end).  Later runs copy the new seed
// into device memory and replay the graph.  Because every draw is keyed by
// (seed, trajectory, net_id, channel, firing index), the outputs equal those
// of one rtssa_simulate per item with the same seed and net_id.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <string>
#include <vector>

#include "internal.h"

namespace {

struct class_key {
    int mapping;    // RTSSA_MAP_*
    int a, b;       // thread: padded (M, N); wave / workgroup: lanes per trajectory, 0;
                    // tree methods: 64, the power-of-two channel range
    int method;     // RTSSA_METHOD_*: the tree methods have classes of their own
    // Class order is launch order.  The tree methods' classes (long, one
    // wavefront per trajectory) go first: launched after the others they
    // start late and set the step time (2.63 s against 3.25 s per step on
    // 4096 random networks with the lazy form above 512 channels), largest
    // channel range first; the random-time classes follow, lightest first.
    bool operator<(const class_key& o) const
    {
        if (method != o.method) return method > o.method;
        if (method != RTSSA_METHOD_RANDOM_TIME) return b > o.b;
        return mapping != o.mapping ? mapping < o.mapping : (a != o.a ? a < o.a : b < o.b);
    }
};

int pad_thread_m(int M) { return M <= 1 ? 1 : (M <= 4 ? M : (M <= 6 ? 6 : 8)); }
int pad_thread_n(int N) { return N <= 1 ? 1 : (N <= 2 ? 2 : (N <= 4 ? 4 : 8)); }

// plan cache: lines "wave <M_lo> <M_hi> <L>" or "workgroup <M_lo> <M_hi> <L>"
struct plan_entry { int mapping, lo, hi, L; };

std::vector<plan_entry> read_plan(const char* path)
{
    std::vector<plan_entry> out;
    if (!path || !*path) return out;
    FILE* f = fopen(path, "r");
    if (!f) return out;
    char kind[32];
    int lo, hi, L;
    while (fscanf(f, "%31s %d %d %d", kind, &lo, &hi, &L) == 4) {
        int m = strcmp(kind, "wave") == 0 ? RTSSA_MAP_WAVE
                                          : (strcmp(kind, "workgroup") == 0 ? RTSSA_MAP_WORKGROUP : 0);
        if (m) out.push_back({m, lo, hi, L});
    }
    fclose(f);
    return out;
}

int plan_lookup(const std::vector<plan_entry>& plan, int mapping, int M)
{
    for (const auto& e : plan)
        if (e.mapping == mapping && M >= e.lo && M <= e.hi) return e.L;
    return 0;
}

// The tree methods' classes: one per power-of-two channel range (at least 64),
// so that each class's LDS tree, and with it the number of wavefronts a CU
// holds, is sized for its own networks rather than the largest of the batch.
int tree_range(int M)
{
    int r = 64;
    while (r < M) r <<= 1;
    return r;
}

class_key classify(const rtssa_network* net, int method, const std::vector<plan_entry>& plan,
                   const rtssa_options& o)
{
    if (method != RTSSA_METHOD_RANDOM_TIME) return {RTSSA_MAP_WAVE, 64, tree_range(net->M), method};
    int mapping = o.mapping ? o.mapping : rt_auto_mapping(net);
    if (mapping == RTSSA_MAP_THREAD && rt_thread_supported(net->M, net->N))
        return {RTSSA_MAP_THREAD, pad_thread_m(net->M), pad_thread_n(net->N), 0};
    if (mapping == RTSSA_MAP_THREAD) mapping = RTSSA_MAP_WAVE;
    if (mapping == RTSSA_MAP_WAVE && (net->M > 512 || net->max_nu > 64))
        mapping = RTSSA_MAP_WORKGROUP;
    if (mapping == RTSSA_MAP_WAVE) {
        int L = plan_lookup(plan, RTSSA_MAP_WAVE, net->M);
        if (L <= 0) L = rt_subwave_lanes(net->M);
        while (L < 64 && (L < net->max_nu || L * 8 < net->M)) L <<= 1;
        return {RTSSA_MAP_WAVE, L, 0, 0};
    }
    int L = plan_lookup(plan, RTSSA_MAP_WORKGROUP, net->M);
    if (L <= 0) L = rt_auto_group_size(net->M);
    return {RTSSA_MAP_WORKGROUP, L, 0, 0};
}

}  // namespace

struct rtssa_batch_class {
    class_key key;
    std::vector<int> members;   // item indices, heaviest first
    int max_M = 0, max_N = 0, max_nu = 0;
    int64_t units = 0;
    rt_class_dev dev{};
    hipStream_t side = nullptr;
    int block_used = 0, grid_used = 0;
    int lazy_grid = 0;          // lazy form: the grid its workspace is sized for
    void* lazy_ws = nullptr;    // lazy form: channel workspace (in the batch's block)
};

struct rtssa_batch {
    std::vector<rtssa_batch_item> items;
    std::vector<rtssa_batch_class> classes;
    rtssa_options opt{};
    void* dev_block = nullptr;     // descriptors, prefix sums, counters, workspaces, key
    uint32_t* key_dev = nullptr;
    rt_ws* ws_dev = nullptr;       // one per class, contiguous
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> joins;
    int device = -1;
    bool holds_nets = false;       // batch_refs of the items' networks taken
};

static int batch_create(const rtssa_batch_item* items, int32_t count, const rtssa_options* opt,
                        const std::vector<plan_entry>& plan, rtssa_batch** out);

extern "C" int rtssa_batch_create(const rtssa_batch_item* items, int32_t count,
                                  const rtssa_options* opt, const char* plan_path,
                                  rtssa_batch** out)
{
    return batch_create(items, count, opt, read_plan(plan_path), out);
}

static int batch_create(const rtssa_batch_item* items, int32_t count, const rtssa_options* opt,
                        const std::vector<plan_entry>& plan, rtssa_batch** out)
{
    if (!out) return rt_fail(RTSSA_E_INVALID, "out is NULL");
    *out = nullptr;
    if (count < 1 || !items) return rt_fail(RTSSA_E_INVALID, "a batch needs at least one item");
    rtssa_options o{};
    if (opt) o = *opt;
    uint64_t maxf = o.max_firings ? o.max_firings : 10000000ull;
    if (maxf > 0xFFFFFFFFull) return rt_fail(RTSSA_E_INVALID, "max_firings must be < 2^32");
    if (o.method != RTSSA_METHOD_RANDOM_TIME)
        return rt_fail(RTSSA_E_UNSUPPORTED, "the batch's method is chosen per item "
                                            "(rtssa_batch_item.method); opt->method must be 0");
    // validate every item (reads each sample grid once)
    for (int i = 0; i < count; ++i) {
        const rtssa_batch_item& b = items[i];
        int rc = rt_check_run(b.net, b.x0, b.x0_per_traj, b.t_end, b.sample_t, b.G,
                              b.traj_offset, b.R);
        if (!rc && b.R > 0) rc = rt_check_grid_host(b.sample_t, b.G, b.t_end);
        const std::string at = "item " + std::to_string(i) + ": ";
        if (rc) return rt_fail(rc, at + rtssa_last_error());
        if (!(b.weight >= 0.0) || !std::isfinite(b.weight))
            return rt_fail(RTSSA_E_INVALID, at + "weight must be finite and >= 0");
        if (b.method != RTSSA_METHOD_RANDOM_TIME && b.method != RTSSA_METHOD_LAZY &&
            b.method != RTSSA_METHOD_DIRECT_TREE)
            return rt_fail(RTSSA_E_UNSUPPORTED, at + "batched items run RANDOM_TIME, LAZY or "
                                                     "DIRECT_TREE");
        if (b.method != RTSSA_METHOD_RANDOM_TIME) {
            if (b.method == RTSSA_METHOD_DIRECT_TREE && b.net->dev.sched_B > 0)
                return rt_fail(RTSSA_E_UNSUPPORTED,
                               at + "the direct method takes no rate schedule");
            if (b.method == RTSSA_METHOD_DIRECT_TREE && (b.T_out || b.tie_step))
                return rt_fail(RTSSA_E_INVALID, at + "the direct method has no T_out or tie_step");
            if (b.R > 0) {
                rc = rt_lazy_prepare(const_cast<rtssa_network*>(b.net));
                if (rc) return rt_fail(rc, at + rtssa_last_error());
            }
        }
    }
    std::map<class_key, std::vector<int>> groups;
    for (int i = 0; i < count; ++i) {
        if (items[i].R <= 0) continue;
        const class_key key = classify(items[i].net, items[i].method, plan, o);
        if (key.method == RTSSA_METHOD_RANDOM_TIME &&
            (key.mapping == RTSSA_MAP_WORKGROUP || key.mapping == RTSSA_MAP_WAVE)) {
            // the workgroup kernels read the network's fixed-stride records,
            // the sub-wave kernel its jump and touch rows
            rtssa_network* n = const_cast<rtssa_network*>(items[i].net);
            const int rc = key.mapping == RTSSA_MAP_WORKGROUP ? rt_group_rows_prepare(n)
                                                              : rt_lazy_prepare(n);
            if (rc) return rt_fail(rc, "item " + std::to_string(i) + ": " + rtssa_last_error());
        }
        groups[key].push_back(i);
    }

    rtssa_batch* B = new rtssa_batch();
    B->items.assign(items, items + count);
    B->opt = o;
    hipGetDevice(&B->device);
    for (auto& kv : groups) {
        rtssa_batch_class c;
        c.key = kv.first;
        c.members = kv.second;
        // heaviest items first so the tail of the queue holds short work (the
        // caller's weight, else M x R)
        auto work = [&](int x) {
            return items[x].weight > 0.0 ? items[x].weight
                                         : (double)items[x].net->M * items[x].R;
        };
        std::stable_sort(c.members.begin(), c.members.end(),
                         [&](int x, int y) { return work(x) > work(y); });
        for (int i : c.members) {
            c.max_M = std::max(c.max_M, items[i].net->M);
            c.max_N = std::max(c.max_N, items[i].net->N);
            c.max_nu = std::max(c.max_nu, items[i].net->max_nu);
            c.units += items[i].R;
        }
        B->classes.push_back(c);
    }
    // one device block: per class items, unit_start, item_next; then the
    // workspaces; then the key
    size_t off = 0;
    std::vector<size_t> o_items, o_start, o_next;
    auto align = [](size_t v) { return (v + 255) / 256 * 256; };
    for (auto& c : B->classes) {
        o_items.push_back(off);
        off = align(off + sizeof(rt_item_dev) * c.members.size());
        o_start.push_back(off);
        off = align(off + sizeof(int64_t) * (c.members.size() + 1));
        o_next.push_back(off);
        off = align(off + sizeof(unsigned long long) * c.members.size());
    }
    // the lazy classes' channel workspaces, sized for their grids
    std::vector<size_t> o_lazy(B->classes.size(), 0);
    for (size_t ci = 0; ci < B->classes.size(); ++ci) {
        auto& c = B->classes[ci];
        if (c.key.method != RTSSA_METHOD_LAZY) continue;
        bool sched = false;
        for (int i : c.members) sched |= items[i].net->dev.sched_B > 0;
        // beside other classes, at most 4 resident wavefronts per CU: a full
        // grid of the lazy kernel (3 per SIMD) would take every SIMD's
        // registers until its class drains, and the small classes, bound by
        // their longest trajectories, would wait for it (measured on 4096
        // random networks: 1.93 s per step against 2.06 s uncapped, 2.7 s at 2)
        const int cap = B->classes.size() > 1 ? 4 : 0;
        int rc = rt_lazy_grid(c.max_N, c.max_M, o.grid, c.units, sched, &c.lazy_grid, cap);
        if (rc) {
            delete B;
            return rc;
        }
        o_lazy[ci] = off;
        off = align(off + rt_lazy_workspace_bytes(c.lazy_grid, c.max_M));
    }
    const size_t o_ws = off;
    off = align(off + sizeof(rt_ws) * std::max<size_t>(1, B->classes.size()));
    const size_t o_key = off;
    off = align(off + 16);
    if (hipMalloc(&B->dev_block, off) != hipSuccess) {
        delete B;
        return rt_fail(RTSSA_E_NOMEM, "batch tables allocation failed");
    }
    char* base = (char*)B->dev_block;
    B->ws_dev = (rt_ws*)(base + o_ws);
    for (size_t ci = 0; ci < B->classes.size(); ++ci)
        if (B->classes[ci].key.method == RTSSA_METHOD_LAZY) B->classes[ci].lazy_ws = base + o_lazy[ci];
    B->key_dev = (uint32_t*)(base + o_key);
    int rc = RTSSA_OK;
    for (size_t ci = 0; ci < B->classes.size() && !rc; ++ci) {
        auto& c = B->classes[ci];
        std::vector<rt_item_dev> dv;
        std::vector<int64_t> starts(1, 0);
        for (int i : c.members) {
            const rtssa_batch_item& b = items[i];
            dv.push_back(rt_make_item(b.net, b.x0, b.x0_per_traj, b.t_end, b.sample_t, b.G,
                                      b.net_id, b.traj_offset, b.R, b.samples, b.s_stride_r,
                                      b.s_stride_g, b.s_stride_n, b.n_out, b.T_out, b.x_final,
                                      b.t_last, b.status, b.seq_hash, b.tie_step));
            starts.push_back(starts.back() + b.R);
        }
        rc = check_hip(hipMemcpy(base + o_items[ci], dv.data(), sizeof(rt_item_dev) * dv.size(),
                                 hipMemcpyHostToDevice), "batch upload");
        if (!rc)
            rc = check_hip(hipMemcpy(base + o_start[ci], starts.data(),
                                     sizeof(int64_t) * starts.size(), hipMemcpyHostToDevice),
                           "batch upload");
        c.dev.items = (const rt_item_dev*)(base + o_items[ci]);
        c.dev.unit_start = (const int64_t*)(base + o_start[ci]);
        c.dev.item_next = (unsigned long long*)(base + o_next[ci]);
        c.dev.ws = B->ws_dev + ci;
        c.dev.count = (int32_t)c.members.size();
        c.dev.exclusive = 1;
        c.dev.max_N = c.max_N;
        c.dev.max_M = c.max_M;
        c.dev.max_firings = (uint32_t)maxf;
        c.dev.has_schedule = 0;
        for (int i : c.members) c.dev.has_schedule |= items[i].net->dev.sched_B > 0;
        if (!rc && ci > 0)
            rc = check_hip(hipStreamCreateWithFlags(&c.side, hipStreamNonBlocking), "stream");
    }
    if (!rc) rc = check_hip(hipEventCreateWithFlags(&B->fork, hipEventDisableTiming), "event");
    for (size_t ci = 0; ci < B->classes.size() && !rc; ++ci) {
        hipEvent_t e = nullptr;
        rc = check_hip(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
        B->joins.push_back(e);
    }
    if (rc) {
        rtssa_batch_destroy(B);
        return rc;
    }
    // the items' descriptors hold each network's device pointers: its
    // schedule must not be reallocated while this batch exists
    for (const auto& it : B->items) ++const_cast<rtssa_network*>(it.net)->batch_refs;
    B->holds_nets = true;
    *out = B;
    return RTSSA_OK;
}

static int batch_enqueue(rtssa_batch* B, hipStream_t stream)
{
    // setup kernels (counters, queues, key) then one persistent kernel per
    // class, each class on its own stream, joined back into `stream`
    int rc = RTSSA_OK;
    for (size_t ci = 0; ci < B->classes.size() && !rc; ++ci) {
        auto& c = B->classes[ci];
        rc = rt_launch_setup(c.dev.ws, c.dev.item_next, c.dev.count, 0u, 0u, B->key_dev, nullptr,
                             nullptr, nullptr, stream);
    }
    if (!rc) rc = check_hip(hipEventRecord(B->fork, stream), "fork");
    for (size_t ci = 1; ci < B->classes.size() && !rc; ++ci)
        rc = check_hip(hipStreamWaitEvent(B->classes[ci].side, B->fork, 0), "fork");
    for (size_t ci = 0; ci < B->classes.size() && !rc; ++ci) {
        auto& c = B->classes[ci];
        hipStream_t s = ci == 0 ? stream : c.side;
        const int block = c.key.mapping == RTSSA_MAP_THREAD ? B->opt.block : c.key.a;
        if (c.key.method == RTSSA_METHOD_LAZY) {
            c.block_used = 64;
            rc = rt_launch_lazy(c.dev, c.max_N, c.max_M, c.lazy_grid, c.units, s, &c.grid_used,
                                c.lazy_ws);
        } else if (c.key.method == RTSSA_METHOD_DIRECT_TREE) {
            c.block_used = 64;
            rc = rt_launch_dmtree(c.dev, c.max_N, c.max_M, B->opt.grid, c.units, s, &c.grid_used);
        } else {
            rc = rt_launch_class(c.key.mapping,
                                 c.key.mapping == RTSSA_MAP_THREAD ? c.key.a : c.max_M,
                                 c.key.mapping == RTSSA_MAP_THREAD ? c.key.b : c.max_N, c.max_nu,
                                 c.dev, block, B->opt.grid, c.units, s, &c.block_used,
                                 &c.grid_used);
        }
        if (!rc && ci > 0) rc = check_hip(hipEventRecord(B->joins[ci], s), "join");
    }
    for (size_t ci = 1; ci < B->classes.size() && !rc; ++ci)
        rc = check_hip(hipStreamWaitEvent(stream, B->joins[ci], 0), "join");
    return rc;
}

extern "C" int rtssa_batch_run(rtssa_batch* B, uint64_t seed, int32_t use_graph,
                               rtssa_stream_t stream_, rtssa_stats* stats)
{
    if (!B) return rt_fail(RTSSA_E_INVALID, "batch is NULL");
    hipStream_t stream = (hipStream_t)stream_;
    if (stats) memset(stats, 0, sizeof(*stats));
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    int rc = check_hip(hipMemcpyAsync(B->key_dev, key, sizeof(key), hipMemcpyHostToDevice, stream),
                       "seed upload");
    if (rc) return rc;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (stats) {
        hipEventCreate(&ev0);
        hipEventCreate(&ev1);
        hipEventRecord(ev0, stream);
    }
    if (use_graph) {
        if (!B->exec) {
            // capture once; the key is read from device memory at run time
            hipStream_t cap = nullptr;
            rc = check_hip(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "stream");
            if (!rc) rc = check_hip(hipStreamBeginCapture(cap, hipStreamCaptureModeGlobal), "capture");
            if (!rc) {
                int rc2 = batch_enqueue(B, cap);
                hipGraph_t g = nullptr;
                rc = check_hip(hipStreamEndCapture(cap, &g), "end capture");
                if (!rc) rc = rc2;
                if (!rc) {
                    B->graph = g;
                    rc = check_hip(hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0),
                                   "graph instantiate");
                } else if (g) {
                    hipGraphDestroy(g);
                }
            }
            if (cap) hipStreamDestroy(cap);
        }
        if (!rc) rc = check_hip(hipGraphLaunch(B->exec, stream), "graph launch");
    } else {
        rc = batch_enqueue(B, stream);
    }
    if (!rc && stats) {
        hipEventRecord(ev1, stream);
        std::vector<rt_ws> h(B->classes.size());
        rc = check_hip(hipMemcpyAsync(h.data(), B->ws_dev, sizeof(rt_ws) * h.size(),
                                      hipMemcpyDeviceToHost, stream), "reading stats");
        if (!rc) rc = check_hip(hipStreamSynchronize(stream), "batch");
        if (!rc) {
            float ms = 0.f;
            hipEventElapsedTime(&ms, ev0, ev1);
            for (const auto& w : h) rt_fill_stats(stats, w);
            stats->kernel_ms = ms;
            stats->mapping = 0;
            stats->grid = (int32_t)B->classes.size();
        }
    }
    if (ev0) hipEventDestroy(ev0);
    if (ev1) hipEventDestroy(ev1);
    return rc;
}

extern "C" int rtssa_batch_info(const rtssa_batch* B, int32_t cls, int32_t* mapping, int32_t* lanes,
                                int32_t* n_items, int64_t* trajectories, int32_t* max_M)
{
    if (!B) return rt_fail(RTSSA_E_INVALID, "batch is NULL");
    if (cls < 0) {
        if (n_items) *n_items = (int32_t)B->classes.size();
        return RTSSA_OK;
    }
    if (cls >= (int)B->classes.size()) return rt_fail(RTSSA_E_INVALID, "no such class");
    const auto& c = B->classes[cls];
    if (mapping) *mapping = c.key.mapping;
    if (lanes) *lanes = c.key.mapping == RTSSA_MAP_THREAD ? 1 : c.key.a;
    if (n_items) *n_items = (int32_t)c.members.size();
    if (trajectories) *trajectories = c.units;
    if (max_M) *max_M = c.max_M;
    return RTSSA_OK;
}

extern "C" int rtssa_batch_class_items(const rtssa_batch* B, int32_t cls, int32_t* items,
                                       int32_t capacity, int32_t* count)
{
    if (!B || !count) return rt_fail(RTSSA_E_INVALID, "batch and count are required");
    if (cls < 0 || cls >= (int)B->classes.size()) return rt_fail(RTSSA_E_INVALID, "no such class");
    const auto& m = B->classes[cls].members;
    *count = (int32_t)m.size();
    if (items)
        for (int32_t i = 0; i < std::min<int32_t>(capacity, (int32_t)m.size()); ++i) items[i] = m[i];
    return RTSSA_OK;
}

extern "C" int rtssa_batch_destroy(rtssa_batch* B)
{
    if (!B) return RTSSA_OK;
    if (B->holds_nets)
        for (const auto& it : B->items) --const_cast<rtssa_network*>(it.net)->batch_refs;
    if (B->exec) hipGraphExecDestroy(B->exec);
    if (B->graph) hipGraphDestroy(B->graph);
    for (auto& c : B->classes)
        if (c.side) hipStreamDestroy(c.side);
    for (auto e : B->joins)
        if (e) hipEventDestroy(e);
    if (B->fork) hipEventDestroy(B->fork);
    if (B->dev_block) hipFree(B->dev_block);
    delete B;
    return RTSSA_OK;
}

// ---------------------------------------------------------------- autotuner
// Size classes present in the items: sub-wave channel counts in (8L/2, 8L]
// (all counts up to 32 for L = 4); workgroup counts in power-of-two ranges
// from (512, 1024] up.  For each class, every feasible lane count is timed on
// a sub-batch of up to `samples` of its items, launched the way the batch
// launches the class (one persistent grid shared by the items, outputs
// dropped, firings capped at 4000 per trajectory); items with a shared x0
// get more trajectories so that the sub-batch fills the device (65536
// trajectories for sub-wavefront classes, 8192 for workgroup classes).  The
// fastest in firings per second goes to the plan file.  Returns the number
// of classes tuned.
extern "C" int rtssa_autotune(const rtssa_batch_item* items, int32_t count, int32_t samples,
                              const char* plan_path, rtssa_stream_t stream_)
{
    if (!items || count < 1 || !plan_path) return rt_fail(RTSSA_E_INVALID, "bad arguments");
    hipStream_t stream = (hipStream_t)stream_;
    struct bucket { int mapping, lo, hi; std::vector<int> members; };
    std::map<std::pair<int, int>, bucket> buckets;
    for (int i = 0; i < count; ++i) {
        const rtssa_network* n = items[i].net;
        if (items[i].R < 1 || items[i].method != RTSSA_METHOD_RANDOM_TIME) continue;
        int m = rt_auto_mapping(n);
        if (m == RTSSA_MAP_THREAD) continue;
        if (m == RTSSA_MAP_WAVE && n->M > 512) m = RTSSA_MAP_WORKGROUP;
        int lo, hi;
        if (m == RTSSA_MAP_WAVE) {
            int L = rt_subwave_lanes(n->M);
            lo = L == 4 ? 1 : 4 * L + 1;
            hi = 8 * L;
        } else {
            hi = 1024;
            while (hi < n->M) hi <<= 1;
            lo = hi == 1024 ? 1 : hi / 2 + 1;
        }
        auto& b = buckets[{m, hi}];
        b.mapping = m;
        b.lo = lo;
        b.hi = hi;
        if ((int)b.members.size() < std::max(1, samples)) b.members.push_back(i);
    }
    std::vector<plan_entry> chosen;
    for (auto& kv : buckets) {
        bucket& b = kv.second;
        int max_nu = 0, max_M = 0;
        std::vector<rtssa_batch_item> sub;
        // enough trajectories to fill the device at every candidate (a
        // too-small sub-batch measures latency, not throughput)
        const int64_t fill = b.mapping == RTSSA_MAP_WAVE ? 65536 : 8192;
        const int64_t per_item = (fill + (int64_t)b.members.size() - 1) / (int64_t)b.members.size();
        for (int i : b.members) {
            rtssa_batch_item it = items[i];
            if (!it.x0_per_traj) it.R = std::max<int64_t>(it.R, per_item);
            // outputs dropped: the tuning runs leave the caller's buffers alone
            it.samples = nullptr;
            it.G = 0;
            it.sample_t = nullptr;
            it.n_out = nullptr;
            it.T_out = nullptr;
            it.x_final = nullptr;
            it.t_last = nullptr;
            it.status = nullptr;
            it.seq_hash = nullptr;
            it.tie_step = nullptr;
            sub.push_back(it);
            max_nu = std::max(max_nu, it.net->max_nu);
            max_M = std::max(max_M, it.net->M);
        }
        std::vector<int> cands;
        if (b.mapping == RTSSA_MAP_WAVE) {
            for (int L = 4; L <= 64; L <<= 1)
                if (8 * L >= max_M && L >= max_nu) cands.push_back(L);
        } else {
            for (int L = 64; L <= 1024; L <<= 1)
                if (rt_group_supported(max_M, L)) cands.push_back(L);
        }
        double best = -1.0;
        int bestL = 0;
        for (int L : cands) {
            rtssa_options o{};
            o.mapping = b.mapping;
            o.max_firings = 4000;
            std::vector<plan_entry> p = {{b.mapping, 1, 1 << 30, L}};
            rtssa_batch* tb = nullptr;
            if (batch_create(sub.data(), (int32_t)sub.size(), &o, p, &tb)) continue;
            rtssa_stats st{};
            const int rc = rtssa_batch_run(tb, 7, 0, (rtssa_stream_t)stream, &st);
            rtssa_batch_destroy(tb);
            if (rc || st.kernel_ms <= 0) continue;
            const double rate = (double)st.firings / st.kernel_ms;
            if (rate > best) { best = rate; bestL = L; }
        }
        if (bestL > 0) chosen.push_back({b.mapping, b.lo, b.hi, bestL});
    }
    FILE* f = fopen(plan_path, "w");
    if (!f) return rt_fail(RTSSA_E_INVALID, std::string("cannot write ") + plan_path);
    for (const auto& e : chosen)
        fprintf(f, "%s %d %d %d\n", e.mapping == RTSSA_MAP_WAVE ? "wave" : "workgroup", e.lo, e.hi,
                e.L);
    fclose(f);
    return (int)chosen.size();
}
