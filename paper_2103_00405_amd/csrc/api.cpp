// api.cpp -- the C ABI: argument validation, mapping choice, launches, stats.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "internal.h"

static thread_local std::string g_last_error = "no error";

int rt_fail(int code, const std::string& msg)
{
    g_last_error = msg;
    return code;
}

extern "C" const char* rtssa_last_error(void) { return g_last_error.c_str(); }
extern "C" const char* rtssa_version(void) { return "rtssa 0.1 (gfx950)"; }

int check_hip(hipError_t e, const char* what)
{
    if (e == hipSuccess) return RTSSA_OK;
    return rt_fail(RTSSA_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Mapping chosen from the network size: thread-per-trajectory for register-
// sized networks, sub-wavefront groups (4..64 lanes) up to 512 channels, a
// workgroup beyond.
int rt_auto_mapping(const rtssa_network* net)
{
    if (rt_thread_supported(net->M, net->N)) return RTSSA_MAP_THREAD;
    if (net->M <= 512 && net->max_nu <= 64) return RTSSA_MAP_WAVE;
    return RTSSA_MAP_WORKGROUP;
}

// Workgroup size of the workgroup mapping when no plan says otherwise: the
// fewest threads that hold every channel in at most 16 slots (up to 4096
// channels; 1024 threads with up to 8 slots beyond).  Fewer, fuller threads
// leave room for more trajectories per CU, which measured faster on every
// size class tried (512..4096 channels).
int rt_auto_group_size(int M)
{
    int L = 64;
    while (L < 256 && 16 * L < M) L <<= 1;
    return 16 * L >= M ? L : 1024;
}

// Lanes per trajectory of the sub-wave mapping: the requested value, or the
// fewest lanes holding every channel in at most 8 slots; never fewer lanes
// than species changed by one reaction.
int rt_pick_lanes(const rtssa_network* net, int requested)
{
    int L = requested > 0 ? requested : rt_subwave_lanes(net->M);
    while (L < 64 && L < net->max_nu) L <<= 1;
    return L;
}

// Launch one class with the given mapping; block = lanes per trajectory for
// the sub-wave mapping, threads per trajectory for the workgroup mapping,
// workgroup size for the thread mapping.
int rt_launch_class(int mapping, int max_M, int max_N, int max_nu, const rt_class_dev& C,
                    int block, int grid, int64_t lanes, hipStream_t stream, int* block_used,
                    int* grid_used, int method)
{
    if (mapping == RTSSA_MAP_THREAD) {
        if (block <= 0) block = 256;
        *block_used = block;
        return rt_launch_thread(max_M, max_N, C, block, grid, stream, grid_used, lanes, method);
    }
    if (method != RTSSA_METHOD_RANDOM_TIME)
        return rt_fail(RTSSA_E_UNSUPPORTED, "the direct method runs only in the thread mapping");
    if (mapping == RTSSA_MAP_WAVE) {
        int L = block > 0 ? block : rt_subwave_lanes(max_M);
        while (L < 64 && L < max_nu) L <<= 1;
        if (L != 4 && L != 8 && L != 16 && L != 32 && L != 64)
            return rt_fail(RTSSA_E_INVALID, "sub-wave lanes per trajectory must be 4..64, a power of 2");
        if (max_M > 8 * L) return rt_fail(RTSSA_E_UNSUPPORTED, "too many channels for this lane count");
        if (max_nu > L) return rt_fail(RTSSA_E_UNSUPPORTED, "a reaction changes more species than lanes");
        *block_used = L;
        return rt_launch_subwave(max_M, C, L, grid, stream, grid_used);
    }
    if (mapping == RTSSA_MAP_WORKGROUP) {
        int L = block > 0 ? block : rt_auto_group_size(max_M);
        if (L != 64 && L != 128 && L != 256 && L != 512 && L != 1024)
            return rt_fail(RTSSA_E_INVALID, "group size must be 64, 128, 256, 512 or 1024");
        if (max_nu > 64) return rt_fail(RTSSA_E_UNSUPPORTED, "a reaction changes more than 64 species");
        *block_used = L;
        // propensities in LDS and one barrier per firing where its LDS fits,
        // else every channel's state in registers
        if (rt_group_lds_kernel_for(max_M, max_N, L, C.has_schedule != 0))
            return rt_launch_group_lds(max_M, max_N, C, L, grid, stream, grid_used);
        return rt_launch_group(max_M, max_N, max_M, C, L, grid, stream, grid_used);
    }
    return rt_fail(RTSSA_E_INVALID, "unknown mapping");
}

// Item descriptor of one run (host copy).
rt_item_dev rt_make_item(const rtssa_network* net, const int32_t* x0, int32_t x0_per_traj,
                         double t_end, const double* sample_t, int32_t G, uint32_t net_id,
                         uint64_t traj_offset, int64_t R, int32_t* samples, int64_t s_stride_r,
                         int64_t s_stride_g, int64_t s_stride_n, uint32_t* n_out, double* T_out,
                         int32_t* x_final, double* t_last, uint8_t* status, uint64_t* seq_hash,
                         uint32_t* tie_step)
{
    rt_item_dev it{};
    it.net = net->dev;
    it.x0 = x0;
    it.x0_per_traj = x0_per_traj;
    it.G = G;
    it.t_end = t_end;
    it.s = sample_t;
    it.net_id = net_id;
    it.traj_offset = (uint32_t)traj_offset;
    it.R = R;
    it.samples = samples;
    it.ss_r = s_stride_r;
    it.ss_g = s_stride_g;
    it.ss_n = s_stride_n;
    it.n_out = n_out;
    it.T_out = T_out;
    it.x_final = x_final;
    it.t_last = t_last;
    it.status = status;
    it.seq_hash = (unsigned long long*)seq_hash;
    it.tie_step = tie_step;
    return it;
}

// Host-side checks of a run's sizes and pointers; the sample grid's values
// stay on the device and are checked there by the setup kernel.
int rt_check_run(const rtssa_network* net, const int32_t* x0, int32_t x0_per_traj, double t_end,
                 const double* sample_t, int32_t G, uint64_t traj_offset, int64_t R)
{
    if (!net) return rt_fail(RTSSA_E_INVALID, "net is NULL");
    if (R < 0 || G < 0) return rt_fail(RTSSA_E_INVALID, "R and G must be >= 0");
    if (!(t_end >= 0.0) || !isfinite(t_end)) return rt_fail(RTSSA_E_INVALID, "t_end must be finite and >= 0");
    if (traj_offset + (uint64_t)R > (1ull << 32))
        return rt_fail(RTSSA_E_INVALID, "traj_offset + R must not exceed 2^32");
    if (R > 0 && !x0 && net->N > 0) return rt_fail(RTSSA_E_INVALID, "x0 is NULL");
    if (G > 0 && !sample_t) return rt_fail(RTSSA_E_INVALID, "sample_t is NULL with G > 0");
    if (x0_per_traj != 0 && x0_per_traj != 1) return rt_fail(RTSSA_E_INVALID, "x0_per_traj must be 0 or 1");
    return RTSSA_OK;
}

// Reads a sample grid from the device and checks it (synchronous).
int rt_check_grid_host(const double* sample_t, int32_t G, double t_end)
{
    if (G <= 0) return RTSSA_OK;
    std::vector<double> s(G);
    int rc = check_hip(hipMemcpy(s.data(), sample_t, sizeof(double) * G, hipMemcpyDeviceToHost),
                       "reading sample_t");
    if (rc) return rc;
    for (int g = 0; g < G; ++g) {
        if (!(s[g] >= 0.0 && s[g] <= t_end))
            return rt_fail(RTSSA_E_INVALID, "sample_t values must lie in [0, t_end]");
        if (g > 0 && s[g] < s[g - 1])
            return rt_fail(RTSSA_E_INVALID, "sample_t must be non-decreasing");
    }
    return RTSSA_OK;
}

void rt_fill_stats(rtssa_stats* stats, const rt_ws& h)
{
    stats->firings += h.firings;
    stats->near_ties += h.near_ties;
    stats->clamps += h.clamps;
    stats->slow_logs += h.slow_logs;
    for (int q = 0; q < 4; ++q) stats->status_count[q] += h.status_count[q];
}


int rt_run_rows(const rtssa_network* net, const rtssa_options& o)
{
    if (o.method == RTSSA_METHOD_LAZY || o.method == RTSSA_METHOD_DIRECT_TREE) return 1;
    if (o.method != RTSSA_METHOD_RANDOM_TIME) return 0;
    const int mapping = o.mapping == RTSSA_MAP_AUTO ? rt_auto_mapping(net) : o.mapping;
    // (also for M = 0: the kernels load the rows of channel 0 before they
    // find that nothing can fire, and the tables then hold one empty row)
    return mapping == RTSSA_MAP_WORKGROUP ? 2 : (mapping == RTSSA_MAP_WAVE ? 1 : 0);
}

bool rt_rows_ready(const rtssa_network* net, int rows)
{
    return rows == 0 || (net->lazy_block && (rows < 2 || net->group_block));
}

int rt_rows_prepare(rtssa_network* net, int rows)
{
    if (rows >= 2) return rt_group_rows_prepare(net);
    if (rows == 1) return rt_lazy_prepare(net);
    return RTSSA_OK;
}

int rt_check_method(const rtssa_network* net, const rtssa_options& o, bool want_T,
                           bool want_tie)
{
    if (o.method != RTSSA_METHOD_RANDOM_TIME && o.method != RTSSA_METHOD_DIRECT &&
        o.method != RTSSA_METHOD_LAZY && o.method != RTSSA_METHOD_DIRECT_TREE)
        return rt_fail(RTSSA_E_INVALID, "unknown method");
    const bool wave_tree = o.method == RTSSA_METHOD_LAZY || o.method == RTSSA_METHOD_DIRECT_TREE;
    if (o.method == RTSSA_METHOD_DIRECT_TREE && (want_T || want_tie))
        return rt_fail(RTSSA_E_INVALID, "the direct method has no internal times or near-ties: "
                                        "T_out and tie_step must be NULL");
    if (wave_tree) {
        if (o.method == RTSSA_METHOD_DIRECT_TREE && net->dev.sched_B > 0)
            return rt_fail(RTSSA_E_UNSUPPORTED, "the direct method takes no rate schedule");
        if (o.mapping != RTSSA_MAP_AUTO && o.mapping != RTSSA_MAP_WAVE)
            return rt_fail(RTSSA_E_UNSUPPORTED, "the tree methods run one wavefront per trajectory");
        if (o.block != 0 && o.block != 64)
            return rt_fail(RTSSA_E_INVALID, "the tree methods' block is 64 lanes");
        if (net->max_nu > 64)
            return rt_fail(RTSSA_E_UNSUPPORTED, "a reaction changes more than 64 species");
    }
    if (o.method == RTSSA_METHOD_DIRECT) {
        if (net->dev.sched_B > 0)
            return rt_fail(RTSSA_E_UNSUPPORTED, "rate schedules run with the random-time method");
        if (want_T || want_tie)
            return rt_fail(RTSSA_E_INVALID, "the direct method has no internal times or near-ties: "
                                            "T_out and tie_step must be NULL");
        if (!rt_thread_supported(net->M, net->N) ||
            (o.mapping != RTSSA_MAP_AUTO && o.mapping != RTSSA_MAP_THREAD))
            return rt_fail(RTSSA_E_UNSUPPORTED, "the channel-order direct method runs only in the "
                                                "thread mapping (M, N <= 8); "
                                                "RTSSA_METHOD_DIRECT_TREE runs larger networks");
    }
    return RTSSA_OK;
}

// Workspace of one run: the counters, descriptor and queue heads, then (LAZY)
// the channel records of the lazy grid that the launch will use.  cap > 0
// bounds the workspace: the lazy grid then keeps only as many resident
// wavefronts as their channel records fit in cap (at least one).
int rt_run_workspace(const rtssa_network* net, int64_t R, const rtssa_options& o, size_t cap,
                     size_t* bytes, int* lazy_grid)
{
    const size_t base = rt_align256(sizeof(rt_run_scratch));
    size_t b = base;
    *lazy_grid = 0;
    if (o.method == RTSSA_METHOD_LAZY && R > 0) {
        int req = o.grid;
        if (cap > 0) {
            const size_t per_wave = rt_lazy_workspace_bytes(1, net->M);
            if (cap < base + rt_align256(per_wave))
                return rt_fail(RTSSA_E_UNSUPPORTED,
                               "the lazy form needs " + std::to_string(base + rt_align256(per_wave)) +
                                   " bytes of workspace for one wavefront; the maximum is " +
                                   std::to_string(cap));
            const int fit = (int)std::min<size_t>((cap - base - 255) / per_wave, 1 << 30);
            req = req > 0 ? std::min(req, fit) : fit;
        }
        int g = 0;
        const int rc = rt_lazy_grid(net->N, net->M, req, R, net->dev.sched_B > 0, &g);
        if (rc) return rc;
        if (cap > 0 && o.grid <= 0) {
            // the device's own resident count when it is below the cap
            int full = 0;
            const int rc2 = rt_lazy_grid(net->N, net->M, 0, R, net->dev.sched_B > 0, &full);
            if (rc2) return rc2;
            g = std::min(g, full);
        }
        *lazy_grid = g;
        b += rt_align256(rt_lazy_workspace_bytes(g, net->M));
    }
    *bytes = b;
    return RTSSA_OK;
}

extern "C" int rtssa_workspace_size(const rtssa_network* net, int64_t R, const rtssa_options* opt,
                                    size_t* bytes)
{
    if (!net || !bytes) return rt_fail(RTSSA_E_INVALID, "NULL argument");
    if (R < 0) return rt_fail(RTSSA_E_INVALID, "R must be >= 0");
    rtssa_options o{};
    if (opt) o = *opt;
    int rc = rt_check_method(net, o, false, false);
    if (rc) return rc;
    rc = rt_rows_prepare(const_cast<rtssa_network*>(net), rt_run_rows(net, o));
    if (rc) return rc;
    int lazy_grid = 0;
    return rt_run_workspace(net, R, o, 0, bytes, &lazy_grid);
}

// One run on a workspace the caller provides (ws, at least the bytes that
// rt_run_workspace reports for lazy_grid): validates, enqueues the setup and
// simulation kernels on the stream; with stats, waits and fills them
// (kernel_ms from two HIP events when time_kernels, else 0).
int rt_simulate_on(const rtssa_network* net, const int32_t* x0, int32_t x0_per_traj,
                   double t_end, const double* sample_t, int32_t G, uint64_t seed,
                   uint32_t net_id, uint64_t traj_offset, int64_t R, int32_t* samples,
                   int64_t s_stride_r, int64_t s_stride_g, int64_t s_stride_n, uint32_t* n_out,
                   double* T_out, int32_t* x_final, double* t_last, uint8_t* status,
                   uint64_t* seq_hash, uint32_t* tie_step, const rtssa_options& o, void* wsp,
                   int lazy_grid, hipStream_t stream, rtssa_stats* stats, bool time_kernels)
{
    const uint64_t maxf = o.max_firings ? o.max_firings : 10000000ull;
    const bool wave_tree = o.method == RTSSA_METHOD_LAZY || o.method == RTSSA_METHOD_DIRECT_TREE;
    const int mapping = o.method == RTSSA_METHOD_DIRECT
                            ? RTSSA_MAP_THREAD
                            : (wave_tree ? RTSSA_MAP_WAVE
                                         : (o.mapping == RTSSA_MAP_AUTO ? rt_auto_mapping(net)
                                                                        : o.mapping));
    rt_run_scratch* sc = (rt_run_scratch*)wsp;
    void* lazy_ws = (char*)wsp + rt_align256(sizeof(rt_run_scratch));
    const rt_item_dev item = rt_make_item(net, x0, x0_per_traj, t_end, sample_t, G, net_id,
                                          traj_offset, R, samples, s_stride_r, s_stride_g,
                                          s_stride_n, n_out, T_out, x_final, t_last, status,
                                          seq_hash, tie_step);
    rt_class_dev C{};
    C.items = &sc->item;
    C.unit_start = sc->unit_start;
    C.item_next = sc->item_next;
    C.ws = &sc->ws;
    C.count = 1;
    C.exclusive = 0;
    C.max_N = net->N;
    C.max_M = net->M;
    C.max_firings = (uint32_t)maxf;
    C.has_schedule = net->dev.sched_B > 0;

    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (stats && time_kernels) {
        hipEventCreate(&ev0);
        hipEventCreate(&ev1);
    }
    int rc = rt_launch_setup(&sc->ws, sc->item_next, 2, (uint32_t)seed, (uint32_t)(seed >> 32),
                             nullptr, &item, &sc->item, sc->unit_start, stream);
    if (!rc && ev0) hipEventRecord(ev0, stream);
    int grid_used = 0, block_used = 0;
    if (!rc && o.method == RTSSA_METHOD_LAZY) {
        block_used = 64;
        rc = rt_launch_lazy(C, net->N, net->M, lazy_grid, R, stream, &grid_used, lazy_ws);
    } else if (!rc && o.method == RTSSA_METHOD_DIRECT_TREE) {
        block_used = 64;
        rc = rt_launch_dmtree(C, net->N, net->M, o.grid, R, stream, &grid_used);
    } else if (!rc) {
        rc = rt_launch_class(mapping, net->M, net->N, net->max_nu, C, o.block, o.grid, R, stream,
                             &block_used, &grid_used, o.method);
    }
    if (!rc && stats) {
        if (ev1) hipEventRecord(ev1, stream);
        rt_ws h{};
        rc = check_hip(hipMemcpyAsync(&h, &sc->ws, sizeof(rt_ws), hipMemcpyDeviceToHost, stream),
                       "reading stats");
        if (!rc) rc = check_hip(hipStreamSynchronize(stream), "simulation");
        if (!rc) {
            float ms = 0.f;
            if (ev0 && ev1) hipEventElapsedTime(&ms, ev0, ev1);
            rt_fill_stats(stats, h);
            stats->kernel_ms = ms;
            stats->mapping = mapping;
            stats->block = block_used;
            stats->grid = grid_used;
            stats->bad_input = h.bad_input ? 1 : 0;
            if (h.bad_input)
                rc = rt_fail(RTSSA_E_INVALID, "sample_t must be non-decreasing and lie in "
                                              "[0, t_end] (checked on the device; nothing ran)");
        }
    }
    if (ev0) hipEventDestroy(ev0);
    if (ev1) hipEventDestroy(ev1);
    return rc;
}

// Argument checks shared by the entry points; *ready: the run has work.
int rt_simulate_checks(const rtssa_network* net, const int32_t* x0, int32_t x0_per_traj,
                       double t_end, const double* sample_t, int32_t G, uint64_t traj_offset,
                       int64_t R, const double* T_out, const uint32_t* tie_step,
                       const rtssa_options& o, bool may_build_rows)
{
    uint64_t maxf = o.max_firings ? o.max_firings : 10000000ull;
    if (maxf > 0xFFFFFFFFull) return rt_fail(RTSSA_E_INVALID, "max_firings must be < 2^32");
    int rc = rt_check_run(net, x0, x0_per_traj, t_end, sample_t, G, traj_offset, R);
    if (rc) return rc;
    rc = rt_check_method(net, o, T_out != nullptr, tie_step != nullptr);
    if (rc) return rc;
    const int rows = rt_run_rows(net, o);
    if (rows && R > 0) {
        if (!may_build_rows && !rt_rows_ready(net, rows))
            return rt_fail(RTSSA_E_INVALID, "the tree methods and the sub-wave and workgroup "
                                            "mappings need the network's rows built first "
                                            "(rtssa_workspace_size)");
        rc = rt_rows_prepare(const_cast<rtssa_network*>(net), rows);
        if (rc) return rc;
    }
    return RTSSA_OK;
}

extern "C" int rtssa_simulate(const rtssa_network* net, const int32_t* x0, int32_t x0_per_traj,
                              double t_end, const double* sample_t, int32_t G, uint64_t seed,
                              uint32_t net_id, uint64_t traj_offset, int64_t R, int32_t* samples,
                              int64_t s_stride_r, int64_t s_stride_g, int64_t s_stride_n,
                              uint32_t* n_out, double* T_out, int32_t* x_final, double* t_last,
                              uint8_t* status, uint64_t* seq_hash, uint32_t* tie_step,
                              const rtssa_options* opt, rtssa_stream_t stream_, rtssa_stats* stats)
{
    hipStream_t stream = (hipStream_t)stream_;
    rtssa_options o{};
    if (opt) o = *opt;
    if (stats) memset(stats, 0, sizeof(*stats));
    if (o.workspace && ((uintptr_t)o.workspace & 255u))
        return rt_fail(RTSSA_E_INVALID, "the workspace must be 256-byte aligned");
    int rc = rt_simulate_checks(net, x0, x0_per_traj, t_end, sample_t, G, traj_offset, R, T_out,
                                tie_step, o, o.workspace == nullptr);
    if (rc || R == 0) return rc;
    size_t need = 0;
    int lazy_grid = 0;
    rc = rt_run_workspace(net, R, o, 0, &need, &lazy_grid);
    if (rc) return rc;
    void* wsp = o.workspace;
    if (wsp) {
        if (o.workspace_bytes < need)
            return rt_fail(RTSSA_E_INVALID, "workspace too small: " + std::to_string(need) +
                                                " bytes needed (rtssa_workspace_size)");
    } else {
        rc = check_hip(hipMallocAsync(&wsp, need, stream), "workspace allocation");
        if (rc) return rc;
    }
    rc = rt_simulate_on(net, x0, x0_per_traj, t_end, sample_t, G, seed, net_id, traj_offset, R,
                        samples, s_stride_r, s_stride_g, s_stride_n, n_out, T_out, x_final, t_last,
                        status, seq_hash, tie_step, o, wsp, lazy_grid, stream, stats);
    if (!o.workspace) hipFreeAsync(wsp, stream);
    return rc;
}

extern "C" int rtssa_score_grad_workspace_size(int64_t R, int32_t M, size_t* bytes)
{
    if (!bytes || R < 1 || M < 1) return rt_fail(RTSSA_E_INVALID, "R, M >= 1 and bytes required");
    *bytes = rt_score_grad_workspace_bytes(R, M);
    return RTSSA_OK;
}

extern "C" int rtssa_score_grad(const double* f, const uint32_t* n, const double* T, int64_t R,
                                int32_t M, int32_t baseline, double* grad, double* se,
                                void* workspace, uint64_t workspace_bytes, rtssa_stream_t stream)
{
    if (!f || !n || !T || !grad) return rt_fail(RTSSA_E_INVALID, "NULL argument");
    if (R < 1 || M < 1) return rt_fail(RTSSA_E_INVALID, "R and M must be >= 1");
    if (baseline != 0 && baseline != 1) return rt_fail(RTSSA_E_INVALID, "baseline must be 0 or 1");
    if (workspace && (workspace_bytes < rt_score_grad_workspace_bytes(R, M) ||
                      ((uintptr_t)workspace & 7u)))
        return rt_fail(RTSSA_E_INVALID, "score workspace too small or misaligned");
    return rt_launch_score_grad(f, n, T, R, M, baseline, grad, se, workspace,
                                (hipStream_t)stream);
}

extern "C" int rtssa_debug_neglog(const uint64_t* m, double* out, uint8_t* slow, int64_t count,
                                  int32_t force_accurate, rtssa_stream_t stream)
{
    if (count < 0 || (count > 0 && (!m || !out))) return rt_fail(RTSSA_E_INVALID, "bad arguments");
    return rt_launch_debug_neglog(m, out, slow, count, force_accurate, (hipStream_t)stream);
}

extern "C" int rtssa_debug_philox(const uint32_t* ctr, uint32_t key0, uint32_t key1, uint32_t* out,
                                  int64_t count, rtssa_stream_t stream)
{
    if (count < 0 || (count > 0 && (!ctr || !out))) return rt_fail(RTSSA_E_INVALID, "bad arguments");
    return rt_launch_debug_philox(ctr, key0, key1, out, count, (hipStream_t)stream);
}

extern "C" int rtssa_debug_select(const double* v, int32_t M, int64_t count, int32_t mapping,
                                  int32_t lanes, int32_t* mu, double* v1, double* v2,
                                  uint8_t* near, rtssa_stream_t stream)
{
    if (count < 0 || M < 0) return rt_fail(RTSSA_E_INVALID, "count and M must be >= 0");
    if (count > 0 && (!mu || !v1 || !v2 || !near || (M > 0 && !v)))
        return rt_fail(RTSSA_E_INVALID, "NULL argument");
    return rt_launch_debug_select(v, M, count, mapping, lanes, mu, v1, v2, near,
                                  (hipStream_t)stream);
}
