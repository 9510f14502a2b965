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

static int check_hip(hipError_t e, const char* what)
{
    if (e == hipSuccess) return RTSSA_OK;
    return rt_fail(RTSSA_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Mapping chosen from the network size: thread-per-trajectory for register-
// sized networks, one wavefront for up to 64 x 16 channels, else a workgroup.
int rt_auto_mapping(const rtssa_network* net)
{
    if (rt_thread_supported(net->M, net->N)) return RTSSA_MAP_THREAD;
    if (net->M <= 512) return RTSSA_MAP_WAVE;
    return RTSSA_MAP_WORKGROUP;
}

int rt_auto_group_size(int M)
{
    if (M <= 1024) return 256;
    if (M <= 4096) return 1024;
    return 1024;
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
    if (!net) return rt_fail(RTSSA_E_INVALID, "net is NULL");
    if (R < 0 || G < 0) return rt_fail(RTSSA_E_INVALID, "R and G must be >= 0");
    if (!(t_end >= 0.0) || !isfinite(t_end)) return rt_fail(RTSSA_E_INVALID, "t_end must be finite and >= 0");
    if (traj_offset + (uint64_t)R > (1ull << 32))
        return rt_fail(RTSSA_E_INVALID, "traj_offset + R must not exceed 2^32");
    if (R > 0 && !x0 && net->N > 0) return rt_fail(RTSSA_E_INVALID, "x0 is NULL");
    if (G > 0 && !sample_t) return rt_fail(RTSSA_E_INVALID, "sample_t is NULL with G > 0");
    if (x0_per_traj != 0 && x0_per_traj != 1) return rt_fail(RTSSA_E_INVALID, "x0_per_traj must be 0 or 1");
    rtssa_options o{};
    if (opt) o = *opt;
    uint64_t maxf = o.max_firings ? o.max_firings : 10000000ull;
    if (maxf > 0xFFFFFFFFull) return rt_fail(RTSSA_E_INVALID, "max_firings must be < 2^32");
    if (stats) memset(stats, 0, sizeof(*stats));
    if (R == 0) return RTSSA_OK;

    // the sample grid must be sorted and inside [0, t_end]
    if (G > 0) {
        std::vector<double> s(G);
        int rc = check_hip(hipMemcpyAsync(s.data(), sample_t, sizeof(double) * G,
                                          hipMemcpyDeviceToHost, stream), "reading sample_t");
        if (!rc) rc = check_hip(hipStreamSynchronize(stream), "reading sample_t");
        if (rc) return rc;
        for (int g = 0; g < G; ++g) {
            if (!(s[g] >= 0.0 && s[g] <= t_end))
                return rt_fail(RTSSA_E_INVALID, "sample_t values must lie in [0, t_end]");
            if (g > 0 && s[g] < s[g - 1])
                return rt_fail(RTSSA_E_INVALID, "sample_t must be non-decreasing");
        }
    }

    int mapping = o.mapping;
    if (mapping == RTSSA_MAP_AUTO)
        mapping = rt_auto_mapping(net);

    rt_ws* ws = nullptr;
    int rc = check_hip(hipMallocAsync((void**)&ws, sizeof(rt_ws), stream), "workspace allocation");
    if (rc) return rc;
    rt_sim_params p{};
    p.x0 = x0;
    p.x0_per_traj = x0_per_traj;
    p.G = G;
    p.t_end = t_end;
    p.s = sample_t;
    p.key0 = (uint32_t)seed;
    p.key1 = (uint32_t)(seed >> 32);
    p.net_id = net_id;
    p.traj_offset = (uint32_t)traj_offset;
    p.R = R;
    p.max_firings = (uint32_t)maxf;
    p.samples = samples;
    p.ss_r = s_stride_r;
    p.ss_g = s_stride_g;
    p.ss_n = s_stride_n;
    p.n_out = n_out;
    p.T_out = T_out;
    p.x_final = x_final;
    p.t_last = t_last;
    p.status = status;
    p.seq_hash = (unsigned long long*)seq_hash;
    p.tie_step = tie_step;
    p.ws = ws;

    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (stats) {
        hipEventCreate(&ev0);
        hipEventCreate(&ev1);
    }
    rc = rt_launch_zero_ws(ws, &p, stream);
    if (!rc && stats) hipEventRecord(ev0, stream);
    int grid_used = 0, block_used = o.block;
    if (!rc) {
        if (mapping == RTSSA_MAP_THREAD) {
            if (block_used <= 0) block_used = 256;
            rc = rt_launch_thread(net, p, block_used, o.grid, stream, &grid_used);
        } else if (mapping == RTSSA_MAP_WAVE || mapping == RTSSA_MAP_WORKGROUP) {
            if (mapping == RTSSA_MAP_WAVE) block_used = 64;
            else if (block_used <= 0) block_used = rt_auto_group_size(net->M);
            if (block_used != 64 && block_used != 256 && block_used != 512 && block_used != 1024)
                rc = rt_fail(RTSSA_E_INVALID, "group size must be 64, 256, 512 or 1024");
            else
                rc = rt_launch_group(net, p, block_used, o.grid, stream, &grid_used);
        } else {
            rc = rt_fail(RTSSA_E_INVALID, "unknown mapping");
        }
    }
    if (!rc && stats) {
        hipEventRecord(ev1, stream);
        rt_ws h{};
        rc = check_hip(hipMemcpyAsync(&h, ws, sizeof(rt_ws), hipMemcpyDeviceToHost, stream),
                       "reading stats");
        if (!rc) rc = check_hip(hipStreamSynchronize(stream), "simulation");
        if (!rc) {
            float ms = 0.f;
            hipEventElapsedTime(&ms, ev0, ev1);
            stats->firings = h.firings;
            stats->near_ties = h.near_ties;
            stats->clamps = h.clamps;
            stats->slow_logs = h.slow_logs;
            for (int q = 0; q < 4; ++q) stats->status_count[q] = h.status_count[q];
            stats->kernel_ms = ms;
            stats->mapping = mapping;
            stats->block = block_used;
            stats->grid = grid_used;
        }
    }
    if (ev0) hipEventDestroy(ev0);
    if (ev1) hipEventDestroy(ev1);
    hipFreeAsync(ws, stream);
    return rc;
}

extern "C" int rtssa_score_grad(const double* f, const uint32_t* n, const double* T, int64_t R,
                                int32_t M, int32_t baseline, double* grad, double* se,
                                rtssa_stream_t stream)
{
    if (!f || !n || !T || !grad) return rt_fail(RTSSA_E_INVALID, "NULL argument");
    if (R < 1 || M < 1) return rt_fail(RTSSA_E_INVALID, "R and M must be >= 1");
    if (baseline != 0 && baseline != 1) return rt_fail(RTSSA_E_INVALID, "baseline must be 0 or 1");
    return rt_launch_score_grad(f, n, T, R, M, baseline, grad, se, (hipStream_t)stream);
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
