// noalloc.hip -- rtssa_simulate_noalloc: one run on a fixed device scratch
// array instead of an allocated workspace, for callers that cannot allocate.
//
// The array lives in this code object (one copy per GPU, held until the
// process ends).  Its device address is resolved once per device, with that
// device current, and kept; host code passes that address to the kernels,
// never the array's name (which is a host-side stand-in).
#include <hip/hip_runtime.h>
#include <string.h>

#include <mutex>
#include <string>

#include "internal.h"

namespace {

static __device__ __align__(256) unsigned char scratch[RTSSA_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array.
int scratch_address(void** out)
{
    int dev = 0;
    int rc = check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (rc) return rc;
    if (dev < 0 || dev >= kMaxDevices) return rt_fail(RTSSA_E_UNSUPPORTED, "device index too large");
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        rc = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "resolving the scratch array");
        if (rc) return rc;
        if (!p || ((uintptr_t)p & 255u))
            return rt_fail(RTSSA_E_HIP, "scratch array address is not 256-byte aligned");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return RTSSA_OK;
}

}  // namespace

extern "C" int rtssa_simulate_noalloc(const rtssa_network* net, const int32_t* x0,
                                      int32_t x0_per_traj, double t_end, const double* sample_t,
                                      int32_t G, uint64_t seed, uint32_t net_id,
                                      uint64_t traj_offset, int64_t R, int32_t* samples,
                                      int64_t s_stride_r, int64_t s_stride_g, int64_t s_stride_n,
                                      uint32_t* n_out, double* T_out, int32_t* x_final,
                                      double* t_last, uint8_t* status, uint64_t* seq_hash,
                                      uint32_t* tie_step, const rtssa_options* opt,
                                      rtssa_stream_t stream_, rtssa_stats* stats)
{
    hipStream_t stream = (hipStream_t)stream_;
    rtssa_options o{};
    if (opt) o = *opt;
    if (stats) memset(stats, 0, sizeof(*stats));
    if (o.workspace)
        return rt_fail(RTSSA_E_INVALID, "rtssa_simulate_noalloc takes no workspace "
                                        "(it runs on the library's scratch array)");
    // the tree methods' rows are never built here (that allocates)
    int rc = rt_simulate_checks(net, x0, x0_per_traj, t_end, sample_t, G, traj_offset, R, T_out,
                                tie_step, o, false);
    if (rc || R == 0) return rc;
    size_t need = 0;
    int lazy_grid = 0;
    rc = rt_run_workspace(net, R, o, RTSSA_NOALLOC_SCRATCH_BYTES, &need, &lazy_grid);
    if (rc) return rc;
    if (need > RTSSA_NOALLOC_SCRATCH_BYTES)
        return rt_fail(RTSSA_E_UNSUPPORTED,
                       "the run needs " + std::to_string(need) + " bytes of scratch; "
                       "rtssa_simulate_noalloc has " +
                           std::to_string((size_t)RTSSA_NOALLOC_SCRATCH_BYTES));
    void* wsp = nullptr;
    rc = scratch_address(&wsp);
    if (rc) return rc;
    return rt_simulate_on(net, x0, x0_per_traj, t_end, sample_t, G, seed, net_id, traj_offset, R,
                          samples, s_stride_r, s_stride_g, s_stride_n, n_out, T_out, x_final,
                          t_last, status, seq_hash, tie_step, o, wsp, lazy_grid, stream, stats,
                          false);
}
