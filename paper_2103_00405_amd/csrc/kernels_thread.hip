// kernels_thread.hip -- thread-per-trajectory mapping for small networks.
//
// One lane owns one trajectory at a time; its whole state (t, X, and per
// channel T_k, P_k, a_k, 1/a_k, n_k) lives in VGPRs, the network tables in
// SGPRs.  The grid is persistent: a lane that finishes a trajectory takes the
// next index from a device work queue, so lanes stay busy despite uneven
// trajectory lengths.  Outputs go straight to the caller's buffers.
//
// The step is the next reaction random time algorithm (section 4, Table 2)
// in the internal-time form of Eq. 14-16: gaps (P_k - T_k)/a_k, argmin
// (Eq. 25), internal-time advance, jump, and one fresh Exp(1) (Eq. 26).
#include <hip/hip_runtime.h>

#include "internal.h"
#include "rt_device.h"

namespace {

constexpr uint32_t kTieNone = 0xFFFFFFFFu;
constexpr unsigned long long kFnvOffset = 0xcbf29ce484222325ull;
constexpr unsigned long long kFnvPrime = 0x100000001b3ull;

// RN((double)h) for h < 2^64: both halves convert exactly, one rounding.
__device__ __forceinline__ double u64_to_f64(uint64_t h)
{
    return fma((double)(uint32_t)(h >> 32), 0x1p32, (double)(uint32_t)h);
}

template <int NT>
__device__ __forceinline__ int32_t pick(const int32_t (&X)[NT], int j)
{
    int32_t v = X[0];
#pragma unroll
    for (int q = 1; q < NT; ++q) v = (j == q) ? X[q] : v;
    return v;
}

// h_k(X) of Eq. 2 with the reaction kind fixed per channel (uniform branch).
template <int NT>
__device__ __forceinline__ double propensity(int kind, int s0, int s1, double c,
                                             const int32_t (&X)[NT])
{
    uint64_t h;
    if (kind == RT_H_ZERO) {
        h = 1;
    } else if (kind == RT_H_ONE) {
        h = (uint32_t)pick(X, s0);
    } else if (kind == RT_H_PAIR) {
        uint32_t x = (uint32_t)pick(X, s0);
        h = ((uint64_t)x * (uint32_t)(x - 1u)) >> 1;   // x = 0 gives 0
    } else {
        h = (uint64_t)(uint32_t)pick(X, s0) * (uint32_t)pick(X, s1);
    }
    return c * u64_to_f64(h);
}

#ifndef RT_THREAD_MIN_WAVES
#define RT_THREAD_MIN_WAVES 4
#endif

template <int MT, int NT>
__global__ __launch_bounds__(256, RT_THREAD_MIN_WAVES) void rt_thread_kernel(
    rt_hot_params H, rt_ws* __restrict__ ws, rt_net_dev net)
{
    const rt_sim_params& P = ws->params;   // read only on rare paths
    // ---- network, uniform across the grid
    int kind[MT], s0[MT], s1[MT], nu[MT][NT];
    double c[MT];
#pragma unroll
    for (int k = 0; k < MT; ++k) {
        if (k < net.M) {
            int2 rr = net.react[k];
            kind[k] = (int)((uint32_t)rr.x >> 29);
            s0[k] = rr.x & RT_SPECIES_MASK;
            s1[k] = rr.y;
            c[k] = net.c[k];
        } else {
            kind[k] = RT_H_ZERO; s0[k] = 0; s1[k] = 0; c[k] = 0.0;   // dead padding channel
        }
#pragma unroll
        for (int j = 0; j < NT; ++j)
            nu[k][j] = (k < net.M && j < net.N) ? net.nu_dense[k * net.N + j] : 0;
    }
    const int N = net.N, M = net.M;
    const bool want_hash = ws->params.seq_hash != nullptr;
    __shared__ uint32_t log_scratch[4][RT_LOG_SCRATCH];     // one slice per wave
    uint32_t* sc = log_scratch[threadIdx.x >> 6];

    // counters live in the device workspace and change only on rare events
    // ---- trajectory state
    int32_t X[NT];
    double T[MT], Pk[MT], a[MT], inv[MT];
    uint32_t n[MT];
#pragma unroll
    for (int j = 0; j < NT; ++j) X[j] = 0;
#pragma unroll
    for (int k = 0; k < MT; ++k) { T[k] = 0.0; Pk[k] = 0.0; a[k] = 0.0; inv[k] = 0.0; n[k] = 0; }
    double t = 0.0, s_next = 0.0;
    int32_t g = 0;
    uint32_t fired = 0, tie = kTieNone, traj = 0;
    unsigned long long hash = kFnvOffset;
    int64_t r = 0;

    auto write_sample = [&](int32_t gg, bool invalid) {
        int32_t* dst = P.samples + r * P.ss_r + (int64_t)gg * P.ss_g;
#pragma unroll
        for (int j = 0; j < NT; ++j)
            if (j < N) dst[j * P.ss_n] = invalid ? -1 : X[j];
    };

    // Each pass is one firing of every active lane.  The common path is
    // straight-line; every rare event (start or end of a trajectory, a sample
    // point, a near-tie, a clamped gap, an overflow, the firing cap) is
    // handled in one branch entered only when some lane of the wave needs it.
    bool active = true, fresh = true, capped = false;
    while (__ballot(active) != 0ull) {
        if (!active) continue;
        // gaps and argmin (lowest k wins ties; d2 = second smallest gap)
        double d1 = __builtin_inf(), d2 = __builtin_inf();
        int mu = 0;
        bool clamped = false;
#pragma unroll
        for (int k = 0; k < MT; ++k) {
            const double raw = (Pk[k] - T[k]) * inv[k];
            double d = raw < 0.0 ? 0.0 : raw;
            d = a[k] == 0.0 ? __builtin_inf() : d;
            const bool lt = d < d1;
            d2 = lt ? d1 : (d < d2 ? d : d2);
            d1 = lt ? d : d1;
            mu = lt ? k : mu;
            clamped = lt ? (raw < 0.0) : clamped;
        }
        const double t_new = t + d1;
        const bool absorbed = d1 == __builtin_inf();
        const bool term = absorbed || t_new > H.t_end;
        // jump v_mu, checked against [0, 2^31 - 1]
        int32_t Xn[NT];
        bool ok = true;
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            int32_t dl = nu[0][j];
#pragma unroll
            for (int k = 1; k < MT; ++k) dl = (mu == k) ? nu[k][j] : dl;
            const int64_t v = (int64_t)X[j] + dl;
            ok = ok && v >= 0 && v <= 0x7FFFFFFF;
            Xn[j] = (int32_t)v;
        }
        const bool live = !fresh && !capped;          // a trajectory is in progress
        const bool event = live && !term;             // this pass may apply an event
        const bool near_tie = event && d2 - d1 <= 1e-12 * d1;
        const bool rare = !live || term || near_tie || clamped || !ok || s_next < t_new;
        if (__builtin_expect(__ballot(rare) != 0ull, 0)) {
            if (event) {
                if (near_tie) {
                    atomicAdd(&ws->near_ties, 1ull);
                    tie = tie == kTieNone ? fired : tie;
                }
                while (s_next < t_new) {
                    if (P.samples) write_sample(g, false);
                    ++g;
                    s_next = g < P.G ? P.s[g] : __builtin_inf();
                }
                if (ok && clamped) atomicAdd(&ws->clamps, 1ull);
            }
            const bool stop = !live || term || !ok;
            if (stop && !fresh) {
                // end of the trajectory
                const int st = capped ? RTSSA_TRAJ_MAX_FIRINGS
                                      : (absorbed ? RTSSA_TRAJ_ABSORBED
                                                  : (term ? RTSSA_TRAJ_OK : RTSSA_TRAJ_OVERFLOW));
                const bool good = st == RTSSA_TRAJ_OK || st == RTSSA_TRAJ_ABSORBED;
                if (P.samples)
                    for (int32_t gg = g; gg < P.G; ++gg) write_sample(gg, !good);
                if (good) {
                    const double dt = H.t_end - t;
#pragma unroll
                    for (int k = 0; k < MT; ++k) T[k] = fma(a[k], dt, T[k]);
                }
                if (P.n_out) {
#pragma unroll
                    for (int k = 0; k < MT; ++k) if (k < M) P.n_out[r * M + k] = n[k];
                }
                if (P.T_out) {
#pragma unroll
                    for (int k = 0; k < MT; ++k) if (k < M) P.T_out[r * M + k] = T[k];
                }
                if (P.x_final) {
#pragma unroll
                    for (int j = 0; j < NT; ++j) if (j < N) P.x_final[r * N + j] = X[j];
                }
                if (P.t_last) P.t_last[r] = t;
                if (P.status) P.status[r] = (uint8_t)st;
                if (P.seq_hash) P.seq_hash[r] = hash;
                if (P.tie_step) P.tie_step[r] = tie;
                atomicAdd(&ws->firings, (unsigned long long)fired);
                atomicAdd(&ws->status_count[st], 1ull);
            }
            if (stop) {
                // take the next trajectory from the work queue
                const int64_t rr = (int64_t)atomicAdd(&ws->next_traj, 1ull);
                fresh = false;
                capped = false;
                active = rr < P.R;
                if (active) {
                    r = rr;
                    traj = H.traj_offset + (uint32_t)rr;
                    const int32_t* x0 = P.x0 + (P.x0_per_traj ? rr * N : 0);
#pragma unroll
                    for (int j = 0; j < NT; ++j) X[j] = j < N ? x0[j] : 0;
                    t = 0.0;
                    g = 0;
                    s_next = P.G > 0 ? P.s[0] : __builtin_inf();
                    fired = 0;
                    tie = kTieNone;
                    hash = kFnvOffset;
#pragma unroll
                    for (int k = 0; k < MT; ++k) {
                        T[k] = 0.0;
                        n[k] = 0;
                        a[k] = propensity<NT>(kind[k], s0[k], s1[k], c[k], X);
                        inv[k] = 1.0 / a[k];
                    }
                    // first internal firing times, one draw at a time
#pragma unroll 1
                    for (int k = 0; k < MT; ++k) {
                        const double E0 = rt_exp1_wave(H.key0, H.key1, traj, H.net_id, (uint32_t)k,
                                                       0u, &ws->slow_logs, sc);
#pragma unroll
                        for (int q = 0; q < MT; ++q) Pk[q] = q == k ? E0 : Pk[q];
                    }
                }
            }
            if (__ballot(stop) != 0ull) continue;   // started lanes compute their first gaps
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
        p_mu = p_mu + rt_exp1_wave(H.key0, H.key1, traj, H.net_id, (uint32_t)mu, n_mu,
                                   &ws->slow_logs, sc);
        // a_k is a pure function of X; inv_k = RN(1 / a_k) (+inf for a dead
        // channel, whose gap is +inf by the a_k = 0 test and never reads it)
#pragma unroll
        for (int k = 0; k < MT; ++k) {
            Pk[k] = (mu == k) ? p_mu : Pk[k];
            a[k] = propensity<NT>(kind[k], s0[k], s1[k], c[k], X);
            inv[k] = 1.0 / a[k];
        }
        capped = fired >= H.max_firings;
    }

}

__global__ void rt_zero_ws_kernel(rt_ws* ws, rt_sim_params params)
{
    unsigned long long* w = (unsigned long long*)ws;
    const int nw = (int)(offsetof(rt_ws, params) / sizeof(unsigned long long));
    for (int i = threadIdx.x; i < nw; i += blockDim.x) w[i] = 0ull;
    if (threadIdx.x == 0) ws->params = params;
}

typedef void (*thread_kernel_t)(rt_hot_params, rt_ws*, rt_net_dev);

template <int MT, int NT>
int launch_mn(const rt_sim_params& p, const rt_net_dev& net, int block, int grid,
              hipStream_t stream, int* grid_used)
{
    thread_kernel_t kfn = rt_thread_kernel<MT, NT>;
    if (grid <= 0) {
        int dev = 0, cus = 0, per_cu = 0;
        hipGetDevice(&dev);
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, block, 0) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        int64_t need = (p.R + block - 1) / block;
        int64_t full = (int64_t)cus * per_cu;
        grid = (int)std::max<int64_t>(1, std::min<int64_t>(need, full));
    }
    if (grid_used) *grid_used = grid;
    rt_hot_params h{};
    h.t_end = p.t_end;
    h.key0 = p.key0;
    h.key1 = p.key1;
    h.net_id = p.net_id;
    h.traj_offset = p.traj_offset;
    h.max_firings = p.max_firings;
    hipLaunchKernelGGL(kfn, dim3(grid), dim3(block), 0, stream, h, p.ws, net);
    return hipGetLastError() == hipSuccess ? RTSSA_OK : rt_fail(RTSSA_E_HIP, "thread kernel launch failed");
}

template <int MT>
int launch_m(int N, const rt_sim_params& p, const rt_net_dev& net, int block, int grid,
             hipStream_t stream, int* gu)
{
    if (N <= 1) return launch_mn<MT, 1>(p, net, block, grid, stream, gu);
    if (N <= 2) return launch_mn<MT, 2>(p, net, block, grid, stream, gu);
    if (N <= 4) return launch_mn<MT, 4>(p, net, block, grid, stream, gu);
    return launch_mn<MT, 8>(p, net, block, grid, stream, gu);
}

}  // namespace

int rt_thread_supported(int M, int N)
{
    return M >= 0 && N >= 0 && M <= RT_THREAD_MAX_M && N <= RT_THREAD_MAX_N;
}

int rt_launch_thread(const rtssa_network* net, const rt_sim_params& p, int block, int grid,
                     hipStream_t stream, int* grid_used)
{
    const int M = net->M, N = net->N;
    if (!rt_thread_supported(M, N))
        return rt_fail(RTSSA_E_UNSUPPORTED, "network too large for the thread mapping");
    if (block <= 0) block = 256;
    if (block > 256 || block % 64)
        return rt_fail(RTSSA_E_INVALID, "thread mapping block must be a multiple of 64, <= 256");
    switch (M) {
        case 0:
        case 1: return launch_m<1>(N, p, net->dev, block, grid, stream, grid_used);
        case 2: return launch_m<2>(N, p, net->dev, block, grid, stream, grid_used);
        case 3: return launch_m<3>(N, p, net->dev, block, grid, stream, grid_used);
        case 4: return launch_m<4>(N, p, net->dev, block, grid, stream, grid_used);
        case 5:
        case 6: return launch_m<6>(N, p, net->dev, block, grid, stream, grid_used);
        default: return launch_m<8>(N, p, net->dev, block, grid, stream, grid_used);
    }
}

int rt_launch_zero_ws(rt_ws* ws, const rt_sim_params* params, hipStream_t stream)
{
    hipLaunchKernelGGL(rt_zero_ws_kernel, dim3(1), dim3(64), 0, stream, ws, *params);
    return hipGetLastError() == hipSuccess ? RTSSA_OK : rt_fail(RTSSA_E_HIP, "workspace clear failed");
}
