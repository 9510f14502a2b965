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
#define RT_HD __device__ __forceinline__
#define RT_LOG_CONST __constant__
#include <hip/hip_runtime.h>

#include "internal.h"
#include "rt_math.h"

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

template <int MT, int NT>
__global__ __launch_bounds__(256) void rt_thread_kernel(rt_sim_params P, rt_net_dev net)
{
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
    const bool want_hash = P.seq_hash != nullptr;

    // ---- lane counters
    unsigned long long c_fired = 0, c_ties = 0, c_clamps = 0, c_slow = 0;
    unsigned long long c_st[4] = {0, 0, 0, 0};

    // ---- trajectory state
    int32_t X[NT];
    double T[MT], Pk[MT], a[MT], inv[MT];
    uint32_t n[MT];
    double t = 0.0, s_next = 0.0;
    int32_t g = 0;
    uint32_t fired = 0, tie = kTieNone, traj = 0;
    unsigned long long hash = kFnvOffset;
    int64_t r = 0;

    auto refresh_rates = [&]() {
#pragma unroll
        for (int k = 0; k < MT; ++k) {
            a[k] = propensity<NT>(kind[k], s0[k], s1[k], c[k], X);
            inv[k] = a[k] > 0.0 ? 1.0 / a[k] : 0.0;
        }
    };
    auto start = [&](int64_t rr) {
        r = rr;
        traj = P.traj_offset + (uint32_t)rr;
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
            bool slow = false;
            Pk[k] = rt_exp1(P.key0, P.key1, traj, P.net_id, (uint32_t)k, 0u, &slow);
            c_slow += slow;
        }
        refresh_rates();
    };
    auto write_sample = [&](int32_t gg, bool invalid) {
        int32_t* dst = P.samples + r * P.ss_r + (int64_t)gg * P.ss_g;
#pragma unroll
        for (int j = 0; j < NT; ++j)
            if (j < N) dst[j * P.ss_n] = invalid ? -1 : X[j];
    };
    auto finish = [&](int st) {
        const bool good = st == RTSSA_TRAJ_OK || st == RTSSA_TRAJ_ABSORBED;
        if (P.samples)
            for (int32_t gg = g; gg < P.G; ++gg) write_sample(gg, !good);
        if (good) {
            const double dt = P.t_end - t;
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
        c_fired += fired;
        c_st[st] += 1;
    };

    int64_t rr = (int64_t)atomicAdd(&P.ws->next_traj, 1ull);
    bool active = rr < P.R;
    if (active) start(rr);

    while (active) {
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
        int st = -1;
        const double t_new = t + d1;
        if (d1 == __builtin_inf()) {
            st = RTSSA_TRAJ_ABSORBED;
        } else if (t_new > P.t_end) {
            st = RTSSA_TRAJ_OK;
        } else {
            if (d2 - d1 <= 1e-12 * d1) {
                c_ties += 1;
                tie = tie == kTieNone ? fired : tie;
            }
            while (s_next < t_new) {
                if (P.samples) write_sample(g, false);
                ++g;
                s_next = g < P.G ? P.s[g] : __builtin_inf();
            }
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
            if (!ok) {
                st = RTSSA_TRAJ_OVERFLOW;
            } else {
                c_clamps += clamped;
                // internal times advance by a_k Delta (Eq. 15); the fired
                // channel lands exactly on its firing internal time
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
                bool slow = false;
                const double E = rt_exp1(P.key0, P.key1, traj, P.net_id, (uint32_t)mu, n_mu, &slow);
                c_slow += slow;
                p_mu = p_mu + E;
#pragma unroll
                for (int k = 0; k < MT; ++k) Pk[k] = (mu == k) ? p_mu : Pk[k];
                refresh_rates();
                if (fired >= P.max_firings) st = RTSSA_TRAJ_MAX_FIRINGS;
            }
        }
        if (st >= 0) {
            finish(st);
            rr = (int64_t)atomicAdd(&P.ws->next_traj, 1ull);
            active = rr < P.R;
            if (active) start(rr);
        }
    }

    // one atomic per counter and wave (lanes are converged here)
    unsigned long long v[8] = {c_fired, c_ties, c_clamps, c_slow, c_st[0], c_st[1], c_st[2], c_st[3]};
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_xor(v[q], off, 64);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&P.ws->firings, v[0]);
        atomicAdd(&P.ws->near_ties, v[1]);
        atomicAdd(&P.ws->clamps, v[2]);
        atomicAdd(&P.ws->slow_logs, v[3]);
#pragma unroll
        for (int q = 0; q < 4; ++q) atomicAdd(&P.ws->status_count[q], v[4 + q]);
    }
}

__global__ void rt_zero_ws_kernel(rt_ws* ws)
{
    unsigned long long* w = (unsigned long long*)ws;
    const int nw = (int)(sizeof(rt_ws) / sizeof(unsigned long long));
    for (int i = threadIdx.x; i < nw; i += blockDim.x) w[i] = 0ull;
}

typedef void (*thread_kernel_t)(rt_sim_params, rt_net_dev);

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
    hipLaunchKernelGGL(kfn, dim3(grid), dim3(block), 0, stream, p, net);
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

int rt_launch_zero_ws(rt_ws* ws, hipStream_t stream)
{
    hipLaunchKernelGGL(rt_zero_ws_kernel, dim3(1), dim3(64), 0, stream, ws);
    return hipGetLastError() == hipSuccess ? RTSSA_OK : rt_fail(RTSSA_E_HIP, "workspace clear failed");
}
