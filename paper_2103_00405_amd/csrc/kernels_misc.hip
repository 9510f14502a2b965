// kernels_misc.hip -- score-function gradient (backward) and test-hook kernels.
#include <hip/hip_runtime.h>
#include <math.h>

#include "internal.h"
#include "rt_device.h"
#include "rt_wave.h"

namespace {

constexpr int kRedBlock = 256;

// Deterministic block sum of f over a contiguous row chunk.
__global__ __launch_bounds__(kRedBlock) void rt_sum_f_kernel(const double* f, int64_t R,
                                                             int64_t chunk, double* part)
{
    __shared__ double sh[kRedBlock];
    const int64_t r0 = (int64_t)blockIdx.x * chunk;
    const int64_t r1 = r0 + chunk < R ? r0 + chunk : R;
    double acc = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += kRedBlock) acc += f[r];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kRedBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Per block and channel: sum_r y_rk and sum_r y_rk^2 with
// y_rk = (f_r - b_r)(n_rk - T_rk), b_r the leave-one-out mean of f.
__global__ __launch_bounds__(kRedBlock) void rt_score_part_kernel(
    const double* f, const uint32_t* n, const double* T, int64_t R, int32_t M,
    int32_t baseline, int64_t chunk, const double* fpart, int nb, double* out)
{
    __shared__ double s1[kRedBlock], s2[kRedBlock];
    double F = 0.0;
    for (int b = 0; b < nb; ++b) F += fpart[b];
    const double denom = R > 1 ? (double)(R - 1) : 1.0;
    const int64_t r0 = (int64_t)blockIdx.x * chunk;
    const int64_t r1 = r0 + chunk < R ? r0 + chunk : R;
    const int kk = M < kRedBlock ? M : kRedBlock;
    const int tpk = kRedBlock / kk;
    const int tid = threadIdx.x;
    for (int kb = 0; kb < M; kb += kk) {
        const int k = kb + tid % kk;
        const int q = tid / kk;
        double a1 = 0.0, a2 = 0.0;
        if (q < tpk && k < M) {
            for (int64_t r = r0 + q; r < r1; r += tpk) {
                const double fr = f[r];
                const double b = baseline ? (F - fr) / denom : 0.0;
                const double y = (fr - b) * ((double)n[r * M + k] - T[r * M + k]);
                a1 += y;
                a2 += y * y;
            }
        }
        s1[tid] = a1;
        s2[tid] = a2;
        __syncthreads();
        if (tid < kk && kb + tid < M) {
            double t1 = 0.0, t2 = 0.0;
            for (int qq = 0; qq < tpk; ++qq) { t1 += s1[qq * kk + tid]; t2 += s2[qq * kk + tid]; }
            out[((int64_t)blockIdx.x * M + kb + tid) * 2 + 0] = t1;
            out[((int64_t)blockIdx.x * M + kb + tid) * 2 + 1] = t2;
        }
        __syncthreads();
    }
}

__global__ void rt_score_final_kernel(const double* part, int nb, int32_t M, int64_t R,
                                      double* grad, double* se)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    double t1 = 0.0, t2 = 0.0;
    for (int b = 0; b < nb; ++b) {
        t1 += part[((int64_t)b * M + k) * 2 + 0];
        t2 += part[((int64_t)b * M + k) * 2 + 1];
    }
    const double Rd = (double)R;
    grad[k] = t1 / Rd;
    if (se) {
        double var = R > 1 ? (t2 - t1 * (t1 / Rd)) / (Rd - 1.0) : 0.0;
        se[k] = var > 0.0 ? sqrt(var / Rd) : 0.0;
    }
}

__global__ __launch_bounds__(256) void rt_debug_neglog_kernel(const uint64_t* m, double* out,
                                                               uint8_t* slow, int64_t count,
                                                               int force)
{
    __shared__ uint32_t log_scratch[4][RT_LOG_SCRATCH];
    __shared__ unsigned long long slow_count[256];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    slow_count[threadIdx.x] = 0ull;
    out[i] = rt_neglog_wave(m[i], force != 0, &slow_count[threadIdx.x],
                            log_scratch[threadIdx.x >> 6]);
    if (slow) slow[i] = slow_count[threadIdx.x] ? 1 : 0;
}

__global__ void rt_debug_philox_kernel(const uint32_t* ctr, uint32_t k0, uint32_t k1,
                                       uint32_t* out, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    rt_u4 c = {ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]};
    rt_u4 w = rt_philox4x32_10(c, k0, k1);
    out[4 * i] = w.x;
    out[4 * i + 1] = w.y;
    out[4 * i + 2] = w.z;
    out[4 * i + 3] = w.w;
}

// ---- the selection step (Eq. 25) and near-tie rule of each mapping, on
// rows of given values (test hook); the same device functions as the kernels
__device__ __forceinline__ void debug_sel_store(int64_t r, const rt_min2& v, int32_t* mu,
                                                double* v1, double* v2, uint8_t* near)
{
    mu[r] = v.k;
    v1[r] = v.d1;
    v2[r] = v.d2;
    near[r] = rt_near_tie(v.d1, v.d2) ? 1 : 0;
}

// thread mapping: one lane per row, channels in order from {+inf, +inf, 0}
__global__ __launch_bounds__(256) void rt_debug_sel_thread_kernel(
    const double* v, int32_t M, int64_t count, int32_t* mu, double* v1, double* v2, uint8_t* near)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= count) return;
    rt_min2 sel{__builtin_inf(), __builtin_inf(), 0};
    for (int k = 0; k < M; ++k) rt_min2_push(sel, v[r * M + k], k);
    debug_sel_store(r, sel, mu, v1, v2, near);
}

// sub-wavefront mapping: W lanes per row, lane l holds channels l + s W
template <int W>
__global__ __launch_bounds__(256) void rt_debug_sel_wave_kernel(
    const double* v, int32_t M, int64_t count, int32_t* mu, double* v1, double* v2, uint8_t* near)
{
    constexpr int LOG2W = __builtin_ctz(W);
    const int li = (int)(threadIdx.x & (W - 1));
    const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> LOG2W;
    rt_min2 loc = rt_min2_empty();
    if (r < count)
        for (int s = 0; li + s * W < M; ++s) rt_min2_push(loc, v[r * M + li + s * W], s);
    loc = rt_min2_slot_to_channel(loc, li, LOG2W);
    loc = rt_min2_allreduce<W>(loc);                 // every lane of the group is active
    if (r < count && li == 0) debug_sel_store(r, loc, mu, v1, v2, near);
}

// workgroup mapping: one row per workgroup of L threads
template <int L>
__global__ __launch_bounds__(L) void rt_debug_sel_group_kernel(
    const double* v, int32_t M, int64_t count, int32_t* mu, double* v1, double* v2, uint8_t* near)
{
    __shared__ rt_min2 wave_min[16];
    const int tid = threadIdx.x;
    const int64_t r = blockIdx.x;
    rt_min2 loc = rt_min2_empty();
    for (int s = 0; tid + s * L < M; ++s) rt_min2_push(loc, v[r * M + tid + s * L], s);
    loc = rt_min2_slot_to_channel(loc, tid, __builtin_ctz(L));
    loc = rt_min2_group_allreduce<L>(loc, wave_min);
    if (tid == 0) debug_sel_store(r, loc, mu, v1, v2, near);
}

// workgroup mapping with the propensities in LDS: the lane's two smallest
// values, then the selection in two single-value reductions
template <int L>
__global__ __launch_bounds__(L) void rt_debug_sel_group_lds_kernel(
    const double* v, int32_t M, int64_t count, int32_t* mu, double* v1, double* v2, uint8_t* near)
{
    __shared__ rt_sel_part part[16];
    const int tid = threadIdx.x;
    const int64_t r = blockIdx.x;
    double d1 = __builtin_inf(), d2 = __builtin_inf();
    int ks = 0;
    for (int s = 0; tid + s * L < M; ++s) {
        const double d = v[r * M + tid + s * L];
        const bool lt = d < d1;
        d2 = fmin(d2, fmax(d1, d));
        d1 = fmin(d1, d);
        ks = lt ? s : ks;
    }
    const rt_min2 sel = rt_select_group<L>(d1, d2, tid + ks * L, part);
    if (tid == 0) debug_sel_store(r, sel, mu, v1, v2, near);
}

typedef void (*debug_sel_t)(const double*, int32_t, int64_t, int32_t*, double*, double*, uint8_t*);

}  // namespace

int rt_launch_debug_select(const double* v, int32_t M, int64_t count, int32_t mapping,
                           int32_t lanes, int32_t* mu, double* v1, double* v2, uint8_t* near,
                           hipStream_t stream)
{
    if (count <= 0) return RTSSA_OK;
    debug_sel_t k = nullptr;
    int64_t blocks = 0;
    int block = 256;
    if (mapping == RTSSA_MAP_THREAD) {
        k = rt_debug_sel_thread_kernel;
        blocks = (count + 255) / 256;
    } else if (mapping == RTSSA_MAP_WAVE) {
        switch (lanes) {
            case 2: k = rt_debug_sel_wave_kernel<2>; break;
            case 4: k = rt_debug_sel_wave_kernel<4>; break;
            case 8: k = rt_debug_sel_wave_kernel<8>; break;
            case 16: k = rt_debug_sel_wave_kernel<16>; break;
            case 32: k = rt_debug_sel_wave_kernel<32>; break;
            case 64: k = rt_debug_sel_wave_kernel<64>; break;
            default: return rt_fail(RTSSA_E_INVALID, "wavefront lanes must be 2..64, a power of 2");
        }
        blocks = (count * lanes + 255) / 256;
    } else if (mapping == RTSSA_MAP_WORKGROUP) {
        switch (lanes) {
            case 64: k = rt_debug_sel_group_kernel<64>; break;
            case 128: k = rt_debug_sel_group_kernel<128>; break;
            case 256: k = rt_debug_sel_group_kernel<256>; break;
            case 512: k = rt_debug_sel_group_kernel<512>; break;
            case 1024: k = rt_debug_sel_group_kernel<1024>; break;
            default: return rt_fail(RTSSA_E_INVALID, "workgroup size must be 64..1024, a power of 2");
        }
        block = lanes;
        blocks = count;
    } else if (mapping == RTSSA_DEBUG_MAP_WORKGROUP_LDS) {
        switch (lanes) {
            case 64: k = rt_debug_sel_group_lds_kernel<64>; break;
            case 128: k = rt_debug_sel_group_lds_kernel<128>; break;
            case 256: k = rt_debug_sel_group_lds_kernel<256>; break;
            case 512: k = rt_debug_sel_group_lds_kernel<512>; break;
            case 1024: k = rt_debug_sel_group_lds_kernel<1024>; break;
            default: return rt_fail(RTSSA_E_INVALID, "workgroup size must be 64..1024, a power of 2");
        }
        block = lanes;
        blocks = count;
    } else {
        return rt_fail(RTSSA_E_INVALID, "unknown mapping");
    }
    if (blocks > 0x7FFFFFFF) return rt_fail(RTSSA_E_INVALID, "too many rows");
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(block), 0, stream, v, M, count, mu, v1, v2,
                       near);
    return hipGetLastError() == hipSuccess ? RTSSA_OK : rt_fail(RTSSA_E_HIP, "launch failed");
}

// blocks of the score reduction: one per 4096 trajectories, 1..256
static int score_blocks(int64_t R)
{
    int64_t nb = (R + 4095) / 4096;
    return (int)(nb > 256 ? 256 : (nb < 1 ? 1 : nb));
}

size_t rt_score_grad_workspace_bytes(int64_t R, int32_t M)
{
    const size_t nb = (size_t)score_blocks(R);
    return sizeof(double) * (nb + nb * (size_t)M * 2);
}

int rt_launch_score_grad(const double* f, const uint32_t* n, const double* T, int64_t R,
                         int32_t M, int32_t baseline, double* grad, double* se,
                         void* workspace, hipStream_t stream)
{
    const int nb = score_blocks(R);
    const int64_t chunk = (R + nb - 1) / nb;
    double* buf = (double*)workspace;
    const size_t bytes = rt_score_grad_workspace_bytes(R, M);
    if (!buf && hipMallocAsync((void**)&buf, bytes, stream) != hipSuccess)
        return rt_fail(RTSSA_E_NOMEM, "score workspace allocation failed");
    double* fpart = buf;
    double* part = buf + nb;
    hipLaunchKernelGGL(rt_sum_f_kernel, dim3(nb), dim3(kRedBlock), 0, stream, f, R, chunk, fpart);
    hipLaunchKernelGGL(rt_score_part_kernel, dim3(nb), dim3(kRedBlock), 0, stream, f, n, T, R, M,
                       baseline, chunk, fpart, nb, part);
    hipLaunchKernelGGL(rt_score_final_kernel, dim3((M + 255) / 256), dim3(256), 0, stream, part,
                       nb, M, R, grad, se);
    hipError_t e = hipGetLastError();
    if (!workspace) hipFreeAsync(buf, stream);
    return e == hipSuccess ? RTSSA_OK : rt_fail(RTSSA_E_HIP, "score kernel launch failed");
}

int rt_launch_debug_neglog(const uint64_t* m, double* out, uint8_t* slow, int64_t count,
                           int force, hipStream_t stream)
{
    if (count <= 0) return RTSSA_OK;
    hipLaunchKernelGGL(rt_debug_neglog_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0,
                       stream, m, out, slow, count, force);
    return hipGetLastError() == hipSuccess ? RTSSA_OK : rt_fail(RTSSA_E_HIP, "launch failed");
}

int rt_launch_debug_philox(const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out,
                           int64_t count, hipStream_t stream)
{
    if (count <= 0) return RTSSA_OK;
    hipLaunchKernelGGL(rt_debug_philox_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0,
                       stream, ctr, k0, k1, out, count);
    return hipGetLastError() == hipSuccess ? RTSSA_OK : rt_fail(RTSSA_E_HIP, "launch failed");
}
