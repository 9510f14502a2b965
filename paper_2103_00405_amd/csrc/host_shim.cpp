// host_shim.cpp -- the kernels' numeric core (rt_math.h) compiled for the CPU,
// exported as test hooks so its bits can be checked without a GPU.
#include <math.h>
#include <stdint.h>

#define RT_HD static inline
#define RT_LOG_CONST static const
#include "rt_math.h"

extern "C" double rtssa_debug_neglog_host(uint64_t m, int32_t force_accurate, int32_t* slow)
{
    bool s = false;
    uint32_t sc[RT_LOG_SCRATCH];
    double v = rt_neglog_u53(m, force_accurate != 0, &s, sc);
    if (slow) *slow = s ? 1 : 0;
    return v;
}

// The fast phase's double-double, for measuring its error margin.
extern "C" void rtssa_debug_neglog_fast_host(uint64_t m, double* yh, double* yl)
{
    int e, i;
    double z;
    rt_neglog_reduce(m, e, i, z);
    rt_neglog_fast(e, i, z, *yh, *yl);
}

extern "C" void rtssa_debug_philox_host(const uint32_t ctr[4], uint32_t key0, uint32_t key1,
                                        uint32_t out[4])
{
    rt_u4 c = {ctr[0], ctr[1], ctr[2], ctr[3]};
    rt_u4 w = rt_philox4x32_10(c, key0, key1);
    out[0] = w.x;
    out[1] = w.y;
    out[2] = w.z;
    out[3] = w.w;
}
