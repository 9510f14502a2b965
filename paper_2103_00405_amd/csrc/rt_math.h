// rt_math.h -- numeric core of the random-time SSA kernels.
//
// Included by the gfx950 kernels (RT_HD = __device__ __forceinline__,
// RT_LOG_CONST = __constant__) and by a host shim used for CPU tests of the
// very same arithmetic (RT_HD = static inline, RT_LOG_CONST = static const).
// Every floating-point step is an IEEE binary64 operation rounded to
// nearest-even; fused multiply-adds appear only as explicit fma() calls and
// the build disables contraction, so both builds produce identical bits.
//
// Contents:
//   rt_philox4x32_10  Philox4x32-10 block function (Salmon, Moraes, Dror &
//                     Shaw, SC'11) -- the counter-based stream of the
//                     unit-exponential internal-time gaps (paper Eq. 23, 26);
//                     rt_xor3 does each round's two xors in one instruction.
//   rt_neglog_u53     correctly rounded -ln(u), u = (m+1) 2^-53, so that a
//                     draw ln(1/r) has one exact binary64 value.
//   rt_draw_m53       the 53-bit integer behind the n-th draw of channel k.
#pragma once
#include <stdint.h>

#ifndef RT_HD
#error "define RT_HD and RT_LOG_CONST before including rt_math.h"
#endif


#include "log_tables.inc"

RT_HD uint64_t rt_d2u(double x) { return __builtin_bit_cast(uint64_t, x); }
RT_HD double rt_u2d(uint64_t x) { return __builtin_bit_cast(double, x); }

// --------------------------------------------------------------- Philox
struct rt_u4 { uint32_t x, y, z, w; };

// a ^ b ^ c; on the GPU one three-input bitwise instruction (v_bitop3_b32
// with truth table 0x96, the parity of its three inputs), which the compiler
// does not form from two xors by itself.
RT_HD uint32_t rt_xor3(uint32_t a, uint32_t b, uint32_t c)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
#else
    return a ^ b ^ c;
#endif
}

// Each round's output words x and z are a product's high half xor a counter
// word xor a key word, with rt_xor3 when XOR3, else two plain xors (the same
// bits).  rt_xor3 runs on the vector unit: a block whose inputs are the same
// in every lane, left to the scalar unit, takes the plain form, and so do the
// kernels where the three-input form measured slower.
template <bool XOR3 = true>
RT_HD rt_u4 rt_philox4x32_10(rt_u4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        rt_u4 o;
        o.x = XOR3 ? rt_xor3((uint32_t)(p1 >> 32), c.y, k0) : (uint32_t)(p1 >> 32) ^ c.y ^ k0;
        o.y = (uint32_t)p1;
        o.z = XOR3 ? rt_xor3((uint32_t)(p0 >> 32), c.w, k1) : (uint32_t)(p0 >> 32) ^ c.w ^ k1;
        o.w = (uint32_t)p0;
        c = o;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// ------------------------------------------------ error-free transforms
// Fast2Sum (Dekker): s + e == a + b exactly when |a| >= |b| or a == 0.
RT_HD void rt_fast2sum(double a, double b, double& s, double& e)
{
    s = a + b;
    double bb = s - a;
    e = b - bb;
}

// TwoSum (Knuth/Moller): s + e == a + b exactly, no ordering needed.
RT_HD void rt_twosum(double a, double b, double& s, double& e)
{
    s = a + b;
    double ap = s - b;
    double bp = s - ap;
    e = (a - ap) + (b - bp);
}

// ------------------------------------- accurate phase: 288-bit fixed point
// Values are two's-complement integers of RT_LOG_LIMBS 32-bit limbs
// (little-endian) in units of 2^-256: 32 integer bits, 256 fraction bits.
// The routines work in a caller-provided buffer of RT_LOG_SCRATCH words (the
// kernels give each wave a slice of LDS and let the lanes that need this
// rare phase take turns), so they add no register pressure to the hot loop.
#define RT_LOG_SCRATCH (2 * RT_LOG_LIMBS + 2)

// p <- c - p
RT_HD void rt_fix_rsub_const(uint32_t* p, const uint32_t* c)
{
    uint64_t borrow = 0;
    #pragma unroll 1
    for (int i = 0; i < RT_LOG_LIMBS; ++i) {
        uint64_t d = (uint64_t)c[i] - p[i] - borrow;
        p[i] = (uint32_t)d;
        borrow = (d >> 32) & 1u;
    }
}

// p <- p + c * s, s a small non-negative integer
RT_HD void rt_fix_add_mul_const(uint32_t* p, const uint32_t* c, uint32_t s)
{
    uint64_t carry = 0;
    #pragma unroll 1
    for (int i = 0; i < RT_LOG_LIMBS; ++i) {
        uint64_t t = (uint64_t)c[i] * s + p[i] + carry;
        p[i] = (uint32_t)t;
        carry = t >> 32;
    }
}

RT_HD void rt_fix_neg(uint32_t* p)
{
    uint64_t carry = 1;
    #pragma unroll 1
    for (int i = 0; i < RT_LOG_LIMBS; ++i) {
        uint64_t t = (uint64_t)(~p[i]) + carry;
        p[i] = (uint32_t)t;
        carry = t >> 32;
    }
}

// p <- p * Z / 2^61 truncated toward zero, |Z| < 2^63: the product of a
// fixed-point value by z = Z 2^-61.  tmp holds RT_LOG_LIMBS + 2 words.
RT_HD void rt_fix_mul_z(uint32_t* p, int64_t Z, uint32_t* tmp)
{
    const bool pneg = (p[RT_LOG_LIMBS - 1] >> 31) != 0;
    const bool neg = pneg != (Z < 0);
    if (pneg) rt_fix_neg(p);
    const uint64_t az = Z < 0 ? (uint64_t)(-Z) : (uint64_t)Z;
    #pragma unroll 1
    for (int i = 0; i < RT_LOG_LIMBS + 2; ++i) tmp[i] = 0;
    #pragma unroll 1
    for (int j = 0; j < 2; ++j) {
        const uint32_t zj = (uint32_t)(az >> (32 * j));
        uint64_t carry = 0;
        #pragma unroll 1
        for (int i = 0; i < RT_LOG_LIMBS; ++i) {
            uint64_t t = (uint64_t)p[i] * zj + tmp[i + j] + carry;
            tmp[i + j] = (uint32_t)t;
            carry = t >> 32;
        }
        tmp[RT_LOG_LIMBS + j] += (uint32_t)carry;
    }
    // shift right by 61 = 32 + 29 bits
    #pragma unroll 1
    for (int i = 0; i < RT_LOG_LIMBS; ++i) p[i] = (tmp[i + 1] >> 29) | (tmp[i + 2] << 3);
    if (neg) rt_fix_neg(p);
}

// Round a non-negative fixed-point value to the nearest binary64 (ties even).
RT_HD double rt_fix_to_double(const uint32_t* a)
{
    int top = -1;
    #pragma unroll 1
    for (int i = RT_LOG_LIMBS - 1; i >= 0 && top < 0; --i)
        if (a[i]) top = 32 * i + (31 - __builtin_clz(a[i]));
    if (top < 0) return 0.0;
    uint64_t mant = 0;
    #pragma unroll 1
    for (int b = top; b > top - 53; --b) {
        uint32_t bit = b >= 0 ? (a[b >> 5] >> (b & 31)) & 1u : 0u;
        mant = (mant << 1) | bit;
    }
    const int rb = top - 53;                        // rounding bit position
    const uint32_t round_bit = rb >= 0 ? (a[rb >> 5] >> (rb & 31)) & 1u : 0u;
    bool sticky = false;
    #pragma unroll 1
    for (int b = rb - 1; b >= 0 && !sticky; --b) sticky = ((a[b >> 5] >> (b & 31)) & 1u) != 0;
    if (round_bit && (sticky || (mant & 1u))) mant += 1;
    int expo = top - 52 - RT_LOG_FRAC;              // value = mant * 2^expo
    if (mant == (1ull << 53)) { mant >>= 1; expo += 1; }
    const double d = (double)mant;                  // exact: mant <= 2^53
    return d * rt_u2d((uint64_t)(1023 + expo) << 52);
}

// -ln(u) = -e ln2 + ln r - ln(1 + z), each term to about 2^-250 absolute, in
// the buffer sc of RT_LOG_SCRATCH words.
RT_HD double rt_neglog_accurate(int e, int i, double z, uint32_t* sc)
{
    uint32_t* p = sc;
    uint32_t* tmp = sc + RT_LOG_LIMBS;
    // z = Z 2^-61 exactly (|z| <= 2^-8 is a multiple of 2^-61)
    const int64_t Z = (int64_t)(z * 0x1p61);
    // Horner: p = sum_{j=0..KMAX} (-z)^j / (j + 1);  ln(1 + z) = z p
    #pragma unroll 1
    for (int q = 0; q < RT_LOG_LIMBS; ++q) p[q] = RT_INVK_FIX[RT_LOG_KMAX][q];
    #pragma unroll 1
    for (int j = RT_LOG_KMAX - 1; j >= 0; --j) {
        rt_fix_mul_z(p, Z, tmp);
        rt_fix_rsub_const(p, RT_INVK_FIX[j]);
    }
    rt_fix_mul_z(p, Z, tmp);                        // p = ln(1 + z)
    rt_fix_neg(p);
    rt_fix_add_mul_const(p, RT_LNR_FIX[i], 1u);     // + ln r
    rt_fix_add_mul_const(p, RT_LN2_FIX, (uint32_t)(-e));  // + (-e) ln 2, e <= 0
    return rt_fix_to_double(p);
}

// ------------------------------------------------- correctly rounded -ln u
// Argument reduction: u = (m + 1) 2^-53 = 2^e f with f in [0.707, 1.414);
// the top 9 mantissa bits give the table index i; z = f r_i - 1 is exact and
// |z| <= 2^-8, so -ln u = -e ln 2 + ln r_i - ln(1 + z).
RT_HD void rt_neglog_reduce(uint64_t m, int& e, int& i, double& z)
{
    const double u = (double)(m + 1) * 0x1p-53;                // exact
    const uint64_t ub = rt_d2u(u);
    e = (int)(ub >> 52) - 1023;
    const uint64_t mf = ub & 0xFFFFFFFFFFFFFull;
    i = (int)(mf >> (52 - RT_LOG_NBITS));
    double f = rt_u2d(mf | 0x3FF0000000000000ull);             // [1, 2)
    if (i >= RT_LOG_I_HALF) { f = f * 0.5; e += 1; }           // [0.707, 1.414)
    z = fma(f, RT_RTAB[i], -1.0);                              // exact, |z| <= 2^-8
}

// Fast phase: -ln u as a double-double yh + yl (|yl| <= ulp(yh)/2) with
// relative error far below 2^-70.
RT_HD void rt_neglog_fast(int e, int i, double z, double& yh, double& yl)
{
    // ln(1 + z) = z - z^2/2 + z^3/3 + z^4 q(z), q to degree 6 (terms to z^10)
    const double z2h = z * z;
    const double z2l = fma(z, z, -z2h);
    const double z3h = z2h * z;
    const double z3l = fma(z2h, z, -z3h) + z2l * z;
    const double t3h = z3h * RT_THIRD_H;
    const double t3l = fma(z3h, RT_THIRD_H, -t3h) + (z3l * RT_THIRD_H + z3h * RT_THIRD_L);
    double q = -0.1;
    q = fma(q, z, 1.0 / 9.0);
    q = fma(q, z, -0.125);
    q = fma(q, z, 1.0 / 7.0);
    q = fma(q, z, -1.0 / 6.0);
    q = fma(q, z, 0.2);
    q = fma(q, z, -0.25);
    const double z4 = z2h * z2h;
    const double tail = z4 * q;
    double s1h, s1l, s2h, s2l;
    rt_fast2sum(z, -0.5 * z2h, s1h, s1l);
    rt_fast2sum(s1h, t3h, s2h, s2l);
    const double low = (((s1l + s2l) + (-0.5 * z2l)) + t3l) + tail;
    // y = -e ln2 + ln r - (s2h + low)
    const double ee = (double)(-e);
    const double A = ee * RT_LN2_H;                            // exact
    double h1, e1, h2, e2;
    rt_twosum(RT_LNR_H[i], -s2h, h1, e1);
    rt_fast2sum(A, h1, h2, e2);
    const double lo = (((RT_LNR_L[i] - low) + e1) + e2) + ee * RT_LN2_L;
    rt_fast2sum(h2, lo, yh, yl);
}

// True when every real within yh + yl +- 2^-70 yh rounds to yh: the interval
// must stay strictly inside the half spacings below and above yh (yh > 0).
RT_HD bool rt_rounding_certain(double yh, double yl)
{
    const uint64_t yb = rt_d2u(yh);
    const double half_up = rt_u2d(((yb >> 52) - 53) << 52);
    const double half_dn = (yb & 0xFFFFFFFFFFFFFull) ? half_up : 0.5 * half_up;
    const double err = yh * 0x1p-70;
    return yl + err < half_up && yl - err > -half_dn;
}

// RN(-ln u) for u = (m + 1) 2^-53, m < 2^53, in one lane: when the fast
// phase cannot certify its rounding the accurate phase decides in sc.
// *slow is set when the accurate phase ran.
RT_HD double rt_neglog_u53(uint64_t m, bool force_accurate, bool* slow, uint32_t* sc)
{
    if (m == 0x1FFFFFFFFFFFFFull) return 0.0;                 // u = 1
    int e, i;
    double z;
    rt_neglog_reduce(m, e, i, z);
    if (!force_accurate) {
        double yh, yl;
        rt_neglog_fast(e, i, z, yh, yl);
        if (rt_rounding_certain(yh, yl)) return yh;
    }
    if (slow) *slow = true;
    return rt_neglog_accurate(e, i, z, sc);
}

// The 53-bit integer m of the draw E(seed, traj, net, k, n): the Philox block
// at counter (n >> 1, k, traj, net) under key (seed_lo, seed_hi); the 64-bit
// word is (w1:w0) for even n and (w3:w2) for odd n; m = word >> 11, and the
// draw is E = RN(-ln((m + 1) 2^-53)).
template <bool XOR3 = true>
RT_HD uint64_t rt_draw_m53(uint32_t k0, uint32_t k1, uint32_t traj, uint32_t net, uint32_t k,
                           uint32_t n)
{
    rt_u4 c = {n >> 1, k, traj, net};
    rt_u4 w = rt_philox4x32_10<XOR3>(c, k0, k1);
    uint64_t word = (n & 1u) ? (((uint64_t)w.w << 32) | w.z) : (((uint64_t)w.y << 32) | w.x);
    return word >> 11;
}
