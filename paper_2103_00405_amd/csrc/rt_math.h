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
//                     unit-exponential internal-time gaps (paper Eq. 23, 26).
//   rt_neglog_u53     correctly rounded -ln(u), u = (m+1) 2^-53, so that a
//                     draw ln(1/r) has one exact binary64 value.
//   rt_exp1           the draw of the n-th refresh of channel k.
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

RT_HD rt_u4 rt_philox4x32_10(rt_u4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        rt_u4 o;
        o.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
        o.y = (uint32_t)p1;
        o.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
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
struct rt_fix { uint32_t w[RT_LOG_LIMBS]; };

RT_HD void rt_fix_load(rt_fix& a, const uint32_t* src)
{
    for (int i = 0; i < RT_LOG_LIMBS; ++i) a.w[i] = src[i];
}

RT_HD void rt_fix_add(rt_fix& a, const rt_fix& b)
{
    uint64_t carry = 0;
    for (int i = 0; i < RT_LOG_LIMBS; ++i) {
        uint64_t s = (uint64_t)a.w[i] + b.w[i] + carry;
        a.w[i] = (uint32_t)s;
        carry = s >> 32;
    }
}

RT_HD void rt_fix_neg(rt_fix& a)
{
    uint64_t carry = 1;
    for (int i = 0; i < RT_LOG_LIMBS; ++i) {
        uint64_t s = (uint64_t)(~a.w[i]) + carry;
        a.w[i] = (uint32_t)s;
        carry = s >> 32;
    }
}

RT_HD void rt_fix_sub(rt_fix& a, const rt_fix& b)
{
    rt_fix nb = b;
    rt_fix_neg(nb);
    rt_fix_add(a, nb);
}

RT_HD bool rt_fix_isneg(const rt_fix& a) { return (a.w[RT_LOG_LIMBS - 1] >> 31) != 0; }

// a <- a * s for a small non-negative integer s (no overflow in use).
RT_HD void rt_fix_mul_small(rt_fix& a, uint32_t s)
{
    uint64_t carry = 0;
    for (int i = 0; i < RT_LOG_LIMBS; ++i) {
        uint64_t p = (uint64_t)a.w[i] * s + carry;
        a.w[i] = (uint32_t)p;
        carry = p >> 32;
    }
}

// a <- a * Z / 2^61 truncated toward zero, for a signed integer |Z| < 2^63: the product of a
// fixed-point value by z = Z 2^-61.  Truncation error below one unit 2^-256.
RT_HD void rt_fix_mul_z(rt_fix& a, int64_t Z)
{
    bool neg = rt_fix_isneg(a) != (Z < 0);
    rt_fix m = a;
    if (rt_fix_isneg(m)) rt_fix_neg(m);
    uint64_t az = Z < 0 ? (uint64_t)(-Z) : (uint64_t)Z;
    uint32_t zl = (uint32_t)az, zh = (uint32_t)(az >> 32);
    // product of RT_LOG_LIMBS limbs by 2 limbs -> RT_LOG_LIMBS + 2 limbs
    uint32_t p[RT_LOG_LIMBS + 2];
    for (int i = 0; i < RT_LOG_LIMBS + 2; ++i) p[i] = 0;
    for (int j = 0; j < 2; ++j) {
        uint32_t zj = j == 0 ? zl : zh;
        uint64_t carry = 0;
        for (int i = 0; i < RT_LOG_LIMBS; ++i) {
            uint64_t t = (uint64_t)m.w[i] * zj + p[i + j] + carry;
            p[i + j] = (uint32_t)t;
            carry = t >> 32;
        }
        p[RT_LOG_LIMBS + j] += (uint32_t)carry;
    }
    // shift right by 61 = 32 + 29 bits
    for (int i = 0; i < RT_LOG_LIMBS; ++i) {
        uint32_t lo = p[i + 1], hi = (i + 2 < RT_LOG_LIMBS + 2) ? p[i + 2] : 0u;
        m.w[i] = (lo >> 29) | (hi << 3);
    }
    if (neg) rt_fix_neg(m);
    a = m;
}

// Round a non-negative fixed-point value to the nearest binary64 (ties even).
RT_HD double rt_fix_to_double(const rt_fix& a)
{
    int top = -1;
    for (int i = RT_LOG_LIMBS - 1; i >= 0 && top < 0; --i)
        if (a.w[i]) top = 32 * i + (31 - __builtin_clz(a.w[i]));
    if (top < 0) return 0.0;
    // bit b of the integer is a.w[b / 32] >> (b % 32)
    uint64_t mant = 0;
    for (int b = top; b > top - 53; --b) {
        uint32_t bit = b >= 0 ? (a.w[b >> 5] >> (b & 31)) & 1u : 0u;
        mant = (mant << 1) | bit;
    }
    int rb = top - 53;                       // rounding bit position
    uint32_t round_bit = rb >= 0 ? (a.w[rb >> 5] >> (rb & 31)) & 1u : 0u;
    bool sticky = false;
    for (int b = rb - 1; b >= 0 && !sticky; --b)
        sticky = ((a.w[b >> 5] >> (b & 31)) & 1u) != 0;
    if (round_bit && (sticky || (mant & 1u))) mant += 1;
    int expo = top - 52 - RT_LOG_FRAC;       // value = mant * 2^expo
    if (mant == (1ull << 53)) { mant >>= 1; expo += 1; }
    // mant < 2^53 is exact in binary64; scaling by a power of two is exact
    double d = (double)mant;
    uint64_t scale_bits = (uint64_t)(1023 + expo) << 52;   // expo within normal range here
    return d * rt_u2d(scale_bits);
}

// -ln(u) = -e ln2 + ln r - ln(1 + z), each term to about 2^-250 absolute.
RT_HD double rt_neglog_accurate(int e, int i, double z)
{
    // z = Z 2^-61 exactly (|z| <= 2^-8 is a multiple of 2^-61)
    int64_t Z = (int64_t)(z * 0x1p61);
    // Horner: p = sum_{j=0..KMAX} (-z)^j / (j + 1);  ln(1 + z) = z p
    rt_fix p;
    rt_fix_load(p, RT_INVK_FIX[RT_LOG_KMAX]);
    for (int j = RT_LOG_KMAX - 1; j >= 0; --j) {
        rt_fix_mul_z(p, Z);
        rt_fix c;
        rt_fix_load(c, RT_INVK_FIX[j]);
        rt_fix_sub(c, p);
        p = c;
    }
    rt_fix_mul_z(p, Z);                       // p = ln(1 + z)
    rt_fix y;
    rt_fix_load(y, RT_LN2_FIX);
    rt_fix_mul_small(y, (uint32_t)(-e));      // -e ln 2, e <= 0
    rt_fix lnr;
    rt_fix_load(lnr, RT_LNR_FIX[i]);
    rt_fix_add(y, lnr);
    rt_fix_sub(y, p);
    return rt_fix_to_double(y);
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

// RN(-ln u) for u = (m + 1) 2^-53, m < 2^53.  When the fast phase cannot
// certify its rounding (about one call in 2^17) the accurate phase decides.
// *slow is set when the accurate phase ran.
RT_HD double rt_neglog_u53(uint64_t m, bool force_accurate, bool* slow)
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
    return rt_neglog_accurate(e, i, z);
}

// E(seed, traj, net, k, n): block at counter (n >> 1, k, traj, net) under key
// (seed_lo, seed_hi); the 64-bit word is (w1:w0) for even n and (w3:w2) for
// odd n; u = ((word >> 11) + 1) 2^-53.
RT_HD double rt_exp1(uint32_t k0, uint32_t k1, uint32_t traj, uint32_t net, uint32_t k,
                     uint32_t n, bool* slow)
{
    rt_u4 c = {n >> 1, k, traj, net};
    rt_u4 w = rt_philox4x32_10(c, k0, k1);
    uint64_t word = (n & 1u) ? (((uint64_t)w.w << 32) | w.z) : (((uint64_t)w.y << 32) | w.x);
    return rt_neglog_u53(word >> 11, false, slow);
}
