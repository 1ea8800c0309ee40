// aca_device.h -- device-side arithmetic of the method (gfx950).
//
// The two per-arrival computations of Section 3, Eq. (5): a counter-based
// draw r(c, n) for cell c's n-th arrival, and the exponential gap
// -ln(r) / lambda to its next arrival.  Written for this library; the
// serial oracle implements the same contract separately.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace aca {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  The key is uniform
// across the wavefront, so its Weyl schedule stays in scalar registers; each
// round costs two 32x32->64 multiplies and two three-input XORs (gfx950's
// v_bitop3_b32 with truth table 0x96) per lane.
struct Draw {
    uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ Draw philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                              uint32_t c3, uint32_t key_lo,
                                              uint32_t key_hi)
{
    constexpr uint32_t kMulA = 0xD2511F53u;   // multiplies word 0
    constexpr uint32_t kMulB = 0xCD9E8D57u;   // multiplies word 2
    constexpr uint32_t kWeylA = 0x9E3779B9u;
    constexpr uint32_t kWeylB = 0xBB67AE85u;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint32_t ka = key_lo + kWeylA * (uint32_t)round;
        const uint32_t kb = key_hi + kWeylB * (uint32_t)round;
        uint64_t prodA = (uint64_t)kMulA * c0;
        uint64_t prodB = (uint64_t)kMulB * c2;
        if (round == 9) {
            // keep the last round's products whole: one v_mad_u64_u32 each
            // instead of separate quarter-rate high and low multiplies
            __asm__("" : "+v"(prodA));
            __asm__("" : "+v"(prodB));
        }
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(prodB >> 32), c1, ka, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(prodA >> 32), c3, kb, 0x96);
        c1 = (uint32_t)prodB;
        c3 = (uint32_t)prodA;
        c0 = n0;
        c2 = n2;
    }
    return Draw{c0, c1, c2, c3};
}

// -ln u for u = (2 (w >> 12) + 1) 2^-53, in binary64 with every operation
// rounded separately (no contraction), in this order:
//   u = f 2^e, f in [1,2); f > sqrt2 -> f/2, e+1
//   s = (f-1)/(f+1), z = s^2
//   p = 1/21; p = p z + 1/19; ...; p = p z + 1/3
//   lf = 2 (s + s (z p));  ln u = e ln2_head + (e ln2_tail + lf)
// ln f = 2 atanh(s); the series tail beyond z^10/21 is below 1e-18 relative.
__device__ __forceinline__ double neg_log_u53(uint64_t w)
{
    constexpr double kRoot2 = 0x1.6a09e667f3bcdp+0;          // nearest sqrt(2)
    constexpr double kLn2Head = 0x1.62e42fefa4000p-1;        // 39 bits of ln 2
    constexpr double kLn2Tail = -0x1.8432a1b0e2634p-43;      // ln 2 - head
    const uint64_t odd = ((w >> 12) << 1) | 1ull;             // < 2^53: exact
    const double u = (double)odd * 0x1p-53;
    const uint64_t bits = (uint64_t)__double_as_longlong(u);
    int e = (int)(bits >> 52) - 1023;                         // u is normal
    double f = __longlong_as_double(
        (long long)((bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull));
    if (f > kRoot2) {
        f = f * 0.5;
        e = e + 1;
    }
    const double num = f - 1.0;
    const double den = f + 1.0;
    // s = num / den, the IEEE quotient, by the hardware's division sequence
    // (reciprocal, two Newton steps, one fused correction) without its
    // operand scaling and special-value fix-up: here den is in [1.70, 2.42]
    // and num is 0 or at least 2^-53 in magnitude, so neither step changes
    // anything and the result is bit for bit the compiler's num / den.
    double r = __builtin_amdgcn_rcp(den);
    r = __builtin_fma(__builtin_fma(-den, r, 1.0), r, r);
    r = __builtin_fma(__builtin_fma(-den, r, 1.0), r, r);
    const double q0 = num * r;
    const double s = __builtin_fma(__builtin_fma(-den, q0, num), r, q0);
    const double z = s * s;
    double p = 1.0 / 21.0;
    p = p * z; p = p + 1.0 / 19.0;
    p = p * z; p = p + 1.0 / 17.0;
    p = p * z; p = p + 1.0 / 15.0;
    p = p * z; p = p + 1.0 / 13.0;
    p = p * z; p = p + 1.0 / 11.0;
    p = p * z; p = p + 1.0 / 9.0;
    p = p * z; p = p + 1.0 / 7.0;
    p = p * z; p = p + 1.0 / 5.0;
    p = p * z; p = p + 1.0 / 3.0;
    double t = z * p;
    t = s * t;
    double lf = s + t;
    lf = lf + lf;
    const double ed = (double)e;
    const double head = ed * kLn2Head;
    const double tail = ed * kLn2Tail;
    return -(head + (tail + lf));
}

// Exponential gap from the first two draw words (w = w1:w0), rate lambda.
__device__ __forceinline__ double arrival_gap(uint32_t w0, uint32_t w1, double rate,
                                              bool unit_rate)
{
    const double e = neg_log_u53(((uint64_t)w1 << 32) | (uint64_t)w0);
    return unit_rate ? e : e / rate;
}

}  // namespace aca
