// mc_math.h -- arithmetic shared by the kernels of the library (device code).
//
//  * Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11): ten rounds of two
//    32x32->64 products and xors, key bumped by the golden-ratio and
//    sqrt(3)-1 Weyl constants.
//  * exp(d) for d in [-23, 0] and ln(h) for integers h >= 1 by a fixed sequence
//    of binary64 operations (Cody-Waite reduction + Taylor series; the atanh
//    series of ln((1+s)/(1-s))), so that thresholds and weights come out the
//    same bits on every IEEE-754 machine.  The library is compiled with
//    -ffp-contract=off: every fused multiply-add below is written out.
//  * the Metropolis threshold tau(d) (acceptance rule min(1, w'/w), Sec. 4.2
//    of the paper, as an integer compare against a 32-bit uniform word).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcgpu {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kWeyl0 = 0x9E3779B9u;
constexpr uint32_t kWeyl1 = 0xBB67AE85u;

// Random-word domains (the fourth counter word).
constexpr uint32_t kDomSweep = 0u;
constexpr uint32_t kDomInit = 1u;
constexpr uint32_t kDomJoin = 2u;

__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        // one 32x32->64 product per lane and word (v_mad_u64_u32)
        const uint64_t p0 = (uint64_t)kPhiloxM0 * c.x;
        const uint64_t p1 = (uint64_t)kPhiloxM1 * c.z;
        // three-input xors as one v_bitop3_b32 each (truth table 0x96 = a ^ b ^ c)
        c = make_uint4(__builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c.y, k0, 0x96), (uint32_t)p1,
                       __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c.w, k1, 0x96), (uint32_t)p0);
        k0 += kWeyl0;
        k1 += kWeyl1;
    }
    return c;
}

__device__ __forceinline__ uint32_t word_of(uint4 v, uint32_t i) {
    return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}

// ---------------------------------------------------------------------------
// exp: x = k ln2 + r, |r| <= ln2/2; ln 2 = head + tail with head = RN(ln 2).
// P(r) = sum_{i=0}^{13} r^i / i!, Horner with fma; result P * 2^k.
// ---------------------------------------------------------------------------
constexpr double kLn2Head = 0x1.62e42fefa39efp-1;
constexpr double kLn2Tail = 0x1.abc9e3b39803fp-56;
constexpr double kInvLn2 = 0x1.71547652b82fep+0;

__device__ __forceinline__ double det_exp(double x) {
    if (x < -745.0) return 0.0;
    // 1/i! as correctly rounded quotients (i! exact in binary64 up to 13!).
    constexpr double c0 = 1.0, c1 = 1.0, c2 = 1.0 / 2.0, c3 = 1.0 / 6.0, c4 = 1.0 / 24.0, c5 = 1.0 / 120.0,
                     c6 = 1.0 / 720.0, c7 = 1.0 / 5040.0, c8 = 1.0 / 40320.0, c9 = 1.0 / 362880.0,
                     c10 = 1.0 / 3628800.0, c11 = 1.0 / 39916800.0, c12 = 1.0 / 479001600.0,
                     c13 = 1.0 / 6227020800.0;
    const double k = rint(x * kInvLn2);
    double r = fma(-k, kLn2Head, x);
    r = fma(-k, kLn2Tail, r);
    double p = c13;
    p = fma(p, r, c12);
    p = fma(p, r, c11);
    p = fma(p, r, c10);
    p = fma(p, r, c9);
    p = fma(p, r, c8);
    p = fma(p, r, c7);
    p = fma(p, r, c6);
    p = fma(p, r, c5);
    p = fma(p, r, c4);
    p = fma(p, r, c3);
    p = fma(p, r, c2);
    p = fma(p, r, c1);
    p = fma(p, r, c0);
    return ldexp(p, (int)k);
}

// ---------------------------------------------------------------------------
// ln h, h >= 1: h = f 2^e, f moved into [sqrt(1/2), sqrt(2)); s = (f-1)/(f+1);
// ln f = 2s (1 + z/3 + z^2/5 + ... + z^11/23), z = s^2, evaluated as
// fma(2s*z, q, 2s) with q = 1/3 + z/5 + ... by Horner; then + e ln 2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double det_log(int64_t h) {
    int e;
    double f = frexp((double)h, &e);
    if (f < 0x1.6a09e667f3bcdp-1) {
        f = f * 2.0;
        e = e - 1;
    }
    const double s = (f - 1.0) / (f + 1.0);
    const double z = s * s;
    double q = 1.0 / 23.0;
    q = fma(q, z, 1.0 / 21.0);
    q = fma(q, z, 1.0 / 19.0);
    q = fma(q, z, 1.0 / 17.0);
    q = fma(q, z, 1.0 / 15.0);
    q = fma(q, z, 1.0 / 13.0);
    q = fma(q, z, 1.0 / 11.0);
    q = fma(q, z, 1.0 / 9.0);
    q = fma(q, z, 1.0 / 7.0);
    q = fma(q, z, 1.0 / 5.0);
    q = fma(q, z, 1.0 / 3.0);
    const double s2 = s + s;
    const double lnf = fma(s2 * z, q, s2);
    const double de = (double)e;
    return fma(de, kLn2Head, fma(de, kLn2Tail, lnf));
}

// Metropolis threshold of a change d of ln w: accept iff u <= tau(d).
__device__ __forceinline__ uint32_t tau_of(double d) {
    if (d >= 0.0) return 0xFFFFFFFFu;
    if (d < -23.0) return 0u;  // exp(-23) * 2^32 < 1
    const double v = floor(det_exp(d) * 4294967296.0);
    return v >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)v;
}

}  // namespace mcgpu
