// Device-side random numbers and elementary functions for the WBRW kernels.
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the
// multiply-xor bijection with multipliers 0xD2511F53 / 0xCD9E8D57 and Weyl key
// increments 0x9E3779B9 / 0xBB67AE85.  Counter = (id_lo, id_hi, step,
// tag<<28 | event<<8 | sub), key = (seed, instance): every particle lineage
// draws from its own stream, independent of where it sits in memory.
//
// log, sin and cos are evaluated by fixed sequences of IEEE double operations
// (no fused multiply-add: this file must be compiled with -ffp-contract=off):
//   log y = e ln2 + 2 atanh f,  y = m 2^e, m in [sqrt(1/2), sqrt(2)),
//           f = (m-1)/(m+1), atanh series through f^23;
//   sin/cos: a = n pi/2 + r with pi/2 split in three (33 + 33 + 53 bits),
//           Taylor series through r^19 (sin) and r^20 (cos).
// The same sequences give the same bits on any IEEE-754 machine, which is
// what lets the GPU ensemble be compared bit for bit with a CPU reference.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wbrw {

enum : uint32_t {
    kTagStep = 0u, kTagRegen = 1u, kTagInit = 2u, kTagBoot = 3u,
    kTagRound = 4u, kTagChild = 5u, kTagGhost = 6u, kTagHist = 7u, kTagReject = 8u, kTagDeriv = 9u
};

struct W4 { uint32_t a, b, c, d; };

__device__ __forceinline__ W4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)c0 * 0xD2511F53ull;
        const uint64_t p1 = (uint64_t)c2 * 0xCD9E8D57ull;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return W4{c0, c1, c2, c3};
}

__device__ __forceinline__ uint32_t ctr_word(uint32_t tag, uint32_t event, uint32_t sub)
{
    return (tag << 28) | ((event & 0xFFFFFu) << 8) | (sub & 0xFFu);
}

__device__ __forceinline__ W4 draw(uint64_t id, uint32_t step, uint32_t tag, uint32_t event,
                                   uint32_t sub, uint32_t seed, uint32_t inst)
{
    return philox4x32_10((uint32_t)id, (uint32_t)(id >> 32), step, ctr_word(tag, event, sub),
                         seed, inst);
}

// (hi:lo) >> 11 scaled by 2^-53: a uniform on [0,1) with 53 random bits.
__device__ __forceinline__ double unit53(uint32_t lo, uint32_t hi)
{
    const uint64_t v = ((((uint64_t)hi) << 32) | (uint64_t)lo) >> 11;
    return (double)v * 0x1p-53;
}

__device__ __forceinline__ double ln_series(double y)
{
    int ex;
    double m = frexp(y, &ex);
    if (m < 0x1.6a09e667f3bcdp-1) {   // below sqrt(1/2): move to [sqrt(1/2), 1)
        m = m + m;
        ex = ex - 1;
    }
    const double f = (m - 1.0) / (m + 1.0);
    const double f2 = f * f;
    // sum_{j=0}^{11} f2^j / (2j+1), innermost term first
    double acc = 1.0 / 23.0;
    acc = acc * f2 + 1.0 / 21.0;
    acc = acc * f2 + 1.0 / 19.0;
    acc = acc * f2 + 1.0 / 17.0;
    acc = acc * f2 + 1.0 / 15.0;
    acc = acc * f2 + 1.0 / 13.0;
    acc = acc * f2 + 1.0 / 11.0;
    acc = acc * f2 + 1.0 / 9.0;
    acc = acc * f2 + 1.0 / 7.0;
    acc = acc * f2 + 1.0 / 5.0;
    acc = acc * f2 + 1.0 / 3.0;
    acc = acc * f2 + 1.0;
    const double lnm = (2.0 * f) * acc;
    const double fe = (double)ex;
    // ln2 = 0x1.62e42fee00000p-1 (exact times any exponent) + 0x1.a39ef35793c76p-33
    return fe * 0x1.62e42fee00000p-1 + (fe * 0x1.a39ef35793c76p-33 + lnm);
}

// r = a - n pi/2 and the quadrant n mod 4
__device__ __forceinline__ double quarter_turns(double a, int& quad)
{
    const double n = rint(a * 0x1.45f306dc9c883p-1);   // a * (2/pi)
    double r = a - n * 0x1.921fb54400000p+0;
    r = r - n * 0x1.0b4611a600000p-34;
    r = r - n * 0x1.3198a2e037073p-69;
    quad = (int)((long long)n & 3);
    return r;
}

__device__ __forceinline__ double taylor_sin(double r)
{
    const double r2 = r * r;
    double acc = -1.0 / 121645100408832000.0;      // -1/19!
    acc = acc * r2 + 1.0 / 355687428096000.0;      //  1/17!
    acc = acc * r2 - 1.0 / 1307674368000.0;        // -1/15!
    acc = acc * r2 + 1.0 / 6227020800.0;           //  1/13!
    acc = acc * r2 - 1.0 / 39916800.0;             // -1/11!
    acc = acc * r2 + 1.0 / 362880.0;               //  1/9!
    acc = acc * r2 - 1.0 / 5040.0;                 // -1/7!
    acc = acc * r2 + 1.0 / 120.0;                  //  1/5!
    acc = acc * r2 - 1.0 / 6.0;                    // -1/3!
    return r + (r * r2) * acc;
}

__device__ __forceinline__ double taylor_cos(double r)
{
    const double r2 = r * r;
    double acc = 1.0 / 2432902008176640000.0;      //  1/20!
    acc = acc * r2 - 1.0 / 6402373705728000.0;     // -1/18!
    acc = acc * r2 + 1.0 / 20922789888000.0;       //  1/16!
    acc = acc * r2 - 1.0 / 87178291200.0;          // -1/14!
    acc = acc * r2 + 1.0 / 479001600.0;            //  1/12!
    acc = acc * r2 - 1.0 / 3628800.0;              // -1/10!
    acc = acc * r2 + 1.0 / 40320.0;                //  1/8!
    acc = acc * r2 - 1.0 / 720.0;                  // -1/6!
    acc = acc * r2 + 1.0 / 24.0;                   //  1/4!
    acc = acc * r2 - 1.0 / 2.0;                    // -1/2!
    return 1.0 + r2 * acc;
}

__device__ __forceinline__ double sin_det(double a)
{
    int q;
    const double r = quarter_turns(a, q);
    if (q == 0) return taylor_sin(r);
    if (q == 1) return taylor_cos(r);
    if (q == 2) return -taylor_sin(r);
    return -taylor_cos(r);
}

__device__ __forceinline__ double cos_det(double a)
{
    int q;
    const double r = quarter_turns(a, q);
    if (q == 0) return taylor_cos(r);
    if (q == 1) return -taylor_sin(r);
    if (q == 2) return -taylor_cos(r);
    return taylor_sin(r);
}

constexpr double kTwoPi = 0x1.921fb54442d18p+2;

}  // namespace wbrw
