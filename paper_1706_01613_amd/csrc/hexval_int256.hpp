// Fixed-width exact integer arithmetic for the device-side exact tier.
//
// Every double is m 2^e with an integer m < 2^53, so the coordinates of one
// element are integers times 2^E, E the smallest such exponent.  With the
// integers below 2^B, the quantities the exact tier needs are bounded by
//   edge component < 2^(B+1), pair sum of two edges < 2^(B+2);
//   V = 4 J at a corner or edge midpoint (the triple products of Section 5;
//     6 products of three factors) < 2^(3B+8);
//   32 b (Table 3: corners 8 V, edges 16 V_e - 4 (V_p + V_q), faces
//     8 sum V_e - 6 sum V_c, centre 4 sum V_e - 5 sum V_c) < 88 V < 2^(3B+15);
//   a quadrangle corner value < 2^(2B+3).
// With B <= kMaxCoordBits = 78 all are below 2^249: two's complement
// addition, subtraction and the low 256 bits of a product are exact.
#pragma once

#include <stdint.h>

#include "hexval_math.hpp"

namespace hexval {

constexpr int kMaxCoordBits = 78;

struct I256 {
    uint64_t w[4];
};

HEXVAL_HD I256 i256_zero() { return {{0, 0, 0, 0}}; }

HEXVAL_HD I256 i256_add(const I256& a, const I256& b)
{
    I256 r;
    uint64_t carry = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint64_t s = a.w[i] + b.w[i];
        const uint64_t c1 = s < a.w[i];
        r.w[i] = s + carry;
        carry = c1 | (r.w[i] < s);
    }
    return r;
}

HEXVAL_HD I256 i256_neg(const I256& a)
{
    I256 r;
    uint64_t carry = 1;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint64_t x = ~a.w[i];
        r.w[i] = x + carry;
        carry = carry && r.w[i] == 0;
    }
    return r;
}

HEXVAL_HD I256 i256_sub(const I256& a, const I256& b) { return i256_add(a, i256_neg(b)); }

HEXVAL_HD uint64_t mul_hi64(uint64_t a, uint64_t b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __umul64hi(a, b);
#else
    return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

// Low 256 bits of a * b (exact for two's complement operands whose product
// fits, see the bounds above).
HEXVAL_HD I256 i256_mul(const I256& a, const I256& b)
{
    uint64_t r[4] = {0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        uint64_t carry = 0;
#pragma unroll
        for (int j = 0; i + j < 4; ++j) {
            const uint64_t lo = a.w[i] * b.w[j];
            const uint64_t hi = mul_hi64(a.w[i], b.w[j]);
            uint64_t s = r[i + j] + lo;
            uint64_t c = s < lo;
            const uint64_t s2 = s + carry;
            c += s2 < s;
            r[i + j] = s2;
            carry = hi + c;
        }
    }
    return {{r[0], r[1], r[2], r[3]}};
}

HEXVAL_HD I256 i256_small(int64_t k)
{
    const uint64_t ext = k < 0 ? ~0ull : 0ull;
    return {{(uint64_t)k, ext, ext, ext}};
}

HEXVAL_HD I256 i256_mul_small(const I256& a, int64_t k) { return i256_mul(a, i256_small(k)); }

// -1, 0 or 1.
HEXVAL_HD int i256_sign(const I256& a)
{
    if (a.w[3] >> 63) return -1;
    return (a.w[0] | a.w[1] | a.w[2] | a.w[3]) ? 1 : 0;
}

// The coordinates c[0..k) as integers x[i] = c[i] 2^-E.  Returns false when a
// coordinate is not finite or the integers would need more than
// kMaxCoordBits bits (the caller falls back to the host tier).
HEXVAL_HD bool i256_coordinates(const double* c, int k, I256* x)
{
    int emin = 0, emax = 0;
    bool any = false;
    for (int i = 0; i < k; ++i) {
        if (!isfinite(c[i])) return false;
        if (c[i] != 0.0) {
            int e;
            frexp(c[i], &e);
            if (!any || e - 53 < emin) emin = e - 53;
            if (!any || e > emax) emax = e;
            any = true;
        }
    }
    if (any && emax - emin > kMaxCoordBits) return false;
    for (int i = 0; i < k; ++i) {
        if (c[i] == 0.0) {
            x[i] = i256_zero();
            continue;
        }
        int e;
        const double f = frexp(fabs(c[i]), &e);
        const uint64_t m = (uint64_t)ldexp(f, 53);
        const int sh = (e - 53) - emin;   // 0 <= sh <= kMaxCoordBits - 53
        I256 v = i256_zero();
        const int word = sh / 64, bits = sh % 64;
        v.w[word] = m << bits;
        if (bits && word + 1 < 4) v.w[word + 1] = m >> (64 - bits);
        x[i] = c[i] < 0 ? i256_neg(v) : v;
    }
    return true;
}

struct I3 {
    I256 x, y, z;
};

HEXVAL_HD I3 i3_sub(const I3& a, const I3& b) { return {i256_sub(a.x, b.x), i256_sub(a.y, b.y), i256_sub(a.z, b.z)}; }
HEXVAL_HD I3 i3_add(const I3& a, const I3& b) { return {i256_add(a.x, b.x), i256_add(a.y, b.y), i256_add(a.z, b.z)}; }

// a . (b x c)
HEXVAL_HD I256 i3_triple(const I3& a, const I3& b, const I3& c)
{
    const I256 x = i256_sub(i256_mul(b.y, c.z), i256_mul(b.z, c.y));
    const I256 y = i256_sub(i256_mul(b.z, c.x), i256_mul(b.x, c.z));
    const I256 z = i256_sub(i256_mul(b.x, c.y), i256_mul(b.y, c.x));
    return i256_add(i256_add(i256_mul(a.x, x), i256_mul(a.y, y)), i256_mul(a.z, z));
}

}  // namespace hexval
