#pragma once

#include <stdint.h>

#include "hexval_int256.hpp"

namespace hexval {

// Device exact tier (also compiled for the host, for tests).
//
// The elements whose floating-point decisions could not be certified are
// settled here in exact integer arithmetic (hexval_int256.hpp): the signs of
// the 20 values (step 2 of Section 6) and of the top-level coefficients
// (step 4), the corner-only test, and quadrangle corner values; elements that
// need subdivision (step 5) go on to exact_device_subdivide.  Coordinates
// spanning more than kMaxCoordBits bits are left to the host tier
// (kHostExact).

constexpr uint8_t kHostExact = 0xFE;        // left to the host tier
constexpr uint8_t kExactSubdivide = 0xFC;   // needs exact subdivision

// Steps 2 and 4 in exact arithmetic.  b: the 27 coefficients times 32 in
// Fig. 3 order (written when subdivision is needed).  Returns 0 (INVALID),
// 1 (VALID), 2 (subdivision needed) or kHostExact; corner_only: 1 when the 8
// corner values are positive (Test 1), else 0.
HEXVAL_HD uint8_t exact_device_top(const double* pts, bool corner_only, I256* b)
{
    I256 c[24];
    if (!i256_coordinates(pts, 24, c)) return kHostExact;
    I3 p[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) p[k] = {c[3 * k], c[3 * k + 1], c[3 * k + 2]};
    const I3 a00 = i3_sub(p[1], p[0]), a10 = i3_sub(p[2], p[3]), a01 = i3_sub(p[5], p[4]), a11 = i3_sub(p[6], p[7]);
    const I3 b00 = i3_sub(p[3], p[0]), b10 = i3_sub(p[2], p[1]), b01 = i3_sub(p[7], p[4]), b11 = i3_sub(p[6], p[5]);
    const I3 c00 = i3_sub(p[4], p[0]), c10 = i3_sub(p[5], p[1]), c01 = i3_sub(p[7], p[3]), c11 = i3_sub(p[6], p[2]);
    // V = 4 J: corners (i,j,k) = 4 triple(a_jk, b_ik, c_ij)
    I256 V[20];
    V[0] = i3_triple(a00, b00, c00);
    V[1] = i3_triple(a00, b10, c10);
    V[2] = i3_triple(a10, b10, c11);
    V[3] = i3_triple(a10, b00, c01);
    V[4] = i3_triple(a01, b01, c00);
    V[5] = i3_triple(a01, b11, c10);
    V[6] = i3_triple(a11, b11, c11);
    V[7] = i3_triple(a11, b01, c01);
    bool corners_pos = true;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        corners_pos = corners_pos && i256_sign(V[k]) > 0;
        V[k] = i256_mul_small(V[k], 4);
    }
    if (!corners_pos) return 0;
    if (corner_only) return 1;
    // edge midpoints: triple products with pair-summed vectors (already 4 J)
    const I3 B0 = i3_add(b00, b10), B1 = i3_add(b01, b11), C0 = i3_add(c00, c10), C1 = i3_add(c01, c11);
    const I3 A0 = i3_add(a00, a10), A1 = i3_add(a01, a11), Cq0 = i3_add(c00, c01), Cq1 = i3_add(c10, c11);
    const I3 Aq0 = i3_add(a00, a01), Aq1 = i3_add(a10, a11), Bq0 = i3_add(b00, b01), Bq1 = i3_add(b10, b11);
    V[8] = i3_triple(a00, B0, C0);
    V[9] = i3_triple(A0, b10, Cq1);
    V[10] = i3_triple(a10, B0, C1);
    V[11] = i3_triple(A0, b00, Cq0);
    V[12] = i3_triple(Aq0, Bq0, c00);
    V[13] = i3_triple(Aq0, Bq1, c10);
    V[14] = i3_triple(Aq1, Bq1, c11);
    V[15] = i3_triple(Aq1, Bq0, c01);
    V[16] = i3_triple(a01, B1, C0);
    V[17] = i3_triple(A1, b11, Cq1);
    V[18] = i3_triple(a11, B1, C1);
    V[19] = i3_triple(A1, b01, Cq0);
#pragma unroll
    for (int k = 8; k < 20; ++k)
        if (i256_sign(V[k]) <= 0) return 0;
    // Table 3 times 32: corners 8 V, edges 16 V_e - 4 (V_p + V_q), faces
    // 8 sum V_e - 6 sum V_c, centre 4 sum V_e - 5 sum V_c
    const int EDGE[12][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 0}, {0, 4}, {1, 5},
                             {2, 6}, {3, 7}, {4, 5}, {5, 6}, {6, 7}, {7, 4}};
    const int FACE_C[6][4] = {{0, 1, 2, 3}, {0, 1, 4, 5}, {1, 2, 5, 6}, {2, 3, 6, 7}, {0, 3, 4, 7}, {4, 5, 6, 7}};
    const int FACE_E[6][4] = {{8, 9, 10, 11}, {8, 12, 13, 16}, {9, 13, 14, 17},
                              {10, 14, 15, 18}, {11, 12, 15, 19}, {16, 17, 18, 19}};
    bool pos = true;
    for (int k = 0; k < 8; ++k) b[k] = i256_mul_small(V[k], 8);
    for (int e = 0; e < 12; ++e) {
        b[8 + e] = i256_sub(i256_mul_small(V[8 + e], 16), i256_mul_small(i256_add(V[EDGE[e][0]], V[EDGE[e][1]]), 4));
        pos = pos && i256_sign(b[8 + e]) > 0;
    }
    for (int f = 0; f < 6; ++f) {
        I256 c4 = i256_zero(), e4 = i256_zero();
        for (int q = 0; q < 4; ++q) {
            c4 = i256_add(c4, V[FACE_C[f][q]]);
            e4 = i256_add(e4, V[FACE_E[f][q]]);
        }
        b[20 + f] = i256_sub(i256_mul_small(e4, 8), i256_mul_small(c4, 6));
        pos = pos && i256_sign(b[20 + f]) > 0;
    }
    I256 sc = i256_zero(), se = i256_zero();
    for (int k = 0; k < 8; ++k) sc = i256_add(sc, V[k]);
    for (int k = 8; k < 20; ++k) se = i256_add(se, V[k]);
    b[26] = i256_sub(i256_mul_small(se, 4), i256_mul_small(sc, 5));
    pos = pos && i256_sign(b[26]) > 0;
    return pos ? 1 : 2;
}

HEXVAL_HD uint8_t exact_device_hex(const double* pts, int max_depth, bool corner_only)
{
    I256 b[27];
    const uint8_t r = exact_device_top(pts, corner_only, b);
    if (r != 2) return r;
    return max_depth <= 0 ? 2 : kExactSubdivide;
}

// ------------------------------------------------------- exact subdivision
//
// De Casteljau at 1/2 in integers: (x0, x1, x2) -> 4 x the left half,
// (4 x0, 2 (x0 + x1), x0 + 2 x1 + x2), so a sub-box of level L carries its
// coefficients times 2^(6L) (times 4 per axis and level; signs are what the
// method uses).  From the root's 32 b < 2^(3B+15) <= 2^249 (B <=
// kMaxCoordBits) the integers stay below 2^(249 + 6L) <= 2^369 up to the
// largest depth cap (20): 384-bit two's complement additions and doublings
// are exact.

constexpr int kWideWords = 6;

struct IW {
    uint64_t w[kWideWords];
};

HEXVAL_HD IW iw_from(const I256& a)
{
    IW r;
    const uint64_t ext = (a.w[3] >> 63) ? ~0ull : 0ull;
#pragma unroll
    for (int i = 0; i < kWideWords; ++i) r.w[i] = i < 4 ? a.w[i] : ext;
    return r;
}

HEXVAL_HD IW iw_add(const IW& a, const IW& b)
{
    IW r;
    uint64_t carry = 0;
#pragma unroll
    for (int i = 0; i < kWideWords; ++i) {
        const uint64_t s = a.w[i] + b.w[i];
        const uint64_t c1 = s < a.w[i];
        r.w[i] = s + carry;
        carry = c1 | (r.w[i] < s);
    }
    return r;
}

// a * 2^s for s in 1..63 (the low 384 bits).
HEXVAL_HD IW iw_shl(const IW& a, int s)
{
    IW r;
    r.w[0] = a.w[0] << s;
#pragma unroll
    for (int i = 1; i < kWideWords; ++i) r.w[i] = (a.w[i] << s) | (a.w[i - 1] >> (64 - s));
    return r;
}

// -1, 0 or 1.
HEXVAL_HD int iw_sign(const IW& a)
{
    if (a.w[kWideWords - 1] >> 63) return -1;
    uint64_t o = 0;
#pragma unroll
    for (int i = 0; i < kWideWords; ++i) o |= a.w[i];
    return o ? 1 : 0;
}

// Tensor index t = i + 3 j + 9 k mirrored along the axes set in `pattern`.
HEXVAL_HD int exact_mirror(int t, int pattern)
{
    int i = t % 3, j = (t / 3) % 3, k = t / 9;
    if (pattern & 1) i = 2 - i;
    if (pattern & 2) j = 2 - j;
    if (pattern & 4) k = 2 - k;
    return i + 3 * j + 9 * k;
}

HEXVAL_HD void iw_left_half4(IW& x0, IW& x1, IW& x2)
{
    const IW s01 = iw_add(x0, x1), s12 = iw_add(x1, x2);
    x2 = iw_add(s01, s12);
    x1 = iw_shl(s01, 1);
    x0 = iw_shl(x0, 2);
}

// Words of one level of the path: 27 coefficients and a 28th word holding
// the next child to visit (w[0]) and the node's orientation (w[1]).
constexpr int kExactDfsWords = 28;

// Step 5 in exact arithmetic, depth first as the recursion of Section 6:
// the children of a box are its 8 octants; a child with a corner coefficient
// <= 0 makes the element INVALID, a child whose other 19 coefficients are > 0
// is retired, any other is split again below the depth cap and counts as
// UNDECIDED at it.  b: the root's 27 coefficients times 32 (Fig. 3 order);
// st: (max_depth + 1) * kExactDfsWords words (the path, one level each).
// A box is stored mirrored along the axes of the octant it came from (its
// orientation), as the level kernel stores them.  Returns 0, 1 or 2.
HEXVAL_HD uint8_t exact_device_subdivide(const I256* b, IW* st, int max_depth)
{
#pragma unroll 1
    for (int a = 0; a < 27; ++a) st[fig3_to_tensor(a)] = iw_from(b[a]);
    st[27].w[0] = 0;
    st[27].w[1] = 0;
    bool undecided = false;
    int L = 0;
    while (L >= 0) {
        IW* nd = st + kExactDfsWords * L;
        const int c = (int)nd[27].w[0];
        if (c == 8) {
            --L;
            continue;
        }
        nd[27].w[0] = (uint64_t)(c + 1);
        const int pat = (int)nd[27].w[1] ^ c;
        IW* ch = nd + kExactDfsWords;
#pragma unroll 1
        for (int k = 0; k < 27; ++k) ch[k] = nd[exact_mirror(k, pat)];
#pragma unroll 1
        for (int jk = 0; jk < 9; ++jk) iw_left_half4(ch[3 * jk], ch[3 * jk + 1], ch[3 * jk + 2]);
#pragma unroll 1
        for (int k = 0; k < 3; ++k)
            for (int i = 0; i < 3; ++i) iw_left_half4(ch[i + 9 * k], ch[i + 3 + 9 * k], ch[i + 6 + 9 * k]);
#pragma unroll 1
        for (int ij = 0; ij < 9; ++ij) iw_left_half4(ch[ij], ch[ij + 9], ch[ij + 18]);
        bool corner_nonpos = false, others_pos = true;
#pragma unroll 1
        for (int k = 0; k < 27; ++k) {
            const int i = k % 3, j = (k / 3) % 3, kk = k / 9;
            const int sg = iw_sign(ch[k]);
            if (i != 1 && j != 1 && kk != 1) corner_nonpos = corner_nonpos || sg <= 0;
            else others_pos = others_pos && sg > 0;
        }
        if (corner_nonpos) return 0;
        if (others_pos) continue;
        if (L + 1 < max_depth) {
            ch[27].w[0] = 0;
            ch[27].w[1] = (uint64_t)c;
            ++L;
        } else {
            undecided = true;
        }
    }
    return undecided ? 2 : 1;
}

// exact_device_hex followed by the exact subdivision where it is needed
// (st as for exact_device_subdivide).
HEXVAL_HD uint8_t exact_device_verdict(const double* pts, int max_depth, IW* st)
{
    I256 b[27];
    const uint8_t r = exact_device_top(pts, false, b);
    if (r != 2) return r;
    if (max_depth <= 0) return 2;
    return exact_device_subdivide(b, st, max_depth);
}

HEXVAL_HD uint8_t exact_device_quad(const double* pts)
{
    I256 c[8];
    if (!i256_coordinates(pts, 8, c)) return kHostExact;
    // Jacobian matrix at corner (xi, eta): x_xi = n2-n1 (eta 0) or n3-n4
    // (eta 1), x_eta = n4-n1 (xi 0) or n3-n2 (xi 1); 0-based points
    const int XI[2][2] = {{1, 0}, {2, 3}}, ETA[2][2] = {{3, 0}, {2, 1}};
    const int C[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
    for (int k = 0; k < 4; ++k) {
        const int* a = XI[C[k][1]];
        const int* b = ETA[C[k][0]];
        const I256 ax = i256_sub(c[2 * a[0]], c[2 * a[1]]), ay = i256_sub(c[2 * a[0] + 1], c[2 * a[1] + 1]);
        const I256 bx = i256_sub(c[2 * b[0]], c[2 * b[1]]), by = i256_sub(c[2 * b[0] + 1], c[2 * b[1] + 1]);
        if (i256_sign(i256_sub(i256_mul(ax, by), i256_mul(ay, bx))) <= 0) return 0;
    }
    return 1;
}

}  // namespace hexval
