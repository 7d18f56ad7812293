#pragma once

#include <stdint.h>

#include "hexval_int256.hpp"

namespace hexval {

// Device exact tier (also compiled for the host, for tests).
//
// The elements whose floating-point decisions could not be certified are
// first settled here in exact integer arithmetic (hexval_int256.hpp): the
// signs of the 20 values (step 2 of Section 6) and of the top-level
// coefficients (step 4), the corner-only test, and quadrangle corner values.
// What needs exact subdivision, or coordinates spanning more than
// kMaxCoordBits bits, is left to the host tier (kHostExact).

constexpr uint8_t kHostExact = 0xFE;   // left to the host tier

HEXVAL_HD uint8_t exact_device_hex(const double* pts, int max_depth, bool corner_only)
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
    // Table 3 times 32 for b_9..b_27: edges 16 V_e - 4 (V_p + V_q), faces
    // 8 sum V_e - 6 sum V_c, centre 4 sum V_e - 5 sum V_c (corners: 8 V > 0)
    const int EDGE[12][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 0}, {0, 4}, {1, 5},
                             {2, 6}, {3, 7}, {4, 5}, {5, 6}, {6, 7}, {7, 4}};
    const int FACE_C[6][4] = {{0, 1, 2, 3}, {0, 1, 4, 5}, {1, 2, 5, 6}, {2, 3, 6, 7}, {0, 3, 4, 7}, {4, 5, 6, 7}};
    const int FACE_E[6][4] = {{8, 9, 10, 11}, {8, 12, 13, 16}, {9, 13, 14, 17},
                              {10, 14, 15, 18}, {11, 12, 15, 19}, {16, 17, 18, 19}};
    bool pos = true;
    for (int e = 0; e < 12; ++e) {
        const I256 b = i256_sub(i256_mul_small(V[8 + e], 16),
                                i256_mul_small(i256_add(V[EDGE[e][0]], V[EDGE[e][1]]), 4));
        pos = pos && i256_sign(b) > 0;
    }
    for (int f = 0; f < 6; ++f) {
        I256 c4 = i256_zero(), e4 = i256_zero();
        for (int q = 0; q < 4; ++q) {
            c4 = i256_add(c4, V[FACE_C[f][q]]);
            e4 = i256_add(e4, V[FACE_E[f][q]]);
        }
        pos = pos && i256_sign(i256_sub(i256_mul_small(e4, 8), i256_mul_small(c4, 6))) > 0;
    }
    I256 sc = i256_zero(), se = i256_zero();
    for (int k = 0; k < 8; ++k) sc = i256_add(sc, V[k]);
    for (int k = 8; k < 20; ++k) se = i256_add(se, V[k]);
    pos = pos && i256_sign(i256_sub(i256_mul_small(se, 4), i256_mul_small(sc, 5))) > 0;
    if (pos) return 1;
    if (max_depth <= 0) return 2;
    return kHostExact;   // exact subdivision: host tier
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
