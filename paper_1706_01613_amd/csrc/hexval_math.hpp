// Per-element arithmetic of the validity test (Johnen, Weill, Remacle, IMR
// 2017), shared by the HIP kernels.  Written as __host__ __device__ so that
// the same operations can be replayed on the CPU by the arithmetic check
// library (host_emul.cpp); every rounding below is explicit (compiled with
// -ffp-contract=off, fused operations written as fma()).
#pragma once

#include <stdint.h>
#include <string.h>
#include <math.h>

#ifndef HEXVAL_HD
#if defined(__HIPCC__)
#define HEXVAL_HD __host__ __device__ __forceinline__
#else
#define HEXVAL_HD inline
#endif
#endif

namespace hexval {

// nextafter(x, -inf) and nextafter(x, +inf) from the bit pattern (one
// integer step away from zero or towards it), without the library call's
// general two-argument handling.
HEXVAL_HD double next_down(double x)
{
    if (x != x || x == -HUGE_VAL) return x;
    int64_t b;
    if (x == 0.0) {
        b = 1;                          // the smallest subnormal, negated below
        double d;
        memcpy(&d, &b, 8);
        return -d;
    }
    memcpy(&b, &x, 8);
    b += x > 0.0 ? -1 : 1;
    double d;
    memcpy(&d, &b, 8);
    return d;
}
HEXVAL_HD double next_up(double x) { return -next_down(-x); }

// u = 2^-53 (binary64 unit roundoff).
constexpr double kU64 = 1.1102230246251565e-16;
// Range guard for the per-direction scales (see bounds below).
constexpr double kScaleLo = 0x1p-300;
constexpr double kScaleHi = 0x1p+300;
// Thresholds in units of u * M^ (derivation in the comment of ElementValues).
constexpr double kTauValue = 16.0;     // values J at corners and edge midpoints
constexpr double kTauCoeff = 256.0;    // top-level coefficients b_9..b_27
constexpr double kTauLevel = 72.0;     // added per subdivision level

struct V3 {
    double x, y, z;
};

HEXVAL_HD V3 sub3(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
HEXVAL_HD V3 add3(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }

// a . (b x c): three fused cross-product components, then a fused dot
// product.  At most 2 + 3 roundings on any product path.
HEXVAL_HD double triple(V3 a, V3 b, V3 c)
{
    const double x = fma(b.y, c.z, -(b.z * c.y));
    const double y = fma(b.z, c.x, -(b.x * c.z));
    const double z = fma(b.x, c.y, -(b.y * c.x));
    return fma(a.z, z, fma(a.y, y, a.x * x));
}

HEXVAL_HD double amax(double m, V3 v)
{
    return fmax(m, fmax(fabs(v.x), fmax(fabs(v.y), fabs(v.z))));
}

// Values and (scaled) Bezier coefficients of one element.
//   c[k]  = J at corner k (paper values/coefficients 1..8)
//   d[k]  = 4 J at edge midpoint 9+k
//   e[k]  = 2 b_{9+k}
//   f[k]  = 4 b_{21+k}
//   z     = 8 b_27
// The scaled forms keep the Table 3 arithmetic exact in the constants:
//   2 b_e = 4 v_e - (v_p + v_q)           (edge e between corners p, q)
//   4 b_f = sum_4 (4 v_e) - 3 sum_4 v_c   (face f: its 4 edges and corners)
//   8 b_27 = sum_12 (4 v_e) - 5 sum_8 v_c
//
// Error bounds (u = 2^-53, S_d = largest |component| of the four edge vectors
// of direction d, M = 6 S_xi S_eta S_zeta, |J| <= M everywhere):
//   corner value:   |c^ - c| <= ((1+u)^3 (1+g5) - 1) M       <= 8.01 u M
//   4 x edge value: operands B, C are pair sums (error g2 of |b0|+|b1|, the
//                   permanent of the magnitudes is 4M):    <= 40.01 u M
//   so values J carry <= 10.01 u M < kTauValue u M^.
//   2 b_e: 40.01 + 2*8.01 + 4 + 4   (u M)                  -> b_e  <= 32.01 u M
//   4 b_f: 3*40.01 + 192.04 + 28                            -> b_f  <= 85.01 u M
//   8 b_27: 5*88.01 + 672.13 + 88                           -> b_27 <= 150.02 u M
//   so top-level coefficients carry < kTauCoeff u M^.
//   A de Casteljau halving along one axis adds <= g2 max|b| <= 22.01 u M
//   (|b| <= 11 M: absolute row sums of Table 3 are at most 11), three axes per
//   level: a sub-box at level L carries < (kTauCoeff + kTauLevel L) u M^.
//   M <= M^ (1 + 6.01 u) with M^ computed from the rounded edge vectors.
// Guard: each S_d in [2^-300, 2^300] (no overflow; underflow errors far below
// u M) and 8 b_27 finite (every value enters it, so NaN/Inf inputs or
// overflow show there).  Outside the guard an element is not certified.
struct ElementValues {
    double c[8];
    double d[12];
    double e[12];
    double f[6];
    double z;
    double scale;   // M^
    bool certified_range;
};

// Section 5: derivative edge vectors of the trilinear map (0-based nodes of
// Appendix A).  xi-edges a_jk (j = eta index, k = zeta index), eta-edges b_ik,
// zeta-edges c_ij; J at corner (i,j,k) is triple(a_jk, b_ik, c_ij) and at an
// edge midpoint the two derivatives across the edge are averages (pair sums).
HEXVAL_HD void element_values(const V3 p[8], ElementValues& r)
{
    const V3 a00 = sub3(p[1], p[0]), a10 = sub3(p[2], p[3]);
    const V3 a01 = sub3(p[5], p[4]), a11 = sub3(p[6], p[7]);
    const V3 b00 = sub3(p[3], p[0]), b10 = sub3(p[2], p[1]);
    const V3 b01 = sub3(p[7], p[4]), b11 = sub3(p[6], p[5]);
    const V3 c00 = sub3(p[4], p[0]), c10 = sub3(p[5], p[1]);
    const V3 c01 = sub3(p[7], p[3]), c11 = sub3(p[6], p[2]);

    r.c[0] = triple(a00, b00, c00);  // (0,0,0)
    r.c[1] = triple(a00, b10, c10);  // (1,0,0)
    r.c[2] = triple(a10, b10, c11);  // (1,1,0)
    r.c[3] = triple(a10, b00, c01);  // (0,1,0)
    r.c[4] = triple(a01, b01, c00);  // (0,0,1)
    r.c[5] = triple(a01, b11, c10);  // (1,0,1)
    r.c[6] = triple(a11, b11, c11);  // (1,1,1)
    r.c[7] = triple(a11, b01, c01);  // (0,1,1)

    const V3 B0 = add3(b00, b10), B1 = add3(b01, b11);     // 2 x_eta,  xi=1/2
    const V3 C0 = add3(c00, c10), C1 = add3(c01, c11);     // 2 x_zeta, xi=1/2
    const V3 A0 = add3(a00, a10), A1 = add3(a01, a11);     // 2 x_xi,   eta=1/2
    const V3 Cq0 = add3(c00, c01), Cq1 = add3(c10, c11);   // 2 x_zeta, eta=1/2
    const V3 Aq0 = add3(a00, a01), Aq1 = add3(a10, a11);   // 2 x_xi,   zeta=1/2
    const V3 Bq0 = add3(b00, b01), Bq1 = add3(b10, b11);   // 2 x_eta,  zeta=1/2

    r.d[0] = triple(a00, B0, C0);     //  9 (1/2,0,0)
    r.d[1] = triple(A0, b10, Cq1);    // 10 (1,1/2,0)
    r.d[2] = triple(a10, B0, C1);     // 11 (1/2,1,0)
    r.d[3] = triple(A0, b00, Cq0);    // 12 (0,1/2,0)
    r.d[4] = triple(Aq0, Bq0, c00);   // 13 (0,0,1/2)
    r.d[5] = triple(Aq0, Bq1, c10);   // 14 (1,0,1/2)
    r.d[6] = triple(Aq1, Bq1, c11);   // 15 (1,1,1/2)
    r.d[7] = triple(Aq1, Bq0, c01);   // 16 (0,1,1/2)
    r.d[8] = triple(a01, B1, C0);     // 17 (1/2,0,1)
    r.d[9] = triple(A1, b11, Cq1);    // 18 (1,1/2,1)
    r.d[10] = triple(a11, B1, C1);    // 19 (1/2,1,1)
    r.d[11] = triple(A1, b01, Cq0);   // 20 (0,1/2,1)

    // Table 3.  Corner pairs of the edges 9..20: (1,2)(2,3)(3,4)(4,1)(1,5)(2,6)
    // (3,7)(4,8)(5,6)(6,7)(7,8)(8,5), 0-based below.
    const double* c = r.c;
    const double s01 = c[0] + c[1], s12 = c[1] + c[2], s23 = c[2] + c[3], s30 = c[3] + c[0];
    const double s04 = c[0] + c[4], s15 = c[1] + c[5], s26 = c[2] + c[6], s37 = c[3] + c[7];
    const double s45 = c[4] + c[5], s56 = c[5] + c[6], s67 = c[6] + c[7], s74 = c[7] + c[4];
    const double* d = r.d;
    r.e[0] = d[0] - s01;
    r.e[1] = d[1] - s12;
    r.e[2] = d[2] - s23;
    r.e[3] = d[3] - s30;
    r.e[4] = d[4] - s04;
    r.e[5] = d[5] - s15;
    r.e[6] = d[6] - s26;
    r.e[7] = d[7] - s37;
    r.e[8] = d[8] - s45;
    r.e[9] = d[9] - s56;
    r.e[10] = d[10] - s67;
    r.e[11] = d[11] - s74;
    // Faces 21..26 = zeta=0, eta=0, xi=1, eta=1, xi=0, zeta=1: their corners
    // and edges (Fig. 3 numbering).
    const double cz0 = s01 + s23, cz1 = s45 + s67;
    const double dz0 = (d[0] + d[2]) + (d[1] + d[3]);
    const double dz1 = (d[8] + d[10]) + (d[9] + d[11]);
    const double dvert = (d[4] + d[5]) + (d[6] + d[7]);
    r.f[0] = fma(-3.0, cz0, dz0);                                   // 21: 1234 | 9 10 11 12
    r.f[1] = fma(-3.0, s01 + s45, (d[0] + d[8]) + (d[4] + d[5]));   // 22: 1256 | 9 13 14 17
    r.f[2] = fma(-3.0, s12 + s56, (d[1] + d[9]) + (d[5] + d[6]));   // 23: 2367 | 10 14 15 18
    r.f[3] = fma(-3.0, s23 + s67, (d[2] + d[10]) + (d[6] + d[7]));  // 24: 3478 | 11 15 16 19
    r.f[4] = fma(-3.0, s30 + s74, (d[3] + d[11]) + (d[4] + d[7]));  // 25: 1458 | 12 13 16 20
    r.f[5] = fma(-3.0, cz1, dz1);                                   // 26: 5678 | 17 18 19 20
    r.z = fma(-5.0, cz0 + cz1, (dz0 + dz1) + dvert);                // 27

    double sx = 0.0, sy = 0.0, sz = 0.0;
    sx = amax(amax(amax(amax(sx, a00), a10), a01), a11);
    sy = amax(amax(amax(amax(sy, b00), b10), b01), b11);
    sz = amax(amax(amax(amax(sz, c00), c10), c01), c11);
    r.scale = (6.0 * sx) * sy * sz;
    r.certified_range = sx >= kScaleLo && sx <= kScaleHi && sy >= kScaleLo && sy <= kScaleHi &&
                        sz >= kScaleLo && sz <= kScaleHi && isfinite(r.z);
}

// Coefficient b_alpha (Fig. 3 order, 0-based) in true scale.
HEXVAL_HD double coefficient(const ElementValues& r, int a)
{
    if (a < 8) return r.c[a];
    if (a < 20) return 0.5 * r.e[a - 8];
    if (a < 26) return 0.25 * r.f[a - 20];
    return 0.125 * r.z;
}

struct Summary {
    double m20;     // min of the 20 values J
    double mb;      // min of b_9..b_27
    double min27;   // min of all 27 coefficients
};

HEXVAL_HD Summary summarize(const ElementValues& r)
{
    double m8 = fmin(fmin(fmin(r.c[0], r.c[1]), fmin(r.c[2], r.c[3])),
                     fmin(fmin(r.c[4], r.c[5]), fmin(r.c[6], r.c[7])));
    double md = r.d[0], me = r.e[0];
#pragma unroll
    for (int k = 1; k < 12; ++k) {
        md = fmin(md, r.d[k]);
        me = fmin(me, r.e[k]);
    }
    double mf = fmin(fmin(r.f[0], r.f[1]), fmin(fmin(r.f[2], r.f[3]), fmin(r.f[4], r.f[5])));
    Summary s;
    s.m20 = fmin(m8, 0.25 * md);
    s.mb = fmin(fmin(0.5 * me, 0.25 * mf), 0.125 * r.z);
    s.min27 = fmin(m8, s.mb);
    return s;
}

// Outcome of the top level (Section 6 steps 2 and 4) with certified decisions.
enum TopState : int {
    kTopInvalid = 0,    // some value certainly <= 0
    kTopValid = 1,      // all values and b_9..b_27 certainly > 0
    kTopUndecided = 2,  // depth cap 0 and some b certainly <= 0
    kTopSubdivide = 3,  // subdivision needed (some b not certainly > 0)
    kTopExact = 4       // not certifiable in floating point: exact tier
};

HEXVAL_HD int top_state(const ElementValues& r, const Summary& s, int max_depth)
{
    if (!r.certified_range) return kTopExact;
    const double tv = kTauValue * kU64 * r.scale;
    const double tb = kTauCoeff * kU64 * r.scale;
    if (s.m20 <= -tv) return kTopInvalid;
    if (!(s.m20 > tv)) return kTopExact;
    if (s.mb > tb) return kTopValid;
    if (max_depth > 0) return kTopSubdivide;
    return s.mb <= -tb ? kTopUndecided : kTopExact;
}

// Tensor index of Fig. 3 node alpha: i + 3 j + 9 k with (i, j, k) in half-steps.
HEXVAL_HD int fig3_to_tensor(int a)
{
    // corners, edges 9-20, faces 21-26, centre
    const int8_t map[27] = {0, 2, 8, 6, 18, 20, 26, 24,
                            1, 5, 7, 3, 9, 11, 17, 15, 19, 23, 25, 21,
                            4, 10, 14, 16, 12, 22,
                            13};
    return map[a];
}

// Threshold of a sub-box at `level` (>= 1), same units as values.
HEXVAL_HD double level_threshold(double scale, int level)
{
    return (kTauCoeff + kTauLevel * level) * kU64 * scale;
}

// Left half of a quadratic Bernstein segment: (x0, (x0+x1)/2, ((x0+x1)/2 + (x1+x2)/2)/2).
HEXVAL_HD void left_half(double& x0, double& x1, double& x2)
{
    const double m01 = 0.5 * (x0 + x1);
    const double m12 = 0.5 * (x1 + x2);
    x2 = 0.5 * (m01 + m12);
    x1 = m01;
}

// Child coefficients in tensor order (t = i + 3 j + 9 k): the (0,0,0) octant of
// the input box by de Casteljau at 1/2 along xi, eta, zeta.  The other octants
// are obtained by mirroring the input (see the subdivision kernel).
HEXVAL_HD void lower_octant(double t[27])
{
#pragma unroll
    for (int jk = 0; jk < 9; ++jk) left_half(t[3 * jk], t[3 * jk + 1], t[3 * jk + 2]);
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int i = 0; i < 3; ++i) left_half(t[i + 9 * k], t[i + 3 + 9 * k], t[i + 6 + 9 * k]);
#pragma unroll
    for (int ij = 0; ij < 9; ++ij) left_half(t[ij], t[ij + 9], t[ij + 18]);
}

}  // namespace hexval

namespace hexval {

// The first-pass quantities only (no coefficient array): the same operations
// and roundings as element_values + summarize, ordered so that the edge
// values are consumed as soon as they are formed (fewer live registers).
// T = double is the FP64 pass; T = float is the FP32 filter, whose edge
// vectors are formed in FP64 and rounded once to FP32 (everything after that
// in FP32 with the same operation order).
template <typename T>
struct LeanT {
    T m20, mb, min27, scale;
    bool certified_range;
};
using LeanResult = LeanT<double>;

template <typename T>
struct W3 {
    T x, y, z;
};

template <typename T>
HEXVAL_HD W3<T> edge_t(V3 a, V3 b)
{
    return {(T)(a.x - b.x), (T)(a.y - b.y), (T)(a.z - b.z)};
}

template <typename T>
HEXVAL_HD W3<T> add_t(W3<T> a, W3<T> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }

template <typename T>
HEXVAL_HD T triple_t(W3<T> a, W3<T> b, W3<T> c)
{
    const T x = fma(b.y, c.z, -(b.z * c.y));
    const T y = fma(b.z, c.x, -(b.x * c.z));
    const T z = fma(b.x, c.y, -(b.y * c.x));
    return fma(a.z, z, fma(a.y, y, a.x * x));
}

template <typename T>
HEXVAL_HD T amax_t(T m, W3<T> v)
{
    return fmax(m, fmax(fabs(v.x), fmax(fabs(v.y), fabs(v.z))));
}

// Scale guard per precision: every per-direction scale inside [lo, hi].
template <typename T> struct Guard;
template <> struct Guard<double> {
    static constexpr double lo = 0x1p-300, hi = 0x1p+300;
};
template <> struct Guard<float> {
    static constexpr float lo = 0x1p-30f, hi = 0x1p+30f;
};

// check_edges: also test the 12 edge-midpoint values in the step-2 minimum.
// Without it an element whose only non-positive value sits at an edge
// midpoint is sent to subdivision, where that midpoint is a corner of a
// level-1 sub-box, so the verdict is the same whenever the depth cap is >= 1.
template <typename T>
HEXVAL_HD LeanT<T> element_lean_t(const V3 p[8], bool check_edges)
{
    const W3<T> a00 = edge_t<T>(p[1], p[0]), a10 = edge_t<T>(p[2], p[3]);
    const W3<T> a01 = edge_t<T>(p[5], p[4]), a11 = edge_t<T>(p[6], p[7]);
    const W3<T> b00 = edge_t<T>(p[3], p[0]), b10 = edge_t<T>(p[2], p[1]);
    const W3<T> b01 = edge_t<T>(p[7], p[4]), b11 = edge_t<T>(p[6], p[5]);
    const W3<T> c00 = edge_t<T>(p[4], p[0]), c10 = edge_t<T>(p[5], p[1]);
    const W3<T> c01 = edge_t<T>(p[7], p[3]), c11 = edge_t<T>(p[6], p[2]);
    const T sx = fmax(fmax(amax_t(fabs(a00.x), a10), amax_t(fabs(a00.y), a01)), amax_t(fabs(a00.z), a11));
    const T sy = fmax(fmax(amax_t(fabs(b00.x), b10), amax_t(fabs(b00.y), b01)), amax_t(fabs(b00.z), b11));
    const T sz = fmax(fmax(amax_t(fabs(c00.x), c10), amax_t(fabs(c00.y), c01)), amax_t(fabs(c00.z), c11));

    const T c0 = triple_t(a00, b00, c00), c1 = triple_t(a00, b10, c10);
    const T c2 = triple_t(a10, b10, c11), c3 = triple_t(a10, b00, c01);
    const T c4 = triple_t(a01, b01, c00), c5 = triple_t(a01, b11, c10);
    const T c6 = triple_t(a11, b11, c11), c7 = triple_t(a11, b01, c01);
    const T s01 = c0 + c1, s12 = c1 + c2, s23 = c2 + c3, s30 = c3 + c0;
    const T s04 = c0 + c4, s15 = c1 + c5, s26 = c2 + c6, s37 = c3 + c7;
    const T s45 = c4 + c5, s56 = c5 + c6, s67 = c6 + c7, s74 = c7 + c4;

    // xi-edge midpoints 9, 11, 17, 19
    const W3<T> B0 = add_t(b00, b10), B1 = add_t(b01, b11);
    const W3<T> C0 = add_t(c00, c10), C1 = add_t(c01, c11);
    const T d0 = triple_t(a00, B0, C0), d2 = triple_t(a10, B0, C1);
    const T d8 = triple_t(a01, B1, C0), d10 = triple_t(a11, B1, C1);
    T md = check_edges ? fmin(fmin(d0, d2), fmin(d8, d10)) : T(0);
    T me = fmin(fmin(d0 - s01, d2 - s23), fmin(d8 - s45, d10 - s67));
    const T h02 = d0 + d2, h810 = d8 + d10, p08 = d0 + d8, p210 = d2 + d10;
    // eta-edge midpoints 10, 12, 18, 20
    const W3<T> A0 = add_t(a00, a10), A1 = add_t(a01, a11);
    const W3<T> Cq0 = add_t(c00, c01), Cq1 = add_t(c10, c11);
    const T d1 = triple_t(A0, b10, Cq1), d3 = triple_t(A0, b00, Cq0);
    const T d9 = triple_t(A1, b11, Cq1), d11 = triple_t(A1, b01, Cq0);
    if (check_edges) md = fmin(md, fmin(fmin(d1, d3), fmin(d9, d11)));
    me = fmin(me, fmin(fmin(d1 - s12, d3 - s30), fmin(d9 - s56, d11 - s74)));
    const T dz0 = h02 + (d1 + d3), dz1 = h810 + (d9 + d11);
    const T p19 = d1 + d9, p311 = d3 + d11;
    // zeta-edge midpoints 13..16
    const W3<T> Aq0 = add_t(a00, a01), Aq1 = add_t(a10, a11);
    const W3<T> Bq0 = add_t(b00, b01), Bq1 = add_t(b10, b11);
    const T d4 = triple_t(Aq0, Bq0, c00), d5 = triple_t(Aq0, Bq1, c10);
    const T d6 = triple_t(Aq1, Bq1, c11), d7 = triple_t(Aq1, Bq0, c01);
    if (check_edges) md = fmin(md, fmin(fmin(d4, d5), fmin(d6, d7)));
    me = fmin(me, fmin(fmin(d4 - s04, d5 - s15), fmin(d6 - s26, d7 - s37)));
    const T v45 = d4 + d5, v67 = d6 + d7;

    const T cz0 = s01 + s23, cz1 = s45 + s67;
    T mf = fmin(fma(T(-3), cz0, dz0), fma(T(-3), cz1, dz1));
    mf = fmin(mf, fmin(fma(T(-3), s01 + s45, p08 + v45), fma(T(-3), s12 + s56, p19 + (d5 + d6))));
    mf = fmin(mf, fmin(fma(T(-3), s23 + s67, p210 + v67), fma(T(-3), s30 + s74, p311 + (d4 + d7))));
    const T z = fma(T(-5), cz0 + cz1, (dz0 + dz1) + (v45 + v67));

    const T m8 = fmin(fmin(fmin(c0, c1), fmin(c2, c3)), fmin(fmin(c4, c5), fmin(c6, c7)));
    LeanT<T> r;
    r.m20 = check_edges ? fmin(m8, T(0.25) * md) : m8;
    r.mb = fmin(fmin(T(0.5) * me, T(0.25) * mf), T(0.125) * z);
    r.min27 = fmin(m8, r.mb);
    r.scale = (T(6) * sx) * sy * sz;
    r.certified_range = sx >= Guard<T>::lo && sx <= Guard<T>::hi && sy >= Guard<T>::lo &&
                        sy <= Guard<T>::hi && sz >= Guard<T>::lo && sz <= Guard<T>::hi && isfinite(z);
    return r;
}

HEXVAL_HD LeanResult element_lean(const V3 p[8], bool check_edges)
{
    return element_lean_t<double>(p, check_edges);
}

// FP32 filter thresholds, in units of u32 M^ (u32 = 2^-24).  Each edge
// component carries one FP64 and one FP32 rounding (relative u32 (1 + 2^-29));
// everything after follows the FP64 derivation with u -> u32, whose
// multipliers (8.01, 40.01, 32.01, 85.01, 150.02) keep their slack at this
// precision (second-order terms are below 1e-5 of the first).  The FP32
// values of the guard keep all products in the normal range with a margin
// far above the underflow error.
constexpr float kU32 = 5.9604644775390625e-08f;   // 2^-24

// Outcome of the FP32 pass: 0 INVALID, 1 VALID (both certain), -1 recheck in FP64.
HEXVAL_HD int filter_state(const LeanT<float>& r)
{
    if (!r.certified_range) return -1;
    const float tv = kTauValue * kU32 * r.scale;
    const float tb = kTauCoeff * kU32 * r.scale;
    if (r.m20 <= -tv) return kTopInvalid;
    if (r.m20 > tv && r.mb > tb) return kTopValid;
    return -1;
}

HEXVAL_HD int lean_state(const LeanResult& r, int max_depth)
{
    if (!r.certified_range) return kTopExact;
    const double tv = kTauValue * kU64 * r.scale;
    const double tb = kTauCoeff * kU64 * r.scale;
    if (r.m20 <= -tv) return kTopInvalid;
    if (!(r.m20 > tv)) return kTopExact;
    if (r.mb > tb) return kTopValid;
    if (max_depth > 0) return kTopSubdivide;
    return r.mb <= -tb ? kTopUndecided : kTopExact;
}

}  // namespace hexval
