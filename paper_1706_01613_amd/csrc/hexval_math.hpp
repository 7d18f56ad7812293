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

// a x b with fused components (the cross product inside triple()), and
// c . X with the fused dot product of triple(): dot(c, cross(a, b)) is
// triple(c, a, b) bit for bit.
HEXVAL_HD V3 cross(V3 a, V3 b)
{
    return {fma(a.y, b.z, -(a.z * b.y)), fma(a.z, b.x, -(a.x * b.z)), fma(a.x, b.y, -(a.y * b.x))};
}
HEXVAL_HD double dot(V3 c, V3 x) { return fma(c.z, x.z, fma(c.y, x.y, c.x * x.x)); }
// c . x + d . y as one fused chain of six products.
HEXVAL_HD double dot2(V3 c, V3 x, V3 d, V3 y)
{
    return fma(d.z, y.z, fma(d.y, y.y, fma(d.x, y.x, fma(c.z, x.z, fma(c.y, x.y, c.x * x.x)))));
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
// of direction d, M = 6 S_xi S_eta S_zeta, |J| <= M everywhere; first-order
// terms, the second-order ones are below 1e-14 of them):
//   corner value:   |c^ - c| <= ((1+u)^3 (1+g5) - 1) M       <= 8.01 u M
//   2 b_e, xi- and eta-edges: a cross component (|X| <= 2 S S') carries
//     <= 3u S S'; the six-product fused chain adds u (6+5+...+1) 2 = 42u to
//     the 6 * 3u = 18u of its operands (units S_xi S_eta S_zeta):
//     60u = 10 u M                                          -> b_e <= 5 u M
//   2 b_e, zeta-edges: the triple of pair sums carries 132u = 22 u M, the
//     corner pair sum 2 * 8.01 + 2, the subtraction 6 (|2 b_e| <= 6 M):
//     46.02 u M                                             -> b_e <= 23.01 u M
//   4 J at an edge midpoint, (2 b_e) + (v_p + v_q): 10 + 18.02 + 4 on xi- and
//     eta-edges; on zeta-edges the pair sum's error cancels (the same rounded
//     sum is subtracted and added back): 22 + 6 + 4.  So values J carry
//     <= 8.01 u M < kTauValue u M^.
//   4 b_f = sum_4 (2 b_e) - sum_4 v_c: edge terms 2 * 10 + 2 * 46.02, their
//     summation 32, the corner sum 2 * 18.02 + 4, the subtraction 28
//     (|4 b_f| <= 28 M): 212.08 u M                         -> b_f <= 53.02 u M
//   8 b_27 = sum_12 (2 b_e) - 2 sum_8 v_c: edge terms 8 * 10 + 4 * 46.02,
//     their summation 136, the corners 2 * 88.08, the final fma 88
//     (|8 b_27| <= 88 M): 664.24 u M                       -> b_27 <= 83.03 u M
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

    // Corner (i,j,k): J = c_ij . X(i,j,k) with X(i,j,k) = a_jk x b_ik.
    const V3 X0 = cross(a00, b00), X1 = cross(a00, b10), X2 = cross(a10, b10), X3 = cross(a10, b00);
    const V3 X4 = cross(a01, b01), X5 = cross(a01, b11), X6 = cross(a11, b11), X7 = cross(a11, b01);
    double* c = r.c;
    c[0] = dot(c00, X0);  // (0,0,0)
    c[1] = dot(c10, X1);  // (1,0,0)
    c[2] = dot(c11, X2);  // (1,1,0)
    c[3] = dot(c01, X3);  // (0,1,0)
    c[4] = dot(c00, X4);  // (0,0,1)
    c[5] = dot(c10, X5);  // (1,0,1)
    c[6] = dot(c11, X6);  // (1,1,1)
    c[7] = dot(c01, X7);  // (0,1,1)

    // Edge midpoints.  4 J at the midpoint of a xi-edge p-q is C . (X_p + X_q)
    // with C the pair sum of the zeta-edges at p and q (linearity of the
    // cross product in its second factor), and of an eta-edge likewise with
    // the first factor; expanding C leaves v_p + v_q plus the two mixed
    // terms, so 2 b_e = 4 v_e - (v_p + v_q) = c_q . X_p + c_p . X_q (c_p the
    // zeta-edge at p) without cancellation.  On a zeta-edge the two factors
    // both change, and 2 b_e = triple(A', B', c) - (v_p + v_q) with the pair
    // sums A', B' across it.  Corner pairs of the edges 9..20 (0-based):
    // (0,1)(1,2)(2,3)(3,0)(0,4)(1,5)(2,6)(3,7)(4,5)(5,6)(6,7)(7,4).
    double* e = r.e;
    e[0] = dot2(c10, X0, c00, X1);    //  9 (1/2,0,0)
    e[1] = dot2(c11, X1, c10, X2);    // 10 (1,1/2,0)
    e[2] = dot2(c11, X3, c01, X2);    // 11 (1/2,1,0)
    e[3] = dot2(c01, X0, c00, X3);    // 12 (0,1/2,0)
    e[8] = dot2(c10, X4, c00, X5);    // 17 (1/2,0,1)
    e[9] = dot2(c11, X5, c10, X6);    // 18 (1,1/2,1)
    e[10] = dot2(c11, X7, c01, X6);   // 19 (1/2,1,1)
    e[11] = dot2(c01, X4, c00, X7);   // 20 (0,1/2,1)
    const V3 Aq0 = add3(a00, a01), Aq1 = add3(a10, a11);   // 2 x_xi,   zeta=1/2
    const V3 Bq0 = add3(b00, b01), Bq1 = add3(b10, b11);   // 2 x_eta,  zeta=1/2
    const double s01 = c[0] + c[1], s12 = c[1] + c[2], s23 = c[2] + c[3], s30 = c[3] + c[0];
    const double s04 = c[0] + c[4], s15 = c[1] + c[5], s26 = c[2] + c[6], s37 = c[3] + c[7];
    const double s45 = c[4] + c[5], s56 = c[5] + c[6], s67 = c[6] + c[7], s74 = c[7] + c[4];
    e[4] = triple(Aq0, Bq0, c00) - s04;   // 13 (0,0,1/2)
    e[5] = triple(Aq0, Bq1, c10) - s15;   // 14 (1,0,1/2)
    e[6] = triple(Aq1, Bq1, c11) - s26;   // 15 (1,1,1/2)
    e[7] = triple(Aq1, Bq0, c01) - s37;   // 16 (0,1,1/2)
    // 4 J at the edge midpoints (the step-2 values)
    const double sp[12] = {s01, s12, s23, s30, s04, s15, s26, s37, s45, s56, s67, s74};
#pragma unroll
    for (int k = 0; k < 12; ++k) r.d[k] = e[k] + sp[k];

    // Table 3 with the 2 b_e above: each corner of a face lies on two of its
    // edges and each corner of the element on three, so
    //   4 b_f = sum_4 (4 v_e) - 3 sum_4 v_c = sum_4 (2 b_e) - sum_4 v_c,
    //   8 b_27 = sum_12 (4 v_e) - 5 sum_8 v_c = sum_12 (2 b_e) - 2 sum_8 v_c.
    // Faces 21..26 = zeta=0, eta=0, xi=1, eta=1, xi=0, zeta=1: their corners
    // and edges (Fig. 3 numbering).
    const double ez0 = (e[0] + e[2]) + (e[1] + e[3]), ez1 = (e[8] + e[10]) + (e[9] + e[11]);
    const double cz0 = s01 + s23, cz1 = s45 + s67;
    r.f[0] = ez0 - cz0;                                          // 21: 1234 | 9 10 11 12
    r.f[1] = ((e[0] + e[8]) + (e[4] + e[5])) - (s01 + s45);      // 22: 1256 | 9 13 14 17
    r.f[2] = ((e[1] + e[9]) + (e[5] + e[6])) - (s12 + s56);      // 23: 2367 | 10 14 15 18
    r.f[3] = ((e[2] + e[10]) + (e[6] + e[7])) - (s23 + s67);     // 24: 3478 | 11 15 16 19
    r.f[4] = ((e[3] + e[11]) + (e[4] + e[7])) - (s30 + s74);     // 25: 1458 | 12 13 16 20
    r.f[5] = ez1 - cz1;                                          // 26: 5678 | 17 18 19 20
    r.z = fma(-2.0, cz0 + cz1, (ez0 + ez1) + ((e[4] + e[5]) + (e[6] + e[7])));   // 27

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
HEXVAL_HD W3<T> cross_t(W3<T> a, W3<T> b)
{
    return {fma(a.y, b.z, -(a.z * b.y)), fma(a.z, b.x, -(a.x * b.z)), fma(a.x, b.y, -(a.y * b.x))};
}

template <typename T>
HEXVAL_HD T dot_t(W3<T> c, W3<T> x)
{
    return fma(c.z, x.z, fma(c.y, x.y, c.x * x.x));
}

template <typename T>
HEXVAL_HD T dot2_t(W3<T> c, W3<T> x, W3<T> d, W3<T> y)
{
    return fma(d.z, y.z, fma(d.y, y.y, fma(d.x, y.x, fma(c.z, x.z, fma(c.y, x.y, c.x * x.x)))));
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
    // zeta-edges first: their pair sums need the edges of both faces, which
    // then need only stay live for their own face
    const W3<T> c00 = edge_t<T>(p[4], p[0]), c10 = edge_t<T>(p[5], p[1]);
    const W3<T> c01 = edge_t<T>(p[7], p[3]), c11 = edge_t<T>(p[6], p[2]);
    const T sz = fmax(fmax(amax_t(fabs(c00.x), c10), amax_t(fabs(c00.y), c01)), amax_t(fabs(c00.z), c11));
    const W3<T> a00 = edge_t<T>(p[1], p[0]), a10 = edge_t<T>(p[2], p[3]);
    const W3<T> a01 = edge_t<T>(p[5], p[4]), a11 = edge_t<T>(p[6], p[7]);
    const T sx = fmax(fmax(amax_t(fabs(a00.x), a10), amax_t(fabs(a00.y), a01)), amax_t(fabs(a00.z), a11));
    const W3<T> b00 = edge_t<T>(p[3], p[0]), b10 = edge_t<T>(p[2], p[1]);
    const W3<T> b01 = edge_t<T>(p[7], p[4]), b11 = edge_t<T>(p[6], p[5]);
    const T sy = fmax(fmax(amax_t(fabs(b00.x), b10), amax_t(fabs(b00.y), b01)), amax_t(fabs(b00.z), b11));
    T t4, t5, t6, t7;
    {
        const W3<T> Aq0 = add_t(a00, a01), Aq1 = add_t(a10, a11);
        const W3<T> Bq0 = add_t(b00, b01), Bq1 = add_t(b10, b11);
        t4 = triple_t(Aq0, Bq0, c00);
        t5 = triple_t(Aq0, Bq1, c10);
        t6 = triple_t(Aq1, Bq1, c11);
        t7 = triple_t(Aq1, Bq0, c01);
    }
    // Corners and the 2 b_e of the xi- and eta-edges of the bottom face
    // (k = 0) and the top face (k = 1), from the corner cross products as in
    // element_values; each face's crosses are consumed as they are formed.
    T c0, c1, c2, c3, e0, e1, e2, e3;
    {
        const W3<T> X0 = cross_t(a00, b00), X1 = cross_t(a00, b10);
        c0 = dot_t(c00, X0);
        c1 = dot_t(c10, X1);
        e0 = dot2_t(c10, X0, c00, X1);
        const W3<T> X3 = cross_t(a10, b00);
        c3 = dot_t(c01, X3);
        e3 = dot2_t(c01, X0, c00, X3);
        const W3<T> X2 = cross_t(a10, b10);
        c2 = dot_t(c11, X2);
        e1 = dot2_t(c11, X1, c10, X2);
        e2 = dot2_t(c11, X3, c01, X2);
    }
    T c4, c5, c6, c7, e8, e9, e10, e11;
    {
        const W3<T> X4 = cross_t(a01, b01), X5 = cross_t(a01, b11);
        c4 = dot_t(c00, X4);
        c5 = dot_t(c10, X5);
        e8 = dot2_t(c10, X4, c00, X5);
        const W3<T> X7 = cross_t(a11, b01);
        c7 = dot_t(c01, X7);
        e11 = dot2_t(c01, X4, c00, X7);
        const W3<T> X6 = cross_t(a11, b11);
        c6 = dot_t(c11, X6);
        e9 = dot2_t(c11, X5, c10, X6);
        e10 = dot2_t(c11, X7, c01, X6);
    }
    const T s01 = c0 + c1, s12 = c1 + c2, s23 = c2 + c3, s30 = c3 + c0;
    const T s04 = c0 + c4, s15 = c1 + c5, s26 = c2 + c6, s37 = c3 + c7;
    const T s45 = c4 + c5, s56 = c5 + c6, s67 = c6 + c7, s74 = c7 + c4;
    // zeta-edges 13..16
    const T e4 = t4 - s04, e5 = t5 - s15, e6 = t6 - s26, e7 = t7 - s37;

    // step 2 with the edge midpoints (4 J = 2 b_e + v_p + v_q)
    T md = T(0);
    if (check_edges) {
        md = fmin(fmin(fmin(e0 + s01, e1 + s12), fmin(e2 + s23, e3 + s30)),
                  fmin(fmin(e4 + s04, e5 + s15), fmin(e6 + s26, e7 + s37)));
        md = fmin(md, fmin(fmin(e8 + s45, e9 + s56), fmin(e10 + s67, e11 + s74)));
    }
    const T me = fmin(fmin(fmin(fmin(e0, e1), fmin(e2, e3)), fmin(fmin(e4, e5), fmin(e6, e7))),
                      fmin(fmin(e8, e9), fmin(e10, e11)));
    // Table 3 in the form of element_values
    const T ez0 = (e0 + e2) + (e1 + e3), ez1 = (e8 + e10) + (e9 + e11);
    const T cz0 = s01 + s23, cz1 = s45 + s67;
    const T e45 = e4 + e5, e67 = e6 + e7;
    T mf = fmin(ez0 - cz0, ez1 - cz1);
    mf = fmin(mf, fmin(((e0 + e8) + e45) - (s01 + s45), ((e1 + e9) + (e5 + e6)) - (s12 + s56)));
    mf = fmin(mf, fmin(((e2 + e10) + e67) - (s23 + s67), ((e3 + e11) + (e4 + e7)) - (s30 + s74)));
    const T z = fma(T(-2), cz0 + cz1, (ez0 + ez1) + (e45 + e67));

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
// component carries one FP64 and one FP32 rounding (relative u32 (1 + 2^-29)),
// which adds 4u to a corner cross component (7u instead of 3u) and doubles the
// error of a pair sum (4u); the FP64 derivation with u -> u32 then gives
// corner values 6.5, xi/eta 2 b_e 16, zeta 2 b_e 55, edge-midpoint values
// 11, b_f 59 and b_27 90.5 (u32 M), inside kTauValue and kTauCoeff with the
// same margin as in FP64 (second-order terms are below 1e-5 of the first).
// The FP32 values of the guard keep all products in the normal range with a
// margin far above the underflow error.
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

// An element the FP32 pass may send to subdivision itself, without the FP64
// recheck: every corner value above twice its FP32 bound and the Bezier
// minimum at or below minus its bound.  Then the FP64 values (within
// kTauValue and kTauCoeff u64 M^ of the exact ones, and those within the
// FP32 bounds of the FP32 values) keep the corner values above their FP64
// bound and the Bezier minimum below its own, so the FP64 evaluation would
// subdivide the element too (lean_state with max_depth > 0).  Subdivision
// recomputes its coefficients in FP64, so its verdict is the same.
HEXVAL_HD bool filter_subdivides(const LeanT<float>& r)
{
    if (!r.certified_range) return false;
    const float tv = kTauValue * kU32 * r.scale;
    const float tb = kTauCoeff * kU32 * r.scale;
    return r.m20 > 2.0f * tv && r.mb <= -tb;
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
