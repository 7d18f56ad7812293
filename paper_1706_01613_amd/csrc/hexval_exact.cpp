// Exact tier of libhexval (host C++): the Section 6 algorithm in integer
// arithmetic for the few elements whose floating-point sign decisions could
// not be certified.
//
// Every double is m 2^e with an integer m, so with E the smallest exponent
// among an element's coordinates all coordinates are integers times 2^E.
// The values of Section 5 (triple products of edge vectors), the Table 3
// combinations (times 32) and de Casteljau halving (times 4 per axis and
// level) then stay integers; only signs are used, so the positive scalings
// do not matter.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "hexval_exact.hpp"

namespace hexval {
namespace {

// Signed big integer, magnitude in base 2^32, little endian.
struct Big {
    int sign = 0;                  // -1, 0, 1
    std::vector<uint32_t> mag;

    static Big from_shifted(uint64_t m, int shift, bool neg)
    {
        Big r;
        if (m == 0) return r;
        r.sign = neg ? -1 : 1;
        const int words = shift / 32, bits = shift % 32;
        r.mag.assign(words, 0u);
        unsigned __int128 v = (unsigned __int128)m << bits;
        while (v) {
            r.mag.push_back((uint32_t)v);
            v >>= 32;
        }
        return r;
    }
};

int cmp_mag(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b)
{
    if (a.size() != b.size()) return a.size() < b.size() ? -1 : 1;
    for (size_t i = a.size(); i-- > 0;)
        if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
    return 0;
}

void trim(std::vector<uint32_t>& a)
{
    while (!a.empty() && a.back() == 0u) a.pop_back();
}

std::vector<uint32_t> add_mag(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b)
{
    std::vector<uint32_t> r(std::max(a.size(), b.size()) + 1, 0u);
    uint64_t carry = 0;
    for (size_t i = 0; i < r.size(); ++i) {
        uint64_t s = carry;
        if (i < a.size()) s += a[i];
        if (i < b.size()) s += b[i];
        r[i] = (uint32_t)s;
        carry = s >> 32;
    }
    trim(r);
    return r;
}

// a - b with |a| >= |b|
std::vector<uint32_t> sub_mag(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b)
{
    std::vector<uint32_t> r(a.size(), 0u);
    int64_t borrow = 0;
    for (size_t i = 0; i < a.size(); ++i) {
        int64_t s = (int64_t)a[i] - borrow - (i < b.size() ? (int64_t)b[i] : 0);
        borrow = s < 0;
        r[i] = (uint32_t)(s + (borrow << 32));
    }
    trim(r);
    return r;
}

Big add(const Big& a, const Big& b)
{
    if (a.sign == 0) return b;
    if (b.sign == 0) return a;
    Big r;
    if (a.sign == b.sign) {
        r.sign = a.sign;
        r.mag = add_mag(a.mag, b.mag);
        return r;
    }
    const int c = cmp_mag(a.mag, b.mag);
    if (c == 0) return r;
    if (c > 0) {
        r.sign = a.sign;
        r.mag = sub_mag(a.mag, b.mag);
    } else {
        r.sign = b.sign;
        r.mag = sub_mag(b.mag, a.mag);
    }
    return r;
}

Big neg(Big a)
{
    a.sign = -a.sign;
    return a;
}

Big sub(const Big& a, const Big& b) { return add(a, neg(b)); }

Big mul(const Big& a, const Big& b)
{
    Big r;
    if (a.sign == 0 || b.sign == 0) return r;
    r.sign = a.sign * b.sign;
    r.mag.assign(a.mag.size() + b.mag.size(), 0u);
    for (size_t i = 0; i < a.mag.size(); ++i) {
        uint64_t carry = 0;
        for (size_t j = 0; j < b.mag.size(); ++j) {
            const uint64_t t = (uint64_t)a.mag[i] * b.mag[j] + r.mag[i + j] + carry;
            r.mag[i + j] = (uint32_t)t;
            carry = t >> 32;
        }
        size_t k = i + b.mag.size();
        while (carry) {
            const uint64_t t = (uint64_t)r.mag[k] + carry;
            r.mag[k] = (uint32_t)t;
            carry = t >> 32;
            ++k;
        }
    }
    trim(r.mag);
    return r;
}

Big mul_small(const Big& a, uint32_t k)
{
    Big r;
    if (a.sign == 0 || k == 0) return r;
    r.sign = a.sign;
    r.mag.assign(a.mag.size() + 1, 0u);
    uint64_t carry = 0;
    for (size_t i = 0; i < a.mag.size(); ++i) {
        const uint64_t t = (uint64_t)a.mag[i] * k + carry;
        r.mag[i] = (uint32_t)t;
        carry = t >> 32;
    }
    r.mag[a.mag.size()] = (uint32_t)carry;
    trim(r.mag);
    return r;
}

struct BV {
    Big x, y, z;
};

BV bsub(const BV& a, const BV& b) { return {sub(a.x, b.x), sub(a.y, b.y), sub(a.z, b.z)}; }
BV badd(const BV& a, const BV& b) { return {add(a.x, b.x), add(a.y, b.y), add(a.z, b.z)}; }

Big triple(const BV& a, const BV& b, const BV& c)
{
    const Big x = sub(mul(b.y, c.z), mul(b.z, c.y));
    const Big y = sub(mul(b.z, c.x), mul(b.x, c.z));
    const Big z = sub(mul(b.x, c.y), mul(b.y, c.x));
    return add(add(mul(a.x, x), mul(a.y, y)), mul(a.z, z));
}

// Tensor index (i + 3 j + 9 k, half-steps) of the 27 Fig. 3 nodes.
const int kTensor[27] = {0, 2, 8, 6, 18, 20, 26, 24, 1, 5, 7, 3, 9, 11,
                         17, 15, 19, 23, 25, 21, 4, 10, 14, 16, 12, 22, 13};

bool is_corner(int t)
{
    const int i = t % 3, j = (t / 3) % 3, k = t / 9;
    return i != 1 && j != 1 && k != 1;
}

int mirror(int t, int pattern)
{
    int i = t % 3, j = (t / 3) % 3, k = t / 9;
    if (pattern & 1) i = 2 - i;
    if (pattern & 2) j = 2 - j;
    if (pattern & 4) k = 2 - k;
    return i + 3 * j + 9 * k;
}

// (x0, x1, x2) -> 4 x left half: (4 x0, 2 (x0 + x1), x0 + 2 x1 + x2)
void left_half4(Big& x0, Big& x1, Big& x2)
{
    const Big s01 = add(x0, x1), s12 = add(x1, x2);
    x2 = add(s01, s12);
    x1 = mul_small(s01, 2);
    x0 = mul_small(x0, 4);
}

struct Tree {
    int max_depth;
    bool undecided = false;

    // true when a sub-box corner value <= 0 was found below `node` (level L)
    bool subdivide(const std::vector<Big>& node, int level)
    {
        for (int c = 0; c < 8; ++c) {
            std::vector<Big> t(27);
            for (int k = 0; k < 27; ++k) t[k] = node[mirror(k, c)];
            for (int jk = 0; jk < 9; ++jk) left_half4(t[3 * jk], t[3 * jk + 1], t[3 * jk + 2]);
            for (int k = 0; k < 3; ++k)
                for (int i = 0; i < 3; ++i) left_half4(t[i + 9 * k], t[i + 3 + 9 * k], t[i + 6 + 9 * k]);
            for (int ij = 0; ij < 9; ++ij) left_half4(t[ij], t[ij + 9], t[ij + 18]);
            bool corner_nonpos = false, others_pos = true;
            for (int k = 0; k < 27; ++k) {
                if (is_corner(k)) corner_nonpos |= t[k].sign <= 0;
                else others_pos &= t[k].sign > 0;
            }
            if (corner_nonpos) return true;
            if (others_pos) continue;
            if (level + 1 < max_depth) {
                // back to canonical orientation for the child
                std::vector<Big> child(27);
                for (int k = 0; k < 27; ++k) child[mirror(k, c)] = t[k];
                if (subdivide(child, level + 1)) return true;
            } else {
                undecided = true;
            }
        }
        return false;
    }
};

}  // namespace

// The 8 points as integers: every coordinate is m 2^e, so all are integer
// multiples of 2^E, E the smallest such exponent.  Returns 3 for a non-finite
// coordinate, 0 when every coordinate is 0 (one point: J = 0), else -1.
static int integer_points(const double pts[24], BV p[8])
{
    int emin = 0;
    bool any = false;
    for (int i = 0; i < 24; ++i) {
        if (!isfinite(pts[i])) return 3;
        if (pts[i] != 0.0) {
            int e;
            frexp(pts[i], &e);
            const int ulp = e - 53;
            if (!any || ulp < emin) emin = ulp;
            any = true;
        }
    }
    if (!any) return 0;
    for (int k = 0; k < 8; ++k) {
        Big c[3];
        for (int d = 0; d < 3; ++d) {
            const double x = pts[3 * k + d];
            if (x == 0.0) continue;
            int e;
            const double f = frexp(fabs(x), &e);
            const uint64_t m = (uint64_t)ldexp(f, 53);
            c[d] = Big::from_shifted(m, (e - 53) - emin, x < 0);
        }
        p[k] = {c[0], c[1], c[2]};
    }
    return -1;
}

uint8_t exact_corner_test(const double pts[24])
{
    BV p[8];
    const int pre = integer_points(pts, p);
    if (pre >= 0) return (uint8_t)pre;
    const BV a00 = bsub(p[1], p[0]), a10 = bsub(p[2], p[3]), a01 = bsub(p[5], p[4]), a11 = bsub(p[6], p[7]);
    const BV b00 = bsub(p[3], p[0]), b10 = bsub(p[2], p[1]), b01 = bsub(p[7], p[4]), b11 = bsub(p[6], p[5]);
    const BV c00 = bsub(p[4], p[0]), c10 = bsub(p[5], p[1]), c01 = bsub(p[7], p[3]), c11 = bsub(p[6], p[2]);
    const Big J[8] = {triple(a00, b00, c00), triple(a00, b10, c10), triple(a10, b10, c11),
                      triple(a10, b00, c01), triple(a01, b01, c00), triple(a01, b11, c10),
                      triple(a11, b11, c11), triple(a11, b01, c01)};
    for (const Big& v : J)
        if (v.sign <= 0) return 0;
    return 1;
}

uint8_t exact_quad(const double pts[8])
{
    // the 2D points as integers (as integer_points does in 3D)
    int emin = 0;
    bool any = false;
    for (int i = 0; i < 8; ++i) {
        if (!isfinite(pts[i])) return 3;
        if (pts[i] != 0.0) {
            int e;
            frexp(pts[i], &e);
            if (!any || e - 53 < emin) emin = e - 53;
            any = true;
        }
    }
    if (!any) return 0;
    Big x[4], y[4];
    for (int k = 0; k < 4; ++k)
        for (int d = 0; d < 2; ++d) {
            const double v = pts[2 * k + d];
            if (v == 0.0) continue;
            int e;
            const double f = frexp(fabs(v), &e);
            (d == 0 ? x[k] : y[k]) = Big::from_shifted((uint64_t)ldexp(f, 53), (e - 53) - emin, v < 0);
        }
    // Jacobian matrix of the bilinear map at corner (xi, eta): columns
    // x_xi = n2-n1 (eta 0) or n3-n4 (eta 1), x_eta = n4-n1 (xi 0) or n3-n2 (xi 1)
    static const int XI[2][2] = {{1, 0}, {2, 3}}, ETA[2][2] = {{3, 0}, {2, 1}};
    static const int C[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
    for (const auto& c : C) {
        const int* a = XI[c[1]];
        const int* b = ETA[c[0]];
        const Big J = sub(mul(sub(x[a[0]], x[a[1]]), sub(y[b[0]], y[b[1]])),
                          mul(sub(y[a[0]], y[a[1]]), sub(x[b[0]], x[b[1]])));
        if (J.sign <= 0) return 0;
    }
    return 1;
}

uint8_t exact_verdict(const double pts[24], int max_depth)
{
    BV p[8];
    const int pre = integer_points(pts, p);
    if (pre >= 0) return (uint8_t)pre;   // 0: all points coincide, J = 0 -> INVALID
    const BV a00 = bsub(p[1], p[0]), a10 = bsub(p[2], p[3]), a01 = bsub(p[5], p[4]), a11 = bsub(p[6], p[7]);
    const BV b00 = bsub(p[3], p[0]), b10 = bsub(p[2], p[1]), b01 = bsub(p[7], p[4]), b11 = bsub(p[6], p[5]);
    const BV c00 = bsub(p[4], p[0]), c10 = bsub(p[5], p[1]), c01 = bsub(p[7], p[3]), c11 = bsub(p[6], p[2]);
    // V = 4 J (2^-3E units): corners 4 triple, edges triple with pair sums.
    Big V[20];
    V[0] = triple(a00, b00, c00);
    V[1] = triple(a00, b10, c10);
    V[2] = triple(a10, b10, c11);
    V[3] = triple(a10, b00, c01);
    V[4] = triple(a01, b01, c00);
    V[5] = triple(a01, b11, c10);
    V[6] = triple(a11, b11, c11);
    V[7] = triple(a11, b01, c01);
    for (int k = 0; k < 8; ++k) V[k] = mul_small(V[k], 4);
    const BV B0 = badd(b00, b10), B1 = badd(b01, b11), C0 = badd(c00, c10), C1 = badd(c01, c11);
    const BV A0 = badd(a00, a10), A1 = badd(a01, a11), Cq0 = badd(c00, c01), Cq1 = badd(c10, c11);
    const BV Aq0 = badd(a00, a01), Aq1 = badd(a10, a11), Bq0 = badd(b00, b01), Bq1 = badd(b10, b11);
    V[8] = triple(a00, B0, C0);
    V[9] = triple(A0, b10, Cq1);
    V[10] = triple(a10, B0, C1);
    V[11] = triple(A0, b00, Cq0);
    V[12] = triple(Aq0, Bq0, c00);
    V[13] = triple(Aq0, Bq1, c10);
    V[14] = triple(Aq1, Bq1, c11);
    V[15] = triple(Aq1, Bq0, c01);
    V[16] = triple(a01, B1, C0);
    V[17] = triple(A1, b11, Cq1);
    V[18] = triple(a11, B1, C1);
    V[19] = triple(A1, b01, Cq0);
    // Step 2
    for (int j = 0; j < 20; ++j)
        if (V[j].sign <= 0) return 0;
    // Table 3 times 32:  corners 8V, edges 16V_e - 4(V_p + V_q),
    // faces 8 sum V_e - 6 sum V_c, centre 4 sum V_e - 5 sum V_c.
    static const int EDGE[12][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 0}, {0, 4}, {1, 5},
                                    {2, 6}, {3, 7}, {4, 5}, {5, 6}, {6, 7}, {7, 4}};
    static const int FACE_C[6][4] = {{0, 1, 2, 3}, {0, 1, 4, 5}, {1, 2, 5, 6},
                                     {2, 3, 6, 7}, {0, 3, 4, 7}, {4, 5, 6, 7}};
    static const int FACE_E[6][4] = {{8, 9, 10, 11}, {8, 12, 13, 16}, {9, 13, 14, 17},
                                     {10, 14, 15, 18}, {11, 12, 15, 19}, {16, 17, 18, 19}};
    Big b[27];
    for (int k = 0; k < 8; ++k) b[k] = mul_small(V[k], 8);
    for (int e = 0; e < 12; ++e)
        b[8 + e] = sub(mul_small(V[8 + e], 16), mul_small(add(V[EDGE[e][0]], V[EDGE[e][1]]), 4));
    Big sc, se;
    for (int f = 0; f < 6; ++f) {
        Big c4, e4;
        for (int q = 0; q < 4; ++q) {
            c4 = add(c4, V[FACE_C[f][q]]);
            e4 = add(e4, V[FACE_E[f][q]]);
        }
        b[20 + f] = sub(mul_small(e4, 8), mul_small(c4, 6));
    }
    for (int k = 0; k < 8; ++k) sc = add(sc, V[k]);
    for (int k = 8; k < 20; ++k) se = add(se, V[k]);
    b[26] = sub(mul_small(se, 4), mul_small(sc, 5));
    // Step 4
    bool pos = true;
    for (int a = 8; a < 27; ++a) pos &= b[a].sign > 0;
    if (pos) return 1;
    if (max_depth <= 0) return 2;
    // Step 5
    std::vector<Big> node(27);
    for (int a = 0; a < 27; ++a) node[kTensor[a]] = b[a];
    Tree tree{max_depth};
    if (tree.subdivide(node, 0)) return 0;
    return tree.undecided ? 2 : 1;
}

}  // namespace hexval
