/*
 * hexval oracle: TEST INFRASTRUCTURE, not part of the library.
 *
 * A plain, slow, scalar FP64 implementation of the validity test of linear
 * hexahedra from A. Johnen, J.-C. Weill, J.-F. Remacle, "Robust and efficient
 * validation of the linear hexahedral element" (IMR 2017).  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark load it;
 * the HIP library never does, and the two share no code.
 *
 * What is computed, in the paper's terms:
 *   - the trilinear map of Appendix A and its Jacobian determinant
 *     J = det[x_xi x_eta x_zeta] (eq. e:det3d), with the partial derivatives
 *     written as bilinear blends of edge vectors (Section 5);
 *   - c_alpha = J(xi_alpha) at the 27 uniformly spaced nodes of the order-2
 *     hexahedron, ordered as in Fig. 3 (Section 3.2);
 *   - b = T c, T the inverse of A_{alpha beta} = B_beta(xi_alpha) (Section 3.2,
 *     Table 1).  T is formed as the tensor product of the 1D inverse of the
 *     order-2 Bernstein collocation matrix on (0, 1/2, 1); tests compare it with
 *     the printed table entry by entry;
 *   - the algorithm of Section 6: INVALID when one of c_1..c_20 is not
 *     positive (step 2), VALID when b_9..b_27 are all positive (step 4), else
 *     recursive subdivision, where the coefficients of a sub-box are obtained
 *     by RESAMPLING J at the sub-box's own 27 nodes and applying T again (the
 *     sub-box form of Section 3; the child formula the paper defers to its
 *     reference [johnen2013] is not used here).
 *
 * Readings of the paper (each also listed in the design notes):
 *   - "negative"/"positive" in Section 6 are read against the strict validity
 *     definition of Section 2 (J > 0): a value <= 0 is INVALID, only > 0
 *     certifies;
 *   - subdivision stops at a depth cap (default 6); an element with no
 *     non-positive value found but a capped ambiguous sub-box is UNDECIDED;
 *   - non-finite coordinates give BAD_INPUT;
 *   - min_coeff is the minimum of the 27 top-level coefficients, always
 *     computed.
 *
 * Exactness: every sign decision compares the FP64 value against a rigorous
 * forward error bound (derived in the comment above `bounds`).  When the value
 * lies inside its bound the element is reported FRAGILE (255) and the Python
 * exact tier (oracle/exact.py, rational arithmetic) recomputes it.  The verdict
 * of the oracle is therefore the verdict of the algorithm in exact arithmetic.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math:
 * the error bounds assume IEEE binary64 round-to-nearest, no fused ops).
 */
#include <stdint.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OV_INVALID = 0, OV_VALID = 1, OV_UNDECIDED = 2, OV_BAD_INPUT = 3, OV_FRAGILE = 255 };

/* Fig. 3: lattice position of node alpha (0-based alpha = paper index - 1),
 * in half-steps 0, 1, 2 along (xi, eta, zeta).  Corners 1-8 follow Appendix A,
 * edge midpoints 9-20 the edges (12)(23)(34)(41)(15)(26)(37)(48)(56)(67)(78)(85),
 * face centres 21-26 the faces zeta=0, eta=0, xi=1, eta=1, xi=0, zeta=1, and 27
 * the centre. */
static const int NODE[27][3] = {
    {0, 0, 0}, {2, 0, 0}, {2, 2, 0}, {0, 2, 0}, {0, 0, 2}, {2, 0, 2}, {2, 2, 2}, {0, 2, 2},
    {1, 0, 0}, {2, 1, 0}, {1, 2, 0}, {0, 1, 0}, {0, 0, 1}, {2, 0, 1},
    {2, 2, 1}, {0, 2, 1}, {1, 0, 2}, {2, 1, 2}, {1, 2, 2}, {0, 1, 2},
    {1, 1, 0}, {1, 0, 1}, {2, 1, 1}, {1, 2, 1}, {0, 1, 1}, {1, 1, 2},
    {1, 1, 1}};

/* Inverse of the 1D collocation matrix [B_j(t_i)], t = 0, 1/2, 1, for the
 * order-2 Bernstein polynomials B_0=(1-t)^2, B_1=2t(1-t), B_2=t^2:
 * at t=1/2 the basis is (1/4, 1/2, 1/4), hence b_1 = 2 c_1 - (c_0 + c_2)/2. */
static const double T1[3][3] = {{1.0, 0.0, 0.0}, {-0.5, 2.0, -0.5}, {0.0, 0.0, 1.0}};

static double T[27][27];
static int T_ready = 0;

static void build_T(void)
{
    for (int a = 0; a < 27; ++a)
        for (int b = 0; b < 27; ++b)
            T[a][b] = T1[NODE[a][0]][NODE[b][0]] * T1[NODE[a][1]][NODE[b][1]] *
                      T1[NODE[a][2]][NODE[b][2]];
    T_ready = 1;
}

/* Edge vectors of the derivatives of the trilinear map (Section 5), 0-based
 * nodes n0..n7 in Appendix A order:
 *   x_xi   = (n1-n0)(1-eta)(1-zeta) + (n2-n3)eta(1-zeta) + (n5-n4)(1-eta)zeta + (n6-n7)eta zeta
 *   x_eta  = (n3-n0)(1-xi)(1-zeta)  + (n2-n1)xi(1-zeta)  + (n7-n4)(1-xi)zeta  + (n6-n5)xi zeta
 *   x_zeta = (n4-n0)(1-xi)(1-eta)   + (n5-n1)xi(1-eta)   + (n7-n3)(1-xi)eta   + (n6-n2)xi eta  */
typedef struct {
    double ex[4][3], ey[4][3], ez[4][3];
    double M;   /* upper bound of 6 S_xi S_eta S_zeta, see `bounds` */
    int in_range;
} Hex;

static void hex_setup(const double p[8][3], Hex* h)
{
    static const int XI[4][2] = {{1, 0}, {2, 3}, {5, 4}, {6, 7}};
    static const int ETA[4][2] = {{3, 0}, {2, 1}, {7, 4}, {6, 5}};
    static const int ZETA[4][2] = {{4, 0}, {5, 1}, {7, 3}, {6, 2}};
    double s[3] = {0.0, 0.0, 0.0};
    for (int e = 0; e < 4; ++e)
        for (int d = 0; d < 3; ++d) {
            h->ex[e][d] = p[XI[e][0]][d] - p[XI[e][1]][d];
            h->ey[e][d] = p[ETA[e][0]][d] - p[ETA[e][1]][d];
            h->ez[e][d] = p[ZETA[e][0]][d] - p[ZETA[e][1]][d];
            s[0] = fmax(s[0], fabs(h->ex[e][d]));
            s[1] = fmax(s[1], fabs(h->ey[e][d]));
            s[2] = fmax(s[2], fabs(h->ez[e][d]));
        }
    /* Range guard: with every per-direction scale in [2^-300, 2^300] no product
     * formed below overflows, and underflow contributes far less than the
     * slack of the bounds.  Outside it the element goes to the exact tier. */
    const double lo = ldexp(1.0, -300), hi = ldexp(1.0, 300);
    h->in_range = 1;
    for (int d = 0; d < 3; ++d)
        if (!(s[d] >= lo && s[d] <= hi)) h->in_range = 0;
    h->M = 6.0 * s[0] * s[1] * s[2];
}

/* J at (xi, eta, zeta); the three derivative vectors are blended from the
 * edge vectors with the bilinear weights, then det[X Y Z] by cofactor
 * expansion along the first column. */
static double jacobian(const Hex* h, double xi, double eta, double zeta)
{
    const double wx[4] = {(1 - eta) * (1 - zeta), eta * (1 - zeta), (1 - eta) * zeta, eta * zeta};
    const double wy[4] = {(1 - xi) * (1 - zeta), xi * (1 - zeta), (1 - xi) * zeta, xi * zeta};
    const double wz[4] = {(1 - xi) * (1 - eta), xi * (1 - eta), (1 - xi) * eta, xi * eta};
    double X[3], Y[3], Z[3];
    for (int d = 0; d < 3; ++d) {
        X[d] = wx[0] * h->ex[0][d] + wx[1] * h->ex[1][d] + wx[2] * h->ex[2][d] + wx[3] * h->ex[3][d];
        Y[d] = wy[0] * h->ey[0][d] + wy[1] * h->ey[1][d] + wy[2] * h->ey[2][d] + wy[3] * h->ey[3][d];
        Z[d] = wz[0] * h->ez[0][d] + wz[1] * h->ez[1][d] + wz[2] * h->ez[2][d] + wz[3] * h->ez[3][d];
    }
    return X[0] * (Y[1] * Z[2] - Y[2] * Z[1]) - X[1] * (Y[0] * Z[2] - Y[2] * Z[0]) +
           X[2] * (Y[0] * Z[1] - Y[1] * Z[0]);
}

/* Samples c (Fig. 3 order) on the box lo + [0, size]^3 and b = T c. */
static void box_coefficients(const Hex* h, const double lo[3], double size, double c[27], double b[27])
{
    const double half = 0.5 * size;
    for (int a = 0; a < 27; ++a)
        c[a] = jacobian(h, lo[0] + NODE[a][0] * half, lo[1] + NODE[a][1] * half,
                        lo[2] + NODE[a][2] * half);
    for (int a = 0; a < 27; ++a) {
        double s = 0.0;
        for (int k = 0; k < 27; ++k) s += T[a][k] * c[k];
        b[a] = s;
    }
}

/*
 * bounds: rigorous forward error bounds for the FP64 values above.
 * u = 2^-53, gamma_k = k u / (1 - k u).  Let S_d be the largest |component|
 * of the four edge vectors of direction d (exact values), M = 6 S_xi S_eta S_zeta.
 *  - Each edge component is one subtraction: relative error <= u.
 *  - A blended derivative component is sum_i w_i e_i with exact dyadic weights,
 *    w_i >= 0, sum w_i = 1: one rounding per product and three per sum, so the
 *    error is <= gamma_5 S_d and |component| <= S_d.
 *  - det by cofactors without fused operations: <= 5 roundings on every
 *    product path, so <= gamma_5 perm(|X|,|Y|,|Z|) <= gamma_5 M (1+gamma_5)^3,
 *    plus the propagated input error M((1+gamma_5)^3 - 1).
 *    Hence |c^ - c| <= M((1+gamma_5)^4 - 1) <= 20.01 u M, and |c| <= M.
 *  - b = T c: the entries of T are signed powers of two (products exact); a
 *    sequential sum of 27 terms adds gamma_26 times the sum of |terms|; the
 *    absolute row sums of T are at most 27 (centre row: 8/8 + 12/2 + 6*2 + 8).
 *    Hence |b^ - b| <= 27 (20.01 u + gamma_26 (1 + 20.01 u)) M <= 1243 u M.
 *    Corner rows of T are unit rows, so corner coefficients carry the bound of c.
 *  - The computed scale M^ = fl(fl(6 S^_xi) S^_eta) S^_zeta with S^ >= (1-u) S
 *    satisfies M <= M^ (1 + 6.01 u).
 * Thresholds used: tau_c = 24 u M^ for values and corner coefficients,
 * tau_b = 1300 u M^ for the other coefficients.  A value x is certainly
 * positive when x > tau, certainly non-positive when x <= -tau, else fragile.
 */
#define U64 (1.0 / 9007199254740992.0) /* 2^-53 */

enum { FL_INVALID = 1, FL_UNDECIDED = 2, FL_FRAGILE = 4 };

typedef struct {
    const Hex* h;
    double tc, tb;
    int max_depth;
    int64_t nodes;         /* sub-boxes whose coefficients were computed */
    int deepest;           /* deepest level of a computed sub-box */
    double witness[3];     /* a point with J <= 0 when INVALID is found */
} Ctx;

static const int CORNER[8][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {0, 1, 0},
                                 {0, 0, 1}, {1, 0, 1}, {1, 1, 1}, {0, 1, 1}};

/* Section 6, recursive_subdivision: the node at `level` on box lo + [0,size]^3
 * is split in 8; a child with a corner coefficient <= 0 proves invalidity; a
 * child whose other 19 coefficients are > 0 is positive; otherwise the child
 * is subdivided while its level is below the cap. */
static int subdivide(Ctx* x, const double lo[3], double size, int level)
{
    int flags = 0;
    const double hs = 0.5 * size;
    for (int ch = 0; ch < 8; ++ch) {
        double clo[3], c[27], b[27];
        for (int d = 0; d < 3; ++d) clo[d] = lo[d] + CORNER[ch][d] * hs;
        box_coefficients(x->h, clo, hs, c, b);
        x->nodes++;
        if (level + 1 > x->deepest) x->deepest = level + 1;
        double mn8 = b[0];
        int arg8 = 0;
        for (int a = 1; a < 8; ++a)
            if (b[a] < mn8) { mn8 = b[a]; arg8 = a; }
        double mn19 = b[8];
        for (int a = 9; a < 27; ++a) mn19 = fmin(mn19, b[a]);
        if (mn8 <= -x->tc) {
            for (int d = 0; d < 3; ++d) x->witness[d] = clo[d] + NODE[arg8][d] * 0.5 * hs;
            return flags | FL_INVALID;
        }
        if (mn8 <= x->tc) { flags |= FL_FRAGILE; continue; }
        if (mn19 > x->tb) continue;
        if (level + 1 < x->max_depth) {
            flags |= subdivide(x, clo, hs, level + 1);
            if (flags & FL_INVALID) return flags;
        } else if (mn19 <= -x->tb) {
            flags |= FL_UNDECIDED;
        } else {
            flags |= FL_FRAGILE;
        }
    }
    return flags;
}

static int all_finite(const double p[8][3])
{
    for (int k = 0; k < 8; ++k)
        for (int d = 0; d < 3; ++d)
            if (!isfinite(p[k][d])) return 0;
    return 1;
}

static void gather(const double* pts, const int32_t* conn, int64_t e, double p[8][3])
{
    for (int k = 0; k < 8; ++k) {
        const double* q = conn ? pts + 3 * (int64_t)conn[8 * e + k] : pts + 24 * e + 3 * k;
        for (int d = 0; d < 3; ++d) p[k][d] = q[d];
    }
}

/* One element, Section 6 steps 1-5.  Returns the verdict code. */
static int check_one(const double p[8][3], int max_depth, double* min_coeff, int* level,
                     int64_t* nodes, double witness[3])
{
    *level = 0;
    *nodes = 0;
    if (!all_finite(p)) { *min_coeff = NAN; return OV_BAD_INPUT; }
    Hex h;
    hex_setup(p, &h);
    double c[27], b[27];
    const double lo[3] = {0.0, 0.0, 0.0};
    box_coefficients(&h, lo, 1.0, c, b);
    double mn = b[0];
    for (int a = 1; a < 27; ++a) mn = fmin(mn, b[a]);
    *min_coeff = mn;
    if (!h.in_range) return OV_FRAGILE;
    Ctx x = {&h, 24.0 * U64 * h.M, 1300.0 * U64 * h.M, max_depth, 0, 0, {0, 0, 0}};
    /* Step 2: the 20 values at corners and edge midpoints. */
    double m20 = c[0];
    int arg = 0;
    for (int a = 1; a < 20; ++a)
        if (c[a] < m20) { m20 = c[a]; arg = a; }
    if (m20 <= -x.tc) {
        for (int d = 0; d < 3; ++d) witness[d] = 0.5 * NODE[arg][d];
        return OV_INVALID;
    }
    if (m20 <= x.tc) return OV_FRAGILE;
    /* Step 4: b_9..b_27. */
    double m19 = b[8];
    for (int a = 9; a < 27; ++a) m19 = fmin(m19, b[a]);
    if (m19 > x.tb) return OV_VALID;
    /* Step 5. */
    if (max_depth <= 0) return m19 <= -x.tb ? OV_UNDECIDED : OV_FRAGILE;
    int f = subdivide(&x, lo, 1.0, 0);
    *nodes = x.nodes;
    *level = x.deepest;
    if (f & FL_INVALID) {
        memcpy(witness, x.witness, sizeof x.witness);
        return OV_INVALID;
    }
    if (f & FL_FRAGILE) return OV_FRAGILE;
    if (f & FL_UNDECIDED) return OV_UNDECIDED;
    return OV_VALID;
}

/* ---- exported entry points (called through ctypes by oracle/__init__.py) ---- */

/* Verdicts for n hexahedra.  pts: [n,8,3] when conn is NULL, else vertex
 * array [*,3] indexed by conn [n,8] (Appendix A corner order).  verdict
 * receives 0 INVALID, 1 VALID, 2 UNDECIDED, 3 BAD_INPUT or 255 FRAGILE (to be
 * settled by the exact tier).  min_coeff: [n] top-level min of the 27
 * coefficients.  level, nodes, witness: optional ([n], [n], [n,3]).
 * Returns the number of FRAGILE elements. */
int64_t oracle_check(const double* pts, const int32_t* conn, int64_t n, int max_depth, int nthreads,
                     uint8_t* verdict, double* min_coeff, int32_t* level, int64_t* nodes,
                     double* witness)
{
    if (!T_ready) build_T();
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int64_t fragile = 0;
#pragma omp parallel for schedule(static) reduction(+ : fragile)
    for (int64_t e = 0; e < n; ++e) {
        double p[8][3], w[3] = {NAN, NAN, NAN}, mn;
        int lv;
        int64_t nd;
        gather(pts, conn, e, p);
        int v = check_one(p, max_depth, &mn, &lv, &nd, w);
        verdict[e] = (uint8_t)v;
        if (min_coeff) min_coeff[e] = mn;
        if (level) level[e] = lv;
        if (nodes) nodes[e] = nd;
        if (witness)
            for (int d = 0; d < 3; ++d) witness[3 * e + d] = w[d];
        if (v == OV_FRAGILE) fragile++;
    }
    return fragile;
}

/* The 27 top-level Bezier coefficients (Fig. 3 order) of n hexahedra: [n,27].
 * samples (optional): the 27 values c = J(xi_alpha), [n,27]. */
void oracle_coefficients(const double* pts, const int32_t* conn, int64_t n, int nthreads,
                         double* coeffs, double* samples)
{
    if (!T_ready) build_T();
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < n; ++e) {
        double p[8][3], c[27];
        const double lo[3] = {0.0, 0.0, 0.0};
        Hex h;
        gather(pts, conn, e, p);
        hex_setup(p, &h);
        box_coefficients(&h, lo, 1.0, c, coeffs + 27 * e);
        if (samples) memcpy(samples + 27 * e, c, sizeof c);
    }
}

/* The bound scale M^ of each element (see `bounds`), [n]. */
void oracle_scale(const double* pts, const int32_t* conn, int64_t n, double* scale)
{
    for (int64_t e = 0; e < n; ++e) {
        double p[8][3];
        Hex h;
        gather(pts, conn, e, p);
        hex_setup(p, &h);
        scale[e] = h.M;
    }
}

/* J at one point of one hexahedron (8 points, Appendix A order). */
double oracle_jacobian(const double* p8, double xi, double eta, double zeta)
{
    double p[8][3];
    Hex h;
    memcpy(p, p8, sizeof p);
    hex_setup(p, &h);
    return jacobian(&h, xi, eta, zeta);
}

/* The matrix T of Table 1 as this file forms it, [27,27] row-major. */
void oracle_T(double* out)
{
    if (!T_ready) build_T();
    memcpy(out, T, sizeof T);
}

/* Error-bound constants, so that tests can check observed error against them:
 * out[0] = tau_c / (u M^), out[1] = tau_b / (u M^), out[2] = u. */
void oracle_bound_constants(double* out)
{
    out[0] = 24.0;
    out[1] = 1300.0;
    out[2] = U64;
}

/* ---- minimum of J to a tolerance -------------------------------------------
 *
 * The bounds of Section 3.1: on any box, the smallest of its 27 Bezier
 * coefficients is a lower bound of J on the box (convex hull property), and
 * each of its 8 corner coefficients is a value of J, so the smallest corner
 * value met anywhere is an upper bound of min J.  Subdividing sharpens both
 * (the method recalled in the introduction, which computes min J to any
 * prescribed tolerance).  Boxes are processed level by level:
 *
 *   U_L  = the smallest corner value over every box of levels 0..L;
 *   a box B of level L is retired when min_27(B) >= U_L - tol, or when L is the
 *        depth cap (then the element is reported as capped); retired boxes
 *        cover the domain, so LB = min over them of min_27(B) <= min J;
 *   every other box is split into its 8 children (level L + 1).
 *
 * The decisions at level L use U_L only (not the corners of level L + 1), so
 * the result does not depend on the order boxes are visited.  Without the
 * cap, every retired box has min_27 >= U_final - tol, hence U_final - LB <= tol.
 * tol = rtol * M^ / 6 (M^ / 6 = S_xi S_eta S_zeta, the element's J scale).
 *
 * Outputs are widened by the error bounds (coefficients tau_b, corner values
 * tau_c: the corner rows of T are unit rows, so a corner coefficient is the
 * sample itself) and rounded outwards: lo <= min J <= hi.
 * status: 0 converged, 1 depth cap reached, 3 non-finite input, 4 a scale
 * outside the guard range (no bounds). */
enum { MJ_CONVERGED = 0, MJ_CAPPED = 1, MJ_BAD_INPUT = 3, MJ_OUT_OF_RANGE = 4 };

typedef struct {
    double lo[3], size, min27;
} MjBox;

static double mj_min27(const double b[27])
{
    double m = b[0];
    for (int a = 1; a < 27; ++a) m = fmin(m, b[a]);
    return m;
}

static double mj_min_corner(const double b[27])
{
    double m = b[0];
    for (int a = 1; a < 8; ++a) m = fmin(m, b[a]);
    return m;
}

static int min_jacobian_one(const double p[8][3], double rtol, int max_depth, double* lo_out,
                            double* hi_out, int* level_out, int64_t* boxes_out)
{
    *lo_out = *hi_out = NAN;
    *level_out = 0;
    *boxes_out = 1;
    if (!all_finite(p)) return MJ_BAD_INPUT;
    Hex h;
    hex_setup(p, &h);
    if (!h.in_range) return MJ_OUT_OF_RANGE;
    const double tol = rtol * h.M / 6.0;
    double c[27], b[27];
    const double root[3] = {0.0, 0.0, 0.0};
    box_coefficients(&h, root, 1.0, c, b);
    double U = mj_min_corner(b);
    double LB = INFINITY;
    int capped = 0;
    int64_t n = 1, cap = 16;
    MjBox* F = (MjBox*)malloc(sizeof(MjBox) * cap);
    F[0].lo[0] = F[0].lo[1] = F[0].lo[2] = 0.0;
    F[0].size = 1.0;
    F[0].min27 = mj_min27(b);
    for (int L = 0; n > 0; ++L) {
        double U_next = U;
        int64_t m = 0, mcap = 16;
        MjBox* G = (MjBox*)malloc(sizeof(MjBox) * mcap);
        for (int64_t i = 0; i < n; ++i) {
            const MjBox* B = &F[i];
            if (B->min27 >= U - tol || L >= max_depth) {
                LB = fmin(LB, B->min27);
                if (!(B->min27 >= U - tol)) capped = 1;
                continue;
            }
            const double hs = 0.5 * B->size;
            for (int ch = 0; ch < 8; ++ch) {
                if (m == mcap) {
                    mcap *= 2;
                    G = (MjBox*)realloc(G, sizeof(MjBox) * mcap);
                }
                MjBox* K = &G[m++];
                for (int d = 0; d < 3; ++d) K->lo[d] = B->lo[d] + CORNER[ch][d] * hs;
                K->size = hs;
                box_coefficients(&h, K->lo, hs, c, b);
                K->min27 = mj_min27(b);
                U_next = fmin(U_next, mj_min_corner(b));
            }
        }
        free(F);
        F = G;
        n = m;
        U = U_next;
        *boxes_out += m;
        if (m > 0) *level_out = L + 1;
    }
    free(F);
    *lo_out = nextafter(LB - 1300.0 * U64 * h.M, -INFINITY);
    *hi_out = nextafter(U + 24.0 * U64 * h.M, INFINITY);
    return capped ? MJ_CAPPED : MJ_CONVERGED;
}

/* Certified bounds of min J over [0,1]^3 for n hexahedra (layout as in
 * oracle_check).  rtol > 0; lo, hi: [n]; status: [n]; level, boxes:
 * optional [n] (deepest level reached, boxes whose coefficients were formed). */
void oracle_min_jacobian(const double* pts, const int32_t* conn, int64_t n, double rtol, int max_depth,
                         int nthreads, double* lo, double* hi, uint8_t* status, int32_t* level,
                         int64_t* boxes)
{
    if (!T_ready) build_T();
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t e = 0; e < n; ++e) {
        double p[8][3];
        int lv;
        int64_t nb;
        gather(pts, conn, e, p);
        const int st = min_jacobian_one(p, rtol, max_depth, lo + e, hi + e, &lv, &nb);
        status[e] = (uint8_t)st;
        if (level) level[e] = lv;
        if (boxes) boxes[e] = nb;
    }
}

/* ---- corner-only test and corner quality ------------------------------------
 *
 * Test 1 of the comparison in Section 7: the 8 corner tetrahedra must have
 * positive volume, i.e. the 8 values of J at the corners (the corner
 * coefficients b_1..b_8) must be positive.  A corner is a point of the
 * element, so the test is a necessary condition of validity: it may accept
 * invalid elements ("false valid") but never rejects a valid one.
 *
 * Corner quality (the measure quoted for Fig. 7): the minimum over the 8
 * corners of the scaled Jacobian J_c / (|e_xi| |e_eta| |e_zeta|), e_* the
 * three edge vectors that leave the corner; a corner with a zero-length edge
 * counts as 0.
 *
 * test1: 1 VALID (all corner values certainly > 0), 0 INVALID (one certainly
 * <= 0), 3 BAD_INPUT (non-finite coordinate), 255 FRAGILE (a corner sign is
 * not certified by tau_c, or a scale outside the guard: the exact tier
 * decides).  quality: NaN for BAD_INPUT and outside the guard range. */
static int corner_test_one(const double p[8][3], double* quality)
{
    *quality = NAN;
    if (!all_finite(p)) return OV_BAD_INPUT;
    Hex h;
    hex_setup(p, &h);
    const double tc = 24.0 * U64 * h.M;
    int certain_pos = 1, certain_neg = 0;
    double q = INFINITY;
    for (int c = 0; c < 8; ++c) {
        const int i = CORNER[c][0], j = CORNER[c][1], k = CORNER[c][2];
        const double J = jacobian(&h, i, j, k);
        if (J <= -tc) certain_neg = 1;
        if (!(J > tc)) certain_pos = 0;
        const double* a = h.ex[j + 2 * k];
        const double* b = h.ey[i + 2 * k];
        const double* z = h.ez[i + 2 * j];
        const double den = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]) *
                           sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]) *
                           sqrt(z[0] * z[0] + z[1] * z[1] + z[2] * z[2]);
        q = fmin(q, den > 0.0 ? J / den : 0.0);
    }
    if (!h.in_range) return OV_FRAGILE;
    *quality = q;
    if (certain_neg) return OV_INVALID;
    if (certain_pos) return OV_VALID;
    return OV_FRAGILE;
}

/* Test 1 and corner quality of n hexahedra (layout as in oracle_check).
 * Returns the number of FRAGILE elements. */
int64_t oracle_corner_test(const double* pts, const int32_t* conn, int64_t n, int nthreads, uint8_t* test1,
                           double* quality)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int64_t fragile = 0;
#pragma omp parallel for schedule(static) reduction(+ : fragile)
    for (int64_t e = 0; e < n; ++e) {
        double p[8][3];
        gather(pts, conn, e, p);
        const int v = corner_test_one(p, quality + e);
        test1[e] = (uint8_t)v;
        if (v == OV_FRAGILE) fragile++;
    }
    return fragile;
}

/* ---- linear quadrangles (Section 2.1) ---------------------------------------
 *
 * The bilinear map of [0,1]^2 with corners n1..n4 at (0,0) (1,0) (1,1) (0,1);
 * its Jacobian matrix has columns x_xi = (n2-n1)(1-eta) + (n3-n4) eta and
 * x_eta = (n4-n1)(1-xi) + (n3-n2) xi, and J = det[x_xi x_eta] is bilinear, so
 * its minimum over the element is one of the four corner values.  Verdict:
 * INVALID when a corner value is <= 0, VALID when all four are > 0 (the same
 * strict reading as for hexahedra).  The corner values come from evaluating
 * the Jacobian matrix at each corner (not from the per-corner cross products
 * the paper writes out).  Error: each edge component is one rounded
 * difference, each product adds one rounding and the difference one more, so
 * |J^ - J| <= ((1+u)^3 - 1) 2 S^2 + u 2 S^2 (1 + 3.01 u) <= 8.001 u S^2, S the
 * largest |component| of the four edge vectors; the threshold is 9 u S^2.
 * min_j: the smallest corner value.  verdict 255 (FRAGILE): a sign not
 * certified (or S outside [2^-450, 2^450]), settled exactly. */
static int quad_one(const double p[4][2], double* min_j)
{
    for (int k = 0; k < 4; ++k)
        if (!isfinite(p[k][0]) || !isfinite(p[k][1])) {
            *min_j = NAN;
            return OV_BAD_INPUT;
        }
    double ex0[2], ex1[2], ey0[2], ey1[2], s = 0.0;
    for (int d = 0; d < 2; ++d) {
        ex0[d] = p[1][d] - p[0][d];   /* eta = 0 */
        ex1[d] = p[2][d] - p[3][d];   /* eta = 1 */
        ey0[d] = p[3][d] - p[0][d];   /* xi = 0 */
        ey1[d] = p[2][d] - p[1][d];   /* xi = 1 */
        s = fmax(s, fmax(fmax(fabs(ex0[d]), fabs(ex1[d])), fmax(fabs(ey0[d]), fabs(ey1[d]))));
    }
    static const int XY[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
    double mn = INFINITY;
    int neg = 0, pos = 1;
    const double tau = 9.0 * U64 * s * s;
    for (int k = 0; k < 4; ++k) {
        const double xi = XY[k][0], eta = XY[k][1];
        double X[2], Y[2];
        for (int d = 0; d < 2; ++d) {
            X[d] = ex0[d] * (1 - eta) + ex1[d] * eta;
            Y[d] = ey0[d] * (1 - xi) + ey1[d] * xi;
        }
        const double J = X[0] * Y[1] - X[1] * Y[0];
        mn = fmin(mn, J);
        if (J <= -tau) neg = 1;
        if (!(J > tau)) pos = 0;
    }
    *min_j = mn;
    /* guard: s^2 must neither overflow nor lose the bound to underflow */
    if (!(s >= ldexp(1.0, -450) && s <= ldexp(1.0, 450))) return OV_FRAGILE;
    if (neg) return OV_INVALID;
    if (pos) return OV_VALID;
    return OV_FRAGILE;
}

/* Quadrangles: pts [n,4,2] when conn is NULL, else [*,2] indexed by conn [n,4]
 * (corners in the order (0,0) (1,0) (1,1) (0,1)).  Returns #FRAGILE. */
int64_t oracle_quad_check(const double* pts, const int32_t* conn, int64_t n, int nthreads, uint8_t* verdict,
                          double* min_j)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int64_t fragile = 0;
#pragma omp parallel for schedule(static) reduction(+ : fragile)
    for (int64_t e = 0; e < n; ++e) {
        double p[4][2];
        for (int k = 0; k < 4; ++k) {
            const double* q = conn ? pts + 2 * (int64_t)conn[4 * e + k] : pts + 8 * e + 2 * k;
            p[k][0] = q[0];
            p[k][1] = q[1];
        }
        const int v = quad_one(p, min_j + e);
        verdict[e] = (uint8_t)v;
        if (v == OV_FRAGILE) fragile++;
    }
    return fragile;
}
