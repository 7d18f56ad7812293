"""Exact tier of the oracle: TEST INFRASTRUCTURE, not part of the library.

The validity algorithm of Johnen, Weill & Remacle (IMR 2017, Section 6) with
every quantity a ``fractions.Fraction``.  Double-precision inputs are exact
rationals, the Bernstein transform T (Section 3.2, Table 1) has rational
entries and subdivision only evaluates J at dyadic points, so every sign
decision below is exact.  The C oracle (hexval_oracle.c) hands elements whose
floating-point decisions are not certified to this module; tests also call it
directly on small inputs.

Steps, in the paper's order and notation:
  * J(xi) = det[x_xi x_eta x_zeta] of the trilinear map of Appendix A, the
    derivatives blended from edge vectors as in Section 5;
  * c_alpha = J at the 27 nodes of Fig. 3, b = T c (Section 3.2);
  * step 2: some c_1..c_20 <= 0 -> INVALID; step 4: all b_9..b_27 > 0 -> VALID;
  * step 5: recursive subdivision; a sub-box's coefficients are T applied to
    J sampled at the sub-box's 27 nodes; a child with a corner coefficient
    <= 0 -> INVALID; a child with b_9..b_27 > 0 is positive; otherwise it is
    subdivided while its level is below the cap, else it is UNDECIDED.
The readings (strict positivity, depth cap, BAD_INPUT, min of the top-level
coefficients) are the same as in the C oracle.
"""
from fractions import Fraction
import math

INVALID, VALID, UNDECIDED, BAD_INPUT = 0, 1, 2, 3

# Fig. 3 node positions in half-steps (0, 1, 2) along xi, eta, zeta.
NODE = [
    (0, 0, 0), (2, 0, 0), (2, 2, 0), (0, 2, 0), (0, 0, 2), (2, 0, 2), (2, 2, 2), (0, 2, 2),
    (1, 0, 0), (2, 1, 0), (1, 2, 0), (0, 1, 0), (0, 0, 1), (2, 0, 1),
    (2, 2, 1), (0, 2, 1), (1, 0, 2), (2, 1, 2), (1, 2, 2), (0, 1, 2),
    (1, 1, 0), (1, 0, 1), (2, 1, 1), (1, 2, 1), (0, 1, 1), (1, 1, 2),
    (1, 1, 1),
]
CORNER = [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)]

_H = Fraction(1, 2)
# Inverse of the 1D order-2 Bernstein collocation matrix on t = 0, 1/2, 1.
T1 = [[Fraction(1), Fraction(0), Fraction(0)],
      [-_H, Fraction(2), -_H],
      [Fraction(0), Fraction(0), Fraction(1)]]
T = [[T1[NODE[a][0]][NODE[b][0]] * T1[NODE[a][1]][NODE[b][1]] * T1[NODE[a][2]][NODE[b][2]]
      for b in range(27)] for a in range(27)]
_T_SPARSE = [[(k, t) for k, t in enumerate(row) if t != 0] for row in T]


def _sub(p, q):
    return (p[0] - q[0], p[1] - q[1], p[2] - q[2])


def edge_vectors(P):
    """The four edge vectors of each derivative (Section 5), 0-based nodes."""
    ex = [_sub(P[1], P[0]), _sub(P[2], P[3]), _sub(P[5], P[4]), _sub(P[6], P[7])]
    ey = [_sub(P[3], P[0]), _sub(P[2], P[1]), _sub(P[7], P[4]), _sub(P[6], P[5])]
    ez = [_sub(P[4], P[0]), _sub(P[5], P[1]), _sub(P[7], P[3]), _sub(P[6], P[2])]
    return ex, ey, ez


def _blend(e, w):
    return tuple(w[0] * e[0][d] + w[1] * e[1][d] + w[2] * e[2][d] + w[3] * e[3][d] for d in range(3))


def det3(X, Y, Z):
    """det[X Y Z] (columns) = X . (Y x Z)."""
    return (X[0] * (Y[1] * Z[2] - Y[2] * Z[1]) - X[1] * (Y[0] * Z[2] - Y[2] * Z[0])
            + X[2] * (Y[0] * Z[1] - Y[1] * Z[0]))


def jacobian(edges, xi, eta, zeta):
    ex, ey, ez = edges
    X = _blend(ex, ((1 - eta) * (1 - zeta), eta * (1 - zeta), (1 - eta) * zeta, eta * zeta))
    Y = _blend(ey, ((1 - xi) * (1 - zeta), xi * (1 - zeta), (1 - xi) * zeta, xi * zeta))
    Z = _blend(ez, ((1 - xi) * (1 - eta), xi * (1 - eta), (1 - xi) * eta, xi * eta))
    return det3(X, Y, Z)


def box_samples(edges, lo, size):
    half = size / 2
    return [jacobian(edges, lo[0] + n[0] * half, lo[1] + n[1] * half, lo[2] + n[2] * half)
            for n in NODE]


def apply_T(c):
    return [sum((t * c[k] for k, t in row), Fraction(0)) for row in _T_SPARSE]


def to_fractions(points):
    """8 points (any nested sequence of floats) -> tuple of Fraction triples, or
    None when a coordinate is not finite."""
    out = []
    for p in points:
        q = []
        for v in p:
            v = float(v)
            if not math.isfinite(v):
                return None
            q.append(Fraction(v))
        out.append(tuple(q))
    return tuple(out)


def coefficients(points):
    """The 27 exact top-level Bezier coefficients (Fig. 3 order) and the 27
    exact samples c."""
    P = to_fractions(points)
    edges = edge_vectors(P)
    c = box_samples(edges, (Fraction(0),) * 3, Fraction(1))
    return apply_T(c), c


class _Tree:
    def __init__(self, edges, max_depth):
        self.edges = edges
        self.max_depth = max_depth
        self.nodes = 0
        self.deepest = 0
        self.undecided = False
        self.witness = None

    def subdivide(self, lo, size, level):
        """True when a non-positive value was found below this node."""
        hs = size / 2
        for ch in CORNER:
            clo = tuple(lo[d] + ch[d] * hs for d in range(3))
            b = apply_T(box_samples(self.edges, clo, hs))
            self.nodes += 1
            self.deepest = max(self.deepest, level + 1)
            m8 = min(range(8), key=lambda a: b[a])
            if b[m8] <= 0:
                self.witness = tuple(clo[d] + NODE[m8][d] * hs / 2 for d in range(3))
                return True
            if min(b[8:]) > 0:
                continue
            if level + 1 < self.max_depth:
                if self.subdivide(clo, hs, level + 1):
                    return True
            else:
                self.undecided = True
        return False


def validity(points, max_depth=6):
    """Exact verdict of one hexahedron (8 points, Appendix A order).

    Returns a dict: verdict (0 INVALID, 1 VALID, 2 UNDECIDED, 3 BAD_INPUT),
    min_coeff (exact Fraction, None for BAD_INPUT), level (deepest sub-box level
    computed), nodes (sub-boxes computed) and witness (a point with J <= 0 when
    INVALID)."""
    P = to_fractions(points)
    if P is None:
        return dict(verdict=BAD_INPUT, min_coeff=None, level=0, nodes=0, witness=None)
    edges = edge_vectors(P)
    zero = (Fraction(0),) * 3
    c = box_samples(edges, zero, Fraction(1))
    b = apply_T(c)
    res = dict(min_coeff=min(b), level=0, nodes=0, witness=None)
    # Step 2: the 20 values at corners and edge midpoints.
    a = min(range(20), key=lambda k: c[k])
    if c[a] <= 0:
        res.update(verdict=INVALID, witness=tuple(Fraction(n, 2) for n in NODE[a]))
        return res
    # Step 4.
    if min(b[8:]) > 0:
        res.update(verdict=VALID)
        return res
    # Step 5.
    if max_depth <= 0:
        res.update(verdict=UNDECIDED)
        return res
    tree = _Tree(edges, max_depth)
    invalid = tree.subdivide(zero, Fraction(1), 0)
    res.update(level=tree.deepest, nodes=tree.nodes)
    if invalid:
        res.update(verdict=INVALID, witness=tree.witness)
    else:
        res.update(verdict=UNDECIDED if tree.undecided else VALID)
    return res


def corner_test(points):
    """Test 1 of Section 7 in exact arithmetic: VALID when the 8 corner values
    of J are all > 0, else INVALID (BAD_INPUT for a non-finite coordinate)."""
    P = to_fractions(points)
    if P is None:
        return BAD_INPUT
    edges = edge_vectors(P)
    for n in NODE[:8]:
        if jacobian(edges, Fraction(n[0], 2), Fraction(n[1], 2), Fraction(n[2], 2)) <= 0:
            return INVALID
    return VALID


def quad_validity(points):
    """Linear quadrangle (Section 2.1) in exact arithmetic: the Jacobian matrix
    of the bilinear map at each corner, VALID when all four determinants are
    > 0, else INVALID (BAD_INPUT for a non-finite coordinate)."""
    P = []
    for p in points:
        if not all(math.isfinite(float(v)) for v in p):
            return BAD_INPUT
        P.append((Fraction(float(p[0])), Fraction(float(p[1]))))
    for xi, eta in ((0, 0), (1, 0), (1, 1), (0, 1)):
        X = [(P[1][d] - P[0][d]) * (1 - eta) + (P[2][d] - P[3][d]) * eta for d in range(2)]
        Y = [(P[3][d] - P[0][d]) * (1 - xi) + (P[2][d] - P[1][d]) * xi for d in range(2)]
        if X[0] * Y[1] - X[1] * Y[0] <= 0:
            return INVALID
    return VALID
