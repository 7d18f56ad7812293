"""Pins of the oracle's constants against the paper's tables and the
mathematics of Sections 3-5 (CPU only)."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import exact
from tests import _ref

pytestmark = pytest.mark.filterwarnings("ignore")


def _frac_matrix(a):
    return [[Fraction(float(x)) for x in row] for row in a]


def _matmul(A, B):
    return [[sum(A[i][k] * B[k][j] for k in range(len(B))) for j in range(len(B[0]))]
            for i in range(len(A))]


def _inverse(A):
    n = len(A)
    M = [list(row) + [Fraction(int(i == j)) for j in range(n)] for i, row in enumerate(A)]
    for c in range(n):
        p = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        piv = M[c][c]
        M[c] = [v / piv for v in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [a - f * b for a, b in zip(M[r], M[c])]
    return [row[n:] for row in M]


def test_node_order_matches_fig3():
    assert [tuple(n) for n in exact.NODE] == _ref.NODES


def test_T_equals_printed_table1():
    printed = _ref.read_table("table1_T.txt", 27, 27)
    assert _frac_matrix(oracle.T_matrix()) == printed
    assert exact.T == printed


def test_T_is_inverse_of_bernstein_collocation():
    # Section 3.2: A_{alpha beta} = B_beta(xi_alpha), T = A^-1.
    A = _ref.collocation_matrix()
    T = _ref.read_table("table1_T.txt", 27, 27)
    I = _matmul(T, A)
    assert all(I[i][j] == (1 if i == j else 0) for i in range(27) for j in range(27))


def _monomial_basis_20():
    """Monomials xi^i eta^j zeta^k (i,j,k <= 2) without the 7 of the Corollary
    of Section 4 (m220 m202 m022 m221 m212 m122 m222)."""
    zero = {(2, 2, 0), (2, 0, 2), (0, 2, 2), (2, 2, 1), (2, 1, 2), (1, 2, 2), (2, 2, 2)}
    return [(i, j, k) for k in range(3) for j in range(3) for i in range(3)
            if (i, j, k) not in zero]


def _derived_Q():
    """Q from first principles: for a basis of the 20-dimensional space of
    Jacobian determinants, Q maps the values at nodes 1..20 to T (values at all
    27 nodes)."""
    T = _ref.read_table("table1_T.txt", 27, 27)
    basis = _monomial_basis_20()
    pts = [tuple(Fraction(c, 2) for c in n) for n in _ref.NODES]
    C = [[p[0] ** m[0] * p[1] ** m[1] * p[2] ** m[2] for m in basis] for p in pts]  # 27x20
    B = _matmul(T, C)
    V = [row for row in C[:20]]
    return _matmul(B, _inverse(V))


def test_Q_equals_printed_table3_and_first_principles():
    printed = _ref.read_table("table3_Q.txt", 27, 20)
    assert _derived_Q() == printed


def test_table2_printed_signs_are_flipped():
    # Section 4: b_21..27 = R b_1..20.  Derive R from Table 3 (b = Q v with
    # b_1..20 = T20 v) and compare with the printed Table 2.
    Q = _ref.read_table("table3_Q.txt", 27, 20)
    T20 = [row[:20] for row in _ref.read_table("table1_T.txt", 27, 27)[:20]]
    R = _matmul(Q[20:], _inverse(T20))
    printed = _ref.read_table("table2_printed.txt", 7, 20, first_row=21)
    assert R == [[-x for x in row] for row in printed]
    assert R != printed


def test_row_sums():
    # Q rows sum to 1 (a constant J has all coefficients equal);
    # absolute row sums 1, 3, 7, 11 for corner, edge, face, centre rows.
    Q = _ref.read_table("table3_Q.txt", 27, 20)
    assert all(sum(r) == 1 for r in Q)
    assert [sum(abs(x) for x in Q[a]) for a in (0, 8, 20, 26)] == [1, 3, 7, 11]


@pytest.mark.parametrize("seed", range(4))
def test_Q_of_20_values_equals_T_of_27_samples_exactly(seed):
    # Corollary of Section 4 + Section 5: for any linear hexahedron the 27
    # coefficients are Q applied to the 20 values at corners and edge midpoints.
    rng = np.random.default_rng(seed)
    P = rng.integers(-40, 41, size=(8, 3)) / 16.0 + np.array(
        [[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0], [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]])
    b, c = exact.coefficients(P)
    Q = _ref.read_table("table3_Q.txt", 27, 20)
    bq = [sum(Q[a][k] * c[k] for k in range(20)) for a in range(27)]
    assert bq == b


def test_tetrahedron_identities_section5():
    # J_1 = det(v12, v14, v15) = 6 vol(n1,n2,n4,n5) and
    # J_9 = 6 vol(n1, n2, (n4+n3)/2, (n5+n6)/2), exact.
    rng = np.random.default_rng(7)
    P = [tuple(Fraction(int(x), 8) for x in row) for row in rng.integers(-30, 31, size=(8, 3))]

    def sub(p, q):
        return tuple(a - b for a, b in zip(p, q))

    def mid(p, q):
        return tuple((a + b) / 2 for a, b in zip(p, q))

    def vol6(a, b, c, d):
        return exact.det3(sub(b, a), sub(c, a), sub(d, a))

    n = P  # 0-based: n1 = P[0]
    b, c = exact.coefficients([[float(x) for x in p] for p in P])
    assert c[0] == vol6(n[0], n[1], n[3], n[4])
    assert c[8] == vol6(n[0], n[1], mid(n[3], n[2]), mid(n[4], n[5]))
    # and against the shape-function form of Appendix A
    assert c[0] == _ref.jacobian_shape(P, Fraction(0), Fraction(0), Fraction(0))
    assert c[8] == _ref.jacobian_shape(P, Fraction(1, 2), Fraction(0), Fraction(0))


def test_samples_match_shape_function_jacobian():
    # The oracle's edge-vector form of the derivatives (Section 5) against the
    # shape-function gradients of Appendix A, all 27 nodes, exact.
    rng = np.random.default_rng(3)
    P = rng.integers(-64, 65, size=(8, 3)) / 32.0
    _, c = exact.coefficients(P)
    Pf = [tuple(Fraction(float(x)) for x in p) for p in P]
    for a, node in enumerate(_ref.NODES):
        xi = [Fraction(v, 2) for v in node]
        assert c[a] == _ref.jacobian_shape(Pf, *xi)
    # the C oracle's samples agree to rounding
    _, cs = oracle.coefficients(P[None], samples=True)
    assert np.allclose(cs[0], [float(x) for x in c], rtol=0, atol=1e-13)
