"""Pins of the oracle's linear-quadrangle validity (Section 2.1) against closed
forms, the paper's corner relation, exact arithmetic and a dense grid (CPU)."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import exact

SQ = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], dtype=np.float64)


def _q(P):
    r = oracle.quad_check(np.asarray(P, dtype=np.float64)[None])
    return int(r["verdict"][0]), float(r["min_j"][0])


def _jacobian_grid(P, m):
    """J of the bilinear map on an (m+1)^2 grid, from the shape functions."""
    t = np.linspace(0, 1, m + 1)
    xi, eta = np.meshgrid(t, t, indexing="ij")
    dxi = [-(1 - eta), (1 - eta), eta, -eta]
    deta = [-(1 - xi), -xi, xi, (1 - xi)]
    Xx = sum(dxi[k] * P[k][0] for k in range(4))
    Xy = sum(dxi[k] * P[k][1] for k in range(4))
    Yx = sum(deta[k] * P[k][0] for k in range(4))
    Yy = sum(deta[k] * P[k][1] for k in range(4))
    return Xx * Yy - Xy * Yx


def _corner_values_exact(P):
    F = [(Fraction(float(x)), Fraction(float(y))) for x, y in P]
    out = []
    for xi, eta in ((0, 0), (1, 0), (1, 1), (0, 1)):
        X = [(F[1][d] - F[0][d]) * (1 - eta) + (F[2][d] - F[3][d]) * eta for d in range(2)]
        Y = [(F[3][d] - F[0][d]) * (1 - xi) + (F[2][d] - F[1][d]) * xi for d in range(2)]
        out.append(X[0] * Y[1] - X[1] * Y[0])
    return out


def test_square_and_parallelogram():
    assert _q(SQ) == (oracle.VALID, 1.0)
    A = np.array([[2.0, 0.5], [-0.3, 1.5]])
    v, m = _q(SQ @ A.T + [3.0, -1.0])
    assert v == oracle.VALID and abs(m - np.linalg.det(A)) < 1e-15


def test_corner_relation_j1_plus_j3_equals_j2_plus_j4():
    # Section 2.1 (the areas of the corner triangles); exact on dyadic input.
    # The relation holds for the corner values, which also shows the corner
    # to which each of the four products belongs.
    # The oracle's min J is the smallest of these values (exact here: dyadic
    # coordinates with few bits), and its verdict their sign.
    rng = np.random.default_rng(3)
    for _ in range(200):
        P = SQ + rng.integers(-8, 9, size=(4, 2)) / 16.0
        J = _corner_values_exact(P)
        assert J[0] + J[2] == J[1] + J[3]
        v, m = _q(P)
        assert m == float(min(J))
        assert v == (oracle.VALID if min(J) > 0 else oracle.INVALID)


def test_reflection_and_bow_tie_and_reflex_corner_are_invalid():
    assert _q(SQ[:, ::-1])[0] == oracle.INVALID                       # reversed orientation
    assert _q(SQ[[0, 1, 3, 2]])[0] == oracle.INVALID                  # self-intersecting
    arrow = np.array([[0, 0], [2, 0], [0.5, 0.5], [0, 2]], dtype=np.float64)
    assert _q(arrow)[0] == oracle.INVALID                             # reflex corner
    P = SQ.copy()
    P[2] = P[1]                                                       # collapsed edge: J = 0
    assert _q(P)[0] == oracle.INVALID


@pytest.mark.parametrize("seed", range(3))
def test_min_over_grid_is_the_min_corner(seed):
    # J is bilinear, so its minimum over [0,1]^2 is a corner value
    rng = np.random.default_rng(40 + seed)
    for _ in range(100):
        P = SQ + rng.uniform(-0.45, 0.45, size=(4, 2))
        v, m = _q(P)
        g = _jacobian_grid(P, 32)
        assert abs(g.min() - m) < 1e-13
        assert v == (oracle.VALID if g.min() > 0 else oracle.INVALID)


def test_exact_on_integer_quads_with_zeros():
    rng = np.random.default_rng(9)
    P = (SQ[None] * 2 + rng.integers(-1, 2, size=(5000, 4, 2))).astype(np.float64)
    r = oracle.quad_check(P)
    ex = np.array([exact.quad_validity(p) for p in P])
    assert np.array_equal(r["verdict"], ex)
    assert r["fragile"].size > 0


def test_connectivity_layout_and_bad_input():
    V = np.array([[0, 0], [1, 0], [2, 0], [0, 1], [1, 1], [2, 1.5]], dtype=np.float64)
    C = np.array([[0, 1, 4, 3], [1, 2, 5, 4]], dtype=np.int32)
    r = oracle.quad_check(V, C)
    assert (r["verdict"] == oracle.VALID).all()
    P = SQ.copy()
    P[1, 0] = np.nan
    v, m = _q(P)
    assert v == oracle.BAD_INPUT and np.isnan(m)
