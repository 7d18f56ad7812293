"""Pins of the oracle's corner-only test (Test 1 of Section 7) and corner
quality (scaled Jacobian at the corners) against the paper, closed forms,
exact arithmetic and an independent evaluation (CPU only)."""
import math

import numpy as np
import pytest

import oracle
from oracle import exact
from tests import _ref
from tests.test_oracle_pins import CUBE, _twisted


def _ct(P):
    r = oracle.corner_test(np.asarray(P, dtype=np.float64)[None])
    return int(r["test1"][0]), float(r["quality"][0])


def _quality_reference(P):
    """Scaled Jacobian at the corners from the shape-function derivative
    (independent of the oracle's edge-vector formulation)."""
    q = math.inf
    for c in _ref.NODES[:8]:
        xi, eta, zeta = (n / 2 for n in c)
        G = _ref.shape_gradients(xi, eta, zeta)
        D = np.array([[sum(G[k][j] * P[k][i] for k in range(8)) for j in range(3)] for i in range(3)])
        den = np.prod(np.linalg.norm(D, axis=0))
        q = min(q, np.linalg.det(D) / den if den > 0 else 0.0)
    return q


def test_fig7_good_corner_quality_but_invalid():
    # Section 7: corner quality 0.64 (truncated: 0.6471) although invalid
    P, _ = _ref.read_figure("fig7.txt")
    t1, q = _ct(P)
    assert 0.64 <= q < 0.65
    assert t1 == oracle.VALID
    assert oracle.check(P[None])["verdict"][0] == oracle.INVALID


@pytest.mark.parametrize("theta", [0, 30, 60, 90, 135, 170, 180])
def test_twisted_cube_quality_closed_form(theta):
    # corner values are all 1; the edges at each corner have lengths 1, 1 and
    # sqrt(2 - cos theta), and they are orthogonal in the J sense
    P, _ = _twisted(theta)
    t1, q = _ct(P)
    assert t1 == oracle.VALID
    assert abs(q - 1.0 / math.sqrt(2.0 - math.cos(math.radians(theta)))) < 1e-15
    full = oracle.check(P[None])["verdict"][0]
    # theta = 180: min J = cos^2(90 deg) = 0 -> invalid, yet every corner is fine
    assert full == (oracle.INVALID if theta == 180 else oracle.VALID)


def test_cube_and_parallelepiped():
    assert _ct(CUBE) == (oracle.VALID, 1.0)
    A = np.array([[2.0, 0.3, -0.1], [0.2, 1.5, 0.4], [-0.3, 0.1, 0.8]])
    t1, q = _ct(CUBE @ A.T + 3.0)
    assert t1 == oracle.VALID
    assert abs(q - np.linalg.det(A) / np.prod(np.linalg.norm(A, axis=0))) < 1e-14


@pytest.mark.parametrize("seed", range(3))
def test_quality_matches_independent_evaluation(seed):
    rng = np.random.default_rng(500 + seed)
    P = CUBE[None] + rng.uniform(-0.45, 0.45, size=(200, 8, 3))
    r = oracle.corner_test(P)
    ref = np.array([_quality_reference(p) for p in P])
    assert np.abs(r["quality"] - ref).max() < 1e-12


def test_necessary_condition_never_false_invalid():
    rng = np.random.default_rng(7)
    P = CUBE[None] + rng.uniform(-0.6, 0.6, size=(20000, 8, 3))
    t1 = oracle.corner_test(P)["test1"]
    v = oracle.check(P)["verdict"]
    assert not np.any((t1 == oracle.INVALID) & (v != oracle.INVALID))
    fv = np.count_nonzero((t1 == oracle.VALID) & (v == oracle.INVALID))
    assert fv > 0                  # the corner test misses some invalid elements
    assert np.all((t1 == oracle.VALID) | (t1 == oracle.INVALID))


def test_exact_corner_signs_on_lattices_and_degenerate_elements():
    rng = np.random.default_rng(11)
    P = (CUBE[None] * 2 + rng.integers(-1, 2, size=(3000, 8, 3))).astype(np.float64)
    P[0, 1] = P[0, 0]                       # coincident corner: J = 0 there -> INVALID
    r = oracle.corner_test(P)
    ex = np.array([exact.corner_test(p) for p in P])
    assert np.array_equal(r["test1"], ex)
    assert r["test1"][0] == oracle.INVALID
    assert r["fragile"].size > 0            # exact zeros need the exact tier


def test_symmetries():
    rng = np.random.default_rng(21)
    P = CUBE + rng.uniform(-0.3, 0.3, size=(8, 3))
    t1, q = _ct(P)
    for sym in _ref.cube_symmetries():
        Q, _ = _ref.apply_symmetry(P, sym)
        tq, qq = _ct(Q)
        if sym[2] > 0:
            assert tq == t1 and abs(qq - q) < 1e-14
        else:
            assert tq == oracle.INVALID


def test_bad_input():
    P = CUBE.copy()
    P[2, 0] = np.inf
    t1, q = _ct(P)
    assert t1 == oracle.BAD_INPUT and math.isnan(q)
