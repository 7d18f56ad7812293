"""Pins of the oracle's minimum-of-J bounds (Section 3.1 bounds sharpened by
subdivision) against closed forms, brute force and invariants (CPU only).

Every case checks the enclosure lo <= min J <= hi, and the width
hi - lo <= tol + margins whenever the element converged
(tol = rtol * M^ / 6)."""
import math

import numpy as np
import pytest

import oracle
from tests import _ref
from tests.test_oracle_pins import CUBE, _prism, _twisted

U = 2.0 ** -53


def _mj(P, rtol=1e-3, max_depth=6):
    r = oracle.min_jacobian(np.asarray(P, dtype=np.float64)[None], rtol=rtol, max_depth=max_depth)
    return {k: v[0] for k, v in r.items()}


def _width_ok(r, P, rtol):
    M = oracle.scale(np.asarray(P)[None])[0]
    # tol + both widenings (coefficients 1300 u M^, corner values 24 u M^) + rounding
    return r["hi"] - r["lo"] <= rtol * M / 6 + 1330 * U * M + 4 * np.spacing(abs(r["hi"]) + abs(r["lo"]))


def test_unit_cube_and_parallelepiped_are_exact_at_level_0():
    r = _mj(CUBE)
    assert r["status"] == oracle.MJ_CONVERGED and r["level"] == 0
    assert r["lo"] <= 1.0 <= r["hi"] and r["hi"] - r["lo"] < 1e-12
    A = np.array([[2.0, 0.3, -0.1], [0.2, 1.5, 0.4], [-0.3, 0.1, 0.8]])
    P = CUBE @ A.T + np.array([5.0, -3.0, 7.0])
    r = _mj(P)
    det = np.linalg.det(A)
    assert r["level"] == 0 and r["lo"] <= det <= r["hi"] and r["hi"] - r["lo"] < 1e-11


@pytest.mark.parametrize("theta", [10, 45, 89, 90, 120, 150, 179])
@pytest.mark.parametrize("rtol", [1e-2, 1e-4])
def test_twisted_cube_min_is_cos_squared_half_angle(theta, rtol):
    P, _ = _twisted(theta)
    exact_min = math.cos(math.radians(theta) / 2) ** 2
    r = _mj(P, rtol=rtol, max_depth=12)
    assert r["status"] == oracle.MJ_CONVERGED
    assert r["lo"] <= exact_min + 1e-15 and exact_min - 1e-15 <= r["hi"]
    assert _width_ok(r, P, rtol)


@pytest.mark.parametrize("eps", [0.25, 2.0 ** -4, 2.0 ** -10, -2.0 ** -6])
def test_sheared_prism_min_eps_at_one_third(eps):
    # J(zeta) = 1 + t zeta + d zeta^2, minimum eps at zeta = 1/3 (not dyadic:
    # reached only in the limit, so the bounds must bracket it)
    P, t, d = _prism(eps)
    rtol = 1e-3
    r = _mj(P, rtol=rtol, max_depth=14)
    assert r["status"] == oracle.MJ_CONVERGED
    assert r["lo"] <= eps <= r["hi"]
    assert _width_ok(r, P, rtol)


def test_depth_cap_is_reported_and_still_encloses():
    P, t, d = _prism(2.0 ** -10)
    r = _mj(P, rtol=1e-9, max_depth=2)
    assert r["status"] == oracle.MJ_CAPPED and r["level"] == 2
    assert r["lo"] <= 2.0 ** -10 <= r["hi"]


@pytest.mark.parametrize("seed", range(4))
def test_brute_force_grid_between_bounds(seed):
    # 65^3 samples hold every box corner down to level 6, so the sampled
    # minimum S satisfies lo <= min J <= S <= hi; with convergence S - lo <= tol
    rng = np.random.default_rng(300 + seed)
    rtol = 1e-3
    for _ in range(6):
        P = CUBE + rng.uniform(-0.45, 0.45, size=(8, 3))
        r = _mj(P, rtol=rtol, max_depth=6)
        S = _ref.jacobian_grid(P, 64).min()
        slack = 1e-12 * max(1.0, abs(S))
        assert r["lo"] <= S + slack
        assert S <= r["hi"] + slack
        if r["status"] == oracle.MJ_CONVERGED:
            assert _width_ok(r, P, rtol)
            assert S - r["lo"] <= rtol * oracle.scale(P[None])[0] / 6 + 1e-11


def test_paper_figures_signs():
    # Fig. 5: invalid although J > 0 at the 27 nodes -> hi < 0 once refined;
    # Fig. 6: valid with negative coefficients -> lo > 0; Fig. 7: invalid.
    for name, sign in (("fig5.txt", -1), ("fig6.txt", 1), ("fig7.txt", -1)):
        P, _ = _ref.read_figure(name)
        r = _mj(P, rtol=1e-4, max_depth=10)
        assert r["status"] == oracle.MJ_CONVERGED, name
        if sign < 0:
            assert r["hi"] < 0, name
        else:
            assert r["lo"] > 0, name


@pytest.mark.parametrize("seed", range(3))
def test_affine_and_symmetry_invariance(seed):
    rng = np.random.default_rng(400 + seed)
    P = CUBE + rng.uniform(-0.3, 0.3, size=(8, 3))
    r = _mj(P, rtol=1e-4, max_depth=8)
    A = np.array([[1.3, 0.2, 0.0], [-0.1, 0.9, 0.3], [0.2, 0.0, 1.1]])
    det = np.linalg.det(A)
    ra = _mj(P @ A.T + 3.0, rtol=1e-4, max_depth=8)
    # both intervals enclose the same min (scaled by det A)
    assert ra["lo"] <= det * r["hi"] + 1e-12 and det * r["lo"] <= ra["hi"] + 1e-12
    for sym in _ref.cube_symmetries():
        if sym[2] < 0:
            continue                     # reflections negate J
        Q, _ = _ref.apply_symmetry(P, sym)
        rq = _mj(Q, rtol=1e-4, max_depth=8)
        assert rq["lo"] <= r["hi"] + 1e-14 and r["lo"] <= rq["hi"] + 1e-14


def test_bad_and_out_of_range_inputs():
    P = CUBE.copy()
    P[3, 1] = np.nan
    r = _mj(P)
    assert r["status"] == oracle.MJ_BAD_INPUT and np.isnan(r["lo"]) and np.isnan(r["hi"])
    r = _mj(CUBE * 1e-100)
    assert r["status"] == oracle.MJ_OUT_OF_RANGE and np.isnan(r["lo"])
