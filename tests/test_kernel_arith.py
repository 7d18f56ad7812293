"""CPU replay of the kernels' arithmetic (libhexval_emul.so) against the
oracle: the error bounds the kernels certify with, their decision logic and
the library's exact tier (CPU only; the GPU parity tests run the kernels)."""
import ctypes
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import exact
from paper_1706_01613_amd import synth
from paper_1706_01613_amd.build import EMUL

CUBE = synth.CUBE


@pytest.fixture(scope="module")
def emul():
    E = ctypes.CDLL(EMUL)
    P = ctypes.c_void_p
    E.hexval_emul_check.argtypes = [P, P, ctypes.c_int64, ctypes.c_int, P, P, P]
    E.hexval_emul_values.argtypes = [P, P, ctypes.c_int64, ctypes.c_int, P, P, P, P]
    E.hexval_emul_exact.argtypes = [P, ctypes.c_int64, ctypes.c_int, P]
    E.hexval_emul_constants.argtypes = [P]
    E.hexval_emul_lean.argtypes = [P, P, ctypes.c_int64, ctypes.c_int, ctypes.c_int, P, P, P, P, P]
    return E


def run_check(E, pts, conn=None, max_depth=6):
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    n = conn.shape[0] if conn is not None else pts.shape[0]
    v = np.empty(n, np.uint8)
    m = np.empty(n)
    st = np.zeros(4, np.int64)
    E.hexval_emul_check(pts.ctypes.data, None if conn is None else conn.ctypes.data, n,
                        max_depth, v.ctypes.data, m.ctypes.data, st.ctypes.data)
    return v, m, st


def values(E, pts):
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 8, 3)
    n = pts.shape[0]
    c = np.empty((n, 27))
    s = np.empty(n)
    E.hexval_emul_values(pts.ctypes.data, None, n, 6, c.ctypes.data, s.ctypes.data, None, None)
    return c, s


def test_independent_hexes_subset_matches_oracle(emul):
    X = synth.independent_hexes(200000, seed=0)
    v, m, st = run_check(emul, X)
    r = oracle.check(X)
    assert (v == r["verdict"]).all()
    b = oracle.coefficients(X)
    assert (np.abs(m - r["min_coeff"]) / np.abs(b).max(1)).max() < 1e-12
    assert st[0] > 0


@pytest.mark.parametrize("max_depth", [0, 1, 2, 6, 9])
def test_tangled_and_lattice_match_oracle(emul, max_depth):
    X = synth.independent_hexes(30000, noise=0.5, seed=max_depth)
    v, _, _ = run_check(emul, X, max_depth=max_depth)
    assert (v == oracle.check(X, max_depth=max_depth)["verdict"]).all()
    V, C = synth.warped_lattice(24, 20, 16, jitter_fraction=0.1, seed=max_depth)
    v, _, _ = run_check(emul, V, C, max_depth=max_depth)
    assert (v == oracle.check(V, C, max_depth=max_depth)["verdict"]).all()


def test_precision_stress_hexes_match_oracle(emul):
    P = synth.near_degenerate_hexes(20000, seed=1)
    v, _, _ = run_check(emul, P)
    r = oracle.check(P)
    assert (v == r["verdict"]).all()
    assert 0.3 < (r["verdict"] == 0).mean() < 0.7


def test_integer_lattice_and_exact_tier(emul):
    rng = np.random.default_rng(4)
    P = (CUBE[None] * 2 + rng.integers(-1, 2, size=(3000, 8, 3))).astype(np.float64)
    v, _, st = run_check(emul, P)
    assert st[2] > 0                       # exact tier used
    assert (v == oracle.check(P)["verdict"]).all()
    # the library's exact tier alone against the oracle's rational tier
    out = np.empty(300, np.uint8)
    emul.hexval_emul_exact(np.ascontiguousarray(P[:300]).ctypes.data, 300, 6, out.ctypes.data)
    assert list(out) == [exact.validity(p)["verdict"] for p in P[:300]]


def test_exact_tier_on_random_and_degenerate(emul):
    X = synth.independent_hexes(200, noise=0.5, seed=3)
    X[:5] = 0.0
    X[5, 2, 1] = np.nan
    out = np.empty(len(X), np.uint8)
    emul.hexval_emul_exact(np.ascontiguousarray(X).ctypes.data, len(X), 4, out.ctypes.data)
    want = [exact.validity(p, max_depth=4)["verdict"] for p in X]
    assert list(out) == want
    assert want[5] == exact.BAD_INPUT and want[0] == exact.INVALID


@pytest.mark.parametrize("kind", ["random", "offset", "flat", "scaled", "stress"])
def test_kernel_error_bounds_hold(emul, kind):
    """|b^ - b| < tau_coeff u M^ for b_9..b_27 and |c^ - c| < tau_value u M^ for
    corner values, with exact ground truth."""
    rng = np.random.default_rng(20 + len(kind))
    n = 50
    X = CUBE[None] + rng.uniform(-0.4, 0.4, size=(n, 8, 3))
    if kind == "offset":
        X = X + rng.uniform(100, 1000, size=(n, 1, 3))
    if kind == "flat":
        X[:, :, 2] *= 1e-9
    if kind == "scaled":
        X = X * 10.0 ** rng.uniform(-3, 3, size=(n, 1, 1))
    if kind == "stress":
        X = synth.near_degenerate_hexes(n, seed=5)
    k = np.empty(5)
    emul.hexval_emul_constants(k.ctypes.data)
    tau_v, tau_b, _, u, _ = k
    c, s = values(emul, X)
    worst = 0.0
    for P, cc, m in zip(X, c, s):
        be, _ = exact.coefficients(P)
        for a in range(27):
            e = abs(Fraction(float(cc[a])) - be[a])
            t = (tau_v if a < 8 else tau_b) * u * m
            worst = max(worst, float(e) / t)
    assert worst < 1.0


def lean(E, pts, precision, check_edges=0):
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 8, 3)
    n = pts.shape[0]
    out = [np.empty(n) for _ in range(4)]
    st = np.empty(n, np.int32)
    E.hexval_emul_lean(pts.ctypes.data, None, n, precision, check_edges,
                       *[o.ctypes.data for o in out], st.ctypes.data)
    return out + [st]


@pytest.mark.parametrize("kind", ["random", "offset", "scaled", "stress", "tangled"])
@pytest.mark.parametrize("precision", [0, 1])
def test_lean_minima_within_certified_bounds(emul, kind, precision):
    """The first-pass minima (FP64 pass and FP32 filter) stay within the
    thresholds the kernels certify with: |m8^ - m8| < tau_value u M^ and
    |mb^ - mb| < tau_coeff u M^, against exact values."""
    rng = np.random.default_rng(40 + len(kind) + precision)
    n = 40
    X = CUBE[None] + rng.uniform(-0.4, 0.4, size=(n, 8, 3))
    if kind == "offset":
        X = X + rng.uniform(100, 1000, size=(n, 1, 3))
    if kind == "scaled":
        X = X * 10.0 ** rng.uniform(-3, 3, size=(n, 1, 1))
    if kind == "stress":
        X = synth.near_degenerate_hexes(n, seed=6)
    if kind == "tangled":
        X = CUBE[None] + rng.uniform(-0.7, 0.7, size=(n, 8, 3))
    k = np.empty(5)
    emul.hexval_emul_constants(k.ctypes.data)
    u = k[3] if precision == 0 else k[4]
    m20, mb, _, scale, _ = lean(emul, X, precision)
    worst = 0.0
    for P, a, b, s in zip(X, m20, mb, scale):
        be, _ = exact.coefficients(P)
        m8e, mbe = min(be[:8]), min(be[8:])
        worst = max(worst, float(abs(Fraction(float(a)) - m8e)) / (k[0] * u * s),
                    float(abs(Fraction(float(b)) - mbe)) / (k[1] * u * s))
    assert worst < 1.0


def test_fp32_filter_decisions_agree_with_oracle(emul):
    X = np.concatenate([synth.independent_hexes(100000, seed=0),
                        synth.near_degenerate_hexes(20000, seed=1),
                        synth.independent_hexes(20000, noise=0.6, seed=2)])
    _, _, _, _, st = lean(emul, X, 1)
    ref = oracle.check(X)["verdict"]
    decided = st >= 0
    assert (st[decided] == ref[decided]).all()
    assert decided.mean() > 0.8
    # the near-degenerate corners are never certified in FP32
    assert not decided[100000:120000].any()


def test_outward_rounding_is_nextafter(emul):
    # the min-J kernels widen their bounds with next_down / next_up, written
    # from the bit pattern: they must equal nextafter towards -inf / +inf
    rng = np.random.default_rng(11)
    special = np.array([0.0, -0.0, 1.0, -1.0, np.inf, -np.inf, np.nan, 5e-324, -5e-324,
                        2.2250738585072014e-308, -2.2250738585072014e-308, np.finfo(float).max,
                        -np.finfo(float).max, 1e-300, 3.5])
    x = np.concatenate([special, rng.integers(0, 2 ** 63, 200000, dtype=np.int64).view(np.float64),
                        -rng.integers(0, 2 ** 63, 200000, dtype=np.int64).view(np.float64)])
    down = np.empty_like(x)
    up = np.empty_like(x)
    emul.hexval_emul_next.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
    emul.hexval_emul_next(x.ctypes.data, x.size, down.ctypes.data, up.ctypes.data)
    with np.errstate(over="ignore", invalid="ignore"):
        want_down = np.nextafter(x, -np.inf)
        want_up = np.nextafter(x, np.inf)
    assert np.array_equal(down.view(np.int64)[~np.isnan(x)], want_down.view(np.int64)[~np.isnan(x)])
    assert np.array_equal(up.view(np.int64)[~np.isnan(x)], want_up.view(np.int64)[~np.isnan(x)])
    assert np.isnan(down[np.isnan(x)]).all() and np.isnan(up[np.isnan(x)]).all()


def test_fp32_filter_sends_to_subdivision_only_what_fp64_subdivides(emul):
    """The FP32 filter lists an element for subdivision itself, without the
    FP64 recheck, only when its corner values are above twice their FP32
    bound and its Bezier minimum at or below minus its bound.  Every such
    element must be one the FP64 pass subdivides too, and one the oracle does
    not decide at the root (Section 6: some coefficient negative, every
    corner positive)."""
    emul.hexval_emul_filter_subdivides.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                                   ctypes.c_void_p, ctypes.c_void_p]
    X = np.concatenate([synth.independent_hexes(60000, seed=3),
                        synth.independent_hexes(60000, noise=0.6, seed=4),
                        synth.near_degenerate_hexes(10000, seed=5),
                        (synth.independent_hexes(20000, noise=0.5, seed=6)
                         * 10.0 ** np.random.default_rng(7).uniform(-3, 3, size=(20000, 1, 1))),
                        synth.independent_hexes(20000, noise=0.5, seed=8) + 1000.0])
    X = np.ascontiguousarray(X)
    n = X.shape[0]
    sub = np.empty(n, np.int32)
    st64 = np.empty(n, np.int32)
    emul.hexval_emul_filter_subdivides(X.ctypes.data, None, n, sub.ctypes.data, st64.ctypes.data)
    flagged = sub == 1
    assert flagged.sum() > 1000
    assert (st64[flagged] == 3).all()            # kTopSubdivide in the FP64 pass
    idx = np.nonzero(flagged)[0][::7]
    r = oracle.check(X[idx], details=True)
    b = oracle.coefficients(X[idx])
    assert (b[:, :8] > 0).all()                  # every corner value positive
    assert (b[:, 8:].min(axis=1) < 0).all()      # and some coefficient negative
    # the oracle subdivides them, or (testing the 12 edge-midpoint values at
    # the root, which the kernels leave to level 1) finds one non-positive
    assert ((r["level"] >= 1) | (r["verdict"] == oracle.INVALID)).all()
