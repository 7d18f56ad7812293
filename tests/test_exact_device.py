"""The device exact tier (fixed-width integer arithmetic), replayed on the
CPU from the same source (libhexval_emul.so), against the oracle's rational
arithmetic: every element it settles gets the exact answer; the others are
left to the host tier (CPU only)."""
import ctypes

import numpy as np
import pytest

import oracle
from oracle import exact
from paper_1706_01613_amd import synth
from paper_1706_01613_amd.build import EMUL

CUBE = synth.CUBE
HOST = 0xFE


@pytest.fixture(scope="module")
def E():
    L = ctypes.CDLL(EMUL)
    P = ctypes.c_void_p
    for f in (L.hexval_emul_exact_device, L.hexval_emul_exact_host):
        f.argtypes = [P, ctypes.c_int64, ctypes.c_int, ctypes.c_int, P]
    return L


def _run(E, fn, pts, mode, max_depth=6):
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    n = pts.shape[0]
    out = np.empty(n, np.uint8)
    getattr(E, fn)(pts.ctypes.data, n, mode, max_depth, out.ctypes.data)
    return out


def _degenerate_integer_hexes(n, seed):
    rng = np.random.default_rng(seed)
    P = (CUBE[None] * 2 + rng.integers(-1, 2, size=(n, 8, 3))).astype(np.float64)
    P[::4, 1] = P[::4, 0]                       # coincident corners: exact zeros
    return P


def test_verdicts_on_integer_and_degenerate_hexes(E):
    P = _degenerate_integer_hexes(3000, 1)
    dev = _run(E, "hexval_emul_exact_device", P, 0)
    settled = dev != HOST
    assert settled.mean() > 0.5                  # step 2 / step 4 decide most of them
    for e in np.nonzero(settled)[0]:
        assert dev[e] == exact.validity(P[e])["verdict"], e
    host = _run(E, "hexval_emul_exact_host", P, 0)
    assert np.array_equal(dev[settled], host[settled])


def test_verdicts_on_scaled_near_degenerate_hexes(E):
    # coordinates of mixed magnitudes: within 2^78 the device settles them,
    # beyond it (very different exponents) it leaves them to the host
    P = synth.near_degenerate_hexes(400, seed=3, rel=1e-14, log10_scale=2.0)
    dev = _run(E, "hexval_emul_exact_device", P, 0)
    for e in np.nonzero(dev != HOST)[0]:
        assert dev[e] == exact.validity(P[e])["verdict"], e
    wide = P.copy()
    wide[:, 3, 0] = 1e-20                         # an exponent 2^-66 next to 2^0
    assert (_run(E, "hexval_emul_exact_device", wide, 0) == HOST).all()


def test_exact_subdivision_settled_on_the_device(E):
    # integer hexes whose top-level coefficients are not all positive (exact
    # UNDECIDED at cap 0) need exact subdivision: the 384-bit depth-first
    # tier decides every one of them on the device, with the rational
    # answer of the oracle, and agrees with the host tier's big integers
    P = _degenerate_integer_hexes(4000, 7)
    cap0 = _run(E, "hexval_emul_exact_device", P, 0, max_depth=0)
    need = np.nonzero(cap0 == 2)[0]
    assert need.size > 20
    for depth in (1, 3, 6):
        dev = _run(E, "hexval_emul_exact_device", P[need], 0, max_depth=depth)
        assert (dev != HOST).all(), depth
        want = [exact.validity(P[e], max_depth=depth)["verdict"] for e in need]
        assert list(dev) == want, depth
        host = _run(E, "hexval_emul_exact_host", P[need], 0, max_depth=depth)
        assert np.array_equal(dev, host), depth
    # the sheared prisms (min J = eps at a non-dyadic point) to the largest
    # cap: their closed-form verdicts (VALID once the sub-boxes are small
    # enough for eps > 0, INVALID for eps < 0, UNDECIDED at caps reached
    # first, and for eps = 0)
    from tests.test_gpu_parity import _prism
    cases = [(0.25, 6, 1), (2.0 ** -10, 6, 1), (-(2.0 ** -10), 6, 0), (2.0 ** -20, 6, 2),
             (-(2.0 ** -20), 6, 2), (0.0, 6, 2), (2.0 ** -20, 20, 1), (-(2.0 ** -20), 20, 0)]
    for eps, depth, want in cases:
        dev = _run(E, "hexval_emul_exact_device", _prism(eps)[None], 0, max_depth=depth)
        assert dev[0] == want, (eps, depth, dev[0])


def test_depth_cap_zero_gives_undecided_exactly(E):
    P, _ = __import__("tests.test_oracle_pins", fromlist=["_twisted"])._twisted(120)
    dev = _run(E, "hexval_emul_exact_device", P[None], 0, max_depth=0)
    assert dev[0] == exact.validity(P, max_depth=0)["verdict"]


def test_corner_test_and_quads(E):
    P = _degenerate_integer_hexes(3000, 2)
    dev = _run(E, "hexval_emul_exact_device", P, 1)
    assert (dev != HOST).all()
    assert np.array_equal(dev, np.array([exact.corner_test(p) for p in P]))
    rng = np.random.default_rng(4)
    Q = (synth.SQUARE[None] * 2 + rng.integers(-1, 2, size=(3000, 4, 2))).astype(np.float64)
    dq = _run(E, "hexval_emul_exact_device", Q, 2)
    assert (dq != HOST).all()
    assert np.array_equal(dq, np.array([exact.quad_validity(q) for q in Q]))


def test_all_points_equal_and_non_finite(E):
    P = np.zeros((2, 8, 3))
    P[1, 5, 2] = np.nan
    dev = _run(E, "hexval_emul_exact_device", P, 0)
    assert dev[0] == 0 and dev[1] == HOST           # the host reports BAD_INPUT
