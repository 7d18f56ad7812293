"""GPU: linear quadrangle validity (Section 2.1) against the oracle: verdicts
bit-exact, min J (the smallest corner value) to 1e-14 of S^2."""
import numpy as np
import pytest

import oracle
from paper_1706_01613_amd import hexval as hx
from paper_1706_01613_amd import synth
from tests._gpu import say, torch_cuda, to_dev

pytestmark = pytest.mark.gpu

_say = say


def _gpu(torch, P, conn=None, **kw):
    v, m, st = hx.quad_check(to_dev(torch, P), None if conn is None else to_dev(torch, conn), stats=True, **kw)
    torch.cuda.synchronize()
    return v.cpu().numpy(), m.cpu().numpy(), st


def _compare(v, m, P, conn=None, label=""):
    ref = oracle.quad_check(P, conn)
    bad = np.nonzero(v != ref["verdict"])[0]
    assert bad.size == 0, f"{label}: {bad.size} verdict mismatches, first {bad[:8]}"
    fin = np.isfinite(ref["min_j"])
    assert np.array_equal(np.isfinite(m), fin), label
    Q = P.reshape(-1, 4, 2) if conn is None else P.reshape(-1, 2)[conn]
    S = np.abs(np.diff(Q[:, [0, 1, 2, 3, 0], :], axis=1)).max(axis=(1, 2))
    err = np.abs(m[fin] - ref["min_j"][fin]) / np.maximum(S[fin] ** 2, 1e-300)
    assert err.max(initial=0.0) <= 1e-14, label
    return ref


def test_quad_independent_against_oracle():
    torch = torch_cuda()
    P = synth.independent_quads(2_000_000, noise=0.4, seed=0)
    v, m, st = _gpu(torch, P)
    _say(f"stats {st}")
    ref = _compare(v, m, P, label="independent")
    assert 0 < np.count_nonzero(ref["verdict"] == oracle.INVALID) < P.shape[0]


def test_quad_lattice_with_validation():
    torch = torch_cuda()
    V, C = synth.quad_lattice(1000, 700, seed=3)
    C[5, 2] = -1
    v, m, _ = _gpu(torch, V, C, validate_indices=True)
    assert v[5] == hx.BAD_INPUT and np.isnan(m[5])
    keep = np.ones(C.shape[0], bool)
    keep[5] = False
    _compare(v[keep], m[keep], V, C[keep], label="lattice")


def test_quad_exact_tier_on_integer_quads():
    torch = torch_cuda()
    rng = np.random.default_rng(5)
    P = (synth.SQUARE[None] * 2 + rng.integers(-1, 2, size=(300000, 4, 2))).astype(np.float64)
    v, m, st = _gpu(torch, P)
    assert st["n_exact"] > 0
    _compare(v, m, P, label="integer")


def test_quad_closed_forms_and_bad_input():
    torch = torch_cuda()
    sq = synth.SQUARE
    A = np.array([[2.0, 0.5], [-0.3, 1.5]])
    P = np.stack([sq, sq @ A.T + 3.0, sq[::-1], sq[[0, 1, 3, 2]],
                  np.array([[0, 0], [2, 0], [0.5, 0.5], [0, 2]], dtype=np.float64), sq])
    P[5, 0, 0] = np.nan
    v, m, _ = _gpu(torch, P)
    assert list(v) == [hx.VALID, hx.VALID, hx.INVALID, hx.INVALID, hx.INVALID, hx.BAD_INPUT]
    assert m[0] == 1.0 and abs(m[1] - np.linalg.det(A)) < 1e-15 and np.isnan(m[5])


def _walk_layouts():
    """Quad lattices whose rows the walk follows (5000 quads a row), cut,
    broken, permuted, and with integer coordinates (exact tier)."""
    V, C = synth.quad_lattice(5000, 40, seed=6, jitter_fraction=0.2, jitter=0.6)
    rng = np.random.default_rng(7)
    Cb = C.copy()
    rows = rng.choice(C.shape[0], C.shape[0] // 10, replace=False)
    Cb[rows] = Cb[rng.integers(0, C.shape[0], rows.size)]
    Cf = C.copy()
    flip = rng.choice(C.shape[0], 300, replace=False)
    Cf[flip] = Cf[flip][:, [3, 2, 1, 0]]
    Vi, Ci = synth.quad_lattice(4200, 10, seed=8, amp=0.0, jitter_fraction=0.3, jitter=1.0)
    Vi = np.rint(Vi)
    return [("lattice", V, C, 5000), ("partial row", V, C[: C.shape[0] - 777], 5000), ("broken", V, Cb, None),
            ("reflected", V, Cf, 5000), ("permuted", V, C[rng.permutation(C.shape[0])], None),
            ("integer", Vi, Ci, 4200), ("tiny", V, C[:9], 0)]


def _gpu_unset(torch, P, conn, walk):
    """quad_check on outputs that start as values no kernel writes (memory
    from torch's allocator may still hold an earlier run's results)."""
    n = conn.shape[0]
    v = torch.full((n,), 0xEE, dtype=torch.uint8, device="cuda")
    m = torch.full((n,), -7.5e300, dtype=torch.float64, device="cuda")
    st = hx.hexval_stats_t()
    opts = hx.make_opts(walk_layers=walk, stream=torch.cuda.current_stream(), stats=st)
    hx.hexval_quad_check(hx.make_mesh(to_dev(torch, P), to_dev(torch, conn)), opts, v, m)
    torch.cuda.synchronize()
    v, m = v.cpu().numpy(), m.cpu().numpy()
    assert not np.any(v == 0xEE) and not np.any(m == -7.5e300), f"walk {walk}: outputs not written"
    return v, m, st.as_dict()


def test_quad_row_walk_equals_plain_tiles_and_oracle():
    # each lane keeps the shared edge of the quads stacked in rows; any
    # connectivity gives the plain pass's results bit for bit
    torch = torch_cuda()
    for label, V, C, stride in _walk_layouts():
        C = np.ascontiguousarray(C.astype(np.int32))
        bv, bm, bst = _gpu_unset(torch, V, C, -1)
        assert bst["walk_layers"] == 0
        _compare(bv, bm, V, C, label=f"{label} plain")
        for walk in (16, 3, 64):
            v, m, st = _gpu_unset(torch, V, C, walk)
            _say(f"quads {label} walk {walk}: stride {st['walk_stride']}, exact {st['n_exact']}")
            assert st["walk_layers"] == (walk if C.shape[0] >= 8 * 4096 else 0)
            if stride is not None and C.shape[0] >= 8 * 4096:
                assert st["walk_stride"] == stride, label
            assert st["n_exact"] == bst["n_exact"]
            assert np.array_equal(v, bv), f"{label}: walk {walk} verdicts differ from plain tiles"
            assert np.array_equal(np.nan_to_num(m, nan=7.0).view(np.int64),
                                  np.nan_to_num(bm, nan=7.0).view(np.int64)), f"{label}: walk {walk} min_j"
