"""GPU: corner-only test (Test 1 of Section 7) and corner quality against the
oracle.  Test-1 results are bit-exact (both sides take exact sign decisions);
the quality agrees to 1e-12 (it lies in [-1, 1])."""
import math
import numpy as np
import pytest

import oracle
from paper_1706_01613_amd import hexval as hx
from paper_1706_01613_amd import synth
from tests import _ref
from tests._gpu import say, torch_cuda, to_dev
from tests.test_oracle_pins import CUBE, _twisted

pytestmark = pytest.mark.gpu

_say = say


def _gpu(torch, P, conn=None, **kw):
    t1, q, st = hx.corner_test(to_dev(torch, P), None if conn is None else to_dev(torch, conn),
                               stats=True, **kw)
    torch.cuda.synchronize()
    return t1.cpu().numpy(), q.cpu().numpy(), st


def _compare(t1, q, P, conn=None, label=""):
    ref = oracle.corner_test(P, conn)
    bad = np.nonzero(t1 != ref["test1"])[0]
    assert bad.size == 0, f"{label}: {bad.size} test-1 mismatches, first {bad[:8]}"
    fin = np.isfinite(ref["quality"])
    assert np.array_equal(np.isfinite(q), fin), label
    assert np.abs(q[fin] - ref["quality"][fin]).max(initial=0.0) <= 1e-12, label
    return ref


def test_corner_independent_hexes_full():
    torch = torch_cuda()
    P = synth.independent_hexes(1000000, seed=0)
    t1, q, st = _gpu(torch, P)
    _say(f"stats {st}")
    _compare(t1, q, P, label="1M independent hexes")


def test_corner_lattice_with_index_validation():
    torch = torch_cuda()
    V, C = synth.warped_lattice(64, 48, 40, seed=5, jitter_fraction=0.05)
    C[17, 3] = V.shape[0] + 5                    # out of range -> BAD_INPUT
    t1, q, _ = _gpu(torch, V, C, validate_indices=True)
    assert t1[17] == hx.BAD_INPUT and math.isnan(q[17])
    keep = np.ones(C.shape[0], bool)
    keep[17] = False
    _compare(t1[keep], q[keep], V, C[keep], label="lattice")


def test_corner_closed_forms_and_figure7():
    torch = torch_cuda()
    thetas = [0, 45, 90, 135, 180]
    P = np.stack([_twisted(t)[0] for t in thetas] + [_ref.read_figure("fig7.txt")[0]])
    t1, q, _ = _gpu(torch, P)
    assert (t1 == hx.VALID).all()
    for k, t in enumerate(thetas):
        assert abs(q[k] - 1 / math.sqrt(2 - math.cos(math.radians(t)))) < 1e-15
    assert 0.64 <= q[-1] < 0.65


def test_corner_exact_tier_beyond_list_capacity():
    # 1.1M translated copies of a cube with two coincident corners (J = 0
    # there, positive elsewhere, so no corner decides it in floating point)
    # and 200k random integer hexes: more elements need exact signs than the
    # exact list holds at once
    torch = torch_cuda()
    rng = np.random.default_rng(13)
    D = CUBE * 2
    D[1] = D[0]
    P = np.concatenate([D[None] + rng.integers(-50, 50, size=(1100000, 1, 3)),
                        CUBE[None] * 2 + rng.integers(-1, 2, size=(200000, 8, 3))]).astype(np.float64)
    t1, q, st = _gpu(torch, P)
    _say(f"stats {st}")
    assert st["n_exact"] > (1 << 20)
    assert not np.any(t1 == 0xFD)                 # nothing left pending
    # the oracle settles these in rational arithmetic: a sample spread over
    # the whole range, including the elements listed after the first batch
    idx = np.sort(rng.choice(P.shape[0], size=5000, replace=False))
    _compare(t1[idx], q[idx], P[idx], label="integer lattice")


def test_corner_test_is_necessary_condition_on_gpu():
    torch = torch_cuda()
    P = synth.independent_hexes(300000, noise=0.6, seed=8)
    t1, _, _ = _gpu(torch, P)
    v, _, _ = hx.check(to_dev(torch, P))
    v = v.cpu().numpy()
    assert not np.any((t1 == hx.INVALID) & (v != hx.INVALID))
    assert np.count_nonzero((t1 == hx.VALID) & (v == hx.INVALID)) > 0


def test_corner_bad_input_and_empty():
    torch = torch_cuda()
    P = synth.independent_hexes(1000, seed=2)
    P[5, 2, 2] = np.nan
    t1, q, _ = _gpu(torch, P)
    assert t1[5] == hx.BAD_INPUT and math.isnan(q[5])
    e = torch.empty((0, 8, 3), dtype=torch.float64, device="cuda")
    t, _, _ = hx.corner_test(e)
    assert t.numel() == 0
