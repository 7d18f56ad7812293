"""GPU: hexval_check_noalloc (fixed scratch array, no allocation) gives the
results of hexval_check_ex on the same input, through the C ABI, on two calls
in a row whose second input is smaller: FP64 with subdivision, the FP32
filter with its recheck list, the exact tier, and deferred rounds past the
fixed capacities."""
import numpy as np
import pytest

from paper_1706_01613_amd import hexval as hx
from paper_1706_01613_amd import synth
from tests._gpu import say, torch_cuda

pytestmark = pytest.mark.gpu

_say = say


def _run(torch, fn, V, C, **kw):
    n = C.shape[0] if C is not None else V.shape[0]
    # outputs start with values no call writes, so a skipped element shows
    v = torch.full((n,), 77, dtype=torch.uint8, device="cuda")
    m = torch.full((n,), 7.5, dtype=torch.float64, device="cuda")
    st = hx.hexval_stats_t()
    opts = hx.make_opts(stream=torch.cuda.current_stream(), stats=st, **kw)
    fn(hx.make_mesh(V, C, n), opts, v, m)
    torch.cuda.synchronize()
    return v, m, st.as_dict()


def _same(torch, got, ref, label):
    v, m, st = got
    vr, mr, _ = ref
    assert torch.equal(v, vr), f"{label}: {int((v != vr).sum())} verdicts differ"
    assert torch.equal(torch.nan_to_num(m, 3.25), torch.nan_to_num(mr, 3.25)), f"{label}: min_coeff differs"
    _say(f"{label}: {v.numel()} elements equal, stats {st}")


def _pair(torch, label, big, small, **kw):
    """Two no-alloc calls in a row (the second on a smaller input), each
    against hexval_check_ex on the same input."""
    for tag, (V, C) in (("first", big), ("second, smaller", small)):
        _say(f"no-alloc {label}: {tag} call")
        got = _run(torch, hx.hexval_check_noalloc, V, C, **kw)
        ref = _run(torch, hx.hexval_check_ex, V, C, **kw)
        _same(torch, got, ref, f"{label} ({tag})")
    return got


def test_noalloc_fp64_lattices_with_subdivision():
    torch = torch_cuda()
    big = synth.warped_lattice_torch(60, 50, 40, jitter=0.4, seed=3)
    small = synth.warped_lattice_torch(21, 17, 9, jitter=0.45, seed=4)
    _, _, st = _pair(torch, "FP64 lattices", big, small)
    assert st["n_subdivided"] > 0


def test_noalloc_fp32_filter_rechecks():
    torch = torch_cuda()
    big = (torch.from_numpy(synth.near_degenerate_hexes(200_000, seed=7)).cuda(), None)
    small = (torch.from_numpy(synth.near_degenerate_hexes(5_003, seed=8)).cuda(), None)
    _, _, st = _pair(torch, "FP32 filter", big, small, precision=hx.FP32_FILTER)
    assert st["n_recheck"] > 0


def test_noalloc_lists_past_capacity_go_to_rounds():
    # 300,000 elements all needing the FP64 recheck: more than the fixed list
    # holds, so later rounds finish them
    torch = torch_cuda()
    big = (torch.from_numpy(synth.near_degenerate_hexes(300_000, seed=17)).cuda(), None)
    small = (torch.from_numpy(synth.near_degenerate_hexes(1_000, seed=18)).cuda(), None)
    for tag, (V, C) in (("first", big), ("second, smaller", small)):
        got = _run(torch, hx.hexval_check_noalloc, V, C, precision=hx.FP32_FILTER)
        ref = _run(torch, hx.hexval_check_ex, V, C, precision=hx.FP32_FILTER)
        _same(torch, got, ref, f"list rounds ({tag})")
        if tag == "first":
            assert got[2]["n_rounds"] > 1


def test_noalloc_small_queue_rounds_and_exact_tier():
    torch = torch_cuda()
    big = synth.warped_lattice_torch(40, 30, 20, jitter=0.45, seed=40)
    small = synth.warped_lattice_torch(12, 11, 10, jitter=0.45, seed=41)
    _, _, st = _pair(torch, "queue of 64", big, small, queue_capacity=64)
    # integer hexes with exact zeros: the device exact tier
    rng = np.random.default_rng(12)
    P = (synth.CUBE[None] * 2 + rng.integers(-1, 2, size=(6000, 8, 3))).astype(np.float64)
    P[::4, 1] = P[::4, 0]
    Pd = torch.from_numpy(P).cuda()
    _, _, st = _pair(torch, "exact tier", (Pd, None), (Pd[:777].contiguous(), None))
    assert st["n_exact"] > 0


def test_noalloc_rejects_sizes_past_its_store():
    torch = torch_cuda()
    V, C = synth.warped_lattice_torch(4, 4, 4, seed=1)
    for kw in ({"max_depth": 9}, {"queue_capacity": (1 << 17) + 1}):
        with pytest.raises(hx.HexvalError) as e:
            _run(torch, hx.hexval_check_noalloc, V, C, **kw)
        assert e.value.status == hx.E_ARG
        assert "hexval_check_noalloc" in str(e.value)
    # an accepted call after the rejected ones
    got = _run(torch, hx.hexval_check_noalloc, V, C, max_depth=8)
    ref = _run(torch, hx.hexval_check_ex, V, C, max_depth=8)
    _same(torch, got, ref, "after rejected calls")
