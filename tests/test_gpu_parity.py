"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Verdicts must be bit-exact (both sides compute the exact-arithmetic verdict);
Bezier coefficients and min_coeff must agree to 1e-12 relative to the
element's largest coefficient.
"""
import math
import numpy as np
import pytest

import oracle
from paper_1706_01613_amd import hexval as hx
from paper_1706_01613_amd import synth
from tests import _ref
from tests._gpu import say, assert_parity, torch_cuda, to_dev

pytestmark = pytest.mark.gpu

CUBE = synth.CUBE

_say = say


def _run(torch, P, conn=None, **kw):
    if conn is None:
        v, m, st = hx.check(to_dev(torch, P), None, stats=True, **kw)
    else:
        v, m, st = hx.check(to_dev(torch, P), to_dev(torch, conn), stats=True, **kw)
    torch.cuda.synchronize()
    return v.cpu().numpy(), m.cpu().numpy(), st


def test_one_million_independent_hexes_full():
    torch = torch_cuda()
    _say("1,000,000 independent hexes, noise 0.35, seed 0")
    P = synth.independent_hexes(1_000_000, seed=0)
    v, m, st = _run(torch, P)
    ref = assert_parity(v, m, P, label="1M independent hexes")
    assert st["n_elements"] == 1_000_000
    # all 27 coefficients
    c = hx.coefficients(to_dev(torch, P)).cpu().numpy()
    b = oracle.coefficients(P)
    err = np.abs(c - b).max(axis=1) / np.abs(b).max(axis=1)
    assert err.max() <= 1e-12
    assert (ref["verdict"] == 0).sum() > 1000 and (ref["verdict"] == 1).sum() > 1000


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 255, 256, 257, 1000, 4099])
def test_ragged_sizes(n):
    torch = torch_cuda()
    _say(f"ragged n={n}")
    P = synth.independent_hexes(n, noise=0.45, seed=n)
    v, m, _ = _run(torch, P)
    assert_parity(v, m, P, label=f"n={n}")


def test_empty_input():
    torch = torch_cuda()
    v = torch.empty(0, dtype=torch.uint8, device="cuda")
    P = torch.empty((0, 8, 3), dtype=torch.float64, device="cuda")
    assert hx.hexval_check(P, None, 0, v, None) == hx.OK


@pytest.mark.parametrize("nx,ny,nz,seed", [(64, 64, 64, 0), (37, 23, 11, 3), (1, 1, 1, 5)])
def test_warped_lattice_connectivity(nx, ny, nz, seed):
    torch = torch_cuda()
    _say(f"lattice {nx}x{ny}x{nz} seed {seed}")
    V, C = synth.warped_lattice(nx, ny, nz, seed=seed, jitter_fraction=0.05)
    v, m, _ = _run(torch, V, C)
    assert_parity(v, m, V, C, label="lattice")


def test_paper_figures():
    torch = torch_cuda()
    P = np.stack([_ref.read_figure(f"fig{k}.txt")[0] for k in (5, 6, 7)])
    v, m, st = _run(torch, P)
    assert list(v) == [hx.INVALID, hx.VALID, hx.INVALID]
    assert_parity(v, m, P, label="figures")
    assert st["max_level"] >= 3


def _twisted(theta):
    c, s = (0.0, 1.0) if theta == 90 else (-1.0, 0.0) if theta == 180 else (
        math.cos(math.radians(theta)), math.sin(math.radians(theta)))
    P = CUBE.copy()
    for k in range(4, 8):
        x, y = P[k, 0] - 0.5, P[k, 1] - 0.5
        P[k, :2] = [0.5 + c * x - s * y, 0.5 + s * x + c * y]
    return P


def _prism(eps):
    d, t = 9.0 * (1.0 - eps), -6.0 * (1.0 - eps)
    R = np.array([[1 + t / 2, 1.0], [t * t / 4 - d, 1 + t / 2]])
    P = CUBE.copy()
    for k in range(4, 8):
        P[k, :2] = 0.5 + R @ (P[k, :2] - 0.5)
    return P


@pytest.mark.parametrize("max_depth", [0, 1, 3, 6, 11])
def test_closed_form_families(max_depth):
    torch = torch_cuda()
    _say(f"families depth {max_depth}")
    fam = [_twisted(t) for t in (30, 90, 120, 179, 180)]
    fam += [_prism(e) for e in (0.25, 2.0 ** -6, 2.0 ** -10, 2.0 ** -20, 0.0, -(2.0 ** -10), -(2.0 ** -20))]
    P = np.stack(fam)
    v, m, _ = _run(torch, P, max_depth=max_depth)
    assert_parity(v, m, P, max_depth=max_depth, label=f"families d={max_depth}")


def test_deepest_depth_cap():
    # the largest cap (20): families that end by level 11 (the flat prism,
    # whose live boxes grow as 4^L, is left out)
    torch = torch_cuda()
    fam = [_twisted(t) for t in (30, 120, 180)]
    fam += [_prism(e) for e in (0.25, 2.0 ** -10, 2.0 ** -20, -(2.0 ** -10), -(2.0 ** -20))]
    P = np.stack(fam)
    v, m, st = _run(torch, P, max_depth=20)
    assert st["max_level"] == 11
    assert_parity(v, m, P, max_depth=20, label="families d=20")


def test_flat_prism_beyond_the_store_goes_depth_first():
    # the eps = 0 prism's ambiguous region is a surface: about 4^L live boxes
    # at level L, 4^8 = 65536 at cap 8, far more than a store of 4096 nodes.
    # Rounds list fewer elements until one alone overflows, then the elements
    # left are decided depth first in bounded memory, with the oracle's
    # verdicts (UNDECIDED for the flat prism).
    torch = torch_cuda()
    fam = [_prism(0.0), _prism(2.0 ** -20), _prism(-(2.0 ** -20)), _twisted(120), _prism(0.25)]
    P = np.stack(fam * 40)
    v, m, st = _run(torch, P, max_depth=8, queue_capacity=4096)
    _say(f"flat prism, cap 8, store 4096: rounds {st['n_rounds']}, verdicts {np.bincount(v, minlength=4)}")
    assert st["n_rounds"] > 1
    assert (v[0::5] == hx.UNDECIDED).all()
    assert_parity(v, m, P, max_depth=8, label="flat prism depth first")


def test_depth_first_in_a_batch_and_with_the_fp32_filter():
    torch = torch_cuda()
    P = np.stack([_prism(0.0), _twisted(179), _prism(2.0 ** -10)] * 20)
    V, C = synth.warped_lattice(20, 20, 20, seed=3, jitter_fraction=0.2)
    pts = [to_dev(torch, P), to_dev(torch, V)]
    conns = [None, to_dev(torch, C)]
    ns = [P.shape[0], C.shape[0]]
    verd = [torch.empty(n, dtype=torch.uint8, device="cuda") for n in ns]
    mins = [torch.empty(n, dtype=torch.float64, device="cuda") for n in ns]
    meshes = [hx.make_mesh(p, c, n) for p, c, n in zip(pts, conns, ns)]
    for prec in (hx.FP64, hx.FP32_FILTER):
        st = hx.hexval_stats_t()
        opts = hx.make_opts(precision=prec, max_depth=8, queue_capacity=4096, stats=st,
                            stream=torch.cuda.current_stream())
        hx.hexval_check_batched(meshes, opts, verd, mins)
        torch.cuda.synchronize()
        assert st.n_rounds > 1
        assert_parity(verd[0].cpu().numpy(), mins[0].cpu().numpy() if prec == hx.FP64 else None, P,
                      max_depth=8, label=f"batched prisms p{prec}")
        assert_parity(verd[1].cpu().numpy(), mins[1].cpu().numpy() if prec == hx.FP64 else None, V, C,
                      max_depth=8, label=f"batched lattice p{prec}")
        v1, _, _ = _run(torch, P, max_depth=8, queue_capacity=4096, precision=prec)
        assert np.array_equal(v1, verd[0].cpu().numpy())


def test_exact_tier_integer_lattice():
    # small-integer hexes: many values exactly 0 -> exact tier on both sides
    torch = torch_cuda()
    rng = np.random.default_rng(1)
    P = (CUBE[None] * 2 + rng.integers(-1, 2, size=(4000, 8, 3))).astype(np.float64)
    P[:50, 3] = P[:50, 0]
    v, m, st = _run(torch, P)
    assert st["n_exact"] > 0
    # the device tier settles every one of them, exact subdivision included
    # (the coordinates span a few bits)
    assert st["n_exact_host"] == 0
    assert_parity(v, m, P, label="integer lattice")


def test_exact_tier_device_and_host_split():
    # the same integer hexes scaled so that one coordinate has a tiny
    # exponent: the span exceeds the device tier's 78 bits and every uncertain
    # element goes to the host; results are the same either way
    torch = torch_cuda()
    rng = np.random.default_rng(2)
    P = (CUBE[None] * 2 + rng.integers(-1, 2, size=(3000, 8, 3))).astype(np.float64)
    v, m, st = _run(torch, P)
    W = P.copy()
    W[:, 0, 2] = np.where(W[:, 0, 2] == 0.0, 2.0 ** -60, W[:, 0, 2])
    vw, mw, stw = _run(torch, W)
    _say(f"device/host split: {st['n_exact']}/{st['n_exact_host']} vs {stw['n_exact']}/{stw['n_exact_host']}")
    assert st["n_exact_host"] == 0 and stw["n_exact_host"] > 0
    assert_parity(v, m, P, label="integer")
    assert_parity(vw, mw, W, label="wide span")


def test_bad_input_and_index_validation():
    torch = torch_cuda()
    P = np.stack([CUBE] * 4)
    P[1, 2, 0] = np.nan
    P[2, 5, 1] = np.inf
    P[3, 0, 2] = -np.inf
    v, m, _ = _run(torch, P)
    assert list(v) == [hx.VALID, hx.BAD_INPUT, hx.BAD_INPUT, hx.BAD_INPUT]
    assert np.isnan(m[1:]).all() and m[0] == 1.0
    V, C = synth.warped_lattice(4, 4, 4, jitter_fraction=0.0)
    C = C.copy()
    C[5, 3] = V.shape[0]          # out of range
    C[9, 0] = -1
    v, m, _ = _run(torch, V, C, validate_indices=True)
    assert v[5] == hx.BAD_INPUT and v[9] == hx.BAD_INPUT and np.isnan(m[[5, 9]]).all()
    ok = np.setdiff1d(np.arange(C.shape[0]), [5, 9])
    assert (v[ok] == hx.VALID).all()


def test_tiny_queue_rounds_give_identical_verdicts():
    torch = torch_cuda()
    _say("tiny queue")
    P = synth.independent_hexes(20000, noise=0.45, seed=9)
    v0, m0, st0 = _run(torch, P)
    v1, m1, st1 = _run(torch, P, queue_capacity=64)
    assert st0["n_rounds"] == 1 and st1["n_rounds"] > 1
    assert (v0 == v1).all() and np.array_equal(m0, m1)
    assert_parity(v1, m1, P, label="tiny queue")


def test_repeated_runs_are_bitwise_identical():
    torch = torch_cuda()
    P = synth.independent_hexes(300000, noise=0.4, seed=2)
    runs = [_run(torch, P)[:2] for _ in range(3)]
    for v, m in runs[1:]:
        assert (v == runs[0][0]).all() and np.array_equal(m, runs[0][1])


def test_concurrent_calls_from_host_threads():
    # four host threads, each on its own stream, call the library at the same
    # time (FP64, FP32 filter, a tiny queue that forces deferred rounds, and
    # min J): every result equals the same call made alone
    import threading
    torch = torch_cuda()
    P0 = to_dev(torch, synth.independent_hexes(200000, noise=0.4, seed=31))
    P1 = to_dev(torch, synth.independent_hexes(150000, noise=0.5, seed=32))
    P2 = to_dev(torch, synth.independent_hexes(20000, noise=0.45, seed=9))
    V, C = synth.warped_lattice(60, 50, 40, seed=33, jitter_fraction=0.05, jitter=0.5)
    Vd, Cd = to_dev(torch, V), to_dev(torch, C)
    jobs = [
        lambda s: hx.check(P0, None, stream=s)[:2],
        lambda s: hx.check(P1, None, precision=hx.FP32_FILTER, stream=s)[:2],
        lambda s: hx.check(P2, None, queue_capacity=64, stream=s)[:2],
        lambda s: hx.min_jacobian(Vd, Cd, rtol=1e-3, stream=s)[:2],
    ]
    alone = [job(torch.cuda.current_stream()) for job in jobs]
    torch.cuda.synchronize()
    alone = [tuple(x.cpu() for x in r) for r in alone]
    for rep in range(3):
        _say(f"concurrent calls, round {rep}")
        out = [None] * len(jobs)
        errors = []

        def run(k):
            try:
                s = torch.cuda.Stream()
                with torch.cuda.stream(s):
                    r = jobs[k](s)
                s.synchronize()
                out[k] = tuple(x.cpu() for x in r)
            except Exception as exc:   # reported below, in the test's thread
                errors.append((k, exc))

        threads = [threading.Thread(target=run, args=(k,)) for k in range(len(jobs))]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        assert not errors, errors
        for k in range(len(jobs)):
            for a, b in zip(out[k], alone[k]):
                assert torch.equal(torch.nan_to_num(a, 7.0) if a.is_floating_point() else a,
                                   torch.nan_to_num(b, 7.0) if b.is_floating_point() else b), (rep, k)


# ------------------------------------------------------------ FP32 filter

U32 = 2.0 ** -24


def _fp32_min_bound(points, conn=None):
    """Bound of the FP32-decided min_coeff: 256 u32 M (M from the oracle's
    scale, within a factor of the kernel's)."""
    return 300.0 * U32 * oracle.scale(points, conn)


@pytest.mark.parametrize("case", ["independent", "lattice", "stress", "tangled"])
def test_fp32_filter_verdicts_identical(case):
    torch = torch_cuda()
    _say(f"fp32 filter {case}")
    conn = None
    if case == "independent":
        P = synth.independent_hexes(300000, seed=0)
    elif case == "lattice":
        P, conn = synth.warped_lattice(48, 40, 32, seed=2)
    elif case == "stress":
        V, C = synth.warped_lattice(40, 40, 40, seed=3)
        P, conn = synth.append_independent(V, C, synth.near_degenerate_hexes(6400, seed=1))
    else:
        P = synth.independent_hexes(100000, noise=0.6, seed=4)
    v, m, st = _run(torch, P, conn, precision=hx.FP32_FILTER)
    v64, m64, _ = _run(torch, P, conn)
    assert (v == v64).all()
    ref = assert_parity(v, None, P, conn, label=f"fp32 {case}")
    bound = _fp32_min_bound(P, conn)
    ok = np.isfinite(ref["min_coeff"])
    assert (np.abs(m[ok] - ref["min_coeff"][ok]) <= bound[ok]).all()
    assert st["n_recheck"] > 0 or case == "lattice"
    if case == "stress":
        # every near-degenerate element goes to the FP64 recheck
        assert st["n_recheck"] >= 6400


def test_fp32_filter_small_list_defers_to_fp64_rounds():
    torch = torch_cuda()
    P = synth.near_degenerate_hexes(20000, seed=7)
    # FP32 filter with a 64-node subdivision queue: deferred FP64 passes
    v, m, st = _run(torch, P, precision=hx.FP32_FILTER, queue_capacity=64)
    assert_parity(v, None, P, label="fp32 rounds")


def test_fp32_filter_full_recheck_list_defers_to_rounds():
    # 300,000 near-degenerate hexes all need the FP64 recheck, far more than
    # the recheck list holds (2^16 entries here): the entries past it are
    # deferred and checked in later rounds, with the verdicts of plain FP64
    torch = torch_cuda()
    P = synth.near_degenerate_hexes(300000, seed=17)
    v32, _, st = _run(torch, P, precision=hx.FP32_FILTER)
    v64, _, _ = _run(torch, P, precision=hx.FP64)
    print(f"stats {st}", flush=True)
    assert st["n_rounds"] > 1
    assert np.array_equal(v32, v64)
    idx = np.arange(0, P.shape[0], 15)
    assert_parity(v32[idx], None, P[idx], label="fp32 list rounds")
