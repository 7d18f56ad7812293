"""The column walk of the first passes (elements stacked with a stride found
from the connectivity; each lane carries the shared face to the element
above) on connectivity layouts that match the walk, break it in places or do
not match it at all: every result equal to the oracle, and to the plain-tile
pass bit for bit (HIP path through the C ABI)."""
import numpy as np
import pytest

import oracle
from paper_1706_01613_amd import hexval as hx
from paper_1706_01613_amd import synth
from tests._gpu import assert_parity, say, to_dev, torch_cuda

pytestmark = pytest.mark.gpu

NX, NY, NZ = 70, 65, 50          # 4550 elements per layer: above the smallest stride walked


def lattice(jitter=0.05, seed=11):
    return synth.warped_lattice(NX, NY, NZ, seed=seed, jitter_fraction=jitter)


# Outputs start as values no kernel writes, so that an element left without a
# result shows (memory from torch's allocator may still hold an earlier
# run's outputs).
V_UNSET, M_UNSET = 0xEE, -7.5e300


def unset_outputs(torch, n):
    return (torch.full((n,), V_UNSET, dtype=torch.uint8, device="cuda"),
            torch.full((n,), M_UNSET, dtype=torch.float64, device="cuda"))


def assert_all_written(v, m, label=""):
    assert not np.any(v == V_UNSET), f"{label}: {np.count_nonzero(v == V_UNSET)} verdicts not written"
    assert not np.any(m == M_UNSET), f"{label}: {np.count_nonzero(m == M_UNSET)} min_coeff not written"


def run(torch, V, C, walk, precision=hx.FP64, max_depth=6):
    n = C.shape[0]
    v, m = unset_outputs(torch, n)
    st = hx.hexval_stats_t()
    opts = hx.make_opts(precision=precision, max_depth=max_depth, walk_layers=walk,
                        stream=torch.cuda.current_stream(), stats=st)
    hx.hexval_check_ex(hx.make_mesh(to_dev(torch, V), to_dev(torch, C)), opts, v, m)
    torch.cuda.synchronize()
    v, m = v.cpu().numpy(), m.cpu().numpy()
    assert_all_written(v, m, f"walk {walk} precision {precision}")
    return v, m, st.as_dict()


def check_layout(torch, V, C, label, expect_stride=None, precisions=(hx.FP64, hx.FP32_FILTER)):
    for prec in precisions:
        base_v, base_m, st0 = run(torch, V, C, -1, prec)
        assert st0["walk_layers"] == 0
        assert_parity(base_v, base_m if prec == hx.FP64 else None, V, C, label=f"{label} plain")
        for walk in (16, 3, 64):
            v, m, st = run(torch, V, C, walk, prec)
            say(f"{label} precision {prec} walk {walk}: stride {st['walk_stride']}, rounds {st['n_rounds']}")
            # meshes of fewer than 8 layers of the smallest stride are not searched
            assert st["walk_layers"] == (walk if C.shape[0] >= 8 * 4096 else 0)
            assert st["n_recheck"] == st0["n_recheck"], "FP32 filter decisions differ"
            if expect_stride is not None:
                assert st["walk_stride"] == expect_stride
            assert np.array_equal(v, base_v), f"{label}: walk {walk} verdicts differ from plain tiles"
            assert np.array_equal(m.view(np.int64), base_m.view(np.int64)), f"{label}: walk {walk} min_coeff"


def test_lattice_walks_with_its_layer_stride():
    torch = torch_cuda()
    V, C = lattice()
    check_layout(torch, V, C, "lattice", expect_stride=NX * NY)


def test_partial_last_layer_and_single_layer_tiles():
    torch = torch_cuda()
    V, C = lattice()
    n = C.shape[0] - 1234
    check_layout(torch, V, C[:n], "partial layer", expect_stride=NX * NY)


def test_permuted_elements_take_the_full_gather():
    torch = torch_cuda()
    V, C = lattice()
    perm = np.random.default_rng(3).permutation(C.shape[0])
    check_layout(torch, V, C[perm], "permuted")


def test_broken_structure_falls_back_per_lane():
    torch = torch_cuda()
    V, C = lattice(jitter=0.2)
    rng = np.random.default_rng(4)
    C = C.copy()
    rows = rng.choice(C.shape[0], C.shape[0] // 10, replace=False)
    C[rows] = C[rng.integers(0, C.shape[0], rows.size)]          # other elements' rows
    flip = rng.choice(C.shape[0], 500, replace=False)
    C[flip] = C[flip][:, [4, 5, 6, 7, 0, 1, 2, 3]]                # reflected: invalid
    check_layout(torch, V, C, "broken", expect_stride=NX * NY)


def test_two_lattices_with_different_layers():
    torch = torch_cuda()
    V1, C1 = lattice(seed=5)
    V2, C2 = synth.warped_lattice(90, 80, 7, seed=6, jitter_fraction=0.3)
    V = np.concatenate([V1, V2])
    C = np.concatenate([C1, C2 + V1.shape[0]]).astype(np.int32)
    check_layout(torch, V, C, "two lattices", expect_stride=NX * NY)


def test_stacked_part_then_independent_near_degenerate_hexes():
    # as the precision-stress mesh: the walk covers the lattice's layers and
    # the appended hexes (every one uncertain in FP32) come as plain tiles
    torch = torch_cuda()
    V, C = lattice()
    V, C = synth.append_independent(V, C, synth.near_degenerate_hexes(9000, seed=8))
    check_layout(torch, V, C, "lattice + near-degenerate", expect_stride=NX * NY)


def test_fp32_rechecks_scattered_over_the_mesh():
    # every vertex jittered: the elements FP32 cannot decide are spread over
    # many waves, which recheck them in FP64 in batches of 64 from a per-wave
    # buffer (the waves where most lanes need it redo them in place)
    torch = torch_cuda()
    V, C = synth.warped_lattice(NX, NY, NZ, seed=19, jitter=0.45, jitter_all=True)
    check_layout(torch, V, C, "scattered rechecks", expect_stride=NX * NY)
    V2, C2 = synth.append_independent(V, C, synth.near_degenerate_hexes(20000, seed=20))
    check_layout(torch, V2, C2, "scattered and clustered rechecks", expect_stride=NX * NY)


def test_small_layers_are_not_walked():
    torch = torch_cuda()
    V, C = synth.warped_lattice(30, 30, 40, seed=7, jitter_fraction=0.1)   # 900 per layer
    check_layout(torch, V, C, "small layers", expect_stride=0)


def test_tiny_and_single_element_meshes():
    torch = torch_cuda()
    V, C = lattice()
    for n in (1, 7, 255, 4551):
        check_layout(torch, V, C[:n], f"first {n}", precisions=(hx.FP64,))


def test_walk_at_depth_cap_zero_and_edges():
    torch = torch_cuda()
    V, C = lattice(jitter=0.4)
    for walk in (-1, 16):
        v, m, _ = run(torch, V, C, walk, max_depth=0)
        assert_parity(v, m, V, C, max_depth=0, label=f"cap 0 walk {walk}")


def test_min_jacobian_walk_equals_plain_tiles():
    torch = torch_cuda()
    V, C = lattice(jitter=0.3)
    pts, conn = to_dev(torch, V), to_dev(torch, C)
    res = {}
    for walk in (-1, 16):
        n = C.shape[0]
        status, lo = unset_outputs(torch, n)
        hi = lo.clone()
        opts = hx.make_opts(walk_layers=walk, stream=torch.cuda.current_stream())
        hx.hexval_min_jacobian(hx.make_mesh(pts, conn, n), opts, 1e-3, lo, hi, status)
        torch.cuda.synchronize()
        res[walk] = (lo.cpu().numpy(), hi.cpu().numpy(), status.cpu().numpy())
        assert_all_written(res[walk][2], res[walk][0], f"min J walk {walk}")
        assert_all_written(res[walk][2], res[walk][1], f"min J walk {walk}")
    for a, b in zip(res[-1], res[16]):
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8))
    ref = oracle.min_jacobian(V, C, rtol=1e-3, max_depth=6)
    lo, hi, _ = res[16]
    assert not np.any((lo > ref["hi"]) | (ref["lo"] > hi)), "disjoint min J intervals"


def batch_run(torch, meshes, walk, precision=hx.FP64, max_depth=6):
    outs = [unset_outputs(torch, C.shape[0]) for _, C in meshes]
    vs = [o[0] for o in outs]
    ms = [o[1] for o in outs]
    descs = [hx.make_mesh(V, C) for V, C in meshes]
    st = hx.hexval_stats_t()
    opts = hx.make_opts(precision=precision, max_depth=max_depth, walk_layers=walk,
                        stream=torch.cuda.current_stream(), stats=st)
    hx.hexval_check_batched(descs, opts, vs, ms)
    torch.cuda.synchronize()
    vs, ms = [v.cpu().numpy() for v in vs], [m.cpu().numpy() for m in ms]
    for k, (v, m) in enumerate(zip(vs, ms)):
        assert_all_written(v, m, f"batched walk {walk} precision {precision} mesh {k}")
    return vs, ms, st


def mixed_batch():
    """Host arrays of a batch: walkable lattices (one cut inside a layer,
    one with broken rows, one followed by near-degenerate hexes), and meshes
    the walk must leave to plain tiles (permuted, small layers, too few
    layers, tiny, empty)."""
    V, C = lattice()
    rng = np.random.default_rng(9)
    Cb = C.copy()
    rows = rng.choice(C.shape[0], C.shape[0] // 10, replace=False)
    Cb[rows] = Cb[rng.integers(0, C.shape[0], rows.size)]
    Vn, Cn = synth.append_independent(*synth.warped_lattice(75, 60, 12, seed=12, jitter_fraction=0.1),
                                      synth.near_degenerate_hexes(5000, seed=13))
    return [
        (V, C),
        synth.warped_lattice(64, 64, 9, seed=14, jitter_fraction=0.3),     # 9 layers of 4096
        (V, C[: C.shape[0] - 1234]),
        (V, Cb),
        (Vn, Cn),
        (V, C[np.random.default_rng(15).permutation(C.shape[0])]),
        synth.warped_lattice(30, 30, 40, seed=16, jitter_fraction=0.1),     # layers of 900
        synth.warped_lattice(80, 70, 6, seed=17, jitter_fraction=0.1),      # 6 layers
        (V, C[:7]),
        (V[:0], C[:0]),
        synth.warped_lattice(100, 90, 10, seed=18, jitter_fraction=0.6),
    ]


@pytest.mark.parametrize("precision", [hx.FP64, hx.FP32_FILTER])
def test_batched_walk_equals_plain_tiles_and_oracle(precision):
    torch = torch_cuda()
    host = mixed_batch()
    meshes = [(to_dev(torch, V), to_dev(torch, C.astype(np.int32))) for V, C in host]
    base_v, base_m, st0 = batch_run(torch, meshes, -1, precision)
    assert st0.walk_layers == 0
    for k, (V, C) in enumerate(host):
        if C.shape[0]:
            assert_parity(base_v[k], base_m[k] if precision == hx.FP64 else None, V, C,
                          label=f"batched plain mesh {k}")
    for walk in (16, 3, 64):
        v, m, st = batch_run(torch, meshes, walk, precision)
        say(f"batched walk {walk} precision {precision}: rechecks {st.n_recheck}, rounds {st.n_rounds}")
        assert st.walk_layers == (walk if precision == hx.FP64 else 0)   # batches walk in FP64 only
        assert st.walk_stride == 0
        assert st.n_recheck == st0.n_recheck, "FP32 filter decisions differ"
        for k in range(len(host)):
            assert np.array_equal(v[k], base_v[k]), f"mesh {k}: walk {walk} verdicts differ from plain tiles"
            assert np.array_equal(m[k].view(np.int64), base_m[k].view(np.int64)), f"mesh {k}: walk {walk} min_coeff"


def test_batched_walk_depth_zero_and_tuned():
    torch = torch_cuda()
    host = mixed_batch()[:6]
    meshes = [(to_dev(torch, V), to_dev(torch, C.astype(np.int32))) for V, C in host]
    for prec in (hx.FP64, hx.FP32_FILTER):
        base_v, base_m, _ = batch_run(torch, meshes, -1, prec, max_depth=0)
        v, m, st = batch_run(torch, meshes, 16, prec, max_depth=0)
        for k in range(len(host)):
            assert np.array_equal(v[k], base_v[k]), f"cap 0 mesh {k}"
        if prec == hx.FP64:
            for k, (V, C) in enumerate(host):
                assert_parity(v[k], m[k], V, C, max_depth=0, label=f"cap 0 mesh {k}")
    # the tuner's choice (walk or not) never changes results
    v, m, st = batch_run(torch, meshes, 0, hx.FP64)
    base_v, base_m, _ = batch_run(torch, meshes, -1, hx.FP64)
    for k in range(len(host)):
        assert np.array_equal(v[k], base_v[k])
        assert np.array_equal(m[k].view(np.int64), base_m[k].view(np.int64))
