"""GPU: the batched entry point (one persistent launch over many meshes)
gives, for every mesh, the results of checking that mesh alone, and they
agree with the oracle; the autotuned launch shape never changes results."""
import numpy as np
import pytest

import oracle
from paper_1706_01613_amd import hexval as hx
from paper_1706_01613_amd import synth
from tests._gpu import say, assert_parity, normwise_error, torch_cuda

U32 = 2.0 ** -24

pytestmark = pytest.mark.gpu

_say = say


def _alone(torch, V, C, **kw):
    v, m, _ = hx.check(V, C, **kw)
    torch.cuda.synchronize()
    return v, m


def _batched(torch, meshes, precision=hx.FP64, stats=None, **kw):
    # outputs start as values no kernel writes (0xEE, NaN): an element left
    # without a result cannot pass on an earlier run's values in reused memory
    vs = [torch.full((C.shape[0] if C is not None else V.shape[0],), 0xEE, dtype=torch.uint8, device="cuda")
          for V, C in meshes]
    ms = [torch.full((v.shape[0],), float("nan"), dtype=torch.float64, device="cuda") for v in vs]
    descs = [hx.make_mesh(V, C) for V, C in meshes]
    opts = hx.make_opts(precision=precision, stream=torch.cuda.current_stream(), stats=stats, **kw)
    hx.hexval_check_batched(descs, opts, vs, ms)
    torch.cuda.synchronize()
    return vs, ms


@pytest.mark.parametrize("precision", [hx.FP64, hx.FP32_FILTER])
def test_batched_equals_alone_and_oracle(precision):
    torch = torch_cuda()
    _say(f"batched 60 meshes precision {precision}")
    meshes = list(synth.batched_meshes_torch(60, lo=1.0, hi=4.5, seed=11))
    # mixed layouts: a few [n,8,3] meshes and an empty one
    for s in range(3):
        P = torch.from_numpy(synth.independent_hexes(500 + 137 * s, noise=0.45, seed=50 + s)).cuda()
        meshes.append((P, None))
    meshes.append((torch.empty((0, 3), dtype=torch.float64, device="cuda"),
                   torch.empty((0, 8), dtype=torch.int32, device="cuda")))
    st = hx.hexval_stats_t()
    vs, ms = _batched(torch, meshes, precision, stats=st)
    assert st.n_elements == sum(v.shape[0] for v in vs)
    for k, ((V, C), v, m) in enumerate(zip(meshes, vs, ms)):
        va, ma = _alone(torch, V, C, precision=precision)
        assert torch.equal(v, va), k
        assert torch.equal(torch.nan_to_num(m, 7.0), torch.nan_to_num(ma, 7.0)), k
    for k in list(range(0, 64, 7)):
        V, C = meshes[k]
        Vh = V.cpu().numpy()
        Ch = C.cpu().numpy() if C is not None else None
        assert_parity(vs[k].cpu().numpy(), ms[k].cpu().numpy() if precision == hx.FP64 else None,
                      Vh, Ch, label=f"mesh {k}")


@pytest.mark.parametrize("precision", [hx.FP64, hx.FP32_FILTER])
def test_batched_connectivity_meshes_equal_alone(precision):
    # every non-empty mesh has trusted connectivity: the first pass
    # prefetches each tile's rows, looking the tile's mesh up first; ragged
    # meshes (many smaller than a tile), empty ones, several launch shapes
    # and the depth-0 variant (edge values in step 2)
    torch = torch_cuda()
    _say(f"batched connectivity-only meshes, precision {precision}")
    meshes = list(synth.batched_meshes_torch(90, lo=0.0, hi=4.2, seed=21))
    empty = (torch.empty((0, 3), dtype=torch.float64, device="cuda"),
             torch.empty((0, 8), dtype=torch.int32, device="cuda"))
    meshes.insert(0, empty)
    meshes.insert(40, empty)
    meshes.append(empty)
    for kw in [{}, {"block_threads": 64, "grid_blocks": 48}, {"block_threads": 128}, {"max_depth": 0}]:
        vs, ms = _batched(torch, meshes, precision, **kw)
        for k, ((V, C), v, m) in enumerate(zip(meshes, vs, ms)):
            va, ma = _alone(torch, V, C, precision=precision, **kw)
            assert torch.equal(v, va), (k, kw)
            assert torch.equal(torch.nan_to_num(m, 7.0), torch.nan_to_num(ma, 7.0)), (k, kw)
    vs, ms = _batched(torch, meshes, precision)
    for k in (1, 17, 52, len(meshes) - 2):
        V, C = meshes[k]
        assert_parity(vs[k].cpu().numpy(), ms[k].cpu().numpy() if precision == hx.FP64 else None,
                      V.cpu().numpy(), C.cpu().numpy(), label=f"mesh {k}")


def test_launch_shape_does_not_change_results():
    torch = torch_cuda()
    V, C = synth.warped_lattice_torch(60, 50, 40, jitter=0.4, seed=3)
    ref = _alone(torch, V, C)
    for block, grid in [(64, 0), (128, 16), (256, 0), (256, 1024), (192, 4096)]:
        v, m = _alone(torch, V, C, block_threads=block, grid_blocks=grid)
        assert torch.equal(v, ref[0]) and torch.equal(m, ref[1]), (block, grid)
    vs, ms = _batched(torch, [(V, C), (V, C)], block_threads=64, grid_blocks=64)
    assert torch.equal(vs[0], ref[0]) and torch.equal(vs[1], ref[0])


@pytest.mark.timeout(1500)
def test_batched_10000_lattices_full_size():
    """10,000 meshes, hex counts log-uniform in [1e2, 1e6] (about 1.1e9 hexes),
    every vertex jittered by U(0, 0.6) cell, cap 6, one persistent launch:
    the FP32-filter batch (the benchmarked configuration) and the FP64 batch
    give bitwise-identical verdicts on every element, and every mesh is
    streamed through the oracle: verdicts bit-exact on all 1.1e9 elements,
    FP64 min_coeff within 1e-12 of each element's largest coefficient, and
    the FP32-decided min_coeff within its forward bound."""
    torch = torch_cuda()
    _say("10,000 jittered lattices: generating the meshes on the device")
    meshes = list(synth.batched_meshes_torch(10000, seed=4))
    total = sum(C.shape[0] for _, C in meshes)
    _say(f"10,000 jittered lattices: {total} hexes")
    st = hx.hexval_stats_t()
    st.timing = 1
    vs32, ms32 = _batched(torch, meshes, hx.FP32_FILTER, stats=st)
    _say(f"10,000 jittered lattices, FP32 filter stats: {st.as_dict()}")
    assert st.n_elements == total and total > 5e8
    st64 = hx.hexval_stats_t()
    vs64, ms64 = _batched(torch, meshes, hx.FP64, stats=st64)
    _say(f"10,000 jittered lattices, FP64 stats: {st64.as_dict()}")
    v32_all, v64_all = torch.cat(vs32), torch.cat(vs64)
    diff = int((v32_all != v64_all).sum())
    assert diff == 0, f"{diff} verdicts differ between the FP32-filter and FP64 batches"
    v64_host = v64_all.cpu().numpy()
    m64_host = torch.cat(ms64).cpu().numpy()
    m32_host = torch.cat(ms32).cpu().numpy()
    del v32_all, v64_all
    offsets = np.cumsum([0] + [C.shape[0] for _, C in meshes])
    worst64 = worst32 = 0.0
    for k, (V, C) in enumerate(meshes):
        a, b = offsets[k], offsets[k + 1]
        if b == a:
            continue
        Vh, Ch = V.cpu().numpy(), C.cpu().numpy()
        ref = oracle.check(Vh, Ch)
        bad = np.nonzero(v64_host[a:b] != ref["verdict"])[0]
        assert bad.size == 0, (f"mesh {k}: {bad.size} verdict mismatches, first ids {bad[:10]}, "
                               f"gpu {v64_host[a:b][bad[:10]]} oracle {ref['verdict'][bad[:10]]}")
        coeffs = oracle.coefficients(Vh, Ch)
        bmax = np.abs(coeffs).max(axis=1)
        del coeffs
        finite = np.isfinite(ref["min_coeff"])
        m64 = m64_host[a:b]
        assert (np.isnan(m64) == ~finite).all(), f"mesh {k}: NaN pattern of min_coeff differs"
        err = normwise_error(m64[finite], bmax[finite], ref["min_coeff"][finite])
        worst64 = max(worst64, float(err.max(initial=0.0)))
        assert worst64 <= 1e-12, f"mesh {k}: FP64 min_coeff error {worst64}"
        # FP32-decided elements: |m32 - m| <= 256 u32 M^ (the kernel bound;
        # 300 u32 with M^ taken from the oracle's edge vectors)
        lim = 300.0 * U32 * oracle.scale(Vh, Ch)
        d32 = np.abs(m32_host[a:b] - ref["min_coeff"])
        assert (d32[finite] <= lim[finite]).all(), f"mesh {k}: FP32 min_coeff outside its bound"
        worst32 = max(worst32, float((d32[finite] / np.where(bmax[finite] > 0, bmax[finite], 1.0)).max(initial=0.0)))
        if k % 500 == 0:
            _say(f"10,000 jittered lattices: oracle done through mesh {k} ({b} hexes), "
                 f"FP64 min err {worst64:.2e}, FP32 min err {worst32:.2e}")
    _say(f"10,000 jittered lattices: all {total} verdicts equal the oracle's; "
         f"FP64 min_coeff err {worst64:.2e}, FP32 {worst32:.2e}")


@pytest.mark.parametrize("precision", [hx.FP64, hx.FP32_FILTER])
def test_batched_tiny_queue_rounds_equal_alone(precision):
    # a 64-node subdivision queue: most listed elements of the batch are
    # deferred when their wave's buffer is appended and checked in later
    # rounds; every mesh still gets the verdicts of checking it alone
    # (lattices jittered like the single-mesh tiny-queue case, whose trees
    # stay shallow enough for such a queue to make progress)
    torch = torch_cuda()
    dims = [(20 + k % 7, 18 + k % 5, 10 + k % 9) for k in range(12)]
    meshes = [synth.warped_lattice_torch(nx, ny, nz, jitter=0.45, seed=40 + k) for k, (nx, ny, nz) in enumerate(dims)]
    st = hx.hexval_stats_t()
    vs, ms = _batched(torch, meshes, precision, stats=st, queue_capacity=64)
    _say(f"tiny queue batch: {st.as_dict()}")
    assert st.n_rounds > 1
    for k, ((V, C), v) in enumerate(zip(meshes, vs)):
        va, _ = _alone(torch, V, C, precision=precision)
        assert torch.equal(v, va), k


def test_batched_without_min_outputs_and_prepared_args():
    # min_coeffs may be omitted; prepared C arrays give the same results on
    # repeated calls
    torch = torch_cuda()
    meshes = list(synth.batched_meshes_torch(25, lo=1.0, hi=4.0, seed=41))
    vs = [torch.empty(C.shape[0], dtype=torch.uint8, device="cuda") for _, C in meshes]
    args = hx.BatchArgs([hx.make_mesh(V, C) for V, C in meshes], vs)
    opts = hx.make_opts(stream=torch.cuda.current_stream())
    for rep in range(2):
        hx.hexval_check_batched(args, opts)
        torch.cuda.synchronize()
        for k, ((V, C), v) in enumerate(zip(meshes, vs)):
            va, _ = _alone(torch, V, C)
            assert torch.equal(v, va), (rep, k)


def test_batched_index_validation():
    # index validation on: a batch whose meshes have an out-of-range index
    # here and there gets BAD_INPUT exactly there, and otherwise the
    # verdicts of each mesh checked alone
    torch = torch_cuda()
    meshes = list(synth.batched_meshes_torch(12, lo=2.0, hi=4.0, seed=51))
    bad = {}
    for k in (2, 7, 11):
        V, C = meshes[k]
        e = C.shape[0] // 2
        C[e, 5] = V.shape[0] + 3
        bad[k] = e
    vs, _ = _batched(torch, meshes, hx.FP64, validate_indices=True)
    for k, ((V, C), v) in enumerate(zip(meshes, vs)):
        va, _ = _alone(torch, V, C, validate_indices=True)
        assert torch.equal(v, va), k
        if k in bad:
            assert int(v[bad[k]]) == hx.BAD_INPUT, k
