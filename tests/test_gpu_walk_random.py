"""Seeded random layouts through the column and row walks: every result
equal to the plain-tile pass bit for bit, with outputs that start as values
no kernel writes (HIP path through the C ABI).  The layouts mix stacked,
jittered, cut, partly permuted and row-replaced meshes, near-degenerate
hexes appended after a lattice, depth caps 0, 3 and 6, single meshes in FP64
and with the FP32 filter (also without the min output), FP64 batches, and
quadrangle meshes."""
import numpy as np
import pytest

from paper_1706_01613_amd import hexval as hx
from paper_1706_01613_amd import synth
from tests._gpu import say, to_dev, torch_cuda

pytestmark = pytest.mark.gpu

V_UNSET, M_UNSET = 0xEE, -7.5e300
N_CASES = 80


def _unset(torch, n):
    return (torch.full((n,), V_UNSET, dtype=torch.uint8, device="cuda"),
            torch.full((n,), M_UNSET, dtype=torch.float64, device="cuda"))


def _written(v, m, label):
    assert not np.any(v == V_UNSET) and not np.any(m == M_UNSET), f"{label}: outputs not written"


def _same(a, b, label):
    (v1, m1), (v2, m2) = a, b
    assert np.array_equal(v1, v2), f"{label}: verdicts differ"
    assert np.array_equal(np.nan_to_num(m1, nan=7.0).view(np.int64),
                          np.nan_to_num(m2, nan=7.0).view(np.int64)), f"{label}: min values differ"


def _layout(rng):
    nx, ny, nz = int(rng.integers(40, 140)), int(rng.integers(40, 140)), int(rng.integers(4, 40))
    seed = int(rng.integers(1 << 30))
    kind = int(rng.integers(0, 3))
    if kind == 0:
        V, C = synth.warped_lattice(nx, ny, nz, seed=seed, jitter_fraction=float(rng.uniform(0, 0.05)))
    elif kind == 1:
        V, C = synth.warped_lattice(nx, ny, nz, seed=seed, jitter=float(rng.uniform(0.05, 0.5)), jitter_all=True)
    else:
        V, C = synth.warped_lattice(nx, ny, nz, seed=seed)
        V, C = synth.append_independent(V, C, synth.near_degenerate_hexes(int(rng.integers(100, 20000)),
                                                                           seed=seed + 1))
    C = C.copy()
    r = rng.random()
    if r < 0.2:
        k = int(rng.integers(1, C.shape[0] // 5))
        rows = rng.choice(C.shape[0], k, replace=False)
        C[rows] = C[rng.integers(0, C.shape[0], k)]
    elif r < 0.3:
        a, b = sorted(int(x) for x in rng.integers(0, C.shape[0], 2))
        C[a:b] = C[a:b][rng.permutation(b - a)]
    if rng.random() < 0.3:
        C = C[: int(rng.integers(1, C.shape[0] + 1))]
    return V, np.ascontiguousarray(C.astype(np.int32))


def _single(torch, Vd, Cd, walk, prec, cap):
    v, m = _unset(torch, Cd.shape[0])
    st = hx.hexval_stats_t()
    opts = hx.make_opts(precision=prec, max_depth=cap, walk_layers=walk,
                        stream=torch.cuda.current_stream(), stats=st)
    hx.hexval_check_ex(hx.make_mesh(Vd, Cd), opts, v, m)
    torch.cuda.synchronize()
    out = (v.cpu().numpy(), m.cpu().numpy())
    _written(*out, f"walk {walk} precision {prec}")
    return out, st


def _verdicts_only(torch, Vd, Cd, walk, prec, cap):
    v, _ = _unset(torch, Cd.shape[0])
    opts = hx.make_opts(precision=prec, max_depth=cap, walk_layers=walk, stream=torch.cuda.current_stream())
    hx.hexval_check_ex(hx.make_mesh(Vd, Cd), opts, v, None)
    torch.cuda.synchronize()
    v = v.cpu().numpy()
    assert not np.any(v == V_UNSET), f"walk {walk} precision {prec}, no min output: verdicts not written"
    return v


def _batch(torch, meshes, walk, cap):
    outs = [_unset(torch, c.shape[0]) for _, c in meshes]
    opts = hx.make_opts(max_depth=cap, walk_layers=walk, stream=torch.cuda.current_stream())
    hx.hexval_check_batched([hx.make_mesh(a, b) for a, b in meshes], opts,
                            [o[0] for o in outs], [o[1] for o in outs])
    torch.cuda.synchronize()
    res = [(v.cpu().numpy(), m.cpu().numpy()) for v, m in outs]
    for k, r in enumerate(res):
        _written(*r, f"batched walk {walk} mesh {k}")
    return res


def _quads(torch, Vd, Cd, walk):
    v, m = _unset(torch, Cd.shape[0])
    opts = hx.make_opts(walk_layers=walk, stream=torch.cuda.current_stream())
    hx.hexval_quad_check(hx.make_mesh(Vd, Cd), opts, v, m)
    torch.cuda.synchronize()
    out = (v.cpu().numpy(), m.cpu().numpy())
    _written(*out, f"quad walk {walk}")
    return out


def test_random_layouts_walk_equals_plain_tiles():
    torch = torch_cuda()
    rng = np.random.default_rng(2024)
    walked = 0
    for case in range(N_CASES):
        V, C = _layout(rng)
        Vd, Cd = to_dev(torch, V), to_dev(torch, C)
        cap = int(rng.choice([0, 3, 6]))
        for prec in (hx.FP64, hx.FP32_FILTER):
            base, bst = _single(torch, Vd, Cd, -1, prec, cap)
            for walk in (16, int(rng.integers(1, 65))):
                out, st = _single(torch, Vd, Cd, walk, prec, cap)
                _same(base, out, f"case {case} precision {prec} walk {walk} cap {cap}")
                assert st.n_recheck == bst.n_recheck
                walked += st.walk_stride > 0
            if case % 5 == 0:
                assert np.array_equal(_verdicts_only(torch, Vd, Cd, 16, prec, cap), base[0]), \
                    f"case {case} precision {prec}: verdicts without the min output differ"
        if case % 4 == 0:
            meshes = [(Vd, Cd)]
            for _ in range(int(rng.integers(1, 5))):
                V2, C2 = _layout(rng)
                meshes.append((to_dev(torch, V2), to_dev(torch, C2)))
            for a, b in zip(_batch(torch, meshes, -1, cap), _batch(torch, meshes, 16, cap)):
                _same(a, b, f"case {case} batch")
        if case % 3 == 0:
            qx, qy = int(rng.integers(4096, 9000)), int(rng.integers(4, 40))
            QV, QC = synth.quad_lattice(qx, qy, seed=int(rng.integers(1 << 30)),
                                        jitter_fraction=float(rng.uniform(0, 0.3)))
            QC = QC.copy()
            if rng.random() < 0.3:
                k = QC.shape[0] // 10
                rows = rng.choice(QC.shape[0], k, replace=False)
                QC[rows] = QC[rng.integers(0, QC.shape[0], k)]
            QVd, QCd = to_dev(torch, QV), to_dev(torch, np.ascontiguousarray(QC.astype(np.int32)))
            _same(_quads(torch, QVd, QCd, -1), _quads(torch, QVd, QCd, 16), f"case {case} quads")
        if case % 20 == 0:
            say(f"random layouts: case {case} done, {walked} walked runs so far")
    assert walked > N_CASES // 2, "too few layouts were walked"
