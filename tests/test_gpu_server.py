"""GPU: the request queue with continuous batching.  Each request's result is
the same alone and in the mix (bitwise: the arithmetic of an element never
depends on what else runs), host-uploaded requests match device-resident
ones, and admission respects the HBM budget."""
import numpy as np
import pytest

from paper_1706_01613_amd import hexval as hx
from paper_1706_01613_amd import loadgen, synth
from tests._gpu import assert_parity, say, torch_cuda

pytestmark = pytest.mark.gpu


_say = say


def _pool(torch, n, seed, lo=3.0, hi=5.3):
    rng = np.random.default_rng(seed)
    sizes = np.rint(10.0 ** rng.uniform(lo, hi, size=n)).astype(int)
    return [synth.near_degenerate_mesh_torch(int(s), seed=seed * 100 + k) for k, s in enumerate(sizes)]


def _alone(torch, V, C, precision):
    v, m, _ = hx.check(V, C, precision=precision)
    torch.cuda.synchronize()
    return v, m


def _templates(meshes, host=False):
    out = []
    for V, C in meshes:
        r = hx.hexval_request_t()
        r.mesh = hx.make_mesh(V, C)
        if host:
            r.mesh.points = None
            r.mesh.connectivity = None
            r.host_points = V.data_ptr()
            r.host_conn = C.data_ptr()
        out.append(r)
    return out


def _outputs(torch, arena, off, n):
    v = arena[off:off + n]
    a = off + (n + 7) // 8 * 8
    m = arena[a:a + 8 * n].view(torch.float64)
    return v, m


@pytest.mark.parametrize("precision", [hx.FP64, hx.FP32_FILTER])
def test_server_mix_equals_alone(precision):
    torch = torch_cuda()
    meshes = _pool(torch, 10, seed=3)
    alone = [_alone(torch, V, C, precision) for V, C in meshes]
    opts = hx.make_opts(precision=precision)
    sv = hx.hexval_server_create(opts, 8 << 30, 4)
    try:
        # 40 requests, all arriving at once (maximal overlap), then 40 spread out
        idx = np.arange(40) % 10
        arrival = np.concatenate([np.zeros(20), np.linspace(0, 0.02, 20)])
        sizes = [meshes[i][1].shape[0] for i in idx]
        arena = torch.empty(loadgen.arena_bytes(sizes), dtype=torch.uint8, device="cuda")
        lat, st, off, wall = loadgen.run(sv, arrival, idx, _templates(meshes), arena)
        torch.cuda.synchronize()
        assert (st == hx.OK).all()
        for k, i in enumerate(idx):
            v, m = _outputs(torch, arena, int(off[k]), sizes[k])
            assert torch.equal(v, alone[i][0]), k
            assert torch.equal(torch.nan_to_num(m, 7.0), torch.nan_to_num(alone[i][1], 7.0)), k
        assert (lat > 0).all()
    finally:
        hx.hexval_server_destroy(sv)
    V, C = meshes[0]
    assert_parity(alone[0][0].cpu().numpy(), None, V.cpu().numpy(), C.cpu().numpy(), label="pool 0")


def test_server_host_upload_and_budget():
    torch = torch_cuda()
    meshes = _pool(torch, 6, seed=5, lo=4.0, hi=5.0)
    host = [(V.cpu().pin_memory(), C.cpu().pin_memory()) for V, C in meshes]
    alone = [_alone(torch, V, C, hx.FP64) for V, C in meshes]
    # budget: the slot workspaces plus room for about one uploaded mesh
    up = max(V.numel() * 8 + C.numel() * 4 for V, C in meshes)
    opts = hx.make_opts()
    per_slot = 2 * (1 << 20) * 272 + 2 ** 16 * 220 + (1 << 20) * 12   # generous estimate
    sv = hx.hexval_server_create(opts, 2 * per_slot + int(1.2 * up) + (64 << 20), 2)
    try:
        idx = np.arange(12) % 6
        sizes = [meshes[i][1].shape[0] for i in idx]
        arena = torch.empty(loadgen.arena_bytes(sizes), dtype=torch.uint8, device="cuda")
        tmpl = _templates(host, host=True)
        for t, (V, C) in zip(tmpl, host):
            t.mesh.n_points = V.shape[0]
        lat, st, off, _ = loadgen.run(sv, np.zeros(12), idx, tmpl, arena)
        torch.cuda.synchronize()
        assert (st == hx.OK).all()
        for k, i in enumerate(idx):
            v, m = _outputs(torch, arena, int(off[k]), sizes[k])
            assert torch.equal(v, alone[i][0]), k
        # a request whose upload can never fit is refused at submission
        big = hx.hexval_request_t()
        big.mesh = hx.hexval_mesh_t(None, 1 << 33, None, 1 << 33)
        big.host_points = host[0][0].data_ptr()
        big.host_conn = host[0][1].data_ptr()
        big.verdicts = arena.data_ptr()
        with pytest.raises(hx.HexvalError) as e:
            hx.hexval_server_submit(sv, big)
        assert e.value.status == hx.E_BUSY
    finally:
        hx.hexval_server_destroy(sv)


def test_server_bad_request_does_not_fail_its_batch():
    # with index validation on, a device-resident request that gives no
    # vertex count passes submission but is refused when run; queued with
    # good requests that arrive at the same time, only it reports the error
    torch = torch_cuda()
    meshes = _pool(torch, 6, seed=9, lo=3.0, hi=4.5)
    alone = [hx.check(V, C, validate_indices=True)[0] for V, C in meshes]
    torch.cuda.synchronize()
    tmpl = _templates(meshes)
    tmpl[3].mesh.n_points = 0
    sv = hx.hexval_server_create(hx.make_opts(validate_indices=True), 8 << 30, 1)
    try:
        idx = np.arange(12) % 6
        sizes = [meshes[i][1].shape[0] for i in idx]
        arena = torch.empty(loadgen.arena_bytes(sizes), dtype=torch.uint8, device="cuda")
        _, st, off, _ = loadgen.run(sv, np.zeros(12), idx, tmpl, arena)
        torch.cuda.synchronize()
        for k, i in enumerate(idx):
            if i == 3:
                assert st[k] == hx.E_ARG, k
            else:
                assert st[k] == hx.OK, k
                v, _ = _outputs(torch, arena, int(off[k]), sizes[k])
                assert torch.equal(v, alone[i]), k
    finally:
        hx.hexval_server_destroy(sv)


def _slot_bytes(opts):
    # the per-slot workspace size, as create reports it when the budget is too small
    with pytest.raises(hx.HexvalError) as e:
        hx.hexval_server_create(opts, 1, 1)
    msg = str(e.value)
    return int(msg[msg.rindex("(") + 1:].split()[0])


def test_server_upload_buffers_fit_the_budget():
    # room for the slot workspaces plus a little over two of the smaller
    # uploads: slots holding upload buffers from earlier requests must give
    # them back for a larger one to run, and every request still completes
    torch = torch_cuda()
    meshes = [synth.near_degenerate_mesh_torch(s, seed=40 + k) for k, s in enumerate((20000, 22000, 36000))]
    host = [(V.cpu().pin_memory(), C.cpu().pin_memory()) for V, C in meshes]
    alone = [_alone(torch, V, C, hx.FP64) for V, C in meshes]
    up = [(V.numel() * 8 + 255) // 256 * 256 + C.numel() * 4 for V, C in meshes]
    opts = hx.make_opts()
    slots = 3
    room = max(up[0] + up[1], up[2]) + 4096
    # buffers for the second and the third request cannot be held together
    assert up[1] + up[2] > room
    sv = hx.hexval_server_create(opts, slots * _slot_bytes(opts) + room, slots)
    try:
        idx = np.array([0, 1, 2, 0, 1, 2, 1, 0, 2, 2, 0, 1])
        sizes = [meshes[i][1].shape[0] for i in idx]
        arena = torch.empty(loadgen.arena_bytes(sizes), dtype=torch.uint8, device="cuda")
        tmpl = _templates(host, host=True)
        for t, (V, C) in zip(tmpl, host):
            t.mesh.n_points = V.shape[0]
        _say("upload buffers: 12 requests, 3 slots")
        _, st, off, _ = loadgen.run(sv, np.zeros(12), idx, tmpl, arena)
        torch.cuda.synchronize()
        assert (st == hx.OK).all()
        for k, i in enumerate(idx):
            v, m = _outputs(torch, arena, int(off[k]), sizes[k])
            assert torch.equal(v, alone[i][0]), k
            assert torch.equal(torch.nan_to_num(m, 7.0), torch.nan_to_num(alone[i][1], 7.0)), k
    finally:
        hx.hexval_server_destroy(sv)


def test_server_ticket_is_forgotten_once_reported():
    torch = torch_cuda()
    V, C = synth.near_degenerate_mesh_torch(3000, seed=77)
    v = torch.empty(C.shape[0], dtype=torch.uint8, device="cuda")
    sv = hx.hexval_server_create(hx.make_opts(), 8 << 30, 2)
    try:
        r = hx.hexval_request_t()
        r.mesh = hx.make_mesh(V, C)
        r.verdicts = v.data_ptr()
        t1 = hx.hexval_server_submit(sv, r)
        assert hx.hexval_server_wait(sv, t1) >= 0.0
        with pytest.raises(hx.HexvalError) as e:
            hx.hexval_server_poll(sv, t1)
        assert e.value.status == hx.E_ARG
        t2 = hx.hexval_server_submit(sv, r)
        assert t2 != t1
        done = False
        while not done:
            done, lat = hx.hexval_server_poll(sv, t2)
        assert lat >= 0.0
        with pytest.raises(hx.HexvalError):
            hx.hexval_server_wait(sv, t2)
        torch.cuda.synchronize()
        assert torch.equal(v, _alone(torch, V, C, hx.FP64)[0])
    finally:
        hx.hexval_server_destroy(sv)
