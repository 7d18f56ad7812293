"""The C ABI library loads, exports every declared symbol and rejects bad
arguments without touching a GPU (CPU only)."""
import ctypes
import os
import re

import pytest

from paper_1706_01613_amd import hexval as hx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hexval.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hexval_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert "hexval_check" in names and "hexval_server_submit" in names
    L = hx.lib()
    for name in names:
        assert hasattr(L, name), name


def test_calibration_library_exports_its_header():
    header = os.path.join(ROOT, "include", "hexval_calib.h")
    text = re.sub(r"/\*.*?\*/", "", open(header).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(hexval_calib_[a-z0-9_]+)\s*\(", text)))
    assert names == ["hexval_calib_copy", "hexval_calib_fp64", "hexval_calib_read"]
    L = ctypes.CDLL(os.path.join(ROOT, "paper_1706_01613_amd", "libhexval_calib.so"))
    for name in names:
        assert hasattr(L, name), name
    # argument errors come back as status 1 without touching a GPU
    f = ctypes.c_float()
    d = ctypes.c_double()
    L.hexval_calib_read.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p]
    assert L.hexval_calib_read(None, 1 << 20, 1, ctypes.byref(f)) == 1
    L.hexval_calib_fp64.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p]
    assert L.hexval_calib_fp64(0, 1, ctypes.byref(f), ctypes.byref(d), ctypes.byref(d)) == 1


def test_struct_layouts_match_header_sizes():
    # int64 alignment: mesh 32 B, opts 56 B, stats 104 B, request 64 B
    assert ctypes.sizeof(hx.hexval_mesh_t) == 32
    assert ctypes.sizeof(hx.hexval_opts_t) == 56
    assert ctypes.sizeof(hx.hexval_stats_t) == 104
    assert ctypes.sizeof(hx.hexval_request_t) == 64


def test_defaults():
    o = hx.hexval_opts_default()
    assert (o.precision, o.max_depth, o.validate_indices, o.queue_capacity) == (hx.FP64, 6, 0, 0)
    assert (o.walk_layers, o.reserved) == (0, 0)


def _status(f, *args):
    try:
        return f(*args)
    except hx.HexvalError as e:
        return e.status


def test_argument_errors_without_gpu():
    L = hx.lib()
    assert L.hexval_check(None, None, 0, None, None) == hx.OK          # n == 0: no-op
    assert L.hexval_check(None, None, -1, None, None) == hx.E_ARG
    assert L.hexval_check(None, None, 5, 1, None) == hx.E_ARG          # NULL points
    assert "points" in hx.hexval_last_error()
    assert L.hexval_check(16, None, 5, None, None) == hx.E_ARG         # NULL verdicts
    assert L.hexval_check_ex(None, None, None, None) == hx.E_ARG
    mesh = hx.hexval_mesh_t(16, 0, None, 4)
    for field, value in [("max_depth", 21), ("max_depth", -1), ("precision", 7),
                         ("block_threads", 100), ("block_threads", 512), ("queue_capacity", -5),
                         ("walk_layers", -2), ("walk_layers", 65), ("reserved", 1)]:
        o = hx.hexval_opts_default()
        setattr(o, field, value)
        assert L.hexval_check_ex(ctypes.byref(mesh), ctypes.byref(o), 32, None) == hx.E_ARG, field
    o = hx.hexval_opts_default()
    o.validate_indices = 1
    mesh = hx.hexval_mesh_t(16, 0, 32, 4)                               # n_points missing
    assert L.hexval_check_ex(ctypes.byref(mesh), ctypes.byref(o), 32, None) == hx.E_ARG
    assert L.hexval_check_batched(None, -1, None, None, None) == hx.E_ARG
    assert L.hexval_coefficients(None, None, None) == hx.E_ARG
    mesh = hx.hexval_mesh_t(16, 0, None, 4)
    assert L.hexval_min_jacobian(None, None, 1e-3, 32, 48, None) == hx.E_ARG
    for rtol in (0.0, -1.0, float("nan"), float("inf")):
        assert L.hexval_min_jacobian(ctypes.byref(mesh), None, rtol, 32, 48, None) == hx.E_ARG
    assert L.hexval_min_jacobian(ctypes.byref(mesh), None, 1e-3, None, 48, None) == hx.E_ARG
    o = hx.hexval_opts_default()
    o.precision = hx.FP32_FILTER
    assert L.hexval_min_jacobian(ctypes.byref(mesh), ctypes.byref(o), 1e-3, 32, 48, None) == hx.E_ARG
    assert L.hexval_quad_check(None, None, 32, None) == hx.E_ARG
    assert L.hexval_quad_check(ctypes.byref(mesh), None, None, None) == hx.E_ARG
    assert L.hexval_corner_test(None, None, 32, None) == hx.E_ARG
    assert L.hexval_corner_test(ctypes.byref(mesh), None, None, None) == hx.E_ARG
    empty = hx.hexval_mesh_t(None, 0, None, 0)
    assert L.hexval_corner_test(ctypes.byref(empty), None, None, None) == hx.OK
    assert L.hexval_min_jacobian(ctypes.byref(empty), None, 1e-3, None, None, None) == hx.OK
    # the allocation-free check: its own limits are argument errors
    assert L.hexval_check_noalloc(None, None, 32, None) == hx.E_ARG
    assert L.hexval_check_noalloc(ctypes.byref(empty), None, None, None) == hx.OK
    for field, value in [("max_depth", 9), ("queue_capacity", (1 << 17) + 1), ("max_depth", 21)]:
        o = hx.hexval_opts_default()
        setattr(o, field, value)
        assert L.hexval_check_noalloc(ctypes.byref(mesh), ctypes.byref(o), 32, None) == hx.E_ARG, field
    o = hx.hexval_opts_default()
    o.max_depth = 9
    L.hexval_check_noalloc(ctypes.byref(mesh), ctypes.byref(o), 32, None)
    assert "hexval_check_noalloc" in hx.hexval_last_error()
    h = ctypes.c_void_p()
    assert L.hexval_server_create(None, 0, 1, ctypes.byref(h)) == hx.E_ARG
    assert L.hexval_server_create(None, 1 << 30, 0, ctypes.byref(h)) == hx.E_ARG
    assert L.hexval_server_destroy(None) == hx.E_ARG


def test_no_device_reports_hip_error():
    torch = pytest.importorskip("torch")
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present; this case covers hosts without one")
    L = hx.lib()
    # valid-looking arguments: the library must stop at the device check
    assert L.hexval_check(16, None, 4, 32, None) == hx.E_HIP
    assert "device" in hx.hexval_last_error()
    mesh = hx.hexval_mesh_t(16, 0, None, 4)
    assert L.hexval_min_jacobian(ctypes.byref(mesh), None, 1e-3, 32, 48, None) == hx.E_HIP
    assert L.hexval_check_noalloc(ctypes.byref(mesh), None, 32, None) == hx.E_HIP
    h = ctypes.c_void_p()
    assert L.hexval_server_create(None, 1 << 34, 2, ctypes.byref(h)) == hx.E_HIP


def test_binding_names_match_the_abi():
    for name in declared_functions():
        if name == "hexval_opts_default":
            continue
        assert hasattr(hx, name), name


def test_batch_args_marshal_once():
    # the prepared C arrays of a batched call hold the meshes and output
    # addresses in order (no GPU: nothing is called)
    meshes = [hx.hexval_mesh_t(1000 + i, 10 + i, 2000 + i, 5 + i) for i in range(7)]
    a = hx.BatchArgs(meshes, [3000 + i for i in range(7)], [4000 + i if i % 2 else 0 for i in range(7)])
    assert a.n == 7
    assert [a.meshes[i].n for i in range(7)] == [5 + i for i in range(7)]
    assert [a.meshes[i].n_points for i in range(7)] == [10 + i for i in range(7)]
    assert [a.verdicts[i] for i in range(7)] == [3000 + i for i in range(7)]
    assert [a.min_coeffs[i] or 0 for i in range(7)] == [4000 + i if i % 2 else 0 for i in range(7)]
    assert hx.BatchArgs(meshes, [1] * 7).min_coeffs is None


def test_missing_library_fails_loudly(tmp_path):
    # without the built library the binding raises; it never falls back to
    # anything else (checked in a fresh interpreter, so that the library this
    # process already loaded does not interfere)
    import subprocess
    import sys
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_1706_01613_amd import hexval as hx\n"
        "hx.LIB_PATH = %r\n"
        "try:\n"
        "    hx.lib()\n"
        "except hx.HexvalError as e:\n"
        "    print('raised', e)\n"
        "    sys.exit(0)\n"
        "sys.exit(1)\n"
    ) % (str(ROOT), str(tmp_path / "libhexval.so"))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "raised" in r.stdout
