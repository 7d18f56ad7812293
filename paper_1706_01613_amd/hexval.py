"""Thin Python binding of libhexval (ctypes; argument marshalling only).

Every function of ``include/hexval.h`` is exposed under the same name.  Array
arguments may be ROCm torch tensors (their ``data_ptr()`` is passed) or raw
integer device addresses; every step of the check runs in the HIP library.
The library is loaded on first use; if it has not been built this raises
``HexvalError`` (there is no fallback).
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhexval.so")

INVALID, VALID, UNDECIDED, BAD_INPUT = 0, 1, 2, 3
OK, E_ARG, E_HIP, E_NOMEM, E_QUEUE, E_BUSY = 0, 1, 2, 3, 4, 5
FP64, FP32_FILTER = 0, 1
MINJ_CONVERGED, MINJ_DEPTH_CAP, MINJ_QUEUE_FULL, MINJ_BAD_INPUT, MINJ_OUT_OF_RANGE = 0, 1, 2, 3, 4
STATUS_NAMES = {0: "OK", 1: "E_ARG", 2: "E_HIP", 3: "E_NOMEM", 4: "E_QUEUE", 5: "E_BUSY"}


class HexvalError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"hexval {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class hexval_mesh_t(ctypes.Structure):
    _fields_ = [("points", ctypes.c_void_p), ("n_points", ctypes.c_int64),
                ("connectivity", ctypes.c_void_p), ("n", ctypes.c_int64)]


class hexval_stats_t(ctypes.Structure):
    _fields_ = [("n_elements", ctypes.c_int64), ("n_subdivided", ctypes.c_int64),
                ("n_nodes", ctypes.c_int64), ("n_exact", ctypes.c_int64),
                ("n_recheck", ctypes.c_int64), ("n_rounds", ctypes.c_int64),
                ("max_level", ctypes.c_int32), ("timing", ctypes.c_int32),
                ("ms_first_pass", ctypes.c_float), ("ms_recheck", ctypes.c_float),
                ("ms_subdivision", ctypes.c_float), ("ms_total", ctypes.c_float),
                ("block_threads", ctypes.c_int32), ("n_exact_host", ctypes.c_int32),
                ("grid_blocks", ctypes.c_int64), ("walk_layers", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("walk_stride", ctypes.c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class hexval_opts_t(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("max_depth", ctypes.c_int32),
                ("validate_indices", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("queue_capacity", ctypes.c_int64), ("grid_blocks", ctypes.c_int64),
                ("stream", ctypes.c_void_p), ("stats", ctypes.POINTER(hexval_stats_t)),
                ("walk_layers", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class hexval_request_t(ctypes.Structure):
    _fields_ = [("mesh", hexval_mesh_t), ("host_points", ctypes.c_void_p),
                ("host_conn", ctypes.c_void_p), ("verdicts", ctypes.c_void_p),
                ("min_coeffs", ctypes.c_void_p)]


_lib = None


def lib():
    """The loaded libhexval (raises HexvalError when it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise HexvalError(E_HIP, f"{LIB_PATH} is not built; run "
                                     "python -m paper_1706_01613_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        sig = {
            "hexval_opts_default": (None, [ctypes.POINTER(hexval_opts_t)]),
            "hexval_check": (ctypes.c_int, [P, P, I64, P, P]),
            "hexval_check_ex": (ctypes.c_int, [ctypes.POINTER(hexval_mesh_t),
                                               ctypes.POINTER(hexval_opts_t), P, P]),
            "hexval_check_batched": (ctypes.c_int, [ctypes.POINTER(hexval_mesh_t), I32,
                                                    ctypes.POINTER(hexval_opts_t), P, P]),
            "hexval_coefficients": (ctypes.c_int, [ctypes.POINTER(hexval_mesh_t), P, P]),
            "hexval_check_noalloc": (ctypes.c_int, [ctypes.POINTER(hexval_mesh_t),
                                                    ctypes.POINTER(hexval_opts_t), P, P]),
            "hexval_quad_check": (ctypes.c_int, [ctypes.POINTER(hexval_mesh_t),
                                                 ctypes.POINTER(hexval_opts_t), P, P]),
            "hexval_corner_test": (ctypes.c_int, [ctypes.POINTER(hexval_mesh_t),
                                                  ctypes.POINTER(hexval_opts_t), P, P]),
            "hexval_min_jacobian": (ctypes.c_int, [ctypes.POINTER(hexval_mesh_t),
                                                   ctypes.POINTER(hexval_opts_t), ctypes.c_double,
                                                   P, P, P]),
            "hexval_server_create": (ctypes.c_int, [ctypes.POINTER(hexval_opts_t), I64, I32,
                                                    ctypes.POINTER(P)]),
            "hexval_server_submit": (ctypes.c_int, [P, ctypes.POINTER(hexval_request_t),
                                                    ctypes.POINTER(ctypes.c_uint64)]),
            "hexval_server_poll": (ctypes.c_int, [P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int),
                                                  ctypes.POINTER(ctypes.c_double)]),
            "hexval_server_wait": (ctypes.c_int, [P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)]),
            "hexval_server_destroy": (ctypes.c_int, [P]),
            "hexval_last_error": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _addr(x):
    """Device address of a torch tensor, an int, or None (NULL)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _check(status):
    if status != OK:
        raise HexvalError(status, lib().hexval_last_error().decode(errors="replace"))
    return status


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def hexval_opts_default():
    o = hexval_opts_t()
    lib().hexval_opts_default(ctypes.byref(o))
    return o


def make_opts(precision=FP64, max_depth=6, validate_indices=False, block_threads=0,
              queue_capacity=0, grid_blocks=0, stream=None, stats=None, walk_layers=0):
    o = hexval_opts_default()
    o.precision = precision
    o.max_depth = max_depth
    o.validate_indices = int(bool(validate_indices))
    o.block_threads = block_threads
    o.queue_capacity = queue_capacity
    o.grid_blocks = grid_blocks
    o.walk_layers = walk_layers
    o.stream = _stream_handle(stream)
    if stats is not None:
        o.stats = ctypes.pointer(stats)
    return o


def make_mesh(points, connectivity=None, n=None, n_points=None):
    if n is None:
        n = connectivity.shape[0] if connectivity is not None else points.shape[0]
    if n_points is None:
        n_points = points.shape[0] if connectivity is not None and hasattr(points, "shape") else 0
    return hexval_mesh_t(_addr(points), int(n_points), _addr(connectivity), int(n))


def hexval_check(points, connectivity, n, verdicts, min_coeffs=None):
    """C: hexval_check.  Raises HexvalError on a non-OK status."""
    return _check(lib().hexval_check(_addr(points), _addr(connectivity), int(n),
                                     _addr(verdicts), _addr(min_coeffs)))


def hexval_check_ex(mesh, opts, verdicts, min_coeffs=None):
    """C: hexval_check_ex (mesh: hexval_mesh_t, opts: hexval_opts_t or None)."""
    return _check(lib().hexval_check_ex(ctypes.byref(mesh), ctypes.byref(opts) if opts else None,
                                        _addr(verdicts), _addr(min_coeffs)))


def hexval_check_noalloc(mesh, opts, verdicts, min_coeffs=None):
    """C: hexval_check_noalloc (mesh: hexval_mesh_t, opts: hexval_opts_t or None)."""
    return _check(lib().hexval_check_noalloc(ctypes.byref(mesh), ctypes.byref(opts) if opts else None,
                                             _addr(verdicts), _addr(min_coeffs)))


class BatchArgs:
    """The C arrays of a hexval_check_batched call, built once: for a batch
    of many meshes checked repeatedly, marshalling the lists on every call
    costs milliseconds of host time."""

    def __init__(self, meshes, verdicts, min_coeffs=None):
        self.n = len(meshes)
        self.meshes = (hexval_mesh_t * self.n)(*meshes)
        self.verdicts = (ctypes.c_void_p * self.n)(*[_addr(x) for x in verdicts])
        self.min_coeffs = ((ctypes.c_void_p * self.n)(*[_addr(x) for x in min_coeffs])
                           if min_coeffs is not None else None)


def hexval_check_batched(meshes, opts, verdicts=None, min_coeffs=None):
    """C: hexval_check_batched.  meshes: a BatchArgs, or a list of
    hexval_mesh_t with verdicts and min_coeffs as lists of tensors/addresses
    (min_coeffs entries may be None)."""
    a = meshes if isinstance(meshes, BatchArgs) else BatchArgs(meshes, verdicts, min_coeffs)
    return _check(lib().hexval_check_batched(a.meshes, a.n, ctypes.byref(opts) if opts else None,
                                             ctypes.cast(a.verdicts, ctypes.c_void_p),
                                             ctypes.cast(a.min_coeffs, ctypes.c_void_p)
                                             if a.min_coeffs is not None else None))


def hexval_coefficients(mesh, stream, coeffs):
    """C: hexval_coefficients."""
    return _check(lib().hexval_coefficients(ctypes.byref(mesh), _stream_handle(stream), _addr(coeffs)))


def hexval_corner_test(mesh, opts, test1, quality=None):
    """C: hexval_corner_test."""
    return _check(lib().hexval_corner_test(ctypes.byref(mesh), ctypes.byref(opts) if opts else None,
                                           _addr(test1), _addr(quality)))


def hexval_quad_check(mesh, opts, verdicts, min_j=None):
    """C: hexval_quad_check."""
    return _check(lib().hexval_quad_check(ctypes.byref(mesh), ctypes.byref(opts) if opts else None,
                                          _addr(verdicts), _addr(min_j)))


def hexval_min_jacobian(mesh, opts, rtol, lo, hi, status=None):
    """C: hexval_min_jacobian."""
    return _check(lib().hexval_min_jacobian(ctypes.byref(mesh), ctypes.byref(opts) if opts else None,
                                            float(rtol), _addr(lo), _addr(hi), _addr(status)))


def hexval_server_create(opts, hbm_budget_bytes, max_slots):
    h = ctypes.c_void_p()
    _check(lib().hexval_server_create(ctypes.byref(opts) if opts else None, int(hbm_budget_bytes),
                                      int(max_slots), ctypes.byref(h)))
    return h


def hexval_server_submit(server, request):
    t = ctypes.c_uint64()
    _check(lib().hexval_server_submit(server, ctypes.byref(request), ctypes.byref(t)))
    return t.value


def hexval_server_poll(server, ticket):
    done = ctypes.c_int()
    lat = ctypes.c_double()
    _check(lib().hexval_server_poll(server, ticket, ctypes.byref(done), ctypes.byref(lat)))
    return bool(done.value), (lat.value if done.value else None)


def hexval_server_wait(server, ticket):
    lat = ctypes.c_double()
    _check(lib().hexval_server_wait(server, ticket, ctypes.byref(lat)))
    return lat.value


def hexval_server_destroy(server):
    return _check(lib().hexval_server_destroy(server))


def hexval_last_error():
    return lib().hexval_last_error().decode(errors="replace")


# ---------------------------------------------------------------- conveniences

def _unset(shape, dtype, device):
    """An output tensor of the allocating helpers below: it starts as a value
    no kernel writes (0xEE for uint8, NaN for float64), so that an element the
    library left without a result shows instead of whatever the memory held
    (torch's allocator hands back earlier tensors' memory)."""
    import torch
    shape = (shape,) if isinstance(shape, int) else tuple(shape)
    return torch.full(shape, 0xEE if dtype == torch.uint8 else float("nan"), dtype=dtype, device=device)


def _after_fill(stream, device):
    """The fills run on torch's current stream: wait for them when the call
    runs on another stream."""
    import torch
    cur = torch.cuda.current_stream(device)
    if stream is not None and _stream_handle(stream) != _stream_handle(cur):
        cur.synchronize()


def check(points, connectivity=None, precision=FP64, max_depth=6, validate_indices=False,
          stream=None, stats=False, block_threads=0, grid_blocks=0, queue_capacity=0,
          want_min=True, walk_layers=0):
    """Allocate outputs (torch, on points' device) and run hexval_check_ex.

    points: [n,8,3] float64 (connectivity None) or [m,3] float64 with
    connectivity [n,8] int32.  Returns (verdicts uint8 [n], min_coeffs float64
    [n] or None, stats dict or None)."""
    import torch
    n = connectivity.shape[0] if connectivity is not None else points.shape[0]
    verdicts = _unset(n, torch.uint8, points.device)
    mins = _unset(n, torch.float64, points.device) if want_min else None
    _after_fill(stream, points.device)
    st = hexval_stats_t()
    st.timing = 1 if stats else 0
    if stream is None:
        stream = torch.cuda.current_stream(points.device)
    opts = make_opts(precision, max_depth, validate_indices, block_threads, queue_capacity,
                     grid_blocks, stream, st, walk_layers)
    hexval_check_ex(make_mesh(points, connectivity, n), opts, verdicts, mins)
    return verdicts, mins, (st.as_dict() if stats else None)


def coefficients(points, connectivity=None, stream=None):
    import torch
    n = connectivity.shape[0] if connectivity is not None else points.shape[0]
    out = _unset((n, 27), torch.float64, points.device)
    _after_fill(stream, points.device)
    if stream is None:
        stream = torch.cuda.current_stream(points.device)
    hexval_coefficients(make_mesh(points, connectivity, n), stream, out)
    return out


def min_jacobian(points, connectivity=None, rtol=1e-3, max_depth=6, validate_indices=False,
                 stream=None, stats=False, queue_capacity=0):
    """Allocate outputs and run hexval_min_jacobian.  Returns (lo, hi, status,
    stats dict or None) as torch tensors on points' device."""
    import torch
    n = connectivity.shape[0] if connectivity is not None else points.shape[0]
    lo = _unset(n, torch.float64, points.device)
    hi = _unset(n, torch.float64, points.device)
    status = _unset(n, torch.uint8, points.device)
    _after_fill(stream, points.device)
    st = hexval_stats_t()
    st.timing = 1 if stats else 0
    if stream is None:
        stream = torch.cuda.current_stream(points.device)
    opts = make_opts(FP64, max_depth, validate_indices, 0, queue_capacity, 0, stream, st)
    hexval_min_jacobian(make_mesh(points, connectivity, n), opts, rtol, lo, hi, status)
    return lo, hi, status, (st.as_dict() if stats else None)


def corner_test(points, connectivity=None, validate_indices=False, stream=None, stats=False,
                want_quality=True):
    """Allocate outputs and run hexval_corner_test.  Returns (test1 uint8,
    quality float64 or None, stats dict or None) on points' device."""
    import torch
    n = connectivity.shape[0] if connectivity is not None else points.shape[0]
    test1 = _unset(n, torch.uint8, points.device)
    quality = _unset(n, torch.float64, points.device) if want_quality else None
    _after_fill(stream, points.device)
    st = hexval_stats_t()
    st.timing = 1 if stats else 0
    if stream is None:
        stream = torch.cuda.current_stream(points.device)
    opts = make_opts(FP64, 6, validate_indices, 0, 0, 0, stream, st)
    hexval_corner_test(make_mesh(points, connectivity, n), opts, test1, quality)
    return test1, quality, (st.as_dict() if stats else None)


def quad_check(points, connectivity=None, validate_indices=False, stream=None, stats=False, want_min=True,
               grid_blocks=0, walk_layers=0):
    """Allocate outputs and run hexval_quad_check.  points: [n,4,2] float64, or
    [m,2] with connectivity [n,4] int32.  Returns (verdicts, min_j or None,
    stats dict or None)."""
    import torch
    n = connectivity.shape[0] if connectivity is not None else points.shape[0]
    verdicts = _unset(n, torch.uint8, points.device)
    min_j = _unset(n, torch.float64, points.device) if want_min else None
    _after_fill(stream, points.device)
    st = hexval_stats_t()
    st.timing = 1 if stats else 0
    if stream is None:
        stream = torch.cuda.current_stream(points.device)
    opts = make_opts(FP64, 6, validate_indices, 0, 0, grid_blocks, stream, st, walk_layers)
    mesh = hexval_mesh_t(_addr(points), int(points.shape[0]) if connectivity is not None else 0,
                         _addr(connectivity), int(n))
    hexval_quad_check(mesh, opts, verdicts, min_j)
    return verdicts, min_j, (st.as_dict() if stats else None)
