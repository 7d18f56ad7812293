"""ctypes wrapper of libhexval_loadgen.so: an open-loop request stream
against a hexval server (benchmark and test driver)."""
import ctypes
import os

import numpy as np

from . import hexval as hx

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhexval_loadgen.so")
_lib = None


def lib():
    global _lib
    if _lib is None:
        hx.lib()  # libhexval first (the generator links against it)
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.hexval_loadgen_run.restype = ctypes.c_int
        L.hexval_loadgen_run.argtypes = [P, ctypes.c_int64, P, P, ctypes.POINTER(hx.hexval_request_t),
                                         ctypes.c_int32, P, ctypes.c_int64, ctypes.c_int32, P, P, P, P]
        _lib = L
    return _lib


def arena_bytes(sizes, want_min=True):
    total = 0
    for m in sizes:
        total += (m + 7) // 8 * 8 + (8 * m if want_min else 0)
        total = (total + 255) // 256 * 256
    return total


def run(server, arrival_s, mesh_idx, pool, arena, want_min=True):
    """Submit request i at arrival_s[i] (seconds) for pool[mesh_idx[i]];
    returns (latency_ms, status, out_offset, wall_s)."""
    arrival = np.ascontiguousarray(arrival_s, dtype=np.float64)
    idx = np.ascontiguousarray(mesh_idx, dtype=np.int32)
    n = arrival.size
    lat = np.zeros(n)
    st = np.zeros(n, np.int32)
    off = np.zeros(n, np.int64)
    wall = ctypes.c_double()
    parr = (hx.hexval_request_t * len(pool))(*pool)
    rc = lib().hexval_loadgen_run(server, n, arrival.ctypes.data, idx.ctypes.data, parr, len(pool),
                                  arena.data_ptr(), arena.numel() * arena.element_size(),
                                  1 if want_min else 0, lat.ctypes.data, st.ctypes.data,
                                  off.ctypes.data, ctypes.byref(wall))
    if rc != hx.OK:
        raise hx.HexvalError(rc, "load generator failed (arena too small?)")
    return lat, st, off, wall.value
