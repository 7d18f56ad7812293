"""CPU oracle for the validity test of linear hexahedra: TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The HIP library never calls it and the
two share no code.  See ``hexval_oracle.c`` (FP64 pass with certified sign
decisions) and ``exact.py`` (rational-arithmetic tier for the elements the FP64
pass cannot certify).
"""
import ctypes
import os
import subprocess

import numpy as np

from . import exact

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hexval_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

INVALID, VALID, UNDECIDED, BAD_INPUT, FRAGILE = 0, 1, 2, 3, 255

_lib = None


def build():
    """Compile the C oracle (gcc, FP64, no contraction, OpenMP)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=c11",
           "-shared", "-fPIC", SRC, "-o", LIB + ".tmp", "-lm"]
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        lib.oracle_check.restype = ctypes.c_int64
        lib.oracle_check.argtypes = [P, P, ctypes.c_int64, ctypes.c_int, ctypes.c_int, P, P, P, P, P]
        lib.oracle_coefficients.restype = None
        lib.oracle_coefficients.argtypes = [P, P, ctypes.c_int64, ctypes.c_int, P, P]
        lib.oracle_scale.restype = None
        lib.oracle_scale.argtypes = [P, P, ctypes.c_int64, P]
        lib.oracle_jacobian.restype = ctypes.c_double
        lib.oracle_jacobian.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        lib.oracle_T.restype = None
        lib.oracle_T.argtypes = [P]
        lib.oracle_bound_constants.restype = None
        lib.oracle_bound_constants.argtypes = [P]
        lib.oracle_quad_check.restype = ctypes.c_int64
        lib.oracle_quad_check.argtypes = [P, P, ctypes.c_int64, ctypes.c_int, P, P]
        lib.oracle_corner_test.restype = ctypes.c_int64
        lib.oracle_corner_test.argtypes = [P, P, ctypes.c_int64, ctypes.c_int, P, P]
        lib.oracle_min_jacobian.restype = None
        lib.oracle_min_jacobian.argtypes = [P, P, ctypes.c_int64, ctypes.c_double, ctypes.c_int,
                                            ctypes.c_int, P, P, P, P, P]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _prep(points, conn):
    points = np.ascontiguousarray(points, dtype=np.float64)
    if conn is None:
        points = points.reshape(-1, 8, 3)
        n = points.shape[0]
    else:
        conn = np.ascontiguousarray(conn, dtype=np.int32).reshape(-1, 8)
        points = points.reshape(-1, 3)
        n = conn.shape[0]
        if n and (conn.min() < 0 or conn.max() >= points.shape[0]):
            raise IndexError("connectivity index out of range")
    return points, conn, n


def element_points(points, conn, e):
    """The 8 points of element e as a (8,3) float64 array."""
    if conn is None:
        return np.asarray(points, dtype=np.float64).reshape(-1, 8, 3)[e]
    return np.asarray(points, dtype=np.float64).reshape(-1, 3)[np.asarray(conn).reshape(-1, 8)[e]]


def check(points, conn=None, max_depth=6, threads=0, details=False, settle_fragile=True):
    """Verdicts of all elements (exact-arithmetic semantics).

    points: [n,8,3] when conn is None, else [m,3] with conn [n,8] int32.
    Returns a dict with ``verdict`` (uint8 [n]), ``min_coeff`` (float64 [n]),
    ``fragile`` (int64 ids settled by the exact tier) and, with details=True,
    ``level``, ``nodes`` and ``witness``."""
    lib = _load()
    points, conn, n = _prep(points, conn)
    verdict = np.empty(n, np.uint8)
    min_coeff = np.empty(n, np.float64)
    level = np.empty(n, np.int32) if details else None
    nodes = np.empty(n, np.int64) if details else None
    witness = np.empty((n, 3), np.float64) if details else None
    lib.oracle_check(_ptr(points), _ptr(conn), n, int(max_depth), int(threads), _ptr(verdict),
                     _ptr(min_coeff), _ptr(level), _ptr(nodes), _ptr(witness))
    fragile = np.nonzero(verdict == FRAGILE)[0]
    if settle_fragile:
        for e in fragile:
            r = exact.validity(element_points(points, conn, e), max_depth)
            verdict[e] = r["verdict"]
            if r["min_coeff"] is None:
                min_coeff[e] = np.nan
            if details:
                level[e] = r["level"]
                nodes[e] = r["nodes"]
                witness[e] = [float(w) for w in r["witness"]] if r["witness"] else [np.nan] * 3
    out = dict(verdict=verdict, min_coeff=min_coeff, fragile=fragile)
    if details:
        out.update(level=level, nodes=nodes, witness=witness)
    return out


def coefficients(points, conn=None, threads=0, samples=False):
    """The 27 top-level Bezier coefficients [n,27] (and the samples c [n,27])."""
    lib = _load()
    points, conn, n = _prep(points, conn)
    b = np.empty((n, 27), np.float64)
    c = np.empty((n, 27), np.float64) if samples else None
    lib.oracle_coefficients(_ptr(points), _ptr(conn), n, int(threads), _ptr(b), _ptr(c))
    return (b, c) if samples else b


def corner_test(points, conn=None, threads=0):
    """The corner-only test (Test 1 of Section 7: all 8 corner values of J
    positive, a necessary condition of validity) and the corner quality (min
    over the corners of the scaled Jacobian).  Returns a dict with ``test1``
    (uint8 [n]: 1 VALID, 0 INVALID, 3 BAD_INPUT; uncertified corner signs are
    settled exactly), ``quality`` (float64 [n], NaN for bad or out-of-range
    input) and ``fragile`` (ids settled exactly)."""
    lib = _load()
    points, conn, n = _prep(points, conn)
    test1 = np.empty(n, np.uint8)
    quality = np.empty(n, np.float64)
    lib.oracle_corner_test(_ptr(points), _ptr(conn), n, int(threads), _ptr(test1), _ptr(quality))
    fragile = np.nonzero(test1 == FRAGILE)[0]
    for e in fragile:
        test1[e] = exact.corner_test(element_points(points, conn, e))
    return dict(test1=test1, quality=quality, fragile=fragile)


def quad_check(points, conn=None, threads=0):
    """Validity of linear quadrangles (Section 2.1): INVALID when a corner
    value of J is <= 0, VALID when all four are > 0; uncertified signs are
    settled exactly.  points: [n,4,2], or [m,2] with conn [n,4] int32.
    Returns a dict with ``verdict`` (uint8 [n]), ``min_j`` (float64 [n]: the
    smallest corner value, which is min J) and ``fragile``."""
    lib = _load()
    points = np.ascontiguousarray(points, dtype=np.float64)
    if conn is None:
        points = points.reshape(-1, 4, 2)
        n = points.shape[0]
    else:
        conn = np.ascontiguousarray(conn, dtype=np.int32).reshape(-1, 4)
        points = points.reshape(-1, 2)
        n = conn.shape[0]
    verdict = np.empty(n, np.uint8)
    min_j = np.empty(n, np.float64)
    lib.oracle_quad_check(_ptr(points), _ptr(conn), n, int(threads), _ptr(verdict), _ptr(min_j))
    fragile = np.nonzero(verdict == FRAGILE)[0]
    for e in fragile:
        q = points[e] if conn is None else points[conn[e]]
        verdict[e] = exact.quad_validity(q)
    return dict(verdict=verdict, min_j=min_j, fragile=fragile)


MJ_CONVERGED, MJ_CAPPED, MJ_BAD_INPUT, MJ_OUT_OF_RANGE = 0, 1, 3, 4


def min_jacobian(points, conn=None, rtol=1e-3, max_depth=6, threads=0):
    """Certified bounds lo <= min J <= hi over [0,1]^3 (Section 3.1 bounds
    sharpened level by level to width rtol * M^/6).  Returns a dict with
    ``lo``, ``hi`` (float64 [n]), ``status`` (uint8 [n]: 0 converged, 1 depth
    cap, 3 non-finite input, 4 out of the guard range), ``level`` and
    ``boxes``."""
    lib = _load()
    points, conn, n = _prep(points, conn)
    lo = np.empty(n, np.float64)
    hi = np.empty(n, np.float64)
    status = np.empty(n, np.uint8)
    level = np.empty(n, np.int32)
    boxes = np.empty(n, np.int64)
    lib.oracle_min_jacobian(_ptr(points), _ptr(conn), n, float(rtol), int(max_depth), int(threads),
                            _ptr(lo), _ptr(hi), _ptr(status), _ptr(level), _ptr(boxes))
    return dict(lo=lo, hi=hi, status=status, level=level, boxes=boxes)


def scale(points, conn=None):
    """The bound scale M^ = 6 S_xi S_eta S_zeta of each element."""
    lib = _load()
    points, conn, n = _prep(points, conn)
    m = np.empty(n, np.float64)
    lib.oracle_scale(_ptr(points), _ptr(conn), n, _ptr(m))
    return m


def jacobian(p8, xi, eta, zeta):
    lib = _load()
    p8 = np.ascontiguousarray(p8, dtype=np.float64).reshape(8, 3)
    return lib.oracle_jacobian(_ptr(p8), float(xi), float(eta), float(zeta))


def T_matrix():
    lib = _load()
    out = np.empty((27, 27), np.float64)
    lib.oracle_T(_ptr(out))
    return out


def bound_constants():
    lib = _load()
    out = np.empty(3, np.float64)
    lib.oracle_bound_constants(_ptr(out))
    return dict(tau_c=out[0], tau_b=out[1], u=out[2])
