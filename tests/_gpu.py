"""Shared helpers for the GPU parity tests."""
import numpy as np
import pytest

import oracle


_capture = None


def set_capture_manager(cm):
    """Called by conftest: pytest's capture manager, so that progress lines
    can bypass output capture."""
    global _capture
    _capture = cm


def say(msg):
    """A progress line that reaches the terminal even while pytest captures
    the test's output (long GPU tests print one at least every minute)."""
    if _capture is not None:
        with _capture.global_and_fixture_disabled():
            print(msg, flush=True)
    else:
        print(msg, flush=True)


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def to_dev(torch, a, dtype=None):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def normwise_error(got, ref_coeffs_max, ref):
    """|got - ref| / max_beta |b_beta| per element (the 1e-12 criterion)."""
    scale = np.where(ref_coeffs_max > 0, ref_coeffs_max, 1.0)
    return np.abs(got - ref) / scale


def assert_parity(verdicts, mins, points, conn=None, max_depth=6, coeff_tol=1e-12, label=""):
    """Verdicts bit-exact with the oracle; min coefficients within coeff_tol
    normwise (relative to the element's largest oracle coefficient)."""
    ref = oracle.check(points, conn, max_depth=max_depth)
    v = np.asarray(verdicts)
    bad = np.nonzero(v != ref["verdict"])[0]
    assert bad.size == 0, (f"{label}: {bad.size} verdict mismatches, first ids {bad[:10]}, "
                           f"gpu {v[bad[:10]]} oracle {ref['verdict'][bad[:10]]}")
    if mins is not None:
        m = np.asarray(mins)
        b = oracle.coefficients(points, conn)
        bmax = np.abs(b).max(axis=1)
        finite = np.isfinite(ref["min_coeff"])
        assert (np.isnan(m) == ~finite).all(), f"{label}: NaN pattern of min_coeff differs"
        err = normwise_error(m[finite], bmax[finite], ref["min_coeff"][finite])
        assert err.max(initial=0.0) <= coeff_tol, f"{label}: min_coeff error {err.max()}"
    return ref
