"""Error measures shared by the GPU parity tests.

Every comparison of a GPU result with the oracle is made per frequency (the
first axis) in three ways:
  frob  relative Frobenius norm of the difference, ||a - b|| / ||b||;
  elem  largest element-wise difference relative to the largest reference
        entry, max|a - b| / max|b|;
  row   the same per row of the second axis (a receiver's spectrum, a row of
        the Hessian, a source's multipliers), max over rows of
        max|a_r - b_r| / max|b_r|, so that an error confined to one receiver or
        one row cannot hide under the norm of the whole frequency slice.
Arrays may be real or complex; nothing is cast to a real type.
"""
import numpy as np


def _c(x):
    x = np.asarray(x)
    return x.astype(np.complex128) if np.iscomplexobj(x) else x.astype(np.float64)


def rel(a, b) -> float:
    a, b = _c(a), _c(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def elem(a, b) -> float:
    a, b = _c(a), _c(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


def row(a, b) -> float:
    """max over the first axis of ``elem`` of each row (a, b at least 2-D)."""
    a, b = _c(a), _c(b)
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    d = np.abs(a - b).max(axis=1)
    m = np.abs(b).max(axis=1)
    keep = m > 0
    if not np.any(keep):
        return float(d.max())
    return float((d[keep] / m[keep]).max())


def per_freq_rel(a, b):
    return [rel(a[f], b[f]) for f in range(np.asarray(a).shape[0])]


def per_freq(a, b):
    """(frob, elem, row) lists over the first axis."""
    a, b = np.asarray(a), np.asarray(b)
    fr = [rel(a[f], b[f]) for f in range(a.shape[0])]
    el = [elem(a[f], b[f]) for f in range(a.shape[0])]
    rw = [row(a[f], b[f]) if a.ndim >= 3 else el[f] for f in range(a.shape[0])]
    return fr, el, rw


def check(a, b, frob, elem_tol, row_tol=None, label=""):
    """Assert the three measures per frequency; returns them for reporting."""
    fr, el, rw = per_freq(a, b)
    print(f"{label}: frob max {max(fr):.3e} elem max {max(el):.3e} row max {max(rw):.3e}", flush=True)
    assert max(fr) < frob, (label, "frob", fr)
    assert max(el) < elem_tol, (label, "elem", el)
    if row_tol is not None:
        assert max(rw) < row_tol, (label, "row", rw)
    return fr, el, rw
