"""Comparison helpers of the parity tests (no arithmetic of the method).

``assert_parity(a, b, tol)`` checks a computed array ``a`` against the oracle's ``b``
both norm-wise, ||a - b||_2 <= tol ||b||_2, and entry by entry,
|a_i - b_i| <= tol (|b_i| + ||b||_inf), so that one wrong entry cannot hide under
the norm of the others.
"""
import numpy as np


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def max_entry_err(a, b):
    """max_i |a_i - b_i| / (|b_i| + ||b||_inf): the entry-wise relative error."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    if b.size == 0:
        return 0.0
    scale = np.abs(b) + max(np.abs(b).max(), np.finfo(np.float64).tiny)
    return float((np.abs(a - b) / scale).max())


def assert_parity(a, b, tol, what=""):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    assert a.shape == b.shape, (what, a.shape, b.shape)
    assert np.all(np.isfinite(a)), f"{what}: non-finite entries"
    r, m = rel(a, b), max_entry_err(a, b)
    assert r <= tol, f"{what}: norm-wise relative error {r:.3e} > {tol:g}"
    assert m <= tol, f"{what}: entry-wise relative error {m:.3e} > {tol:g} (worst entry {int(np.argmax(np.abs(a - b)))})"
    return r, m
