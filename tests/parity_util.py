"""Comparison helpers shared by the GPU parity tests.

``close(a, b, tol)`` asserts both the relative L2 error of the whole field
and the element-wise bound max |a - b| <= tol * max |b|, so an error confined
to a low-amplitude region (the absorbing layer, a shell's interior) cannot
hide inside the norm of the whole field.
"""
import numpy as np


def rel(a, b) -> float:
    a, b = np.ravel(a), np.ravel(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def maxrel(a, b) -> float:
    a, b = np.ravel(a), np.ravel(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


def close(a, b, tol, what="") -> None:
    r, m = rel(a, b), maxrel(a, b)
    assert r <= tol and m <= tol, f"{what} rel L2 {r:.3e}, max-abs {m:.3e} (tol {tol:g})"
