"""Comparison helpers of the GPU parity tests.

Every solution is compared with the oracle's in two norms: the relative
L2 error over the whole field, and the largest pointwise error relative to
the largest oracle value, so that an error confined to a few rows (the
absorbing layer, the rows next to the padding, the last layer of a sweep)
cannot hide inside a small share of the L2 norm.
"""
import numpy as np


def errors(u, ref):
    u = np.asarray(u)
    ref = np.asarray(ref)
    d = u - ref
    return (float(np.linalg.norm(d) / np.linalg.norm(ref)),
            float(np.max(np.abs(d)) / np.max(np.abs(ref))))


def assert_close(u, ref, tol, what=""):
    l2, mx = errors(u, ref)
    assert l2 <= tol and mx <= tol, f"{what}: rel L2 {l2:.3e}, rel max {mx:.3e}, tol {tol:.1e}"
    return l2, mx
