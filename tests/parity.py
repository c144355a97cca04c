"""Comparison bars shared by the GPU parity tests (imported, not collected).

The FP64 bar is element-wise: max_i |x_i - y_i| <= tol * max_i |y_i|, so a
single wrong entry (a ghost row at a subdomain edge, one grid of a batch)
counts in full instead of being averaged into a norm.  The 2-norm ratio is
printed beside it."""

import numpy as np


def rel_inf(a, b):
    """max_i |a_i - b_i| / max_i |b_i| (0 for empty vectors)."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    if b.size == 0:
        return 0.0
    return float(np.abs(a - b).max() / max(float(np.abs(b).max()), 1e-300))


def rel_2(a, b):
    """||a - b||_2 / ||b||_2."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(float(np.linalg.norm(b)), 1e-300))
