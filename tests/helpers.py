"""Shared helpers of the parity tests (layout conversions and error norms only)."""
import numpy as np


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b.ravel())
    return np.linalg.norm((a - b).ravel()) / (den if den > 0 else 1.0)


def absolute_positions(cell, off, n, d):
    """FP64 absolute positions [3, np] of (cell, offset) pairs."""
    c = np.asarray(cell, dtype=np.int64)
    idx = (c % n[0], (c // n[0]) % n[1], c // (n[0] * n[1]))
    return np.stack([(idx[a] + np.asarray(off[a], dtype=np.float64)) * d[a] for a in range(3)])


def periodic_delta(x1, x0, L):
    """x1 - x0 mapped to (-L/2, L/2] per axis."""
    L = np.asarray(L, dtype=np.float64)[:, None]
    dx = x1 - x0
    return dx - L * np.round(dx / L)


def by_id(ids, *arrays):
    order = np.argsort(ids, kind="stable")
    return [a[..., order] for a in arrays]
