"""Shared test helpers (no method arithmetic here)."""
import numpy as np


def field_errors(a, b):
    """Per-field max-relative L-infinity error: max|a - b| / max|b| for every row."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    out = []
    for v in range(b.shape[0]):
        den = np.abs(b[v]).max()
        num = np.abs(a[v] - b[v]).max()
        out.append(0.0 if num == 0 else (num / den if den > 0 else np.inf))
    return np.array(out)


def field_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    out = []
    for v in range(b.shape[0]):
        den = np.linalg.norm(b[v].ravel())
        num = np.linalg.norm((a[v] - b[v]).ravel())
        out.append(0.0 if num == 0 else (num / den if den > 0 else np.inf))
    return np.array(out)
