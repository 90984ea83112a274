"""Helpers shared by the GPU parity tests (device transfers and error norms)."""
import numpy as np


def normwise(a, b):
    """||a - b||_inf / ||b||_inf (0 when both vanish)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.max(np.abs(b)) if b.size else 0.0
    num = np.max(np.abs(a - b)) if b.size else 0.0
    if den == 0.0:
        return num
    return num / den


def field_errors(A, B):
    return [normwise(A[k], B[k]) for k in range(A.shape[0])]
