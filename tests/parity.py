"""Error measures shared by the GPU parity tests (helper module, not collected).

``rel`` is the Frobenius relative error over a whole array.  ``upd`` is the measure for analysis
updates: the larger of the Frobenius error and the worst member's (column's) own relative error,
so a single wrong member column cannot hide behind the other members' norms.  A one-dimensional
array (a mean) is one column.
"""
import numpy as np


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def col_rel(a, b):
    """Worst column's relative error, ||a_i - b_i|| / ||b_i||."""
    a, b = np.asarray(a), np.asarray(b)
    if a.ndim == 1:
        return rel(a, b)
    num = np.linalg.norm(a - b, axis=0)
    den = np.linalg.norm(b, axis=0)
    return float(np.max(num / den))


def upd(a, b):
    return max(rel(a, b), col_rel(a, b))
