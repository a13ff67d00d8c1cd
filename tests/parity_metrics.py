"""Error measures of the GPU parity tests.

rel(a, b) is the worse of two relative errors of `a` against the reference `b`:
  * the relative L2 norm of the difference over the whole field, and
  * the element-wise one, max |a - b| / max |b|,
so a field-wide tolerance also bounds the error at a single particle (a clamp face or a corner
cell), which an L2 norm over N particles alone would let grow to about sqrt(N) times the tolerance.
"""
import numpy as np


def rel_l2(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    d = np.linalg.norm(a - b)
    s = np.linalg.norm(b)
    return d / s if s > 0 else d


def rel_max(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    d = np.abs(a - b).max() if a.size else 0.0
    s = np.abs(b).max() if b.size else 0.0
    return d / s if s > 0 else d


def rel(a, b):
    return max(rel_l2(a, b), rel_max(a, b))
