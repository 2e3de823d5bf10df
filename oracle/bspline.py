"""Cardinal B-splines by their recursive definition (paper Sec. II.A.2, PME
paragraph: the B-splines are built from the recursive definition).

M_2(w) = 1 - |w - 1| on [0, 2], zero elsewhere;
M_n(w) = [w M_{n-1}(w) + (n - w) M_{n-1}(w - 1)] / (n - 1);
dM_n/dw = M_{n-1}(w) - M_{n-1}(w - 1).
"""
from __future__ import annotations

import numpy as np


def M(n: int, w):
    w = np.asarray(w, dtype=np.float64)
    if n == 2:
        return np.where((w >= 0.0) & (w <= 2.0), 1.0 - np.abs(w - 1.0), 0.0)
    return (w * M(n - 1, w) + (n - w) * M(n - 1, w - 1.0)) / (n - 1)


def dM(n: int, w):
    w = np.asarray(w, dtype=np.float64)
    return M(n - 1, w) - M(n - 1, w - 1.0)
