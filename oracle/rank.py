"""Ranking similarity, plain CPU reference (test infrastructure only).

isim_K(x, y) = (1/K) sum_{i=1..K} |X_i delta Y_i| / (2i), the intersection
similarity of Boldi et al. that the paper uses in Sec. 6 to compare two node
rankings; X_i (Y_i) are the i nodes with the largest x (y), delta the symmetric
difference.  Ranks order by value, largest first, ties by lower node index
(-0 and +0 compare equal).  The sets are grown one node at a time and the
symmetric difference is counted from membership flags, exactly as defined.
"""
from __future__ import annotations

import numpy as np


def ranking(x) -> np.ndarray:
    """Node indices by decreasing value, ties by increasing index."""
    x = np.asarray(x, np.float64)
    if not np.all(np.isfinite(x)):
        raise ValueError("non-finite value")
    return np.lexsort((np.arange(len(x)), -x))


def isim(x, y, k: int | None = None) -> float:
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    n = len(x)
    if len(y) != n or n < 1:
        raise ValueError("x and y must have one positive length")
    k = n if k is None else int(k)
    if not 1 <= k <= n:
        raise ValueError("k out of range")
    ox, oy = ranking(x), ranking(y)
    in_x = np.zeros(n, bool)
    in_y = np.zeros(n, bool)
    delta = 0                      # |X_i delta Y_i|
    total = 0.0
    for i in range(1, k + 1):
        a, b = ox[i - 1], oy[i - 1]
        in_x[a] = True
        delta += -1 if in_y[a] else 1
        in_y[b] = True
        delta += -1 if in_x[b] else 1
        total += delta / (2.0 * i)
    return total / k
