"""Adjusted Rand index of Hubert & Arabie (1985), the score of Sec. 5.2 (oracle)."""
from __future__ import annotations

import numpy as np


def _comb2(x):
    x = np.asarray(x, dtype=np.float64)
    return x * (x - 1.0) / 2.0


def adjusted_rand_index(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    _, ai = np.unique(a, return_inverse=True)
    _, bi = np.unique(b, return_inverse=True)
    table = np.zeros((ai.max() + 1, bi.max() + 1))
    np.add.at(table, (ai, bi), 1.0)
    n = a.shape[0]
    sum_ij = _comb2(table).sum()
    sa = _comb2(table.sum(axis=1)).sum()
    sb = _comb2(table.sum(axis=0)).sum()
    expected = sa * sb / _comb2(n)
    top = 0.5 * (sa + sb)
    if top == expected:
        return 1.0
    return float((sum_ij - expected) / (top - expected))
