"""Uniform sampling without replacement, Eq. (4) (oracle; test only).

Sec. 3.2.2 draws n distinct node indices uniformly at random; the sampling
matrix M of Eq. (4) has M_ij = 1 iff j = omega_i.  Reading taken: every node
gets an independent uniform 64-bit key (see ``philox``) and Omega lists the n
nodes with the smallest (key, index) pairs in increasing order, which is a
uniformly random n-subset in uniformly random order.
"""
from __future__ import annotations

import numpy as np

from .philox import sample_keys


def sample(N: int, n: int, seed: int) -> np.ndarray:
    keys = sample_keys(seed, N)
    order = np.lexsort((np.arange(N), keys))
    return order[:n].astype(np.int64)
