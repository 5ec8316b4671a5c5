"""Polynomial graph filtering (oracle; test infrastructure only).

Sec. 2.1 (fast graph filtering): h~(L) X is obtained with p products by L,
never forming h~(L).  With h~ written in the Chebyshev basis on [0, 2],
T_m(L - I) X follows the three-term recurrence

    T_0 = X,   T_1 = (L - I) X = -A X,   T_{m+1} = 2 (L - I) T_m - T_{m-1}
                                                  = -2 A T_m - T_{m-1},

and h~(L) X = sum_{m=0}^{p} a_m T_m.
"""
from __future__ import annotations

import numpy as np


def chebyshev_terms(A, X: np.ndarray, p: int):
    """Yield T_0 X, T_1 X, ..., T_p X (float64)."""
    X = np.asarray(X, dtype=np.float64)
    t_prev = X
    yield t_prev
    if p == 0:
        return
    t_cur = -(A @ X)
    yield t_cur
    for _ in range(1, p):
        t_next = -2.0 * (A @ t_cur) - t_prev
        yield t_next
        t_prev, t_cur = t_cur, t_next


def filter_block(A, X: np.ndarray, a: np.ndarray) -> np.ndarray:
    """h~(L) X = sum_m a_m T_m(L - I) X."""
    p = len(a) - 1
    Y = np.zeros_like(np.asarray(X, dtype=np.float64))
    for m, T in enumerate(chebyshev_terms(A, X, p)):
        Y += a[m] * T
    return Y


def moments(A, R: np.ndarray, p: int) -> np.ndarray:
    """mu_m = <R, T_m(L - I) R> (Frobenius), m = 0..p."""
    return np.array([float(np.sum(R * T)) for T in chebyshev_terms(A, R, p)])


def filter_block_clenshaw(A, X: np.ndarray, a: np.ndarray) -> np.ndarray:
    """h~(L) X by Clenshaw's backward recurrence for Chebyshev sums.

    With x = L - I (so x B = -A B):  b_{p+1} = b_{p+2} = 0,
    b_m = a_m X + 2 x b_{m+1} - b_{m+2} for m = p, ..., 1, and
    h~(L) X = a_0 X + x b_1 - b_2.  The same p products by A as the forward
    recurrence; each step reads one block fewer (no running sum).
    """
    X = np.asarray(X, dtype=np.float64)
    p = len(a) - 1
    if p == 0:
        return a[0] * X
    b2 = np.zeros_like(X)       # b_{m+2}
    b1 = a[p] * X               # b_p
    for m in range(p - 1, 0, -1):
        b0 = a[m] * X - 2.0 * (A @ b1) - b2
        b2, b1 = b1, b0
    return a[0] * X - (A @ b1) - b2
