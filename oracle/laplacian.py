"""Normalized Laplacian of Sec. 2.1 (oracle; test infrastructure only).

L = I - D^-1/2 W D^-1/2 with D_ii = sum over j != i of W_ij.  Its spectrum lies
in [0, 2].  The Chebyshev filters below work on [0, 2] through the shifted
variable x = lambda - 1, i.e. with the operator L - I = -A where
A = D^-1/2 W D^-1/2, so only A is built.

A node of degree zero makes D^-1/2 undefined; the paper assumes such nodes away
(it requires v_k(i) > 0 in Sec. 3.1).  Here its scaling is taken as 0, so its
row and column of A vanish and L_ii = 1: the node is an eigenvector of L with
eigenvalue 1 and never enters a low-pass band below 1.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def degrees(row_ptr, col, w=None) -> np.ndarray:
    """D_ii = sum_{j != i} W_ij in float64 (W_ij = 1 when ``w`` is None)."""
    n = len(row_ptr) - 1
    rows = np.repeat(np.arange(n), np.diff(np.asarray(row_ptr, dtype=np.int64)))
    vals = np.ones(len(col)) if w is None else np.asarray(w, dtype=np.float64)
    off = rows != np.asarray(col)
    return np.bincount(rows[off], weights=vals[off], minlength=n)


def normalized_adjacency(row_ptr, col, w=None):
    """(A, s) with A = S W S and s_i = D_ii^-1/2 (0 for an isolated node)."""
    n = len(row_ptr) - 1
    deg = degrees(row_ptr, col, w)
    s = np.zeros(n)
    nz = deg > 0
    s[nz] = 1.0 / np.sqrt(deg[nz])
    vals = np.ones(len(col)) if w is None else np.asarray(w, dtype=np.float64)
    W = sp.csr_matrix((vals, np.asarray(col), np.asarray(row_ptr)), shape=(n, n))
    W.setdiag(0.0)
    W.eliminate_zeros()
    S = sp.diags(s)
    A = (S @ W @ S).tocsr()
    return A, s


def laplacian_dense(row_ptr, col, w=None) -> np.ndarray:
    """Dense L for closed-form checks on small graphs."""
    A, _ = normalized_adjacency(row_ptr, col, w)
    return np.eye(A.shape[0]) - A.toarray()
