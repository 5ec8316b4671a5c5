"""Interpolation of the reduced indicators, Eq. (5), and hard labels (oracle).

Eq. (5): x_j = argmin ||M x - c_j^r||^2 + gamma x^T g(L) x for each cluster j,
with M the sampling matrix of Eq. (4) and g a polynomial approximation of the
ideal high-pass 1 - h_lambda_k (Sec. 3.2.2).  Setting the gradient to zero
gives the linear system

    (M^T M + gamma g~(L)) x_j = M^T c_j^r,

where M^T M = diag(mask) (mask_i = 1 iff node i is sampled) and M^T c_j^r puts
a 1 at every sampled node that k-means placed in cluster j.  With the
weighted fidelity term of variable-density sampling, the 1s become the
decoder weights of the sampled nodes.

Readings taken:
* g~ = 1 - h~ with the same order and Jackson damping as the low-pass, so the
  matrix is diag(mask) + gamma (I - h~(L)); Jackson damping keeps h~ inside
  (0, 1), so the matrix is symmetric positive definite;
* the paper solves with gmres and mentions conjugate gradient (Sec. 4.4);
  since the system is SPD this uses conjugate gradient per cluster, from
  x = 0, stopping when ||r|| / ||b|| <= tol or after ``max_iter`` iterations;
* Sec. 4.1: node i gets the cluster j maximising x_j(i) / ||x_j||; ties and
  all-zero columns go to the lowest index.
"""
from __future__ import annotations

import numpy as np

from .cheb import filter_block
from .jackson import lowpass_coeffs


def rhs(N: int, omega: np.ndarray, labels_r: np.ndarray, k: int, weights=None) -> np.ndarray:
    """M^T W c_j^r for every j: weight w_s at (omega_s, labels_r[s]) (W = I by default)."""
    B = np.zeros((N, k))
    B[np.asarray(omega), np.asarray(labels_r)] = 1.0 if weights is None else np.asarray(weights)
    return B


def sample_mask(N: int, omega: np.ndarray, weights=None) -> np.ndarray:
    """Diagonal of M^T W M."""
    mask = np.zeros(N)
    mask[np.asarray(omega)] = 1.0 if weights is None else np.asarray(weights)
    return mask


def apply_operator(A, mask: np.ndarray, gamma: float, a: np.ndarray, X: np.ndarray) -> np.ndarray:
    """(diag(mask) + gamma (I - h~(L))) X."""
    return mask[:, None] * X + gamma * (X - filter_block(A, X, a))


def cg(A, mask, gamma, a, B, tol=1e-6, max_iter=1000):
    """Conjugate gradient on every column of B; columns never mix.

    Returns (X, iterations per column, final recursive relative residual per column).
    """
    N, k = B.shape
    X = np.zeros((N, k))
    R = B.copy()
    P = R.copy()
    rr = np.sum(R * R, axis=0)
    bnorm = np.sqrt(rr)
    active = bnorm > 0.0
    iters = np.zeros(k, dtype=np.int64)
    relres = np.zeros(k)
    for it in range(1, max_iter + 1):
        if not active.any():
            break
        cols = np.nonzero(active)[0]
        Pa = P[:, cols]
        AP = apply_operator(A, mask, gamma, a, Pa)
        pAp = np.sum(Pa * AP, axis=0)
        alpha = rr[cols] / pAp
        X[:, cols] += alpha * Pa
        R[:, cols] -= alpha * AP
        rr_new = np.sum(R[:, cols] * R[:, cols], axis=0)
        rel = np.sqrt(rr_new) / bnorm[cols]
        relres[cols] = rel
        iters[cols] = it
        done = rel <= tol
        beta = rr_new / rr[cols]
        P[:, cols] = R[:, cols] + beta * Pa
        rr[cols] = rr_new
        active[cols[done]] = False
    return X, iters, relres


def hard_labels(X: np.ndarray) -> np.ndarray:
    """argmax_j X_ij / ||X_j||; zero columns never win unless all are zero."""
    norms = np.sqrt(np.sum(X * X, axis=0))
    Z = np.full_like(X, -np.inf)
    nz = norms > 0.0
    Z[:, nz] = X[:, nz] / norms[nz]
    lab = np.argmax(Z, axis=1)
    if not nz.any():
        lab[:] = 0
    return lab


def interpolate(A, lam_k, p, gamma, omega, labels_r, k, tol=1e-6, max_iter=1000, weights=None,
                damping: bool = True):
    """Eq. (5) for every cluster; with ``weights`` (w_s > 0 per sampled node)
    the fidelity term is Puy et al.'s weighted ||W^(1/2) (M x - c_j^r)||^2
    used with variable-density sampling: (M^T W M + gamma g~(L)) x = M^T W c_j^r."""
    N = A.shape[0]
    mask = sample_mask(N, omega, weights)
    a = lowpass_coeffs(lam_k, p, damping)
    B = rhs(N, omega, labels_r, k, weights)
    X, iters, relres = cg(A, mask, gamma, a, B, tol, max_iter)
    return X, hard_labels(X), iters, relres
