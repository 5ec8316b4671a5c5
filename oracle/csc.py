"""Compressive spectral clustering, Alg. 2, end to end (oracle; test only).

Steps as in the paper:
 1. estimate lambda_k by eigencount dichotomy (``eigencount``);
 2. Jackson-Chebyshev coefficients of h_lambda_k of order p (``jackson``);
 3. d Gaussian signals with variance 1/d (stream FEAT, sub-stream 0);
 4. Y = h~(L) R and unit-norm rows (a zero row stays zero);
 5. n nodes sampled uniformly without replacement (``sampling``), or by
    variable-density sampling on the squared feature norms;
 6. k-means on the n sampled features (``kmeans``);
 7. Tikhonov interpolation of the k reduced indicators, then hard labels.

Parameters default to the paper's n = 2 k log k, p = 50, gamma = 1e-3; the
number of features is a parameter (the paper's default is 4 log n, its Thm 3.2
is stated with log N), and n_c = 2 log N count signals.  Logs are natural.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .cheb import filter_block
from .eigencount import count_signals, estimate_lambda_k
from .interp import interpolate
from .jackson import lowpass_coeffs
from .kmeans import kmeans
from .laplacian import normalized_adjacency
from .philox import FEAT, gaussian_block
from .sampling import sample, sample_density


def default_n(k: int) -> int:
    """n = ceil(2 k ln k) sampled nodes (Alg. 2), at least k (the formula gives
    none for k = 1)."""
    return max(k, int(math.ceil(2.0 * k * math.log(k))))


def features(A, lam: float, p: int, d: int, seed: int, with_norms: bool = False,
             damping: bool = True):
    """Rows of h~_lam(L) R scaled to unit length (Alg. 2 steps 3-4); with
    ``with_norms`` also the squared row norms before scaling (the estimates of
    v_k(i)^2, Sec. 4.1)."""
    R = gaussian_block(seed, A.shape[0], d, 0, FEAT)
    Y = filter_block(A, R, lowpass_coeffs(lam, p, damping))
    sq = np.sum(Y * Y, axis=1)
    nrm = np.sqrt(sq)
    F = np.zeros_like(Y)
    nz = nrm > 0.0
    F[nz] = Y[nz] / nrm[nz, None]
    return (F, sq) if with_norms else F


@dataclass
class Result:
    lam: float
    bisect_steps: int
    bisect_trace: list
    bisect_converged: bool
    omega: np.ndarray
    features_sampled: np.ndarray
    labels_r: np.ndarray
    inertia: float
    X: np.ndarray
    labels: np.ndarray
    cg_iters: np.ndarray
    cg_relres: np.ndarray


def run(row_ptr, col, k: int, d: int, seed: int, p: int = 50, n: int | None = None,
        gamma: float = 1e-3, n_c: int | None = None, tol: float = 1e-6, max_iter: int = 1000,
        max_steps: int = 30, replicates: int = 20, kmeans_iter: int = 100, lam: float | None = None,
        sampling: str = "uniform", damping: bool = True):
    """Alg. 2.  ``sampling="density"`` draws the n nodes by variable-density
    sampling on the squared feature norms and uses the weighted fidelity term
    in Eq. (5) (``sampling.sample_density``)."""
    A, _ = normalized_adjacency(row_ptr, col)
    N = A.shape[0]
    n = default_n(k) if n is None else n
    n_c = count_signals(N) if n_c is None else n_c
    if lam is None:
        lam, steps, trace, conv = estimate_lambda_k(A, k, p, n_c, seed, max_steps,
                                                    damping=damping)
    else:
        steps, trace, conv = 0, [], True
    F, sq = features(A, lam, p, d, seed, with_norms=True, damping=damping)
    weights = None
    if sampling == "density":
        omega, weights = sample_density(sq, n, seed)
    else:
        omega = sample(N, n, seed)
    Fr = F[omega]
    labels_r, _, inertia = kmeans(Fr, k, seed, replicates, kmeans_iter)
    X, labels, iters, relres = interpolate(A, lam, p, gamma, omega, labels_r, k, tol, max_iter,
                                           weights, damping)
    return Result(lam, steps, trace, conv, omega, Fr, labels_r, inertia, X, labels, iters, relres)
