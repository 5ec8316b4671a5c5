"""Estimate of lambda_k by eigencount and dichotomy (oracle; test only).

Sec. 4.3: filtering random signals by the low-pass h~_lambda estimates the
number of eigenvalues of L in [0, lambda]; starting from lambda = 2 and halving
the interval, the search stops once that number equals k.  For each lambda the
paper filters 2 log N random signals.

Readings taken where the paper is not explicit:
* the estimator is Hutchinson's, count(lambda) = sum_{i,l} R_il (h~_lambda(L) R)_il
  for R with iid N(0, 1/n_c) entries, whose mean is tr h~_lambda(L);
* fresh signals for every tested lambda: sub-stream t of stream COUNT at step t;
* the bracket starts as [0, 2] (count(2) = N >= k needs no pass), so the first
  tested point is lambda = 1;
* the search stops when floor(count + 1/2) = k and returns that lambda; when the
  count is below k the lower end moves up, otherwise the upper end moves down;
  after ``max_steps`` tested points it returns the upper end.
"""
from __future__ import annotations

import math

import numpy as np

from .cheb import filter_block
from .jackson import lowpass_coeffs
from .philox import COUNT, gaussian_block


def count_signals(N: int) -> int:
    """n_c = ceil(2 ln N) random signals per tested lambda (Sec. 4.3), at least
    one (the formula gives none for N = 1)."""
    return max(1, int(math.ceil(2.0 * math.log(N))))


def eigencount(A, lam: float, p: int, R: np.ndarray, damping: bool = True) -> float:
    a = lowpass_coeffs(lam, p, damping)
    return float(np.sum(R * filter_block(A, R, a)))


def estimate_lambda_k(A, k: int, p: int, n_c: int, seed: int, max_steps: int = 30,
                      bracket=(0.0, 2.0), damping: bool = True):
    """Returns (lambda_hat, steps_used, [(lambda_t, count_t)], converged)."""
    N = A.shape[0]
    lo, hi = float(bracket[0]), float(bracket[1])
    trace = []
    for t in range(1, max_steps + 1):
        mid = 0.5 * (lo + hi)
        R = gaussian_block(seed, N, n_c, t, COUNT)
        c = eigencount(A, mid, p, R, damping)
        trace.append((mid, c))
        if math.floor(c + 0.5) == k:
            return mid, t, trace, True
        if c < k:
            lo = mid
        else:
            hi = mid
    return hi, max_steps, trace, False


def estimate_lambda_k_kpm(A, k: int, p: int, n_c: int, seed: int, max_steps: int = 30,
                          n_signals_pass: int | None = None):
    """One-pass form of the dichotomy (kernel polynomial method).

    count(lambda) = sum_m a_m(lambda) mu_m with mu_m = <R, T_m(L - I) R> holds
    for every lambda with the same signals R (Sec. 4.3's count written in the
    Chebyshev basis), so one moment pass serves every tested lambda and the
    dichotomy, with the rules of ``estimate_lambda_k``, becomes scalar work.
    Reading taken: the pass uses the first dichotomy pass's signals (sub-stream
    1 of stream COUNT), with ``n_signals_pass`` columns (default n_c).

    Returns (lambda_hat, tested points, [(lambda_t, count_t)], converged, mu).
    """
    from .cheb import moments

    N = A.shape[0]
    nc = n_c if n_signals_pass is None else n_signals_pass
    R = gaussian_block(seed, N, nc, 1, COUNT)
    mu = moments(A, R, p)
    lo, hi = 0.0, 2.0
    trace = []
    for t in range(1, max_steps + 1):
        mid = 0.5 * (lo + hi)
        c = float(np.dot(lowpass_coeffs(mid, p), mu))
        trace.append((mid, c))
        if math.floor(c + 0.5) == k:
            return mid, t, trace, True, mu
        if c < k:
            lo = mid
        else:
            hi = mid
    return hi, max_steps, trace, False, mu
