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
from dataclasses import dataclass

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


@dataclass
class Search:
    """Outcome of a dichotomy: the estimate, the number of tested points (one
    eigencount pass each), the (lambda_t, count_t) of every test, whether a
    count rounded to k, whether a given bracket missed lambda_k, the bracket
    the learned search started from, and the interval (lo, hi) whose midpoint
    each test evaluated."""
    lam: float
    steps: int
    trace: list
    found: bool
    missed: bool = False
    bracket: tuple | None = None
    intervals: list | None = None


def _test(A, lam, p, n_c, seed, t, k, damping):
    R = gaussian_block(seed, A.shape[0], n_c, t, COUNT)
    c = eigencount(A, lam, p, R, damping)
    return c, math.floor(c + 0.5) == k


def dichotomy(A, k: int, p: int, n_c: int, seed: int, max_steps: int = 30, bracket=None,
              damping: bool = True) -> Search:
    """The dichotomy of Sec. 4.3 from [0, 2], or from a caller's bracket.

    Test t (t = 1, 2, ...) evaluates the midpoint of the current interval with
    fresh signals (sub-stream t).  Reading for a caller's bracket: if its
    max_steps tests all fall on the same side of k, lambda_k is not inside it,
    and the search starts again from [0, 2] with the following sub-streams,
    for at most max_steps further tests."""
    lo, hi = (0.0, 2.0) if bracket is None else (float(bracket[0]), float(bracket[1]))
    trace, ivs = [], []
    t = 0
    missed = False
    for attempt in range(2 if bracket is not None else 1):
        sides = set()
        for _ in range(max_steps):
            t += 1
            mid = 0.5 * (lo + hi)
            c, stop = _test(A, mid, p, n_c, seed, t, k, damping)
            trace.append((mid, c))
            ivs.append((lo, hi))
            if stop:
                return Search(mid, t, trace, True, missed, intervals=ivs)
            if c < k:
                lo = mid
                sides.add("below")
            else:
                hi = mid
                sides.add("above")
        if bracket is None or attempt == 1 or len(sides) == 2:
            break
        missed = True
        lo, hi = 0.0, 2.0
    return Search(hi, t, trace, False, missed, intervals=ivs)


def estimate_lambda_k(A, k: int, p: int, n_c: int, seed: int, max_steps: int = 30,
                      bracket=None, damping: bool = True):
    """Returns (lambda_hat, steps_used, [(lambda_t, count_t)], converged)."""
    r = dichotomy(A, k, p, n_c, seed, max_steps, bracket, damping)
    return r.lam, r.steps, r.trace, r.found


def estimate_lambda_k_learned(A, k: int, p: int, n_c: int, seed: int, theta,
                              max_steps: int = 30) -> Search:
    """Dichotomy of Sec. 4.3 started from a bracket proposed by the lambda_k
    network (the paper only remarks that a better estimate of lambda_k would
    help, Sec. 5.2; this search is the library's reading of that remark).

    1. Test 1 is the plain search's first test, lambda = 1 with sub-stream 1;
       if its count rounds to k the search ends there.
    2. Otherwise the count at 1 says which half of [0, 2] holds lambda_k.
       The moments of that same pass give the count curve c(lambda) of those
       signals at every lambda, its root lambda_0 and the spread s
       (mlp.count_root); the network maps the pass's features to two offsets
       y, and the bracket is [lambda_0 + s min(y), lambda_0 + s max(y)] cut to
       the half.  If that leaves less than 1/1024, the bracket is
       lambda_0 (moved into the half) plus or minus max(s, 1/1024), cut to
       the half.
    3. Tests 2, 3, ... bisect inside with fresh signals (sub-stream t), with
       the plain stopping rule.  If the first four tests inside the bracket
       all fall on the same side of k (the interval is then a sixteenth of
       the bracket), the search reopens, once, onto the rest of the half on
       that side (from the bracket's upper end to the top of the half when
       the counts were below k, from the bottom of the half to the bracket's
       lower end when above); that reopening marks a bracket miss.
    4. After max_steps tests in all, the upper end is returned.

    theta: the network's float parameters (mlp.N_PARAMS), evaluated in
    float64 here.  Returns a Search whose ``bracket`` is the bracket of step 2
    ((1, 1) when test 1 stopped)."""
    from .cheb import moments
    from . import mlp

    N = A.shape[0]
    R = gaussian_block(seed, N, n_c, 1, COUNT)
    mu = moments(A, R, p)
    c1 = float(np.dot(lowpass_coeffs(1.0, p), mu))
    trace, ivs = [(1.0, c1)], [(0.0, 2.0)]
    if math.floor(c1 + 0.5) == k:
        return Search(1.0, 1, trace, True, False, (1.0, 1.0), ivs)
    half = (1.0, 2.0) if c1 < k else (0.0, 1.0)
    lam0, s = mlp.count_root(mu, p, k, n_c)
    y, _ = mlp.forward(np.asarray(theta, dtype=np.float64), mlp.features(mu, N, k).reshape(1, -1))
    ya, yb = sorted((float(y[0, 0]), float(y[0, 1])))
    lo, hi = max(lam0 + s * ya, half[0]), min(lam0 + s * yb, half[1])
    if not hi - lo >= 1.0 / 1024:
        centre = min(max(lam0, half[0]), half[1])
        width = max(s, 1.0 / 1024)
        lo, hi = max(half[0], centre - width), min(half[1], centre + width)
    lo0, hi0 = lo, hi
    below = above = reopened = False
    t = 1
    while t < max_steps:
        t += 1
        mid = 0.5 * (lo + hi)
        c, stop = _test(A, mid, p, n_c, seed, t, k, True)
        trace.append((mid, c))
        ivs.append((lo, hi))
        if stop:
            return Search(mid, t, trace, True, reopened, (lo0, hi0), ivs)
        if c < k:
            lo, below = mid, True
        else:
            hi, above = mid, True
        if not reopened and not (below and above) and t - 1 >= 4:
            reopened = True
            if below and hi0 < half[1]:
                lo, hi = hi0, half[1]
            elif above and lo0 > half[0]:
                lo, hi = half[0], lo0
    return Search(hi, t, trace, False, reopened, (lo0, hi0), ivs)


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
