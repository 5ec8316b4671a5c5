"""Rounding-aware k-means parity (Alg. 2 step 6) of the library against the oracle.

The oracle forms the k-means++ running sums of the D^2 weights as the plain
index-order prefix sum; the library sums them in blocks of 32 points.  Both
are the same sum in real arithmetic, and each computed running sum of n
non-negative terms lies within (n - 1) 2^-53 of the total of the exact one
(recursive summation bound), as does u * total.  A pick of the library can
therefore differ from the oracle's only where u * total lies within
4 n 2^-53 * total of the oracle's running sum at the smaller of the two picks;
after such a pick the two replicates follow different centres and are not
compared further.

Lloyd's iterations and the choice of the best replicate have no such freedom:
started from the library's own picks, the oracle must reproduce its labels
and inertia bit for bit.
"""
from __future__ import annotations

import numpy as np

from oracle import kmeans

EPS = 2.0 ** -53


def check_seeding(X: np.ndarray, k: int, seed: int, picks: np.ndarray) -> list[bool]:
    """Compares the library's picks (replicates x k) with the oracle's seeding.
    Returns, per replicate, whether every pick agreed; asserts that every
    disagreement is a near-tie of the running sums."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    same = []
    for r in range(picks.shape[0]):
        rec: list = []
        kmeans.seed_plusplus(X, k, seed, r, record=rec)
        agree = True
        for c, (pick, target, cum) in enumerate(rec):
            lib_pick = int(picks[r, c])
            if lib_pick == pick:
                continue
            assert target is not None, (r, c, pick, lib_pick, "no sum decides this pick")
            j = min(pick, lib_pick)
            gap = abs(cum[j] - target)
            assert gap <= 4 * n * EPS * cum[-1], (r, c, pick, lib_pick, gap / cum[-1])
            agree = False
            break
        same.append(agree)
    return same


def check_lloyd(X: np.ndarray, picks: np.ndarray, labels: np.ndarray, inertia: float,
                max_iter: int = 100) -> None:
    """The oracle's Lloyd iterations and best-replicate choice from the
    library's picks give the library's labels and inertia exactly."""
    X = np.asarray(X, dtype=np.float64)
    lab, _, inn = kmeans.best_of(X, [X[picks[r]] for r in range(picks.shape[0])], max_iter)
    assert np.array_equal(lab, labels)
    assert inn == inertia, (inn, inertia)


def check_kmeans(X, k, seed, picks, labels, inertia, max_iter=100) -> list[bool]:
    """Both checks; where every pick of every replicate agrees, the plain oracle
    k-means gives the library's result as well."""
    same = check_seeding(X, k, seed, picks)
    check_lloyd(X, picks, labels, inertia, max_iter)
    if all(same):
        lab, _, inn = kmeans.kmeans(np.asarray(X, np.float64), k, seed, picks.shape[0], max_iter)
        assert np.array_equal(lab, labels) and inn == inertia
    return same
