"""k-means on the sampled features, Alg. 2 step 6 (oracle; test only).

The paper runs Matlab's kmeans with 20 replicates (Sec. 5) and leaves the rest
to that routine.  Reading taken here, fixed to the last rounding so that an
independent implementation can reproduce it exactly from the same inputs:

* squared distances sum (x_j - c_j)^2 over coordinates j in increasing order;
* k-means++ seeding per replicate r: draw u_0 at counter (0, r, KMEANS, 0) and
  take point floor(u_0 n) as the first centre; then for centre c = 1..k-1 draw
  u_c, form the running sums, in index order, of each point's squared distance
  to its nearest chosen centre (D^2 weighting), and take the first point whose
  running sum exceeds u_c times the total (the last point with a non-zero
  distance if none does; point floor(u_c n) if the total is 0);
* Lloyd iterations, at most ``max_iter`` (Matlab's default is 100): assign each
  point to its nearest centre (lowest index on ties); stop when no assignment
  changed (and the previous update re-seeded nothing); otherwise recompute each
  centre as the mean of its points, summed in index order; an empty cluster,
  taken in increasing order, is re-seeded with the point farthest from its
  current centre (lowest index on ties), which moves to it;
* the replicate with the smallest inertia (sum of squared distances to the
  assigned centres, in index order) wins; ties keep the earlier replicate.
"""
from __future__ import annotations

import math

import numpy as np

from .philox import KMEANS, uniform


def sqdist(X: np.ndarray, c: np.ndarray) -> np.ndarray:
    acc = np.zeros(X.shape[0])
    for j in range(X.shape[1]):
        diff = X[:, j] - c[j]
        acc = acc + diff * diff
    return acc


def seed_plusplus(X: np.ndarray, k: int, seed: int, r: int, record: list | None = None) -> np.ndarray:
    """k-means++ centres of replicate r.  With ``record`` (a list), appends for
    every centre c the tuple (pick, target, cum): the chosen point, u_c times
    the total and the running sums it was compared with (None for c = 0 and
    for a zero total, where no sum decides the pick)."""
    n = X.shape[0]
    u = uniform(seed, 0, r, KMEANS)
    first = min(int(math.floor(u * n)), n - 1)
    centres = [X[first].copy()]
    if record is not None:
        record.append((first, None, None))
    mind = sqdist(X, centres[0])
    for c in range(1, k):
        u = uniform(seed, c, r, KMEANS)
        cum = np.cumsum(mind)  # plain running sums in index order
        total = cum[-1]
        target = None
        if total == 0.0:
            pick = min(int(math.floor(u * n)), n - 1)
        else:
            target = u * total
            pick = int(np.searchsorted(cum, target, side="right"))
            if pick >= n:
                pick = int(np.nonzero(mind > 0.0)[0][-1])
        if record is not None:
            record.append((pick, target, cum if target is not None else None))
        centres.append(X[pick].copy())
        mind = np.minimum(mind, sqdist(X, centres[-1]))
    return np.array(centres)


def sqdist_rows(X: np.ndarray, P: np.ndarray) -> np.ndarray:
    """Row-wise squared distance between X[i] and P[i], coordinates in order."""
    acc = np.zeros(X.shape[0])
    for j in range(X.shape[1]):
        diff = X[:, j] - P[:, j]
        acc = acc + diff * diff
    return acc


def assign(X: np.ndarray, C: np.ndarray) -> np.ndarray:
    D = np.zeros((X.shape[0], C.shape[0]))
    for j in range(X.shape[1]):
        diff = X[:, j, None] - C[None, :, j]
        D = D + diff * diff
    return np.argmin(D, axis=1)


def lloyd(X: np.ndarray, C: np.ndarray, max_iter: int):
    C = C.copy()
    k = C.shape[0]
    labels = None
    reseeded = False
    for _ in range(max_iter):
        new = assign(X, C)
        if labels is not None and not reseeded and np.array_equal(new, labels):
            break
        labels = new
        counts = np.bincount(labels, minlength=k)
        for c in range(k):
            if counts[c] > 0:
                C[c] = np.cumsum(X[labels == c], axis=0)[-1] / counts[c]
        reseeded = bool(np.any(counts == 0))
        for c in range(k):
            if counts[c] == 0:
                d = sqdist_rows(X, C[labels])
                far = int(np.argmax(d))
                C[c] = X[far]
                counts[labels[far]] -= 1
                labels[far] = c
                counts[c] = 1
    inertia = float(np.cumsum(sqdist_rows(X, C[labels]))[-1])
    return labels, C, inertia


def best_of(X: np.ndarray, seeds, max_iter: int = 100):
    """Lloyd from each replicate's initial centres (in replicate order); returns
    (labels, centres, inertia) of the smallest inertia, the earliest on ties."""
    X = np.asarray(X, dtype=np.float64)
    best = None
    for C0 in seeds:
        lab, C, inertia = lloyd(X, np.asarray(C0, dtype=np.float64), max_iter)
        if best is None or inertia < best[2]:
            best = (lab, C, inertia)
    return best


def kmeans(X: np.ndarray, k: int, seed: int, replicates: int = 20, max_iter: int = 100):
    """Returns (labels, centres, inertia) of the best replicate."""
    X = np.asarray(X, dtype=np.float64)
    return best_of(X, (seed_plusplus(X, k, seed, r) for r in range(replicates)), max_iter)
