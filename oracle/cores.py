"""Community cores (oracle; test only).

The paper's conclusion proposes to repeat the feature filtering with new
random signals and the clustering of the sampled nodes, to keep the sets of
nodes that are always clustered together, and to interpolate from these
stable cores only.  Readings taken:

* T runs on the same lambda and the same sampled nodes; run t draws its
  signals with seed_t = (seed + t * 0x9E3779B97F4A7C15) mod 2^64 (run 0 is the
  plain run) and clusters with k-means under the same seed;
* two sampled nodes are always clustered together iff their labels agree in
  every run, i.e. they share the label tuple (l_0(i), ..., l_{T-1}(i));
* the cores are the k largest tuple classes, ties broken by the smallest
  sample position of a member; core c (0 = largest) labels its members c;
  sampled nodes outside the cores take no part in the interpolation.
"""
from __future__ import annotations

import numpy as np

GOLDEN = 0x9E3779B97F4A7C15


def run_seed(seed: int, t: int) -> int:
    return (int(seed) + t * GOLDEN) % (1 << 64)


def core_labels(L: np.ndarray, k: int) -> np.ndarray:
    """L: T x n labels of the sampled nodes; returns int[n], -1 outside the cores."""
    L = np.asarray(L, dtype=np.int64)
    T, n = L.shape
    classes = {}
    for s in range(n):
        key = tuple(int(x) for x in L[:, s])
        classes.setdefault(key, []).append(s)
    ranked = sorted(classes.values(), key=lambda m: (-len(m), m[0]))
    out = np.full(n, -1, dtype=np.int64)
    for c, members in enumerate(ranked[:k]):
        out[members] = c
    return out


def run(row_ptr, col, k: int, d: int, seed: int, T: int, p: int = 50, n: int | None = None,
        gamma: float = 1e-3, replicates: int = 20, **kw):
    """Alg. 2 with community cores: returns (labels, lambda, omega, core labels)."""
    from . import csc, interp, kmeans, laplacian, sampling
    from .eigencount import count_signals, estimate_lambda_k

    A, _ = laplacian.normalized_adjacency(row_ptr, col)
    N = A.shape[0]
    n = csc.default_n(k) if n is None else n
    lam, _, _, _ = estimate_lambda_k(A, k, p, count_signals(N), seed)
    omega = sampling.sample(N, n, seed)
    L = np.stack([kmeans.kmeans(csc.features(A, lam, p, d, run_seed(seed, t))[omega], k, seed,
                                replicates)[0] for t in range(T)])
    cl = core_labels(L, k)
    keep = cl >= 0
    X, labels, _, _ = interp.interpolate(A, lam, p, gamma, omega[keep], cl[keep], k)
    return labels, lam, omega, cl
