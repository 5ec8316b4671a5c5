"""Node sampling for Alg. 2 step 5 (oracle; test only).

Sec. 3.2.2 draws n distinct node indices uniformly at random; the sampling
matrix M of Eq. (4) has M_ij = 1 iff j = omega_i.  Reading taken: every node
gets an independent uniform 64-bit key (see ``philox``) and Omega lists the n
nodes with the smallest (key, index) pairs in increasing order, which is a
uniformly random n-subset in uniformly random order.
"""
from __future__ import annotations

import numpy as np

from .philox import SAMPLE, philox4x64, sample_keys


def sample(N: int, n: int, seed: int) -> np.ndarray:
    keys = sample_keys(seed, N)
    order = np.lexsort((np.arange(N), keys))
    return order[:n].astype(np.int64)


def density_keys(w: np.ndarray, seed: int) -> np.ndarray:
    """Exponential-race keys E_i / w_i of variable-density sampling.

    E_i = -ln(u_i) with u_i = ((x0 >> 11) + 1) 2^-53 in (0, 1], x0 the first
    Philox word at counter (i, 1, SAMPLE, 0); nodes with w_i <= 0 (or not
    finite) get +inf.
    """
    w = np.asarray(w, dtype=np.float64)
    N = w.size
    i = np.arange(N, dtype=np.uint64)
    x0, _, _, _ = philox4x64(i, 1, SAMPLE, 0, np.uint64(seed), 0)
    u = ((x0 >> np.uint64(11)) + np.uint64(1)).astype(np.float64) * 2.0**-53
    E = -np.log(u)
    keys = np.full(N, np.inf)
    ok = np.isfinite(w) & (w > 0.0)
    keys[ok] = E[ok] / w[ok]
    return keys


def sample_density(w: np.ndarray, n: int, seed: int):
    """Variable-density sampling of n distinct nodes, P(i drawn next) proportional to w_i.

    The paper (Sec. 3.2.3) leaves the optimal distribution to Puy et al.: it
    follows the local cumulative coherence, p_i = v_k(i)^2 / k, and Sec. 4.1
    notes that v_k(i) is estimated by the norm of row i of the filtered random
    signals, so w_i = ||(h~(L) R)_i||^2.  Reading taken: n distinct nodes by
    successive sampling (each next node drawn with probability proportional to
    w among the nodes not yet drawn), realised as an exponential race: the n
    smallest keys E_i / w_i (ties by index), in increasing key order.

    Returns (omega, decoder weights): the weights 1 / (N p_i) = mean(w) / w_i
    of the sampled nodes, which turn Eq. (5)'s fidelity term into Puy et al.'s
    weighted one (uniform w gives weights 1).
    """
    w = np.asarray(w, dtype=np.float64)
    keys = density_keys(w, seed)
    order = np.lexsort((np.arange(w.size), keys))
    omega = order[:n].astype(np.int64)
    mean = float(np.sum(w)) / w.size
    with np.errstate(divide="ignore"):
        dw = np.where(w[omega] > 0.0, mean / w[omega], 0.0)
    return omega, dw
