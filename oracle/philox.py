"""Philox4x64-10 and the draws built from it (oracle; test infrastructure only).

Philox4x64-R is the counter-based generator of Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3" (SC'11).  A 256-bit counter
(c0, c1, c2, c3) and a 128-bit key (k0, k1) go through R = 10 rounds; each
round forms the two 128-bit products M0*c0 and M1*c2 and sets

    (c0, c1, c2, c3) <- (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0))

and then bumps the key by the Weyl constants (W0, W1).  The four output words
are the final counter state.

The paper draws Gaussian random signals with mean 0 and variance 1/d (Sec. 3.1,
Alg. 2 step 3) and samples nodes uniformly without replacement (Sec. 3.2.2);
it does not fix a generator.  This module fixes one so that two independent
implementations can draw the same numbers:

* key = (seed, 0);
* Gaussian entry (i, j) of an N x w block for sub-stream t of stream S uses the
  counter (i*w + j, t, S, 0); with words x0, x1,
  u1 = ((x0 >> 11) + 1) * 2^-53 in (0, 1], u2 = (x1 >> 11) * 2^-53 in [0, 1),
  z = sqrt(-2 ln u1) cos(2 pi u2) / sqrt(w)   (Box-Muller);
* the sampling key of node i is x0 at counter (i, 0, SAMPLE, 0);
* a uniform draw for k-means++ uses x0 at counter (j, r, KMEANS, 0):
  u = (x0 >> 11) * 2^-53.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)

COUNT, FEAT, SAMPLE, KMEANS, MLP = 1, 2, 3, 4, 5


def _mulhilo(a: np.ndarray, m: np.uint64):
    """128-bit product of uint64 arrays with a constant, as (hi, lo) words."""
    a = a.astype(np.uint64)
    a_lo = a & _LO32
    a_hi = a >> _S32
    m_lo = m & _LO32
    m_hi = m >> _S32
    t = a_lo * m_lo
    u = a_hi * m_lo + (t >> _S32)
    v = a_lo * m_hi + (u & _LO32)
    hi = a_hi * m_hi + (u >> _S32) + (v >> _S32)
    lo = a * m  # wraps modulo 2^64
    return hi, lo


def philox4x64(c0, c1, c2, c3, k0, k1, rounds: int = 10):
    """Philox4x64-``rounds`` of broadcastable uint64 counters and keys."""
    with np.errstate(over="ignore"):
        c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) for x in (c0, c1, c2, c3))
        c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
        k0 = np.uint64(k0)
        k1 = np.uint64(k1)
        for _ in range(rounds):
            hi0, lo0 = _mulhilo(c0, M0)
            hi1, lo1 = _mulhilo(c2, M1)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
            k0 = np.uint64(k0 + W0)
            k1 = np.uint64(k1 + W1)
    return c0, c1, c2, c3


def gaussian_block(seed: int, n_rows: int, w: int, t: int, stream: int) -> np.ndarray:
    """n_rows x w block of N(0, 1/w) entries for sub-stream ``t`` of ``stream``."""
    e = np.arange(n_rows * w, dtype=np.uint64)
    x0, x1, _, _ = philox4x64(e, np.uint64(t), np.uint64(stream), np.uint64(0), np.uint64(seed), 0)
    u1 = ((x0 >> np.uint64(11)) + np.uint64(1)).astype(np.float64) * 2.0**-53
    u2 = (x1 >> np.uint64(11)).astype(np.float64) * 2.0**-53
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    return (z / np.sqrt(float(w))).reshape(n_rows, w)


def sample_keys(seed: int, N: int) -> np.ndarray:
    """64-bit sampling key of every node."""
    i = np.arange(N, dtype=np.uint64)
    x0, _, _, _ = philox4x64(i, 0, SAMPLE, 0, np.uint64(seed), 0)
    return x0


def uniform(seed: int, j: int, r: int, stream: int) -> float:
    """One uniform draw in [0, 1) at counter (j, r, stream, 0)."""
    x0, _, _, _ = philox4x64(np.uint64(j), np.uint64(r), np.uint64(stream), 0, np.uint64(seed), 0)
    return float(int(x0) >> 11) * 2.0**-53
