"""Seeded synthetic graphs in CSR form.

Every generator returns an undirected, unweighted graph without self-loops as a
symmetric CSR pattern (``row_ptr`` int32[N+1], ``col`` int32[nnz], column
indices sorted within each row) plus the planted community of every node.
Node ids are randomly permuted, so community membership carries no locality in
memory, as for a graph read from disk.

Models
------
* Stochastic block model (SBM), Sec. 5.1 of the paper: edge probability q1
  inside a community and q2 = eps * q1 across, parameterised by eps and the
  mean degree s; eps_c = (s - sqrt s) / (s + sqrt s (k - 1)) is the
  detectability threshold quoted there.  q1 is set so that the expected mean
  degree is exactly s.  Edges are drawn per block pair as a binomial edge count
  followed by that many distinct uniformly chosen vertex pairs, which is the
  same distribution as one Bernoulli trial per pair, in O(N + E).
* Chung-Lu graph with power-law expected degrees and planted blocks (a skewed
  degree workload that the paper does not use): weights
  w_i = c (i0 + i)^(-1/(gamma-1)) fitted to a mean and a maximum degree; a
  global Poisson edge multiset with endpoints drawn proportionally to w (the
  Norros-Reittu form of Chung-Lu, edge probability 1 - exp(-w_i w_j / S)),
  plus, inside each block, extra Poisson edges carrying (boost - 1) times the
  same rate, so that pairs inside a block connect about ``boost`` times more
  often.  Multi-edges and self-loops are dropped.
* k disconnected random regular blocks (the eps = 0 case of Sec. 3.2.1).
* Batches of SBMs with per-graph random N, k and s.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Graph:
    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    truth: np.ndarray
    k: int
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))


def _rng(seed: int, tag: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(tag)])))


def eps_critical(s: float, k: int) -> float:
    """Detectability threshold of the SBM quoted in Sec. 5.1 (Decelle et al.)."""
    rs = math.sqrt(s)
    return (s - rs) / (s + rs * (k - 1))


def csr_from_edges(n: int, u: np.ndarray, v: np.ndarray):
    """Symmetric CSR pattern from an undirected edge multiset.

    Self-loops and repeated edges are dropped; columns are sorted per row.
    """
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    a = np.minimum(u, v)
    b = np.maximum(u, v)
    key = np.unique(a * n + b)
    a = key // n
    b = key - a * n
    rows = np.concatenate([a, b])
    cols = np.concatenate([b, a])
    key = np.sort(rows * n + cols)
    rows = key // n
    cols = key - rows * n
    if cols.shape[0] >= 2**31:
        raise ValueError("graph has 2^31 or more stored entries")
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return row_ptr.astype(np.int32), cols.astype(np.int32)


def _relabel(n, u, v, truth_block_order, rng):
    """Apply a uniformly random node permutation."""
    perm = rng.permutation(n).astype(np.int64)
    truth = np.empty(n, dtype=np.int32)
    truth[perm] = truth_block_order
    return perm[u], perm[v], truth


def _tri_decode(t: np.ndarray):
    """Index t of the pair (u, v), u > v >= 0, in the order t = u(u-1)/2 + v."""
    u = np.floor((1.0 + np.sqrt(1.0 + 8.0 * t.astype(np.float64))) / 2.0).astype(np.int64)
    for _ in range(3):
        hi = u * (u - 1) // 2 > t
        u = np.where(hi, u - 1, u)
        lo = (u + 1) * u // 2 <= t
        u = np.where(lo, u + 1, u)
    v = t - u * (u - 1) // 2
    return u, v


def sbm(N: int, k: int, s: float, eps: float, seed: int, sizes=None, name: str = "sbm") -> Graph:
    """Stochastic block model with mean degree ``s`` and ratio ``eps`` = q2/q1."""
    rng = _rng(seed, 0x5B3)
    if sizes is None:
        base, rem = divmod(N, k)
        sizes = [base + 1] * rem + [base] * (k - rem)
    sizes = np.asarray(sizes, dtype=np.int64)
    if sizes.sum() != N or sizes.shape[0] != k or np.any(sizes < 1):
        raise ValueError("community sizes must be positive and sum to N")
    offs = np.zeros(k + 1, dtype=np.int64)
    np.cumsum(sizes, out=offs[1:])
    within = float(np.sum(sizes * (sizes - 1)))
    across = float(np.sum(sizes * (N - sizes)))
    q1 = s * N / (within + eps * across)
    q2 = eps * q1
    if q1 > 1.0:
        raise ValueError("mean degree too large for the community sizes")

    ia, ib = np.triu_indices(k)
    ia = ia.astype(np.int64)
    ib = ib.astype(np.int64)
    same = ia == ib
    M = np.where(same, sizes[ia] * (sizes[ia] - 1) // 2, sizes[ia] * sizes[ib])
    q = np.where(same, q1, q2)
    want = rng.binomial(M, q).astype(np.int64)
    base_key = np.zeros(M.shape[0] + 1, dtype=np.int64)
    np.cumsum(M, out=base_key[1:])

    keys = np.empty(0, dtype=np.int64)
    need = want.copy()
    for _ in range(64):
        tot = int(need.sum())
        if tot == 0:
            break
        pair = np.repeat(np.arange(M.shape[0], dtype=np.int64), need)
        pos = np.floor(rng.random(tot) * M[pair]).astype(np.int64)
        pos = np.minimum(pos, M[pair] - 1)
        keys = np.unique(np.concatenate([keys, base_key[pair] + pos]))
        have = np.bincount(np.searchsorted(base_key, keys, side="right") - 1, minlength=M.shape[0])
        need = want - have[: M.shape[0]]
    else:
        raise RuntimeError("SBM edge sampling did not settle")

    pair = np.searchsorted(base_key, keys, side="right") - 1
    pos = keys - base_key[pair]
    a = ia[pair]
    b = ib[pair]
    u = np.empty_like(pos)
    v = np.empty_like(pos)
    sm = a == b
    tu, tv = _tri_decode(pos[sm])
    u[sm] = offs[a[sm]] + tu
    v[sm] = offs[a[sm]] + tv
    nb = sizes[b[~sm]]
    u[~sm] = offs[a[~sm]] + pos[~sm] // nb
    v[~sm] = offs[b[~sm]] + pos[~sm] % nb

    truth_bo = np.repeat(np.arange(k, dtype=np.int32), sizes)
    u, v, truth = _relabel(N, u, v, truth_bo, rng)
    row_ptr, col = csr_from_edges(N, u, v)
    return Graph(N, row_ptr, col, truth, k, name,
                 dict(model="sbm", s=s, eps=eps, q1=q1, q2=q2, seed=seed, sizes=sizes.tolist()))


def sbm_config(N: int, k: int, s: float = 16.0, seed: int = 0, eps_factor: float = 0.25) -> Graph:
    """SBM with equal communities at eps = eps_factor * eps_c (the paper uses eps_c / 4)."""
    eps = eps_factor * eps_critical(s, k)
    return sbm(N, k, s, eps, seed, name=f"sbm_N{N}_k{k}_s{s:g}")


def _fit_powerlaw_offset(N, mean_deg, max_deg, g):
    i = np.arange(N, dtype=np.float64)

    def mean_w(i0):
        return float(np.mean(max_deg * (i0 / (i0 + i)) ** g))

    lo, hi = 1e-6, float(N)
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if mean_w(mid) < mean_deg:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def chung_lu_blocks(N: int, k: int, mean_deg: float = 20.0, max_deg: float = 2000.0,
                    exponent: float = 2.5, boost: float = 20.0, seed: int = 0,
                    name: str = "chunglu") -> Graph:
    """Chung-Lu graph with power-law expected degrees and ``k`` planted blocks."""
    rng = _rng(seed, 0xC1)
    g = 1.0 / (exponent - 1.0)
    i0 = _fit_powerlaw_offset(N, mean_deg, max_deg, g)
    w = max_deg * (i0 / (i0 + np.arange(N, dtype=np.float64))) ** g
    lab = rng.permutation(np.arange(N, dtype=np.int64) % k)
    S = w.sum()
    Sb = np.bincount(lab, weights=w, minlength=k)
    # expected degree of i: w_i (1 + (boost - 1) S_b(i) / S); rescale to the target mean
    scale = mean_deg / float(np.mean(w * (1.0 + (boost - 1.0) * Sb[lab] / S)))
    w *= scale
    S = w.sum()
    Sb = np.bincount(lab, weights=w, minlength=k)

    cw = np.cumsum(w)
    m_glob = int(rng.poisson(S / 2.0))
    ug = np.searchsorted(cw, rng.random(m_glob) * S, side="right")
    vg = np.searchsorted(cw, rng.random(m_glob) * S, side="right")

    order = np.argsort(lab, kind="stable")
    cwo = np.cumsum(w[order])
    bstart = np.zeros(k + 1, dtype=np.int64)
    np.cumsum(np.bincount(lab, minlength=k), out=bstart[1:])
    before = np.concatenate([[0.0], cwo])[bstart[:-1]]
    m_b = rng.poisson((boost - 1.0) * Sb * Sb / (2.0 * S))
    blk = np.repeat(np.arange(k, dtype=np.int64), m_b)

    def draw(blk_ids):
        t = before[blk_ids] + rng.random(blk_ids.shape[0]) * Sb[blk_ids]
        j = np.searchsorted(cwo, t, side="right")
        j = np.clip(j, bstart[blk_ids], bstart[blk_ids + 1] - 1)
        return order[j]

    ub = draw(blk)
    vb = draw(blk)
    ug = np.minimum(ug, N - 1)
    vg = np.minimum(vg, N - 1)
    u = np.concatenate([ug, ub]).astype(np.int64)
    v = np.concatenate([vg, vb]).astype(np.int64)
    u, v, truth = _relabel(N, u, v, lab.astype(np.int32), rng)
    row_ptr, col = csr_from_edges(N, u, v)
    return Graph(N, row_ptr, col, truth, k, name,
                 dict(model="chung_lu_blocks", mean_deg=mean_deg, max_deg=max_deg,
                      exponent=exponent, boost=boost, i0=i0, seed=seed))


def disconnected_regular(k: int, block_size: int, degree: int, seed: int = 0,
                         name: str = "regular_blocks") -> Graph:
    """k disconnected random ``degree``-regular blocks of ``block_size`` nodes each."""
    import networkx as nx

    rng = _rng(seed, 0x7E6)
    us, vs = [], []
    for b in range(k):
        gb = nx.random_regular_graph(degree, block_size, seed=int(rng.integers(0, 2**31 - 1)))
        e = np.asarray(list(gb.edges()), dtype=np.int64).reshape(-1, 2)
        us.append(e[:, 0] + b * block_size)
        vs.append(e[:, 1] + b * block_size)
    N = k * block_size
    truth_bo = np.repeat(np.arange(k, dtype=np.int32), block_size)
    u, v, truth = _relabel(N, np.concatenate(us), np.concatenate(vs), truth_bo, rng)
    row_ptr, col = csr_from_edges(N, u, v)
    return Graph(N, row_ptr, col, truth, k, name,
                 dict(model="disconnected_regular", degree=degree, block_size=block_size, seed=seed))


def sbm_batch_specs(G: int = 64, seed: int = 0, n_range=(2000, 200000), k_range=(10, 100),
                    s_range=(8.0, 32.0), eps_factor: float = 0.25):
    """(N, k, s, eps, graph seed) of every graph of ``sbm_batch``, without drawing edges."""
    rng = _rng(seed, 0xBA7C)
    out = []
    for g in range(G):
        N = int(rng.integers(n_range[0], n_range[1] + 1))
        k = int(rng.integers(k_range[0], k_range[1] + 1))
        s = float(rng.uniform(s_range[0], s_range[1]))
        out.append((N, k, s, eps_factor * eps_critical(s, k), seed + g))
    return out


def sbm_batch(G: int = 64, seed: int = 0, n_range=(2000, 200000), k_range=(10, 100),
              s_range=(8.0, 32.0), eps_factor: float = 0.25, only=None):
    """Batch of SBMs with N, k, s drawn uniformly per graph; graph g uses seed + g.
    ``only`` (a list of positions in the batch) draws just those graphs, the
    same as the full batch holds at those positions."""
    specs = sbm_batch_specs(G, seed, n_range, k_range, s_range, eps_factor)
    pick = range(G) if only is None else only
    return [sbm(*specs[g][:4], specs[g][4], name=f"batch{g}_N{specs[g][0]}_k{specs[g][1]}")
            for g in pick]
