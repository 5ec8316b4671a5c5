"""Pins of the community-core reading (oracle)."""
import itertools
import math

import numpy as np

import synth
from oracle import cores, csc, metrics


def _brute(L, k):
    T, n = L.shape
    same = np.array([[np.all(L[:, i] == L[:, j]) for j in range(n)] for i in range(n)])
    classes, seen = [], set()
    for i in range(n):
        if i in seen:
            continue
        m = [j for j in range(n) if same[i, j]]
        seen.update(m)
        classes.append(m)
    classes.sort(key=lambda m: (-len(m), m[0]))
    out = -np.ones(n, dtype=int)
    for c, m in enumerate(classes[:k]):
        out[m] = c
    return out


def test_core_labels_match_the_pairwise_definition():
    rng = np.random.default_rng(0)
    for trial in range(30):
        T, n, k = rng.integers(1, 4), rng.integers(5, 40), rng.integers(2, 6)
        L = rng.integers(0, k, size=(T, n))
        assert np.array_equal(cores.core_labels(L, k), _brute(L, k))


def test_single_run_keeps_every_node():
    L = np.array([[2, 0, 1, 1, 2, 2, 0]])
    cl = cores.core_labels(L, 3)
    assert np.all(cl >= 0)
    assert metrics.adjusted_rand_index(cl, L[0]) == 1.0
    assert cl.tolist() == [0, 1, 2, 2, 0, 0, 1]  # largest class first, ties by first position


def test_unstable_nodes_are_dropped():
    L = np.array([[0, 0, 0, 1, 1, 1, 0],
                  [5, 5, 5, 2, 2, 2, 2]])  # the last node changes company
    cl = cores.core_labels(L, 2)
    assert cl.tolist() == [0, 0, 0, 1, 1, 1, -1]


def test_cores_recover_disconnected_blocks():
    gr = synth.disconnected_regular(5, 80, 6, seed=1)
    d = int(math.ceil(4 * math.log(gr.n)))
    labels, lam, omega, cl = cores.run(gr.row_ptr, gr.col, 5, d, 2, T=3, replicates=5)
    assert metrics.adjusted_rand_index(labels, gr.truth) == 1.0
    assert np.all(cl >= 0)
    assert cores.run_seed(7, 0) == 7 and cores.run_seed(2**64 - 1, 1) == (2**64 - 1 + cores.GOLDEN) % 2**64


def test_library_core_grouping_matches_oracle():
    from paper_1602_02018_amd import api

    rng = np.random.default_rng(1)
    for _ in range(200):
        T, n, k = rng.integers(1, 4), rng.integers(1, 60), rng.integers(1, 8)
        L = rng.integers(0, k + 1, size=(T, n))
        assert np.array_equal(api.community_cores(L, k), cores.core_labels(L, k))
