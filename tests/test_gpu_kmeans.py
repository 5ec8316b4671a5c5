"""k-means on the GPU against the host form and the float64 oracle.  The host
and GPU forms run the same sums in the same order, so their labels and
inertia must be bit-identical; against the oracle (plain prefix sums in the
seeding) the picks agree up to near-ties of the running sums and Lloyd from
the same picks agrees exactly (tests/kmeans_parity.py)."""
import numpy as np
import pytest
import torch

from kmeans_parity import check_kmeans

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_1602_02018_amd import api as a

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return a


def _blobs(seed, n, d, k, spread=0.3):
    rng = np.random.default_rng(seed)
    centers = rng.normal(size=(k, d))
    X = centers[rng.integers(0, k, n)] + spread * rng.normal(size=(n, d))
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    return X.astype(np.float32)


@pytest.mark.parametrize("seed,n,d,k,reps", [
    (0, 47, 28, 10, 20),      # plain configuration
    (3, 300, 12, 25, 20),
    (5, 922, 47, 100, 20),    # 1e5-node SBM configuration
    (7, 2761, 56, 250, 4),    # 1e6-node configuration
    (1, 5000, 8, 20, 3),      # more points than the LDS copy of the D^2 weights
    (2, 33, 5, 33, 5),        # k = n
    (4, 1024, 48, 64, 6),     # largest seeding with the points in registers
    (10, 32, 6, 5, 4),        # one full block of the seeding sums
    (11, 64, 6, 7, 4),        # two full blocks
    (12, 1, 3, 1, 2),         # one point, one cluster
    (6, 1025, 49, 40, 4),     # just past it in both n and d
    (8, 700, 49, 30, 4),      # past it in d only
    (13, 3000, 8, 300, 2),    # member lists by a scan of the labels: (blocks x k) counts past LDS
    (14, 9000, 6, 12, 2),     # labels past the update's LDS copy: the scan over global memory
])
def test_device_kmeans_is_bit_identical_to_host(api, seed, n, d, k, reps):
    X = _blobs(seed, n, d, k)
    lab_h, in_h = api.kmeans_reduced(X, k, seed, replicates=reps)
    Xd = torch.as_tensor(X, device="cuda")
    lab_d, in_d = api.kmeans_reduced_device(Xd, k, seed, replicates=reps)
    assert np.array_equal(lab_h, lab_d)
    assert in_h == in_d
    picks = api.kmeans_seeds_device(Xd, k, seed, replicates=reps)
    assert np.array_equal(picks, api.kmeans_seeds(X, k, seed, replicates=reps))
    check_kmeans(X, k, seed, picks, lab_d, in_d)


def test_device_kmeans_duplicates_ties_and_reseeds(api):
    # few distinct points: zero D^2 totals, exact distance ties, empty clusters
    rng = np.random.default_rng(11)
    base = rng.normal(size=(4, 6)).astype(np.float32)
    X = base[rng.integers(0, 4, 40)]
    for k in (3, 6, 9):
        lab_h, in_h = api.kmeans_reduced(X, k, 4, replicates=6)
        lab_d, in_d = api.kmeans_reduced_device(torch.as_tensor(X, device="cuda"), k, 4,
                                                replicates=6)
        assert np.array_equal(lab_h, lab_d) and in_h == in_d
        picks = api.kmeans_seeds_device(torch.as_tensor(X, device="cuda"), k, 4, replicates=6)
        check_kmeans(X, k, 4, picks, lab_d, in_d)


def test_device_kmeans_matches_oracle(api):
    X = _blobs(9, 200, 16, 12)
    Xd = torch.as_tensor(X, device="cuda")
    lab_d, in_d = api.kmeans_reduced_device(Xd, 12, 9)
    same = check_kmeans(X, 12, 9, api.kmeans_seeds_device(Xd, 12, 9), lab_d, in_d)
    assert all(same)


def test_device_kmeans_iteration_cap(api):
    X = _blobs(4, 500, 10, 30, spread=1.0)
    for mi in (1, 2, 3):
        lab_h, in_h = api.kmeans_reduced(X, 30, 2, replicates=3, max_iter=mi)
        lab_d, in_d = api.kmeans_reduced_device(torch.as_tensor(X, device="cuda"), 30, 2,
                                                replicates=3, max_iter=mi)
        assert np.array_equal(lab_h, lab_d) and in_h == in_d
        picks = api.kmeans_seeds(X, 30, 2, replicates=3)
        check_kmeans(X, 30, 2, picks, lab_d, in_d, max_iter=mi)


def test_batched_device_kmeans_matches_single(api):
    Xs = [_blobs(s, n, d, k) for s, n, d, k in ((0, 47, 28, 10), (1, 300, 12, 25), (2, 90, 30, 7))]
    ks, seeds = [10, 25, 7], [0, 5, 9]
    labs, inert = api.kmeans_reduced_device_batched([torch.as_tensor(x, device="cuda") for x in Xs],
                                                    ks, seeds)
    for X, k, sd, l, i in zip(Xs, ks, seeds, labs, inert):
        l2, i2 = api.kmeans_reduced(X, k, sd)
        assert np.array_equal(l, l2) and i == i2
