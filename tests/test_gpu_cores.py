"""Community cores on the GPU against the float64 oracle, and what they change
on a harder SBM (eps = eps_c / 2): recovery against the planted communities
with and without cores, reported."""
import math

import numpy as np
import pytest
import torch

import synth
from search_compare import compare_with
from oracle import cores, eigencount, kmeans, laplacian, metrics
from oracle import csc as ocsc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_1602_02018_amd import api as a

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return a


def test_cores_end_to_end_match_oracle(api):
    """Community cores step by step against the oracle, then end to end: the
    dichotomy; each of the T runs' features and k-means partitions of the
    sampled nodes; the core grouping (integer work, bit-exact given the same
    run labels); the interpolation from the cores; the final labels."""
    gr = synth.sbm_config(1000, 10, seed=0)
    k, p, seed, T, reps = 10, 50, 0, 3, 5
    d = int(math.ceil(4 * math.log(gr.n)))
    g = api.Graph(gr.row_ptr, gr.col)
    A, _ = laplacian.normalized_adjacency(gr.row_ptr, gr.col)
    labels, lam, omega, cl = cores.run(gr.row_ptr, gr.col, k, d, seed, T=T, replicates=reps)
    res = api.run(g, k, d, seed, cores=T, replicates=reps)
    if not compare_with(res.bisection.trace, res.lam, res.bisection.steps,
                        eigencount.dichotomy(A, k, p, api.count_signals(gr.n), seed), k):
        pytest.skip("a near-tie count parted the two searches")
    assert np.array_equal(res.omega.cpu().numpy(), omega)
    om_t = torch.as_tensor(omega, device="cuda")
    runs_gpu, runs_ref = [], []
    for t in range(T):
        st = cores.run_seed(seed, t)
        Fr = ocsc.features(A, lam, p, d, st)[omega]
        F = api.filter(g, lam, p, d, st, rows=om_t, normalize=True)
        assert np.linalg.norm(F.cpu().numpy() - Fr) <= 1e-4 * np.linalg.norm(Fr)
        lg, _ = api.kmeans_reduced_device(F.contiguous(), k, seed, replicates=reps)
        lr = kmeans.kmeans(Fr, k, seed, reps)[0]
        assert metrics.adjusted_rand_index(lg, lr) >= 0.99, t
        runs_gpu.append(lg)
        runs_ref.append(lr)
    assert np.array_equal(api.community_cores(np.stack(runs_ref), k), cl)
    keep = cl >= 0
    it = api.interpolate(g, lam, p, 1e-3, omega[keep], cl[keep], k)
    assert metrics.adjusted_rand_index(it.labels.cpu().numpy(), labels) >= 0.99
    same_runs = all(metrics.adjusted_rand_index(a, b) == 1.0 for a, b in zip(runs_gpu, runs_ref))
    ari = metrics.adjusted_rand_index(res.labels.cpu().numpy(), labels)
    print(f"end to end: runs partitioned alike {same_runs}, ARI vs oracle {ari:.4f}")
    if same_runs:  # the same partitions give the same cores, whatever the label numbers
        assert ari >= 0.99
    assert metrics.adjusted_rand_index(res.labels.cpu().numpy(), gr.truth) > 0.9


def test_cores_on_a_harder_sbm(api):
    gr = synth.sbm_config(1000, 20, seed=3, eps_factor=0.5)
    d = int(math.ceil(4 * math.log(gr.n)))
    g = api.Graph(gr.row_ptr, gr.col)
    plain, with_cores = [], []
    for seed in range(4):
        a = api.run(g, 20, d, seed, replicates=5)
        b = api.run(g, 20, d, seed, cores=3, replicates=5)
        plain.append(metrics.adjusted_rand_index(a.labels.cpu().numpy(), gr.truth))
        with_cores.append(metrics.adjusted_rand_index(b.labels.cpu().numpy(), gr.truth))
    print("ARI vs truth, plain:", np.round(plain, 4), "cores T=3:", np.round(with_cores, 4))
    assert np.mean(with_cores) >= np.mean(plain) - 0.05
