"""Community cores on the GPU against the float64 oracle, and what they change
on a harder SBM (eps = eps_c / 2): recovery against the planted communities
with and without cores, reported."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import cores, metrics

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_1602_02018_amd import api as a

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return a


def test_cores_end_to_end_match_oracle(api):
    gr = synth.sbm_config(1000, 10, seed=0)
    d = int(math.ceil(4 * math.log(gr.n)))
    g = api.Graph(gr.row_ptr, gr.col)
    res = api.run(g, 10, d, 0, cores=3, replicates=5)
    labels, lam, omega, cl = cores.run(gr.row_ptr, gr.col, 10, d, 0, T=3, replicates=5)
    assert abs(res.lam - lam) <= 2.0 / 2 ** res.bisection.steps + 1e-12
    assert metrics.adjusted_rand_index(res.labels.cpu().numpy(), labels) >= 0.9
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
