"""One-pass KPM dichotomy on the GPU against the float64 oracle: the same
moments (within the moment tolerance), the same tested points while the
counts stay clear of the decision boundaries, lambda within one bracket
width; and its cost: one pass instead of one per tested point."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import eigencount, laplacian, metrics

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_1602_02018_amd import api as a

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return a


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_kpm_dichotomy_matches_oracle(api, seed):
    gr = synth.sbm_config(1000, 10, seed=seed)
    A, _ = laplacian.normalized_adjacency(gr.row_ptr, gr.col)
    g = api.Graph(gr.row_ptr, gr.col)
    n_c = api.count_signals(gr.n)
    res = api.estimate_lambda_k_kpm(g, 10, 50, n_c, seed)
    lam, steps, trace, conv, mu = eigencount.estimate_lambda_k_kpm(A, 10, 50, n_c, seed)
    assert np.max(np.abs(res.moments - mu)) <= 1e-5 * mu[0]
    # identical decisions unless an oracle count sits within the count tolerance of a boundary
    for (lg, cg), (lo, co) in zip(res.trace, trace):
        if lg != lo:
            break
        assert abs(cg - co) <= 1e-3 * (1 + abs(co))
    assert abs(res.lam - lam) <= 2.0 / 2 ** min(res.steps, steps)


def test_kpm_first_count_is_the_plain_first_count(api):
    gr = synth.sbm_config(1000, 10, seed=0)
    g = api.Graph(gr.row_ptr, gr.col)
    n_c = api.count_signals(gr.n)
    kpm = api.estimate_lambda_k_kpm(g, 10, 50, n_c, 0)
    plain = api.estimate_lambda_k(g, 10, 50, n_c, 0)
    assert kpm.trace[0][0] == plain.trace[0][0] == 1.0
    assert abs(kpm.trace[0][1] - plain.trace[0][1]) <= 1e-9 * abs(plain.trace[0][1])


def test_kpm_end_to_end_and_passes(api):
    gr = synth.sbm_config(1000, 10, seed=0)
    g = api.Graph(gr.row_ptr, gr.col)
    d = int(math.ceil(4 * math.log(gr.n)))
    a = api.run(g, 10, d, 0, lambda_method="kpm")
    b = api.run(g, 10, d, 0)
    assert metrics.adjusted_rand_index(a.labels.cpu().numpy(), gr.truth) > 0.9
    assert metrics.adjusted_rand_index(a.labels.cpu().numpy(), b.labels.cpu().numpy()) > 0.9
