"""Grouped eigencount passes of the dichotomies: several consecutive tests'
signals filtered side by side in one wider pass.  Each test still draws the
signals of its own sub-stream and keeps its own moments, so the tested
points, the counts (up to the grouping of float64 partial sums) and the
result are those of one pass per test, for every group size, with and
without a caller bracket, in the plain and the learned dichotomy."""
import numpy as np
import pytest
import torch

import synth
from oracle import eigencount, philox
from oracle import laplacian
from paper_1602_02018_amd import _lib

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_1602_02018_amd import api as a

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    yield a
    a.set_tuning(_lib.TUNE_COUNT_GROUP, 4)


def _runs(api, fn):
    out = {}
    try:
        for gsize in (1, 2, 3, 4):
            api.set_tuning(_lib.TUNE_COUNT_GROUP, gsize)
            out[gsize] = fn()
    finally:
        api.set_tuning(_lib.TUNE_COUNT_GROUP, 4)
    return out


def _same_search(a, b, mid_rtol=0.0):
    """Same decisions; tested points equal (the learned bracket comes from a
    network evaluated on the first test's moments, whose float64 sums are
    grouped differently, so there they agree to mid_rtol)."""
    assert a.steps == b.steps and a.status == b.status
    assert abs(a.lam - b.lam) <= mid_rtol * abs(b.lam)
    ta, tb = np.asarray(a.trace), np.asarray(b.trace)
    assert np.allclose(ta[:, 0], tb[:, 0], rtol=mid_rtol, atol=0.0)
    assert np.allclose(ta[:, 1], tb[:, 1], rtol=1e-10, atol=1e-9)


@pytest.mark.parametrize("n,k,bracket", [(1000, 10, None), (3000, 12, None), (1000, 10, (1.5, 2.0)),
                                         (1000, 10, (0.25, 0.75))])
def test_grouped_dichotomy_is_the_plain_one(api, n, k, bracket):
    gr = synth.sbm_config(n, k, seed=2)
    g = api.Graph(gr.row_ptr, gr.col)
    n_c = api.count_signals(gr.n)  # 14 or 17: not a multiple of 4 for n = 3000
    res = _runs(api, lambda: api.estimate_lambda_k(g, k, 50, n_c, 3, max_steps=12, bracket=bracket))
    for gsize in (2, 3, 4):
        _same_search(res[1], res[gsize])
    # and each tested point's count is the oracle's on that test's own signals
    A, _ = laplacian.normalized_adjacency(gr.row_ptr, gr.col)
    for t in (1, len(res[4].trace)):
        mid, cnt = res[4].trace[t - 1]
        R = philox.gaussian_block(3, gr.n, n_c, t, philox.COUNT)
        ref = eigencount.eigencount(A, mid, 50, R)
        assert abs(cnt - ref) <= 1e-3 * (1 + abs(ref))


def test_grouped_moments_of_the_first_test(api):
    gr = synth.sbm_config(2000, 10, seed=5)
    g = api.Graph(gr.row_ptr, gr.col)
    res = _runs(api, lambda: api.estimate_lambda_k(g, 10, 60, 15, 1, max_steps=6))
    m1 = np.asarray(res[1].moments)
    for gsize in (2, 3, 4):
        assert np.allclose(np.asarray(res[gsize].moments), m1, rtol=1e-12, atol=1e-12 * abs(m1[0]))
    _, mref = api.eigencount(g, 0.5, 60, 15, 1, 1)
    assert np.allclose(m1, mref, rtol=1e-12, atol=1e-12 * abs(mref[0]))


def test_grouped_learned_dichotomy(api):
    from paper_1602_02018_amd import learned

    mlp = learned.load_params(torch.device("cuda"))
    gr = synth.sbm_config(5000, 20, seed=7)
    g = api.Graph(gr.row_ptr, gr.col)
    n_c = api.count_signals(gr.n)
    res = _runs(api, lambda: api.estimate_lambda_k_learned(g, 20, 50, n_c, 4, mlp))
    for gsize in (2, 3, 4):
        _same_search(res[1], res[gsize], mid_rtol=1e-9)


def test_group_knob_range(api):
    lib = _lib.lib()
    assert api.get_tuning(_lib.TUNE_COUNT_GROUP) == 4
    assert lib.csc_set_tuning(_lib.TUNE_COUNT_GROUP, 0) == _lib.CSC_E_INVALID_ARG
    assert lib.csc_set_tuning(_lib.TUNE_COUNT_GROUP, 5) == _lib.CSC_E_INVALID_ARG
    assert api.get_tuning(_lib.TUNE_BATCH_COUNT_GROUP) == 1
    assert lib.csc_set_tuning(_lib.TUNE_BATCH_COUNT_GROUP, 0) == _lib.CSC_E_INVALID_ARG
    assert lib.csc_set_tuning(_lib.TUNE_BATCH_COUNT_GROUP, 5) == _lib.CSC_E_INVALID_ARG
    assert api.get_tuning(_lib.TUNE_BATCH_COUNT_GROUP) == 1
