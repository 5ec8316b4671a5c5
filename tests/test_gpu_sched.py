"""Row schedule of the step kernels (a memory-access order, not part of the
method): rows in chunks of 4096, each chunk by decreasing degree.

* csc_row_schedule gives exactly the stable sort of each chunk by degree and
  the exact degree skew of the natural order (integer sums); the binding
  attaches the schedule to skewed graphs only;
* every step result is unchanged by the walk order: each row still sums its
  neighbours in CSR order, so filtered blocks and features are bit for bit
  the same with the schedule off, on for panels of exactly 8 rows per wave and on for every
  multi-row panel; eigencount moments differ only by the grouping of their
  float64 partial sums;
* on a skewed-degree graph (Chung-Lu) the same holds, and the batched calls
  still match the single ones.
"""
import numpy as np
import pytest
import torch

import synth
from paper_1602_02018_amd import _lib

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_1602_02018_amd import api as a

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    yield a
    a.set_tuning(_lib.TUNE_ROW_SCHED, 1)
    a.set_panel_width(0)


@pytest.fixture(scope="module")
def skewed():
    return synth.chung_lu_blocks(20000, 20, seed=3)


def _ref_schedule(row_ptr):
    deg = np.diff(np.asarray(row_ptr, dtype=np.int64))
    n = deg.size
    out = []
    for b in range(0, n, 4096):
        idx = np.arange(b, min(n, b + 4096))
        out.append(idx[np.lexsort((idx, -deg[idx]))])
    return np.concatenate(out)


def _ref_skew(row_ptr):
    deg = np.diff(np.asarray(row_ptr, dtype=np.int64))
    pad = (-deg.size) % 8
    grp = np.concatenate([deg, np.zeros(pad, np.int64)]).reshape(-1, 8)
    return 8.0 * grp.max(axis=1).sum() / deg.sum()


@pytest.mark.parametrize("which", ["sbm", "skewed"])
def test_schedule_is_the_chunked_degree_sort(api, which, skewed):
    gr = synth.sbm_config(9000, 10, seed=1) if which == "sbm" else skewed
    g = api.Graph(gr.row_ptr, gr.col)
    got = g.sched.cpu().numpy()
    assert np.array_equal(got, _ref_schedule(gr.row_ptr))
    assert np.array_equal(np.sort(got), np.arange(gr.n))
    assert g.skew == pytest.approx(_ref_skew(gr.row_ptr), rel=1e-12)
    attached = g.c.sched is not None and g.c.sched != 0
    assert attached == (which == "skewed"), g.skew


@pytest.mark.parametrize("d,pw", [(28, 32), (47, 48), (56, 64), (13, 16)])
def test_features_identical_under_every_walk(api, skewed, d, pw):
    g = api.Graph(skewed.row_ptr, skewed.col)
    g.use_schedule(True)
    api.set_panel_width(pw)
    try:
        outs = []
        for mode in (0, 1, 2):
            api.set_tuning(_lib.TUNE_ROW_SCHED, mode)
            outs.append(api.filter(g, 0.3, 50, d, 5, rows=None, normalize=False))
            outs.append(api.filter(g, 0.3, 50, d, 5, rows=api.sample(g.n, 200, 1)))
        assert torch.equal(outs[0], outs[2]) and torch.equal(outs[0], outs[4])
        assert torch.equal(outs[1], outs[3]) and torch.equal(outs[1], outs[5])
    finally:
        api.set_tuning(_lib.TUNE_ROW_SCHED, 1)
        api.set_panel_width(0)


def test_moments_differ_only_by_float64_grouping(api, skewed):
    g = api.Graph(skewed.row_ptr, skewed.col)
    g.use_schedule(True)
    n_c = api.count_signals(g.n)
    try:
        api.set_tuning(_lib.TUNE_ROW_SCHED, 0)
        c0, m0 = api.eigencount(g, 0.4, 50, n_c, 2, 3)
        api.set_tuning(_lib.TUNE_ROW_SCHED, 2)
        c2, m2 = api.eigencount(g, 0.4, 50, n_c, 2, 3)
    finally:
        api.set_tuning(_lib.TUNE_ROW_SCHED, 1)
    assert np.max(np.abs(m2 - m0)) <= 1e-12 * abs(m0[0])
    assert abs(c2 - c0) <= 1e-9 * (1 + abs(c0))


def test_batched_filter_follows_the_same_walk(api, skewed):
    graphs = [skewed, synth.chung_lu_blocks(7000, 10, seed=4)]
    G = [api.Graph(x.row_ptr, x.col) for x in graphs]
    for g in G:
        g.use_schedule(True)
    rows = [None, None]
    Ys = api.filter_batched(G, [0.3, 0.45], 50, [28, 28], [1, 2], rows)
    for i, g in enumerate(G):
        ref = api.filter(g, [0.3, 0.45][i], 50, 28, [1, 2][i], rows=None)
        assert torch.equal(Ys[i], ref)


def test_schedule_argument_errors(api):
    lib = _lib.lib()
    assert lib.csc_row_schedule(0, None, None, None, None, 0, None) == _lib.CSC_E_INVALID_ARG
    assert api.get_tuning(_lib.TUNE_ROW_SCHED) == 1
    assert lib.csc_set_tuning(_lib.TUNE_ROW_SCHED, 3) == _lib.CSC_E_INVALID_ARG
