"""Batched form: G graphs of uneven size in one launch per step, repeated
passes replayed from captured HIP graphs.  Every output must be bit-identical
to the single-graph call with the same arguments, with graphs on and off, on
several calls in a row."""
import contextlib
import math

import numpy as np
import pytest
import torch

import synth
from oracle import metrics

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_1602_02018_amd import api as a

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    yield a


@pytest.fixture(scope="module")
def batch():
    specs = [(700, 5, 12.0), (1000, 10, 16.0), (1500, 8, 20.0), (333, 3, 10.0), (2500, 20, 16.0),
             (4000, 12, 24.0)]
    gs = [synth.sbm(N, k, s, 0.25 * synth.eps_critical(s, k), seed=i, name=f"b{i}")
          for i, (N, k, s) in enumerate(specs)]
    gs.append(synth.chung_lu_blocks(1037, 7, mean_deg=6.0, max_deg=80.0, seed=2))
    return gs


def _graphs(api, batch):
    return [api.Graph(g.row_ptr, g.col) for g in batch]


@contextlib.contextmanager
def _count_group(api, size):
    """Both dichotomies run `size` tests per eigencount pass."""
    from paper_1602_02018_amd import _lib

    api.set_tuning(_lib.TUNE_COUNT_GROUP, size)
    api.set_tuning(_lib.TUNE_BATCH_COUNT_GROUP, size)
    try:
        yield
    finally:
        api.set_tuning(_lib.TUNE_COUNT_GROUP, 4)
        api.set_tuning(_lib.TUNE_BATCH_COUNT_GROUP, 1)


def _set_graphs(api, on):
    from paper_1602_02018_amd import _lib

    api.set_tuning(_lib.TUNE_HIP_GRAPHS, 1 if on else 0)


@pytest.mark.parametrize("use_graphs", [1, 0])
@pytest.mark.parametrize("group", [1, 4])
def test_batched_dichotomy_matches_single(api, batch, use_graphs, group):
    _set_graphs(api, use_graphs)
    try:
        G = _graphs(api, batch)
        ks = [g.k for g in batch]
        ncs = [api.count_signals(g.n) for g in batch]
        seeds = list(range(10, 10 + len(batch)))
        for _ in range(2):  # two calls in a row
            with _count_group(api, group):
                res = api.estimate_lambda_k_batched(G, ks, 50, ncs, seeds)
                refs = [api.estimate_lambda_k(g, ks[i], 50, ncs[i], seeds[i])
                        for i, g in enumerate(G)]
            for i, g in enumerate(G):
                ref = refs[i]
                assert res[i].lam == ref.lam and res[i].steps == ref.steps
                assert res[i].status == ref.status
                assert [tuple(t) for t in res[i].trace] == [tuple(t) for t in ref.trace]
                assert np.array_equal(res[i].moments, ref.moments)
    finally:
        _set_graphs(api, 1)


def test_batched_dichotomy_workspace_follows_group_size(api, batch):
    """The workspace is sized for the current tests per pass; a call given the
    size for one test per pass after the knob went up is refused, unlaunched."""
    from paper_1602_02018_amd import _lib

    lib = _lib.lib()
    G = _graphs(api, batch)
    ga = api._graphs(G)
    ns = np.ascontiguousarray([api.count_signals(g.n) for g in batch], dtype=np.int32)
    ks = np.ascontiguousarray([g.k for g in batch], dtype=np.int32)
    sd = np.arange(len(batch), dtype=np.uint64)
    size = {}
    try:
        for gsize in (1, 4):
            api.set_tuning(_lib.TUNE_BATCH_COUNT_GROUP, gsize)
            size[gsize] = lib.csc_estimate_workspace_bytes_batched(
                ga, len(G), ns.ctypes.data_as(_lib.pi), 50)
        assert size[4] > size[1] > 0
        ws = torch.empty(size[1], dtype=torch.uint8, device="cuda")
        Gn = len(G)
        lam, steps, status = np.zeros(Gn), np.zeros(Gn, np.int32), np.zeros(Gn, np.int32)
        rc = lib.csc_estimate_lambda_k_batched(
            ga, Gn, ks.ctypes.data_as(_lib.pi), 50, ns.ctypes.data_as(_lib.pi),
            sd.ctypes.data_as(_lib.pu), 30, None, None, lam.ctypes.data_as(_lib.pd),
            steps.ctypes.data_as(_lib.pi), None, None, status.ctypes.data_as(_lib.pi),
            ws.data_ptr(), ws.numel(), None)
        assert rc == _lib.CSC_E_INVALID_ARG
    finally:
        api.set_tuning(_lib.TUNE_BATCH_COUNT_GROUP, 1)


def _tiny_batch():
    """Degenerate graphs (an isolated node, a 2-path, a 5-cycle, a 13-path)
    beside one ordinary SBM, with their k."""
    def path(N, cyc=False):
        u = np.arange(N if cyc else N - 1)
        return synth.csr_from_edges(N, u, (u + 1) % N)

    tiny = [(synth.csr_from_edges(1, np.zeros(0, np.int64), np.zeros(0, np.int64)), 1),
            (path(2), 2), (path(5, cyc=True), 2), (path(13), 3)]
    sb = synth.sbm(700, 5, 12.0, 0.25 * synth.eps_critical(12.0, 5), seed=9)
    return tiny + [((sb.row_ptr, sb.col), sb.k)]


@pytest.mark.parametrize("group", [1, 4])
def test_batched_dichotomy_tiny_graphs(api, group):
    """Degenerate sizes in a batch: each graph's search equals its single call
    at the same group size, bit for bit."""
    items = _tiny_batch()
    G = [api.Graph(rp, cl) for (rp, cl), _ in items]
    ks = [k for _, k in items]
    ns = [len(rp) - 1 for (rp, _), _ in items]
    ncs = [api.count_signals(n) for n in ns]
    seeds = list(range(20, 20 + len(items)))
    with _count_group(api, group):
        res = api.estimate_lambda_k_batched(G, ks, 50, ncs, seeds)
        refs = [api.estimate_lambda_k(g, ks[i], 50, ncs[i], seeds[i]) for i, g in enumerate(G)]
    for i, ref in enumerate(refs):
        assert (res[i].lam, res[i].steps, res[i].status) == (ref.lam, ref.steps, ref.status)
        assert [tuple(t) for t in res[i].trace] == [tuple(t) for t in ref.trace]
        assert np.array_equal(res[i].moments, ref.moments)


@pytest.mark.parametrize("group", [1, 4])
def test_batched_dichotomy_with_brackets(api, batch, group):
    """Missed brackets restart on [0, 2] (with 6 tests per attempt a restart
    falls inside a group of 4); tested points and counts equal the single
    call's at the same group size."""
    G = _graphs(api, batch)
    ks = [g.k for g in batch]
    ncs = [api.count_signals(g.n) for g in batch]
    seeds = [3] * len(batch)
    brackets = [(1.5, 2.0) if i % 2 else (0.0, 1.0) for i in range(len(batch))]
    with _count_group(api, group):
        res = api.estimate_lambda_k_batched(G, ks, 50, ncs, seeds, max_steps=6, brackets=brackets)
        refs = [api.estimate_lambda_k(g, ks[i], 50, ncs[i], seeds[i], max_steps=6,
                                      bracket=brackets[i]) for i, g in enumerate(G)]
    for i, ref in enumerate(refs):
        assert (res[i].lam, res[i].steps, res[i].status) == (ref.lam, ref.steps, ref.status)
        assert [tuple(t) for t in res[i].trace] == [tuple(t) for t in ref.trace]


def test_batched_features_match_single(api, batch):
    G = _graphs(api, batch)
    lams = [0.3 + 0.05 * i for i in range(len(batch))]
    ds = [int(math.ceil(4 * math.log(g.n))) for g in batch]
    seeds = list(range(len(batch)))
    rows = [api.sample(g.n, min(g.n, 40 + 7 * i), seeds[i]) for i, g in enumerate(batch)]
    Ys = api.filter_batched(G, lams, 50, ds, seeds, rows)
    for i, g in enumerate(G):
        ref = api.filter(g, lams[i], 50, ds[i], seeds[i], rows=rows[i])
        assert torch.equal(Ys[i], ref)


@pytest.mark.parametrize("use_graphs", [1, 0])
@pytest.mark.parametrize("method", [2, 1, 0])
def test_batched_interpolation_matches_single(api, batch, use_graphs, method):
    _set_graphs(api, use_graphs)
    try:
        G = _graphs(api, batch)
        ks = [g.k for g in batch]
        lams = [0.35] * len(batch)
        omegas, labs = [], []
        for i, g in enumerate(batch):
            n = min(g.n, api.default_n(max(ks[i], 2)) + 5)
            omegas.append(api.sample(g.n, n, i))
            labs.append(np.arange(n) % ks[i])
        for _ in range(2):
            res = api.interpolate_batched(G, lams, 50, 1e-3, omegas, labs, ks, method=method)
            for i, g in enumerate(G):
                ref = api.interpolate(g, lams[i], 50, 1e-3, omegas[i], labs[i], ks[i], method=method)
                assert torch.equal(res[i].X, ref.X)
                assert torch.equal(res[i].labels, ref.labels)
                assert np.array_equal(res[i].iters, ref.iters)
                assert np.array_equal(res[i].relres, ref.relres)
                assert res[i].status == ref.status
    finally:
        _set_graphs(api, 1)


@pytest.mark.parametrize("method", [2, 1, 0])
def test_batched_interpolation_max_iter(api, batch, method):
    G = _graphs(api, batch)
    ks = [g.k for g in batch]
    omegas = [api.sample(g.n, min(g.n, 30), i) for i, g in enumerate(batch)]
    labs = [np.arange(30) % k for k in ks]
    res = api.interpolate_batched(G, [0.4] * len(batch), 50, 1e-3, omegas, labs, ks, tol=1e-12,
                                  max_iter=3, method=method)
    for i, g in enumerate(G):
        ref = api.interpolate(g, 0.4, 50, 1e-3, omegas[i], labs[i], ks[i], tol=1e-12, max_iter=3,
                              method=method)
        assert res[i].status == ref.status
        assert torch.equal(res[i].X, ref.X)


def test_batched_kmeans_matches_single(api):
    rng = np.random.default_rng(0)
    Fs = [rng.normal(size=(n, d)).astype(np.float32) for n, d in ((47, 28), (300, 12), (90, 30))]
    ks, seeds = [10, 25, 7], [0, 5, 9]
    labs, inert = api.kmeans_reduced_batched(Fs, ks, seeds)
    for F, k, sd, l, i in zip(Fs, ks, seeds, labs, inert):
        l2, i2 = api.kmeans_reduced(F, k, sd)
        assert np.array_equal(l, l2) and i == i2


def test_run_batched_matches_run(api, batch):
    G = _graphs(api, batch)
    ks = [g.k for g in batch]
    ds = [int(math.ceil(4 * math.log(g.n))) for g in batch]
    seeds = list(range(len(batch)))
    res = api.run_batched(G, ks, ds, seeds, replicates=5)
    for i, g in enumerate(G):
        ref = api.run(g, ks[i], ds[i], seeds[i], replicates=5)
        assert res[i].lam == ref.lam
        assert torch.equal(res[i].labels, ref.labels)
        if batch[i].meta.get("model") == "sbm":
            assert metrics.adjusted_rand_index(res[i].labels.cpu().numpy(), batch[i].truth) > 0.5
