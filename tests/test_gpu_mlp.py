"""GPU parity of the bracket network's kernels against the float64 oracle, and
of the learned dichotomy's batched form against its single-graph form."""
import math

import numpy as np
import pytest
import torch

import synth
from paper_1602_02018_amd import _lib
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_1602_02018_amd import api as a

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return a


def _theta(seed=0, scale=0.2):
    return np.random.default_rng(seed).normal(scale=scale, size=omlp.N_PARAMS).astype(np.float32)


@pytest.mark.parametrize("B", [1, 37, 300])
def test_forward_matches_oracle(api, B):
    th = _theta(B)
    X = np.random.default_rng(B + 1).normal(size=(B, 52)).astype(np.float32)
    Y = api.mlp_forward(torch.tensor(th, device="cuda"), torch.tensor(X, device="cuda")).cpu().numpy()
    ref, _ = omlp.forward(th.astype(np.float64), X.astype(np.float64))
    np.testing.assert_allclose(Y, ref, rtol=1e-5, atol=1e-5 * np.abs(ref).max())


@pytest.mark.parametrize("B", [5, 256, 2000])
def test_loss_and_gradient_match_oracle(api, B):
    th = _theta(7)
    rng = np.random.default_rng(B)
    X = rng.normal(size=(B, 52)).astype(np.float32)
    t = rng.uniform(0.1, 0.9, size=B).astype(np.float32)
    loss, g = api.mlp_loss_grad(torch.tensor(th, device="cuda"), torch.tensor(X, device="cuda"),
                                torch.tensor(t, device="cuda"))
    Lref, gref = omlp.loss_and_grad(th.astype(np.float64), X.astype(np.float64), t.astype(np.float64))
    assert abs(loss - Lref) <= 1e-5 * (1 + abs(Lref))
    g = g.cpu().numpy()
    # per parameter block, relative to the block's largest gradient
    off = 0
    for shape in omlp.SHAPES:
        n = int(np.prod(shape))
        gb, rb = g[off:off + n], gref[off:off + n]
        assert np.max(np.abs(gb - rb)) <= 2e-4 * np.max(np.abs(rb)) + 1e-9, shape
        off += n


def test_adam_matches_oracle(api):
    th = _theta(3)
    rng = np.random.default_rng(4)
    X = rng.normal(size=(64, 52)).astype(np.float32)
    t = rng.uniform(0.1, 0.9, size=64).astype(np.float32)
    p = torch.tensor(th, device="cuda")
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    Xd, td = torch.tensor(X, device="cuda"), torch.tensor(t, device="cuda")
    th64, m64, v64 = th.astype(np.float64), np.zeros(omlp.N_PARAMS), np.zeros(omlp.N_PARAMS)
    for step in range(1, 4):
        _, g = api.mlp_loss_grad(p, Xd, td)
        api.mlp_adam_step(p, g, m, v, step, 1e-3)
        # the oracle steps with the GPU's gradient, so only Adam's arithmetic is compared
        th64, m64, v64 = omlp.adam_step(th64, g.cpu().numpy().astype(np.float64), m64, v64, step, 1e-3)
        np.testing.assert_allclose(p.cpu().numpy(), th64, rtol=0, atol=2e-6)


def test_training_reduces_the_loss(api):
    from paper_1602_02018_amd import learned

    rng = np.random.default_rng(0)
    X = rng.normal(size=(500, 52)).astype(np.float32)
    y = (0.4 + 0.1 * np.tanh(X[:, 0])).astype(np.float32)
    params, hist = learned.train(X, y, steps=400)
    assert hist[-1][1] < 0.5 * hist[0][1]


def test_learned_batched_matches_single(api):
    from paper_1602_02018_amd import learned

    gs = [synth.sbm_config(N, k, seed=i) for i, (N, k) in enumerate(((2000, 10), (5000, 25), (3000, 12)))]
    G = [api.Graph(g.row_ptr, g.col) for g in gs]
    params = torch.tensor(learned.init_params(1), device="cuda")
    ks = [g.k for g in gs]
    ncs = [api.count_signals(g.n) for g in gs]
    for group in (1, 4):  # tests per eigencount pass, the same in both forms
        api.set_tuning(_lib.TUNE_COUNT_GROUP, group)
        api.set_tuning(_lib.TUNE_BATCH_COUNT_GROUP, group)
        try:
            res = api.estimate_lambda_k_batched(G, ks, 50, ncs, [5, 6, 7], mlp_params=params)
            refs = [(api.estimate_lambda_k_learned(g, ks[i], 50, ncs[i], 5 + i, params),
                     api.estimate_lambda_k(g, ks[i], 50, ncs[i], 5 + i)) for i, g in enumerate(G)]
        finally:
            api.set_tuning(_lib.TUNE_COUNT_GROUP, 4)
            api.set_tuning(_lib.TUNE_BATCH_COUNT_GROUP, 1)
        _check_learned_batched(res, refs, ks)


def _check_learned_batched(res, refs, ks):
    for i, (ref, plain) in enumerate(refs):
        assert (res[i].lam, res[i].steps, res[i].status) == (ref.lam, ref.steps, ref.status)
        assert [tuple(t) for t in res[i].trace] == [tuple(t) for t in ref.trace]
        # the first pass is the plain dichotomy's first test
        assert ref.trace[0] == plain.trace[0]
        assert abs(round(ref.trace[-1][1]) - ks[i]) == 0 or ref.status != 0
