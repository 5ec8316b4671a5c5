"""The library's lambda_k searches against the oracle's (Sec. 4.3): the
dichotomy inside a caller's bracket with its restart, and the learned search
(single and batched) with networks whose outputs are planted (W3 = 0, biases
chosen) or random.  The weights are seeded inputs, not the trained file.

Rule (as for the plain dichotomy): tested points agree (to 2e-5 where the
network's bracket enters: the GPU evaluates it from float32 moments and a
float32 network, the oracle in float64), counts agree to 1e-3 (1 + |count|),
and every decision agrees unless the oracle's count lies within twice that
margin of k - 1/2, k + 1/2 or k; after such a near-tie the two searches may
part, and the estimates then lie within the width of the interval at that
point.
"""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import eigencount, laplacian, mlp

pytestmark = pytest.mark.gpu

K, P = 10, 50


@pytest.fixture(scope="module")
def api():
    from paper_1602_02018_amd import api as a

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return a


@pytest.fixture(scope="module")
def graphs():
    out = []
    for n, k, seed in ((1000, 10, 0), (3000, 20, 4), (1500, 12, 7)):
        gr = synth.sbm_config(n, k, seed=seed)
        A, _ = laplacian.normalized_adjacency(gr.row_ptr, gr.col)
        out.append((gr, A, k, seed))
    return out


def compare(trace, lam, steps, ref, k, mid_tol=2e-5, tol=1e-3):
    """Returns True when every decision agreed (then the estimates agree)."""
    for s, ((lg, cg), (lo_, co)) in enumerate(zip(trace, ref.trace)):
        assert abs(lg - lo_) <= mid_tol, (s, lg, lo_)
        assert abs(cg - co) <= tol * (1 + abs(co)), (s, cg, co)
        dg = (math.floor(cg + 0.5) == k, cg < k)
        do = (math.floor(co + 0.5) == k, co < k)
        if dg != do:
            near = min(abs(co - (k - 0.5)), abs(co - (k + 0.5)), abs(co - k))
            assert near <= 2 * tol * (1 + abs(co)), (s, cg, co)
            if not ref.missed:  # both searches continue inside the interval of this test
                a, b = ref.intervals[s]
                assert abs(lam - ref.lam) <= (b - a) + mid_tol
            return False
    assert steps == ref.steps
    assert abs(lam - ref.lam) <= mid_tol
    return True


def planted(y_lo, y_hi):
    theta = np.zeros(mlp.N_PARAMS, dtype=np.float32)
    theta[-2:] = (y_lo, y_hi)
    return theta


def random_net(seed, scale=0.2):
    return (np.random.default_rng(seed).normal(size=mlp.N_PARAMS) * scale).astype(np.float32)


NETS = {
    "holding": planted(-10.0, 15.0),
    "above": planted(12.0, 20.0),
    "below": planted(-20.0, -8.0),
    "narrow": planted(0.0, 0.0),
    "random5": random_net(5),
    "random9": random_net(9, 0.5),
}


@pytest.mark.parametrize("net", list(NETS))
def test_learned_search_matches_oracle(api, graphs, net):
    gr, A, k, seed = graphs[0]
    g = api.Graph(gr.row_ptr, gr.col)
    nc = eigencount.count_signals(gr.n)
    theta = NETS[net]
    res = api.estimate_lambda_k_learned(g, k, P, nc, seed, torch.as_tensor(theta, device="cuda"))
    ref = eigencount.estimate_lambda_k_learned(A, k, P, nc, seed, theta)
    assert abs(res.bracket[0] - ref.bracket[0]) <= 2e-5 and abs(res.bracket[1] - ref.bracket[1]) <= 2e-5
    if compare(res.trace, res.lam, res.steps, ref, k):
        from paper_1602_02018_amd import _lib

        assert (res.status == _lib.CSC_W_BRACKET_MISS) == ref.missed
        if net in ("above", "below"):
            assert ref.missed


@pytest.mark.parametrize("net", ["holding", "above", "random5"])
def test_batched_learned_search_matches_oracle(api, graphs, net):
    gs = [api.Graph(gr.row_ptr, gr.col) for gr, _, _, _ in graphs]
    ks = [k for _, _, k, _ in graphs]
    seeds = [s for _, _, _, s in graphs]
    ncs = [eigencount.count_signals(gr.n) for gr, _, _, _ in graphs]
    theta = NETS[net]
    out = api.estimate_lambda_k_batched(gs, ks, P, ncs, seeds,
                                        mlp_params=torch.as_tensor(theta, device="cuda"))
    for (gr, A, k, seed), nc, res in zip(graphs, ncs, out):
        ref = eigencount.estimate_lambda_k_learned(A, k, P, nc, seed, theta)
        compare(res.trace, res.lam, res.steps, ref, k)


@pytest.mark.parametrize("bracket", [(1.5, 2.0), (0.0, 0.1), (0.25, 0.75)])
def test_caller_bracket_search_matches_oracle(api, graphs, bracket):
    gr, A, k, seed = graphs[0]
    g = api.Graph(gr.row_ptr, gr.col)
    nc = eigencount.count_signals(gr.n)
    res = api.estimate_lambda_k(g, k, P, nc, seed, max_steps=12, bracket=bracket)
    ref = eigencount.dichotomy(A, k, P, nc, seed, max_steps=12, bracket=bracket)
    if compare(res.trace, res.lam, res.steps, ref, k, mid_tol=0.0):
        from paper_1602_02018_amd import _lib

        assert (res.status == _lib.CSC_W_BRACKET_MISS) == ref.missed


def test_caller_bracket_trace_buffer_holds_both_searches(api, graphs):
    """The header sizes trace_out at 4 max_steps doubles: a missed bracket runs
    up to 2 max_steps tests.  A sentinel after that size stays untouched."""
    import ctypes as C

    from paper_1602_02018_amd import _lib

    gr, A, k, seed = graphs[0]
    g = api.Graph(gr.row_ptr, gr.col)
    nc = eigencount.count_signals(gr.n)
    ms = 3
    buf = np.full(4 * ms + 8, -7.0)
    lam, steps = C.c_double(), C.c_int32()
    br = np.array([1.5, 2.0])
    ws = torch.empty(api.lib().csc_estimate_workspace_bytes(gr.n, nc, P), dtype=torch.uint8, device="cuda")
    st = api.lib().csc_estimate_lambda_k(g.ref, k, P, nc, seed, ms, br.ctypes.data_as(_lib.pd),
                                         C.byref(lam), C.byref(steps), buf.ctypes.data_as(_lib.pd),
                                         None, C.c_void_p(ws.data_ptr()), ws.numel(),
                                         C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == _lib.CSC_W_BRACKET_MISS and ms < steps.value <= 2 * ms
    assert np.all(buf[4 * ms:] == -7.0)
    assert np.all(buf[: 2 * steps.value] != -7.0)
