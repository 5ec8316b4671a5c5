"""Pins of the oracle's lambda_k searches (Sec. 4.3) beyond the plain
dichotomy from [0, 2]: the search inside a caller's bracket (with its restart
when the bracket misses lambda_k) and the search from the network's bracket.

Every count is checked against the Hutchinson count written with the dense
eigendecomposition, sum_l (U^T R)_l^2 h~_lambda(lambda_l); every estimate
against the spectrum (lambda_k <= estimate <= lambda_{k+1}); the network's
bracket against the root of that dense count curve, found by a library root
finder.  The networks used here have W3 = 0, so their two outputs are exactly
the biases b3 and the bracket is planted where a test needs it.
"""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

import synth
from oracle import eigencount, jackson, laplacian, mlp, philox


@pytest.fixture(scope="module")
def sbm():
    g = synth.sbm_config(1000, 10, seed=0)
    A, _ = laplacian.normalized_adjacency(g.row_ptr, g.col)
    ev, U = np.linalg.eigh(laplacian.laplacian_dense(g.row_ptr, g.col))
    return g, A, ev, U


def dense_count(U, ev, lam, p, R):
    """Hutchinson count from the spectrum: sum_l ||(U^T R)_l||^2 h~_lam(lambda_l)."""
    h = jackson.evaluate(jackson.lowpass_coeffs(lam, p), ev)
    return float(np.sum((U.T @ R) ** 2 * h[:, None]))


def check_trace(trace, U, ev, p, n_c, seed, first_t=1):
    for t, (lt, ct) in enumerate(trace, start=first_t):
        R = philox.gaussian_block(seed, U.shape[0], n_c, t, philox.COUNT)
        ref = dense_count(U, ev, lt, p, R)
        assert abs(ct - ref) <= 1e-8 * max(1.0, abs(ref)), (t, lt, ct, ref)


def planted(y_lo, y_hi):
    theta = np.zeros(mlp.N_PARAMS)
    theta[-2:] = (y_lo, y_hi)  # b3; W3 = 0, so the outputs are exactly b3
    return theta.astype(np.float32)


K, P = 10, 50


def test_caller_bracket_holding_lambda_k(sbm):
    g, A, ev, U = sbm
    nc = eigencount.count_signals(g.n)
    r = eigencount.dichotomy(A, K, P, nc, 0, bracket=(0.25, 0.75))
    assert r.found and not r.missed
    assert ev[K - 1] <= r.lam <= ev[K]
    lo, hi = 0.25, 0.75
    for lt, ct in r.trace:
        assert lt == 0.5 * (lo + hi)
        lo, hi = (lt, hi) if ct < K else (lo, lt)
    check_trace(r.trace, U, ev, P, nc, 0)


@pytest.mark.parametrize("bracket,side", [((1.5, 2.0), "above"), ((0.0, 0.1), "below")])
def test_caller_bracket_missing_lambda_k_restarts_from_0_2(sbm, bracket, side):
    g, A, ev, U = sbm
    nc = eigencount.count_signals(g.n)
    r = eigencount.dichotomy(A, K, P, nc, 0, max_steps=12, bracket=bracket)
    assert r.missed and r.found
    first = r.trace[:12]
    assert all((c > K) if side == "above" else (c < K) for _, c in first)
    assert r.trace[12][0] == 1.0  # the restart tests the midpoint of [0, 2] next
    assert ev[K - 1] <= r.lam <= ev[K]
    check_trace(r.trace, U, ev, P, nc, 0)  # sub-streams continue across the restart
    # the compatibility wrapper reports the same search
    lam, steps, trace, ok = eigencount.estimate_lambda_k(A, K, P, nc, 0, 12, bracket)
    assert (lam, steps, ok) == (r.lam, r.steps, r.found) and trace == r.trace


def test_exhausted_caller_bracket_returns_upper_end(sbm):
    g, A, ev, U = sbm
    nc = eigencount.count_signals(g.n)
    r = eigencount.dichotomy(A, K, P, nc, 0, max_steps=1, bracket=(1.5, 2.0))
    assert r.missed and not r.found and r.steps == 2 and r.lam == 1.0


def _root(U, ev, R, k):
    return brentq(lambda lam: dense_count(U, ev, lam, P, R) - k, 0.0, 2.0, xtol=1e-14)


def test_count_root_is_the_root_of_the_dense_count_curve(sbm):
    g, A, ev, U = sbm
    nc = eigencount.count_signals(g.n)
    R = philox.gaussian_block(0, g.n, nc, 1, philox.COUNT)
    from oracle import cheb

    lam0, s = mlp.count_root(cheb.moments(A, R, P), P, K, nc)
    assert abs(lam0 - _root(U, ev, R, K)) <= 1e-9
    h = 1e-3
    slope = (dense_count(U, ev, lam0 + h, P, R) - dense_count(U, ev, lam0 - h, P, R)) / (2 * h)
    assert abs(s - math.sqrt(2 * K / nc) / slope) <= 1e-6 * s


# the first pass's count curve has its root lambda_0 = 0.345 with s = 0.0128
# on this graph; lambda_10 = 0.35 and lambda_11 = 0.54, and the later tests'
# counts round to k = 10 around 0.42-0.47
@pytest.mark.parametrize("ys,missed", [((-10.0, 15.0), False), ((12.0, 20.0), True),
                                       ((-20.0, -8.0), True), ((0.0, 0.0), None)])
def test_learned_search_from_planted_brackets(sbm, ys, missed):
    g, A, ev, U = sbm
    nc = eigencount.count_signals(g.n)
    R1 = philox.gaussian_block(0, g.n, nc, 1, philox.COUNT)
    c1 = dense_count(U, ev, 1.0, P, R1)
    assert c1 > K  # lambda_k lies in the lower half
    r = eigencount.estimate_lambda_k_learned(A, K, P, nc, 0, planted(*ys))
    from oracle import cheb

    lam0 = _root(U, ev, R1, K)
    _, s = mlp.count_root(cheb.moments(A, R1, P), P, K, nc)
    lo, hi = max(lam0 + s * ys[0], 0.0), min(lam0 + s * ys[1], 1.0)  # cut to the lower half
    if not hi - lo >= 1.0 / 1024:
        w = max(s, 1.0 / 1024)
        lo, hi = max(0.0, lam0 - w), min(1.0, lam0 + w)
    lo0, hi0 = r.bracket
    assert abs(lo0 - lo) <= 1e-8 and abs(hi0 - hi) <= 1e-8, (r.bracket, lo, hi)
    assert r.found and ev[K - 1] <= r.lam <= ev[K]
    if missed is not None:
        assert r.missed == missed
    assert r.trace[0][0] == 1.0
    check_trace(r.trace, U, ev, P, nc, 0)
    # tests 2.. bisect inside the bracket until the reopening
    lo, hi = lo0, hi0
    for j, (lt, ct) in enumerate(r.trace[1:], start=1):
        assert abs(lt - 0.5 * (lo + hi)) <= 1e-15
        lo, hi = (lt, hi) if ct < K else (lo, lt)
        if r.missed and j == 4:
            assert all(c > K for _, c in r.trace[1:5]) or all(c < K for _, c in r.trace[1:5])
            lo, hi = (0.0, lo0) if r.trace[4][1] > K else (hi0, 1.0)


def test_learned_search_stops_at_the_first_test(sbm):
    g, A, ev, U = sbm
    nc = eigencount.count_signals(g.n)
    R1 = philox.gaussian_block(0, g.n, nc, 1, philox.COUNT)
    k = int(math.floor(dense_count(U, ev, 1.0, P, R1) + 0.5))
    r = eigencount.estimate_lambda_k_learned(A, k, P, nc, 0, planted(-1.0, 1.0))
    assert r.found and r.lam == 1.0 and r.steps == 1 and r.bracket == (1.0, 1.0)


def test_learned_search_with_a_random_network_still_brackets_lambda_k(sbm):
    g, A, ev, U = sbm
    nc = eigencount.count_signals(g.n)
    theta = (np.random.default_rng(5).normal(size=mlp.N_PARAMS) * 0.2).astype(np.float32)
    r = eigencount.estimate_lambda_k_learned(A, K, P, nc, 0, theta)
    assert r.found and ev[K - 1] <= r.lam <= ev[K]
    assert r.steps <= 30
    check_trace(r.trace, U, ev, P, nc, 0)
