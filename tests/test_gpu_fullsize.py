"""Parity at full size, in the launch configuration the benchmark times
(built-in panel widths and tuning), on outputs the float64 oracle can compute
one by one (single columns of a filtered block: columns never mix), and via
identities that hold at any size."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import cheb, interp, jackson, laplacian, philox, sampling

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_1602_02018_amd import api as a

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return a


@pytest.fixture(scope="module")
def sbm1e5():
    gr = synth.sbm_config(100000, 100, seed=0)
    A, _ = laplacian.normalized_adjacency(gr.row_ptr, gr.col)
    return gr, A


@pytest.fixture(scope="module")
def chunglu1e6():
    gr = synth.chung_lu_blocks(1000000, 250, seed=0)
    A, _ = laplacian.normalized_adjacency(gr.row_ptr, gr.col)
    return gr, A


def _columns_check(api, g, A, w, p, lam, cols, seed=1):
    R = api.gaussian_block(g.n, w, seed, 0, 2)
    a = jackson.lowpass_coeffs(lam, p)
    Y = api.filter_block(g, a, R)
    Rh = R.cpu().numpy().astype(np.float64)
    Yh = Y.cpu().numpy()
    for c in cols:
        ref = cheb.filter_block(A, Rh[:, c:c + 1], a)[:, 0]
        err = np.linalg.norm(Yh[:, c] - ref) / np.linalg.norm(ref)
        assert err <= 1e-4, (c, err)
    return R, Y, a


def test_sbm_1e5_feature_and_cg_width_columns(api, sbm1e5):
    gr, A = sbm1e5
    g = api.Graph(gr.row_ptr, gr.col)
    _columns_check(api, g, A, 47, 50, 0.3867, (0, 23, 46))
    _columns_check(api, g, A, 100, 50, 0.3867, (0, 57, 99))


def test_sbm_1e5_count_pass_moments(api, sbm1e5):
    gr, A = sbm1e5
    g = api.Graph(gr.row_ptr, gr.col)
    n_c = api.count_signals(gr.n)
    cnt, mom = api.eigencount(g, 0.4, 50, n_c, 0, 1)
    R = philox.gaussian_block(0, gr.n, n_c, 1, philox.COUNT)
    ref = cheb.moments(A, R, 50)
    assert np.max(np.abs(mom - ref)) <= 1e-5 * ref[0]


def test_sbm_1e5_sampling_and_interpolation(api, sbm1e5):
    gr, A = sbm1e5
    g = api.Graph(gr.row_ptr, gr.col)
    k, d, lam = 100, 47, 0.38671875
    n = api.default_n(k)
    omega = api.sample(gr.n, n, 0)
    assert np.array_equal(omega.cpu().numpy(), sampling.sample(gr.n, n, 0))
    F = api.filter(g, lam, 50, d, 0, rows=omega)
    lab_r, _ = api.kmeans_reduced(F, k, 0)
    res = api.interpolate(g, lam, 50, 1e-3, omega, lab_r, k)
    assert res.status == 0 and np.all(res.relres <= 1e-6)
    # true residual of three columns with the float64 operator
    mask = np.zeros(gr.n)
    mask[omega.cpu().numpy()] = 1.0
    B = interp.rhs(gr.n, omega.cpu().numpy(), lab_r, k)
    X = res.X.cpu().numpy().astype(np.float64)
    a = jackson.lowpass_coeffs(lam, 50)
    for c in (0, 41, 99):
        r = interp.apply_operator(A, mask, 1e-3, a, X[:, c:c + 1])[:, 0] - B[:, c]
        assert np.linalg.norm(r) / np.linalg.norm(B[:, c]) <= 1e-4
    res2 = api.interpolate(g, lam, 50, 1e-3, omega, lab_r, k)
    assert torch.equal(res.labels, res2.labels) and torch.equal(res.X, res2.X)
    # the same solve on the graph in community order (the benchmarked launch)
    F_all = api.filter(g, lam, 50, d, 0, rows=None)
    # all rows by Clenshaw, sampled rows by the forward recurrence: float32 rounding apart
    Fg = api.gather_rows(F_all, omega)
    assert torch.linalg.norm(Fg - F) <= 1e-4 * torch.linalg.norm(F)
    order, frac = api.community_order(g, F_all, omega, lab_r, k, want_frac=True)
    assert frac > 0.4  # most edges of this SBM stay inside a community
    res3 = api.interpolate(g, lam, 50, 1e-3, omega, lab_r, k, order=order)
    assert res3.status == 0 and np.all(res3.relres <= 1e-6)
    X3 = res3.X.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(X3 - X) <= 1e-3 * np.linalg.norm(X)
    agree = float((res3.labels == res.labels).float().mean())
    assert agree >= 0.99, agree
    for c in (0, 41, 99):
        r = interp.apply_operator(A, mask, 1e-3, a, X3[:, c:c + 1])[:, 0] - B[:, c]
        assert np.linalg.norm(r) / np.linalg.norm(B[:, c]) <= 1e-4
    # the side-by-side CGs reach the same solution
    res4 = api.interpolate(g, lam, 50, 1e-3, omega, lab_r, k, order=order, method=0)
    assert res4.status == 0 and res3.iters.max() < res4.iters.max()
    X4 = res4.X.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(X4 - X3) <= 1e-2 * np.linalg.norm(X3)


@pytest.mark.slow
def test_chunglu_1e6_filter_columns_and_moment_identity(api, chunglu1e6):
    gr, A = chunglu1e6
    g = api.Graph(gr.row_ptr, gr.col)
    R, Y, a = _columns_check(api, g, A, 56, 60, 0.2, (0, 55))
    # identity between two kernels: <R, h~(L) R> from the filter output equals
    # sum_m a_m mu_m from the moment pass on the same signals
    n_c = 28
    cnt, mom = api.eigencount(g, 0.2, 60, n_c, 4, 9)
    Rc = api.gaussian_block(gr.n, n_c, 4, 9, 1)
    Yc = api.filter_block(g, a, Rc)
    direct = float(torch.sum(Rc.double() * Yc.double()))
    bound = 1e-5 * float(torch.linalg.norm(Rc)) * float(torch.linalg.norm(Yc)) + 1e-3 * (1 + abs(cnt))
    assert abs(direct - cnt) <= bound, (direct, cnt, bound)


@pytest.mark.slow
def test_chunglu_1e6_sampling_and_cg(api, chunglu1e6):
    gr, A = chunglu1e6
    g = api.Graph(gr.row_ptr, gr.col)
    k, lam = 250, 0.2
    n = api.default_n(k)
    omega = api.sample(gr.n, n, 0)
    assert np.array_equal(omega.cpu().numpy(), sampling.sample(gr.n, n, 0))
    lab_r = np.arange(n) % k
    res = api.interpolate(g, lam, 60, 1e-3, omega, lab_r, k, tol=1e-6)
    assert res.status == 0 and np.all(res.relres <= 1e-6)
    mask = np.zeros(gr.n)
    mask[omega.cpu().numpy()] = 1.0
    B = interp.rhs(gr.n, omega.cpu().numpy(), lab_r, k)
    X = res.X.cpu().numpy().astype(np.float64)
    a = jackson.lowpass_coeffs(lam, 60)
    for c in (0, 249):
        r = interp.apply_operator(A, mask, 1e-3, a, X[:, c:c + 1])[:, 0] - B[:, c]
        assert np.linalg.norm(r) / np.linalg.norm(B[:, c]) <= 1e-4


def test_autotuner_records_a_width_and_keeps_results(api, sbm1e5):
    gr, A = sbm1e5
    g = api.Graph(gr.row_ptr, gr.col)
    X = api.gaussian_block(gr.n, 47, 3, 0, 2)
    a = jackson.lowpass_coeffs(0.4, 20)
    before = api.filter_block(g, a, X)
    try:
        pw, xcd, us = api.autotune(g, 47, 0, reps=5)
        assert pw % 4 == 0 and 4 <= pw <= 256 and us > 0
        assert api.panel_width(gr.n, 47, gr.nnz) == pw
        after = api.filter_block(g, a, X)
        # each output element sums its row's neighbours in CSR order whatever the panel width
        assert torch.equal(before, after)
    finally:
        api.autotune_clear()
