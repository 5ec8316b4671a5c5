"""GPU parity: every libcsc call against the CPU float64 oracle on the same
seeded inputs, at sizes the oracle finishes in seconds.

Tolerances (float32 GPU arithmetic against float64):
* Gaussian blocks: float32 rounding of the same float64 draw, |diff| <= 2^-23 |z|;
* filtered blocks and features: relative Frobenius error <= 1e-4;
* moments mu_m = <R, T_m R>: |diff| <= 1e-5 mu_0 (mu_0 = ||R||_F^2);
* eigencount: |diff| <= 1e-3 (1 + |count|); the dichotomy takes the same
  decisions unless the oracle's count lies within that margin of k - 1/2,
  k + 1/2 or k, and then the estimate stays within one bracket width;
* sampled indices: bit-exact; k-means labels from identical inputs: exact;
* interpolation: labels at ARI >= 0.99 against the oracle's, recursive
  residual <= tol, and X within 1e-3 relative Frobenius error.
"""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import cheb, eigencount, interp, jackson, kmeans, laplacian, metrics, philox, sampling
from oracle import csc as ocsc
from kmeans_parity import check_kmeans

pytestmark = pytest.mark.gpu

PANEL_WIDTHS = (4, 8, 12, 16, 28, 32, 48, 64, 100, 256)


@pytest.fixture(scope="module")
def api():
    from paper_1602_02018_amd import api as a

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    yield a
    a.set_panel_width(0)


@pytest.fixture(scope="module")
def cfg1():
    return synth.sbm_config(1000, 10, seed=0)


@pytest.fixture(scope="module")
def ragged():
    # N not a multiple of any tile height; a few isolated nodes
    g = synth.chung_lu_blocks(1037, 7, mean_deg=6.0, max_deg=80.0, seed=2)
    assert (g.degrees() == 0).any()
    return g


def _A(g):
    return laplacian.normalized_adjacency(g.row_ptr, g.col)[0]


def _relfro(x, ref):
    return float(np.linalg.norm(np.asarray(x, np.float64) - ref) / np.linalg.norm(ref))


# ------------------------------------------------------------- Laplacian ---

def test_laplacian_values(api, ragged):
    g = api.Graph(ragged.row_ptr, ragged.col)
    A, s = laplacian.normalized_adjacency(ragged.row_ptr, ragged.col)
    np.testing.assert_allclose(g.dinv_sqrt.cpu().numpy(), s, rtol=2e-7, atol=0)
    val = g.val.cpu().numpy()[: g.nnz]
    np.testing.assert_allclose(val, A.data, rtol=4e-7, atol=0)


def test_laplacian_weighted_and_diagonal(api):
    row_ptr = np.array([0, 2, 4, 5], dtype=np.int32)
    col = np.array([0, 1, 0, 2, 1], dtype=np.int32)
    w = np.array([9.0, 2.0, 2.0, 3.0, 3.0], dtype=np.float32)
    g = api.Graph(row_ptr, col, weights=w)
    A, s = laplacian.normalized_adjacency(row_ptr, col, w.astype(np.float64))
    dense = np.zeros((3, 3))
    val = g.val.cpu().numpy()
    for i in range(3):
        for e in range(row_ptr[i], row_ptr[i + 1]):
            dense[i, col[e]] = val[e]
    np.testing.assert_allclose(dense, A.toarray(), rtol=1e-6, atol=1e-7)


def test_laplacian_rejects_malformed_csr(api):
    from paper_1602_02018_amd import CscError

    with pytest.raises(CscError):
        api.Graph(np.array([0, 2, 1], np.int32), np.array([1, 0], np.int32))
    with pytest.raises(CscError):
        api.Graph(np.array([0, 1, 2], np.int32), np.array([1, 5], np.int32))


def test_laplacian_strict_check_rejects_loops_asymmetry_and_unsorted_rows(api, ragged, cfg1):
    """check = 2: the undirected graph without self-loops of Sec. 2.1."""
    from paper_1602_02018_amd import CscError, _lib

    for gr in (ragged, cfg1):  # the synthetic workloads pass
        api.Graph(gr.row_ptr, gr.col, check_csr=2)
    loop = (np.array([0, 2, 3], np.int32), np.array([0, 1, 0], np.int32))  # (0,0) stored
    api.Graph(*loop, check_csr=1)  # accepted, its value set to 0
    cases = {
        "self-loop": loop,
        "asymmetric": (np.array([0, 1, 2, 2], np.int32), np.array([1, 2], np.int32)),
        "unsorted": (np.array([0, 2, 3, 4], np.int32), np.array([2, 1, 0, 0], np.int32)),
        "duplicate": (np.array([0, 2, 4], np.int32), np.array([1, 1, 0, 0], np.int32)),
    }
    for name, (rp, cl) in cases.items():
        with pytest.raises(CscError) as e:
            api.Graph(rp, cl, check_csr=2)
        assert e.value.status == _lib.CSC_E_GRAPH, name
    # symmetric structure with unequal weights
    rp, cl = np.array([0, 1, 2], np.int32), np.array([1, 0], np.int32)
    api.Graph(rp, cl, weights=np.array([2.0, 2.0], np.float32), check_csr=2)
    with pytest.raises(CscError):
        api.Graph(rp, cl, weights=np.array([2.0, 3.0], np.float32), check_csr=2)


# --------------------------------------------------------------- random ----

@pytest.mark.parametrize("n,w,t,sid", [(1000, 28, 0, 2), (333, 5, 3, 1), (1, 1, 0, 2)])
def test_gaussian_block_matches_oracle(api, n, w, t, sid):
    R = api.gaussian_block(n, w, 7, t, sid).cpu().numpy().astype(np.float64)
    ref = philox.gaussian_block(7, n, w, t, sid)
    assert np.all(np.abs(R - ref) <= 2.0**-23 * np.abs(ref) + 1e-30)


# ----------------------------------------------------------- filtering -----

@pytest.mark.parametrize("pw", PANEL_WIDTHS)
@pytest.mark.parametrize("w", [1, 5, 13, 47, 70])
def test_filter_block_all_panel_widths(api, ragged, pw, w):
    api.set_panel_width(pw)
    try:
        g = api.Graph(ragged.row_ptr, ragged.col)
        X = api.gaussian_block(ragged.n, w, 11, 0, 2)
        a = jackson.lowpass_coeffs(0.45, 30)
        Y = api.filter_block(g, a, X).cpu().numpy()
        ref = cheb.filter_block(_A(ragged), X.cpu().numpy().astype(np.float64), a)
        assert _relfro(Y, ref) <= 1e-4
    finally:
        api.set_panel_width(0)


@pytest.mark.parametrize("lam,p", [(0.3, 50), (1.0, 1), (1.7, 2), (0.05, 60), (2.0, 5), (0.0, 5)])
def test_filter_block_orders_and_cutoffs(api, cfg1, lam, p):
    g = api.Graph(cfg1.row_ptr, cfg1.col)
    X = api.gaussian_block(cfg1.n, 28, 3, 0, 2)
    a = jackson.lowpass_coeffs(lam, p)
    Y = api.filter_block(g, a, X).cpu().numpy()
    ref = cheb.filter_block(_A(cfg1), X.cpu().numpy().astype(np.float64), a)
    if np.linalg.norm(ref) == 0.0:
        assert np.all(Y == 0.0)
    else:
        assert _relfro(Y, ref) <= 1e-4


def test_filter_block_on_graph_without_edges(api):
    N = 300
    g = api.Graph(np.zeros(N + 1, np.int32), np.zeros(0, np.int32))
    X = api.gaussian_block(N, 6, 1, 0, 2)
    a = jackson.lowpass_coeffs(1.3, 20)
    Y = api.filter_block(g, a, X).cpu().numpy()
    # L = I: every eigenvalue is 1, so the filter is the scalar h~(1)
    np.testing.assert_allclose(Y, jackson.evaluate(a, 1.0) * X.cpu().numpy(), rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("normalize", [True, False])
@pytest.mark.parametrize("d", [28, 130])  # rows written in one LDS chunk, or two (d > 128)
def test_feature_pass_all_rows(api, cfg1, normalize, d):
    p, seed, lam = 50, 0, 0.46875
    g = api.Graph(cfg1.row_ptr, cfg1.col)
    F = api.filter(g, lam, p, d, seed, normalize=normalize).cpu().numpy()
    R = philox.gaussian_block(seed, cfg1.n, d, 0, philox.FEAT)
    Y = cheb.filter_block(_A(cfg1), R, jackson.lowpass_coeffs(lam, p))
    ref = ocsc.features(_A(cfg1), lam, p, d, seed) if normalize else Y
    assert _relfro(F, ref) <= 1e-4
    if normalize:
        np.testing.assert_allclose(np.linalg.norm(F, axis=1), 1.0, atol=1e-6)


def test_feature_pass_sampled_rows(api, ragged):
    d, p, seed, lam = 20, 40, 4, 0.6
    g = api.Graph(ragged.row_ptr, ragged.col)
    rows = sampling.sample(ragged.n, 77, 1)
    Fs = api.filter(g, lam, p, d, seed, rows=rows, normalize=True).cpu().numpy()
    Fall = api.filter(g, lam, p, d, seed, normalize=True).cpu().numpy()
    ref = ocsc.features(_A(ragged), lam, p, d, seed)[rows]
    assert _relfro(Fs, ref) <= 1e-4
    # the sampled-row epilogue (forward recurrence) and the full pass (Clenshaw
    # by default) agree to float32 rounding
    assert _relfro(Fs, Fall[rows].astype(np.float64)) <= 1e-4


# ---------------------------------------------------------- eigencount -----

@pytest.mark.parametrize("pw", PANEL_WIDTHS)
def test_moments_match_oracle(api, ragged, pw):
    api.set_panel_width(pw)
    try:
        g = api.Graph(ragged.row_ptr, ragged.col)
        n_c, p, seed, t = 14, 50, 5, 3
        cnt, mom = api.eigencount(g, 0.5, p, n_c, seed, t)
        R = philox.gaussian_block(seed, ragged.n, n_c, t, philox.COUNT)
        ref = cheb.moments(_A(ragged), R, p)
        assert np.max(np.abs(mom - ref)) <= 1e-5 * ref[0]
        cref = float(np.dot(jackson.lowpass_coeffs(0.5, p), ref))
        assert abs(cnt - cref) <= 1e-3 * (1 + abs(cref))
        assert abs(cref - eigencount.eigencount(_A(ragged), 0.5, p, R)) < 1e-9 * (1 + abs(cref))
    finally:
        api.set_panel_width(0)


def _check_bisection(gpu, ref_trace, k, tol):
    ok_until = len(ref_trace)
    for s, ((lg, cg), (lo, co)) in enumerate(zip(gpu.trace, ref_trace)):
        assert lg == lo, (s, lg, lo)
        assert abs(cg - co) <= tol * (1 + abs(co))
        dg = (math.floor(cg + 0.5) == k, cg < k)
        do = (math.floor(co + 0.5) == k, co < k)
        if dg != do:
            near = min(abs(co - (k - 0.5)), abs(co - (k + 0.5)), abs(co - k))
            assert near <= 2 * tol * (1 + abs(co))
            ok_until = s
            break
    return ok_until


def test_bisection_matches_oracle(api, cfg1):
    g = api.Graph(cfg1.row_ptr, cfg1.col)
    k, p, seed = 10, 50, 0
    n_c = eigencount.count_signals(cfg1.n)
    res = api.estimate_lambda_k(g, k, p, n_c, seed)
    lam, steps, trace, ok = eigencount.estimate_lambda_k(_A(cfg1), k, p, n_c, seed)
    stop = _check_bisection(res, trace, k, 1e-3)
    if stop == len(trace):
        assert res.lam == lam and res.steps == steps and res.status == 0
    else:
        assert abs(res.lam - lam) <= 2.0 / 2 ** (stop + 1)
    R = philox.gaussian_block(seed, cfg1.n, n_c, 1, philox.COUNT)
    np.testing.assert_allclose(res.moments, cheb.moments(_A(cfg1), R, p), atol=1e-5 * cfg1.n)


def test_bisection_exhaustion_and_bracket_miss(api, cfg1):
    from paper_1602_02018_amd import _lib

    g = api.Graph(cfg1.row_ptr, cfg1.col)
    n_c = eigencount.count_signals(cfg1.n)
    res = api.estimate_lambda_k(g, 10, 50, n_c, 0, max_steps=1)
    assert res.steps == 1 and res.trace[0][0] == 1.0
    assert res.status == _lib.CSC_W_BISECT_EXHAUSTED and res.lam == 1.0  # count(1) >> 10
    # a bracket far above lambda_k: every count exceeds k, the search falls back to [0, 2]
    res = api.estimate_lambda_k(g, 10, 50, n_c, 0, max_steps=4, bracket=(1.5, 2.0))
    assert res.status == _lib.CSC_W_BRACKET_MISS
    assert all(c > 10 for _, c in res.trace[:4])
    assert res.trace[4][0] == 1.0
    # every test t drew the signals of sub-stream t, across the restart too
    # (the next test's signals are drawn ahead while a test runs)
    for t in (1, 4, 5, 6):
        mid, cnt = res.trace[t - 1]
        R = philox.gaussian_block(0, cfg1.n, n_c, t, philox.COUNT)
        ref = eigencount.eigencount(_A(cfg1), mid, 50, R)
        assert abs(cnt - ref) <= 1e-3 * (1 + abs(ref)), (t, cnt, ref)
    # a bracket holding lambda_k gives the same decisions as the oracle inside it
    res = api.estimate_lambda_k(g, 10, 50, n_c, 0, bracket=(0.25, 0.75))
    lam, steps, trace, ok = eigencount.estimate_lambda_k(_A(cfg1), 10, 50, n_c, 0, bracket=(0.25, 0.75))
    stop = _check_bisection(res, trace, 10, 1e-3)
    if stop == len(trace):
        assert res.lam == lam


# ------------------------------------------------------------ sampling -----

@pytest.mark.parametrize("N,n,seed", [(1000, 47, 0), (100000, 922, 0), (1037, 1, 3), (1037, 1037, 3),
                                      (5000, 4999, 9), (1, 1, 0), (100000, 30000, 2)])
def test_sampling_bit_exact(api, N, n, seed):
    idx = api.sample(N, n, seed).cpu().numpy()
    assert np.array_equal(idx, sampling.sample(N, n, seed))


# ------------------------------------------------------------- k-means -----

def test_kmeans_on_gpu_features_matches_oracle_given_same_input(api, cfg1):
    g = api.Graph(cfg1.row_ptr, cfg1.col)
    omega = api.sample(cfg1.n, 47, 0)
    Fd = api.filter(g, 0.46875, 50, 28, 0, rows=omega)
    F = Fd.cpu().numpy()
    lab, inertia = api.kmeans_reduced_device(Fd.contiguous(), 10, 0)
    same = check_kmeans(F, 10, 0, api.kmeans_seeds_device(Fd.contiguous(), 10, 0), lab, inertia)
    assert all(same)
    # and the float64 oracle features give the same clustering
    Fo = ocsc.features(_A(cfg1), 0.46875, 50, 28, 0)[sampling.sample(cfg1.n, 47, 0)]
    lab_o, _, _ = kmeans.kmeans(Fo, 10, 0)
    assert metrics.adjusted_rand_index(lab, lab_o) == 1.0


# ------------------------------------------------------- interpolation -----

@pytest.mark.parametrize("pw", [4, 8, 16, 0])
@pytest.mark.parametrize("method", [0, 1, 2])
def test_interpolation_matches_oracle(api, cfg1, pw, method):
    api.set_panel_width(pw)
    try:
        g = api.Graph(cfg1.row_ptr, cfg1.col)
        k, p, lam, gamma = 10, 50, 0.46875, 1e-3
        omega = sampling.sample(cfg1.n, 47, 0)
        A = _A(cfg1)
        lab_r, _, _ = kmeans.kmeans(ocsc.features(A, lam, p, 28, 0)[omega], k, 0)
        res = api.interpolate(g, lam, p, gamma, omega, lab_r, k, tol=1e-6, method=method)
        X, lab, iters, relres = interp.interpolate(A, lam, p, gamma, omega, lab_r, k, tol=1e-6)
        assert res.status == 0
        assert np.all(res.relres <= 1e-6) and np.all(res.iters >= 1)
        if method == 0:
            # the same iteration as the oracle's: same iteration counts, iterates close
            assert np.all(np.abs(res.iters - iters) <= 2)
            assert _relfro(res.X.cpu().numpy(), X) <= 1e-3
        else:
            # another Krylov method for the same system: fewer iterations; compare
            # with the solution the oracle reaches at a tolerance far below 1e-6
            assert res.iters.max() < iters.max()
            Xt, _, _, _ = interp.interpolate(A, lam, p, gamma, omega, lab_r, k, tol=1e-12)
            assert _relfro(res.X.cpu().numpy(), Xt) <= 1e-3
        assert metrics.adjusted_rand_index(res.labels.cpu().numpy(), lab) >= 0.99
        # true residual with the float64 operator
        mask = np.zeros(cfg1.n)
        mask[omega] = 1.0
        B = interp.rhs(cfg1.n, omega, lab_r, k)
        Xg = res.X.cpu().numpy().astype(np.float64)
        tr = np.linalg.norm(interp.apply_operator(A, mask, gamma, jackson.lowpass_coeffs(lam, p), Xg) - B,
                            axis=0) / np.linalg.norm(B, axis=0)
        assert np.all(tr <= 1e-4)
    finally:
        api.set_panel_width(0)


def test_interpolation_single_cluster_and_max_iter(api, cfg1):
    from paper_1602_02018_amd import _lib

    g = api.Graph(cfg1.row_ptr, cfg1.col)
    omega = sampling.sample(cfg1.n, 20, 1)
    res = api.interpolate(g, 0.4, 50, 1e-3, omega, np.zeros(20, np.int32), 1, tol=1e-6)
    assert res.status == 0 and np.all(res.labels.cpu().numpy() == 0)
    res = api.interpolate(g, 0.4, 50, 1e-3, omega, np.arange(20) % 3, 3, tol=1e-12, max_iter=2,
                          method=0)
    assert res.status == _lib.CSC_W_NOT_CONVERGED and np.all(res.iters == 2)
    X, lab, iters, relres = interp.interpolate(_A(cfg1), 0.4, 50, 1e-3, omega, np.arange(20) % 3, 3,
                                               tol=1e-12, max_iter=2)
    assert _relfro(res.X.cpu().numpy(), X) <= 1e-4
    for method in (1, 2):
        res = api.interpolate(g, 0.4, 50, 1e-3, omega, np.arange(20) % 3, 3, tol=1e-12, max_iter=2,
                              method=method)
        assert res.status == _lib.CSC_W_NOT_CONVERGED and np.all(res.iters == 2)


@pytest.mark.parametrize("method", [0, 1, 2])
def test_interpolation_cluster_without_samples(api, cfg1, method):
    # cluster 2 has no sampled node: b_2 = 0, its column stays 0 and never wins
    g = api.Graph(cfg1.row_ptr, cfg1.col)
    omega = sampling.sample(cfg1.n, 30, 2)
    lab_r = np.arange(30) % 2
    res = api.interpolate(g, 0.46875, 50, 1e-3, omega, lab_r, 3, method=method)
    X = res.X.cpu().numpy()
    assert np.all(X[:, 2] == 0.0) and res.iters[2] == 0
    assert set(np.unique(res.labels.cpu().numpy())) <= {0, 1}


# -------------------------------------------------------------- Alg. 2 -----

@pytest.mark.parametrize("seed", [0, 1])
def test_end_to_end_plain_config(api, cfg1, seed):
    d = int(math.ceil(4 * math.log(cfg1.n)))
    g = api.Graph(cfg1.row_ptr, cfg1.col)
    res = api.run(g, 10, d, seed)
    ref = ocsc.run(cfg1.row_ptr, cfg1.col, 10, d, seed)
    assert abs(res.lam - ref.lam) <= 2.0 / 2 ** min(res.bisection.steps, ref.bisect_steps)
    assert np.array_equal(res.omega.cpu().numpy(), ref.omega)
    ari = metrics.adjusted_rand_index(res.labels.cpu().numpy(), ref.labels)
    assert ari >= 0.99
    assert metrics.adjusted_rand_index(res.labels.cpu().numpy(), cfg1.truth) > 0.9


def test_end_to_end_disconnected_blocks_exact(api):
    gr = synth.disconnected_regular(6, 80, 6, seed=3)
    d = int(math.ceil(4 * math.log(gr.n)))
    g = api.Graph(gr.row_ptr, gr.col)
    res = api.run(g, 6, d, 3, replicates=5)
    assert metrics.adjusted_rand_index(res.labels.cpu().numpy(), gr.truth) == 1.0


def test_determinism(api, ragged):
    g = api.Graph(ragged.row_ptr, ragged.col)
    a = api.filter(g, 0.5, 50, 13, 9).cpu().numpy()
    b = api.filter(g, 0.5, 50, 13, 9).cpu().numpy()
    assert np.array_equal(a, b)
    c1, m1 = api.eigencount(g, 0.5, 50, 14, 2, 1)
    c2, m2 = api.eigencount(g, 0.5, 50, 14, 2, 1)
    assert c1 == c2 and np.array_equal(m1, m2)


@pytest.mark.parametrize("xcd", [0, 1, 2])
@pytest.mark.parametrize("nt", [0, 1])
@pytest.mark.parametrize("pw", [8, 28, 52, 100, 256])
def test_tuning_knobs_do_not_change_results(api, ragged, xcd, nt, pw):
    from paper_1602_02018_amd import _lib

    keys = (_lib.TUNE_XCD_ORDER, _lib.TUNE_NONTEMPORAL, _lib.TUNE_PANEL_WIDTH)
    old = [api.get_tuning(k) for k in keys]
    try:
        for k, v in zip(keys, (xcd, nt, pw)):
            api.set_tuning(k, v)
        g = api.Graph(ragged.row_ptr, ragged.col)
        X = api.gaussian_block(ragged.n, 37, 2, 0, 2)
        a = jackson.lowpass_coeffs(0.7, 20)
        Y = api.filter_block(g, a, X).cpu().numpy()
        ref = cheb.filter_block(_A(ragged), X.cpu().numpy().astype(np.float64), a)
        assert _relfro(Y, ref) <= 1e-4
        cnt, mom = api.eigencount(g, 0.5, 30, 11, 5, 1)
        R = philox.gaussian_block(5, ragged.n, 11, 1, philox.COUNT)
        mref = cheb.moments(_A(ragged), R, 30)
        assert np.max(np.abs(mom - mref)) <= 1e-5 * mref[0]
    finally:
        for k, v in zip(keys, old):
            api.set_tuning(k, v)


def test_jacobi_block_cg_needs_no_more_iterations(api, cfg1):
    """The preconditioned block CG solves the same system in at most as many
    iterations as the plain one (the diagonal maps sampled and unsampled rows
    to one scale)."""
    g = api.Graph(cfg1.row_ptr, cfg1.col)
    omega = sampling.sample(cfg1.n, 47, 0)
    lab_r = cfg1.truth[omega]
    a = api.interpolate(g, 0.46875, 50, 1e-3, omega, lab_r, 10, method=1)
    b = api.interpolate(g, 0.46875, 50, 1e-3, omega, lab_r, 10, method=2)
    print("block CG iterations, plain / Jacobi:", a.iters.max(), b.iters.max())
    assert a.status == 0 and b.status == 0
    assert b.iters.max() <= a.iters.max()
    assert _relfro(b.X.cpu().numpy(), a.X.cpu().numpy()) <= 1e-3


def _tiny(N, kind):
    """Small graphs: a path, a cycle, two disjoint triangles, an edgeless set."""
    if kind == "path":
        u = np.arange(N - 1)
        v = u + 1
    elif kind == "cycle":
        u = np.arange(N)
        v = (u + 1) % N
    elif kind == "triangles":
        u = np.array([0, 1, 2, 3, 4, 5])
        v = np.array([1, 2, 0, 4, 5, 3])
    else:
        u = v = np.zeros(0, np.int64)
    return synth.csr_from_edges(N, u, v)


@pytest.mark.parametrize("N,kind,k", [(1, "none", 1), (2, "path", 1), (2, "path", 2), (5, "cycle", 2),
                                      (6, "triangles", 2), (13, "path", 3), (7, "none", 3)])
def test_end_to_end_tiny_graphs(api, N, kind, k):
    """Degenerate sizes run through every step: the same lambda_k, samples and
    labels (up to relabelling) as the oracle, with n = N sampled nodes."""
    row_ptr, col = _tiny(N, kind)
    g = api.Graph(row_ptr, col)
    d, n = 3, N
    res = api.run(g, k, d, 0, n=n, replicates=3)
    ref = ocsc.run(row_ptr, col, k, d, 0, n=n, replicates=3)
    assert abs(res.lam - ref.lam) <= 2.0 / 2 ** min(res.bisection.steps, ref.bisect_steps)
    assert np.array_equal(res.omega.cpu().numpy(), ref.omega)
    lab = res.labels.cpu().numpy()
    assert lab.shape == (N,) and lab.min() >= 0 and lab.max() < k
    if N > 1:
        assert metrics.adjusted_rand_index(lab, ref.labels) >= 0.99


@pytest.fixture(scope="module", params=[129, 300])
def multi_panel(request):
    """k = 129 or 300 columns on a 3000-node SBM and the oracle's tight
    solution.  k = 129: the Gram matrices' second 128-column tile holds one
    column (the symmetric ones sum the tiles on and below the diagonal and
    mirror the rest); k = 300: three tiles, two panels."""
    gr = synth.sbm(3000, 30, 16.0, 0.25 * synth.eps_critical(16.0, 30), seed=4)
    k, n = request.param, 1200
    omega = sampling.sample(gr.n, n, 5)
    lab_r = np.arange(n) % k
    Xt, lab, _, _ = interp.interpolate(_A(gr), 0.6, 30, 1e-3, omega, lab_r, k, tol=1e-12)
    return gr, k, omega, lab_r, Xt, lab


@pytest.mark.parametrize("method", [1, 2])
def test_block_interpolation_with_several_panels(api, multi_panel, method):
    """k = 300 columns span two panels of the block layout (widths up to
    256): the Gram matrices and block products cross panel boundaries; k = 129
    puts one column in the Gram matrices' second tile."""
    gr, k, omega, lab_r, Xt, lab = multi_panel
    g = api.Graph(gr.row_ptr, gr.col)
    if k == 300:
        assert api.panel_width(gr.n, k, gr.nnz) < k  # more than one panel
    res = api.interpolate(g, 0.6, 30, 1e-3, omega, lab_r, k, method=method)
    assert res.status == 0 and np.all(res.relres <= 1e-6)
    assert _relfro(res.X.cpu().numpy(), Xt) <= 1e-3
    assert metrics.adjusted_rand_index(res.labels.cpu().numpy(), lab) >= 0.99
