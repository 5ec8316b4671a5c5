"""Pins of the CPU oracle against things other than itself.

Each test checks one oracle function against a library routine, a closed form
fixed by the paper's definitions, a statistical property, or brute force on a
tiny input, so that a dropped term, a wrong sign or index or a transposed
operand in the oracle fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.stats as st

import synth
from oracle import cheb, eigencount, interp, jackson, kmeans, laplacian, metrics, philox, sampling
from oracle import csc as ocsc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- Philox ----

@pytest.mark.parametrize("seed,ctr", [(0, 0), (7, 5), (2**63 + 11, 2**40 + 3), (123, 2**64 - 5)])
def test_philox_matches_numpy(seed, ctr):
    # numpy's Philox is Philox4x64-10; its j-th output block is the bijection
    # applied to (counter + 1 + j) with 256-bit carry.
    g = np.random.Philox(key=np.array([seed, 0], dtype=np.uint64),
                         counter=np.array([ctr % 2**64, 0, 0, 0], dtype=np.uint64))
    raw = g.random_raw(12).reshape(3, 4)
    for j in range(3):
        c = ctr + 1 + j
        c0, c1 = c % 2**64, c // 2**64
        out = philox.philox4x64(np.uint64(c0), np.uint64(c1), 0, 0, np.uint64(seed), 0)
        assert [int(x) for x in out] == [int(x) for x in raw[j]]


def test_philox_high_counter_words_match_numpy():
    g = np.random.Philox(key=np.array([99, 0], dtype=np.uint64),
                         counter=np.array([41, 6, 3, 0], dtype=np.uint64))
    raw = g.random_raw(4)
    out = philox.philox4x64(np.uint64(42), 6, 3, 0, np.uint64(99), 0)
    assert [int(x) for x in out] == [int(x) for x in raw]


def test_philox_vectorised_equals_scalar():
    c = np.arange(50, dtype=np.uint64) * np.uint64(2**37 + 5)
    v = philox.philox4x64(c, 3, 1, 0, np.uint64(17), 0)
    for i in (0, 13, 49):
        s = philox.philox4x64(np.uint64(c[i]), 3, 1, 0, np.uint64(17), 0)
        assert all(int(v[w][i]) == int(s[w]) for w in range(4))


def test_gaussian_block_distribution():
    w = 40
    Z = philox.gaussian_block(5, 5000, w, 0, philox.FEAT)
    assert Z.shape == (5000, w)
    x = Z.ravel() * math.sqrt(w)
    assert abs(x.mean()) < 5.0 / math.sqrt(x.size)
    assert abs(x.var() - 1.0) < 5.0 * math.sqrt(2.0 / x.size)
    assert st.kstest(x, "norm").pvalue > 1e-3
    # columns uncorrelated, different sub-streams and streams independent
    C = np.corrcoef(Z[:, :5].T)
    assert np.max(np.abs(C - np.eye(5))) < 0.06
    Z2 = philox.gaussian_block(5, 5000, w, 1, philox.FEAT)
    Z3 = philox.gaussian_block(5, 5000, w, 0, philox.COUNT)
    assert abs(np.corrcoef(Z.ravel(), Z2.ravel())[0, 1]) < 0.01
    assert abs(np.corrcoef(Z.ravel(), Z3.ravel())[0, 1]) < 0.01


def test_uniform_draws_range_and_mean():
    u = np.array([philox.uniform(3, j, 0, philox.KMEANS) for j in range(4000)])
    assert u.min() >= 0.0 and u.max() < 1.0
    assert st.kstest(u, "uniform").pvalue > 1e-3


# -------------------------------------------------------------- Laplacian ---

def test_normalized_laplacian_matches_networkx():
    import networkx as nx

    g = synth.sbm_config(300, 5, s=8.0, seed=3)
    L = laplacian.laplacian_dense(g.row_ptr, g.col)
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    rows = np.repeat(np.arange(g.n), g.degrees())
    G.add_edges_from(zip(rows.tolist(), g.col.tolist()))
    Lnx = nx.normalized_laplacian_matrix(G, nodelist=range(g.n)).toarray()
    if (g.degrees() == 0).any():
        # networkx leaves an isolated node's row at 0; the oracle puts 1 on the diagonal
        iso = np.nonzero(g.degrees() == 0)[0]
        Lnx[iso, iso] = 1.0
    np.testing.assert_allclose(L, Lnx, atol=1e-14)


def test_laplacian_spectrum_in_0_2_with_zero_eigenvalue():
    g = synth.sbm_config(400, 4, s=10.0, seed=1)
    ev = np.linalg.eigvalsh(laplacian.laplacian_dense(g.row_ptr, g.col))
    assert ev[0] > -1e-12 and ev[-1] < 2.0 + 1e-12
    assert abs(ev[0]) < 1e-10


def test_isolated_node_is_eigenvalue_one():
    row_ptr = np.array([0, 1, 2, 2], dtype=np.int32)  # nodes 0-1 joined, node 2 alone
    col = np.array([1, 0], dtype=np.int32)
    L = laplacian.laplacian_dense(row_ptr, col)
    np.testing.assert_allclose(L, [[1, -1, 0], [-1, 1, 0], [0, 0, 1]], atol=1e-15)


def test_weighted_degrees_exclude_diagonal():
    row_ptr = np.array([0, 2, 4], dtype=np.int32)
    col = np.array([0, 1, 0, 1], dtype=np.int32)
    w = np.array([5.0, 2.0, 2.0, 7.0])
    np.testing.assert_allclose(laplacian.degrees(row_ptr, col, w), [2.0, 2.0])
    A, s = laplacian.normalized_adjacency(row_ptr, col, w)
    np.testing.assert_allclose(A.toarray(), [[0, 1.0], [1.0, 0]])


# ---------------------------------------------------- Jackson-Chebyshev -----

@pytest.mark.parametrize("lc", [0.1, 0.37, 1.0, 1.6])
def test_chebyshev_coefficients_match_quadrature(lc):
    # (2/pi) int_{-1}^{1} h(x) T_m(x) / sqrt(1-x^2) dx computed by adaptive quadrature
    # in the angle variable x = cos t, where the integrand is piecewise smooth.
    from scipy.integrate import quad

    p = 12
    c = jackson.cheb_step_coeffs(lc, p)
    tc = math.acos(lc - 1.0)
    for m in range(p + 1):
        val, _ = quad(lambda t: math.cos(m * t), tc, math.pi, limit=200)
        ref = val / math.pi if m == 0 else 2.0 * val / math.pi
        assert abs(c[m] - ref) < 1e-12


@pytest.mark.parametrize("p", [5, 20, 50, 60])
def test_jackson_factors_are_sine_window_autocorrelation(p):
    # Jackson kernel = |sum_nu a_nu e^{i nu phi}|^2 with a_nu = sin(pi (nu+1)/(p+2)),
    # nu = 0..p; its normalised Fourier coefficients are the damping factors.
    nu = np.arange(p + 1)
    a = np.sin(np.pi * (nu + 1) / (p + 2))
    ref = np.array([np.dot(a[: p + 1 - m], a[m:]) for m in range(p + 1)]) / np.dot(a, a)
    np.testing.assert_allclose(jackson.jackson_factors(p), ref, atol=1e-13)


def test_jackson_kernel_positive():
    p = 30
    g = jackson.jackson_factors(p)
    t = np.linspace(0.0, np.pi, 301)
    m = np.arange(1, p + 1)
    for y in (0.0, 0.7, 2.5):
        K = g[0] + 2.0 * (np.cos(np.multiply.outer(t, m)) * np.cos(m * y)) @ g[1:]
        assert K.min() > -1e-12


def test_lowpass_bounds_monotone_and_limits():
    p = 50
    lam = np.linspace(0.0, 2.0, 20001)
    prev = None
    for lc in (0.05, 0.3, 0.5, 1.0, 1.5, 1.95):
        h = jackson.evaluate(jackson.lowpass_coeffs(lc, p), lam)
        assert h.min() > 0.0 and h.max() < 1.0
        assert abs(jackson.evaluate(jackson.lowpass_coeffs(lc, p), lc) - 0.5) < 0.02
        if prev is not None:
            assert np.all(h >= prev - 1e-12)
        prev = h
    np.testing.assert_allclose(jackson.evaluate(jackson.lowpass_coeffs(2.0, p), lam), 1.0, atol=1e-14)
    np.testing.assert_allclose(jackson.evaluate(jackson.lowpass_coeffs(0.0, p), lam), 0.0, atol=1e-14)


def test_undamped_series_overshoots():
    lam = np.linspace(0.0, 2.0, 20001)
    h = jackson.evaluate(jackson.lowpass_coeffs(0.5, 50, damping=False), lam)
    assert h.max() > 1.05 and h.min() < -0.03


# ------------------------------------------------------------- filtering ----

def _eig(g):
    L = laplacian.laplacian_dense(g.row_ptr, g.col)
    return np.linalg.eigh(L)


@pytest.fixture(scope="module")
def small_sbm():
    g = synth.sbm_config(600, 6, s=12.0, seed=4)
    ev, U = _eig(g)
    A, _ = laplacian.normalized_adjacency(g.row_ptr, g.col)
    return g, A, ev, U


def test_filter_equals_spectral_closed_form(small_sbm):
    g, A, ev, U = small_sbm
    R = philox.gaussian_block(1, g.n, 9, 0, philox.FEAT)
    for lc, p in ((0.3, 50), (1.2, 17), (0.7, 1), (0.7, 0)):
        a = jackson.lowpass_coeffs(lc, p)
        Y = cheb.filter_block(A, R, a)
        Yref = U @ (jackson.evaluate(a, ev)[:, None] * (U.T @ R))
        assert np.linalg.norm(Y - Yref) <= 1e-12 * np.linalg.norm(Yref)


def test_filter_error_within_em_bound(small_sbm):
    # Eq. (8): with e_m = sup over the spectrum of |h~ - h|, ||(h~(L) - h(L)) R||_F <= e_m ||R||_F
    g, A, ev, U = small_sbm
    R = philox.gaussian_block(2, g.n, 7, 0, philox.FEAT)
    lc = 0.5 * (ev[5] + ev[6])
    a = jackson.lowpass_coeffs(lc, 50)
    err = jackson.evaluate(a, ev) - (ev <= lc)
    e_m = np.max(np.abs(err))
    diff = cheb.filter_block(A, R, a) - U @ ((ev <= lc)[:, None] * (U.T @ R))
    assert np.linalg.norm(diff) <= e_m * np.linalg.norm(R) * (1 + 1e-12)
    assert e_m < 0.5


def test_moments_match_spectral_form(small_sbm):
    g, A, ev, U = small_sbm
    R = philox.gaussian_block(3, g.n, 5, 1, philox.COUNT)
    mu = cheb.moments(A, R, 20)
    P = np.sum((U.T @ R) ** 2, axis=1)
    t = np.arccos(np.clip(ev - 1.0, -1, 1))
    ref = np.array([np.sum(P * np.cos(m * t)) for m in range(21)])
    np.testing.assert_allclose(mu, ref, rtol=1e-11, atol=1e-11 * ref[0])


# ------------------------------------------------------------- eigencount ---

def test_hutchinson_count_statistics(small_sbm):
    g, A, ev, U = small_sbm
    n_c = eigencount.count_signals(g.n)
    lc = 0.5 * (ev[5] + ev[6])
    hv = jackson.evaluate(jackson.lowpass_coeffs(lc, 50), ev)
    tr = hv.sum()
    sd = math.sqrt(2.0 * np.sum(hv ** 2) / n_c)
    ests = []
    for t in range(1, 41):
        R = philox.gaussian_block(11, g.n, n_c, t, philox.COUNT)
        ests.append(eigencount.eigencount(A, lc, 50, R))
    ests = np.array(ests)
    assert np.all(np.abs(ests - tr) <= 5 * sd)
    assert abs(ests.mean() - tr) <= 5 * sd / math.sqrt(len(ests))
    assert 0.5 * sd < ests.std() < 2.0 * sd
    assert abs(tr - np.sum(ev <= lc)) < 1.0


def test_bisection_on_disconnected_blocks():
    g = synth.disconnected_regular(5, 60, 6, seed=2)
    ev, _ = _eig(g)
    assert np.all(np.abs(ev[:5]) < 1e-10) and ev[5] > 0.2
    A, _ = laplacian.normalized_adjacency(g.row_ptr, g.col)
    lam, steps, trace, ok = eigencount.estimate_lambda_k(A, 5, 50, eigencount.count_signals(g.n), 0)
    assert ok and ev[4] <= lam < ev[5]
    assert round(trace[-1][1]) == 5
    lo, hi = 0.0, 2.0
    for lt, ct in trace:  # tested points are the successive midpoints of the bracket
        assert lt == 0.5 * (lo + hi)
        lo, hi = (lt, hi) if ct < 5 else (lo, lt)


def test_bisection_exhaustion_returns_upper_end(small_sbm):
    g, A, ev, U = small_sbm
    lam, steps, trace, ok = eigencount.estimate_lambda_k(A, 6, 50, 12, 0, max_steps=1)
    assert steps == 1 and len(trace) == 1 and trace[0][0] == 1.0
    if not ok:
        assert lam == (1.0 if trace[0][1] >= 6 else 2.0)


def test_bisection_brackets_lambda_k_on_sbm():
    g = synth.sbm_config(1000, 10)
    ev, _ = _eig(g)
    A, _ = laplacian.normalized_adjacency(g.row_ptr, g.col)
    lam, steps, trace, ok = eigencount.estimate_lambda_k(A, 10, 50, eigencount.count_signals(g.n), 0)
    assert ok and ev[9] <= lam <= ev[10]


# --------------------------------------------------------------- sampling ---

def test_sampling_brute_force_definition():
    N, n, seed = 37, 9, 4
    keys = [int(x) for x in philox.sample_keys(seed, N)]
    ref = sorted(range(N), key=lambda i: (keys[i], i))[:n]
    assert sampling.sample(N, n, seed).tolist() == ref


def test_sampling_distinct_and_uniform():
    N, n = 50, 10
    counts = np.zeros(N)
    first = np.zeros(N)
    for seed in range(3000):
        om = sampling.sample(N, n, seed)
        assert len(set(om.tolist())) == n and om.min() >= 0 and om.max() < N
        counts[om] += 1
        first[om[0]] += 1
    assert st.chisquare(counts).pvalue > 1e-3
    assert st.chisquare(first).pvalue > 1e-3


# ----------------------------------------------------------------- k-means --

def _blobs(seed=0, n=300, d=6, k=4, spread=0.05):
    rng = np.random.default_rng(seed)
    centers = rng.normal(size=(k, d))
    lab = rng.integers(0, k, n)
    return centers[lab] + spread * rng.normal(size=(n, d)), lab


def test_lloyd_matches_sklearn_from_same_init():
    from sklearn.cluster import KMeans

    X, _ = _blobs(spread=0.6, k=5)
    C0 = X[[3, 50, 100, 150, 200]]
    lab, C, inertia = kmeans.lloyd(X, C0, 100)
    km = KMeans(5, init=C0, n_init=1, algorithm="lloyd", tol=0.0, max_iter=100).fit(X)
    assert np.array_equal(lab, km.labels_)
    np.testing.assert_allclose(C, km.cluster_centers_, atol=1e-12)
    assert abs(inertia - km.inertia_) < 1e-9 * inertia


def test_plusplus_second_centre_weights_are_squared_distances():
    X = np.array([[0.0], [1.0], [3.0]])
    hits = {1: 0, 2: 0}
    for seed in range(6000):
        C = kmeans.seed_plusplus(X, 2, seed, 0)
        if C[0, 0] == 0.0:
            hits[int(np.nonzero(X[:, 0] == C[1, 0])[0][0])] += 1
    tot = hits[1] + hits[2]
    assert tot > 1500
    assert abs(hits[2] / tot - 0.9) < 0.03  # D^2 weights 1 : 9; D weights would give 0.75


@pytest.mark.parametrize("n,k", [(2, 2), (33, 5), (100, 10), (922, 40)])
def test_plusplus_pick_is_where_the_exact_prefix_sum_passes_the_target(n, k):
    """Each k-means++ pick is the first point whose running D^2 weight exceeds
    u_c times the total: checked against exactly rounded prefix sums (fsum)
    of squared distances recomputed from the chosen centres, away from
    rounding-level ties."""
    rng = np.random.default_rng(n)
    X = rng.normal(size=(n, 3))
    rec = []
    kmeans.seed_plusplus(X, k, 7, 0, record=rec)
    picks = [p for p, _, _ in rec]
    for c in range(1, k):
        pick, target, cum = rec[c]
        C = X[picks[:c]]
        w = np.min(((X[:, None, :] - C[None, :, :]) ** 2).sum(-1), axis=1)
        exact = np.array([math.fsum(w[: i + 1]) for i in range(n)])
        assert np.all(np.abs(cum - exact) <= n * np.finfo(float).eps * exact[-1])
        u = target / cum[-1]
        t = u * exact[-1]
        above = np.nonzero(exact > t)[0]
        ref = int(above[0]) if above.size else int(np.nonzero(w > 0)[0][-1])
        near = np.min(np.abs(exact - t)) <= 4 * n * np.finfo(float).eps * exact[-1]
        assert pick == ref or near, (c, pick, ref)


def test_kmeans_recovers_blobs_and_picks_lowest_inertia():
    X, lab = _blobs(seed=3, k=6, spread=0.02)
    out, C, inertia = kmeans.kmeans(X, 6, seed=1, replicates=5)
    assert metrics.adjusted_rand_index(out, lab) == 1.0
    inertias = [kmeans.lloyd(X, kmeans.seed_plusplus(X, 6, 1, r), 100)[2] for r in range(5)]
    assert inertia == min(inertias)


def test_empty_cluster_reseeded_with_farthest_point():
    X = np.array([[0.0], [0.1], [10.0]])
    C0 = np.array([[0.05], [100.0]])  # the second centre captures nobody
    lab, C, inertia = kmeans.lloyd(X, C0, 10)
    assert sorted(np.bincount(lab, minlength=2).tolist()) == [1, 2]
    assert lab[2] != lab[0] and lab[0] == lab[1]
    np.testing.assert_allclose(inertia, 2 * 0.05 ** 2, atol=1e-15)


# ------------------------------------------------------------ interpolation --

def test_cg_matches_dense_solve(small_sbm):
    g, A, ev, U = small_sbm
    k, gamma = 6, 1e-3
    omega = sampling.sample(g.n, 40, 2)
    lab_r = np.arange(40) % k
    lc = 0.5 * (ev[5] + ev[6])
    a = jackson.lowpass_coeffs(lc, 50)
    mask = np.zeros(g.n)
    mask[omega] = 1.0
    B = interp.rhs(g.n, omega, lab_r, k)
    X, iters, relres = interp.cg(A, mask, gamma, a, B, tol=1e-10, max_iter=5000)
    H = U @ np.diag(jackson.evaluate(a, ev)) @ U.T
    M = np.diag(mask) + gamma * (np.eye(g.n) - H)
    Xref = np.linalg.solve(M, B)
    assert np.all(relres <= 1e-10)
    cond = np.linalg.cond(M)
    assert np.linalg.norm(X - Xref) <= 10 * cond * 1e-10 * np.linalg.norm(Xref)
    true_res = np.linalg.norm(M @ X - B, axis=0) / np.linalg.norm(B, axis=0)
    assert np.all(true_res < 1e-8)


def test_rhs_places_sampled_indicators():
    B = interp.rhs(6, np.array([4, 1, 3]), np.array([1, 0, 1]), 2)
    ref = np.zeros((6, 2))
    ref[4, 1] = ref[1, 0] = ref[3, 1] = 1.0
    np.testing.assert_array_equal(B, ref)


def test_hard_labels_definition():
    X = np.array([[1.0, 0.0, 0.0], [0.5, 2.0, 0.0], [0.0, 0.0, 0.0], [1.0, 2.0, 0.0]])
    # column norms 1.5 and sqrt(8); column 2 is all zeros and never wins; row 2 ties -> 0
    lab = interp.hard_labels(X)
    assert lab.tolist() == [0, 1, 0, 1]  # 1/1.5 < 2/sqrt(8) on the last row
    assert interp.hard_labels(np.array([[3.0, 3.0]])).tolist() == [0]


# ----------------------------------------------------------------- metrics --

def test_ari_matches_sklearn():
    from sklearn.metrics import adjusted_rand_score

    rng = np.random.default_rng(0)
    for _ in range(20):
        a = rng.integers(0, 5, 200)
        b = np.where(rng.random(200) < 0.7, a, rng.integers(0, 7, 200))
        assert abs(metrics.adjusted_rand_index(a, b) - adjusted_rand_score(a, b)) < 1e-12
    assert metrics.adjusted_rand_index([0, 0, 1, 1], [5, 5, 2, 2]) == 1.0


# -------------------------------------------------------- whole algorithm ---

def test_global_coherence_of_equal_disconnected_blocks():
    # Sec. 3.2.3: for k equal disconnected regular clusters nu_k = sqrt(k)
    g = synth.disconnected_regular(4, 50, 5, seed=1)
    ev, U = _eig(g)
    v = np.linalg.norm(U[:, :4], axis=1)
    assert abs(math.sqrt(g.n) * v.max() - 2.0) < 1e-9


@pytest.mark.parametrize("seed", range(10))
def test_csc_recovers_disconnected_blocks(seed):
    g = synth.disconnected_regular(6, 80, 6, seed=seed)
    d = int(math.ceil(4 * math.log(g.n)))
    r = ocsc.run(g.row_ptr, g.col, 6, d, seed, replicates=5)
    assert metrics.adjusted_rand_index(r.labels, g.truth) == 1.0
    assert np.all(r.cg_relres <= 1e-6)


def test_csc_on_plain_config_recovers_communities():
    g = synth.sbm_config(1000, 10)
    r = ocsc.run(g.row_ptr, g.col, 10, int(math.ceil(4 * math.log(1000))), 0)
    assert metrics.adjusted_rand_index(r.labels, g.truth) > 0.9
    assert len(set(r.omega.tolist())) == ocsc.default_n(10) == 47


def test_jl_distance_preservation_ideal_filter():
    # Thm 3.2 with eps = 0.5, beta = 1: d > (4 + 2 beta) / (eps^2/2 - eps^3/3) log N
    g = synth.sbm_config(150, 3, s=10.0, seed=5)
    ev, U = _eig(g)
    k = 3
    Uk = U[:, :k]
    v = np.linalg.norm(Uk, axis=1)
    eps, beta = 0.5, 1.0
    d = int(math.ceil((4 + 2 * beta) / (eps ** 2 / 2 - eps ** 3 / 3) * math.log(g.n)))
    Yk = Uk / v[:, None]
    fails = 0
    trials = 10
    for t in range(trials):
        R = philox.gaussian_block(t, g.n, d, 0, philox.FEAT)
        Ft = (Uk @ (Uk.T @ R)) / v[:, None]
        D = np.linalg.norm(Yk[:, None, :] - Yk[None, :, :], axis=2)
        Dt = np.linalg.norm(Ft[:, None, :] - Ft[None, :, :], axis=2)
        m = D > 1e-9
        ratio = Dt[m] / D[m]
        fails += int(not (ratio.min() >= 1 - eps and ratio.max() <= 1 + eps))
    assert fails <= max(1, int(trials * g.n ** -beta * 10))


def test_golden_fixtures_parse():
    sizes = [int(x) for x in open(os.path.join(GOLDEN, "hetero_sizes.txt")).read().split("\n")[1].split()]
    assert len(sizes) == 20 and sum(sizes) == 1000
    g = synth.sbm(1000, 20, 16.0, 0.02, seed=0, sizes=sizes)
    assert np.bincount(g.truth).tolist() == sizes
    d = json.load(open(os.path.join(GOLDEN, "alg2_defaults.json")))
    assert d["p"] == 50 and d["gamma"] == 1e-3


def test_clenshaw_filter_equals_forward_recurrence_and_spectral_definition():
    from oracle import cheb, jackson, laplacian

    g = synth.sbm_config(400, 5, seed=7)
    A, _ = laplacian.normalized_adjacency(g.row_ptr, g.col)
    X = np.random.default_rng(1).normal(size=(g.n, 3))
    for lam, p in ((0.3, 50), (1.2, 7), (0.05, 1), (0.7, 2)):
        a = jackson.lowpass_coeffs(lam, p)
        Yc = cheb.filter_block_clenshaw(A, X, a)
        Yf = cheb.filter_block(A, X, a)
        assert np.linalg.norm(Yc - Yf) <= 1e-12 * np.linalg.norm(Yf)
        ev, U = np.linalg.eigh(laplacian.laplacian_dense(g.row_ptr, g.col))
        h = np.polynomial.chebyshev.chebval(ev - 1.0, a)
        Yd = U @ (h[:, None] * (U.T @ X))
        assert np.linalg.norm(Yc - Yd) <= 1e-10 * np.linalg.norm(Yd)
    a0 = np.array([0.25])
    assert np.array_equal(cheb.filter_block_clenshaw(A, X, a0), 0.25 * X)


def test_one_pass_kpm_dichotomy():
    from oracle import eigencount, laplacian

    g = synth.disconnected_regular(5, 60, 6, seed=2)
    A, _ = laplacian.normalized_adjacency(g.row_ptr, g.col)
    ev = np.linalg.eigvalsh(laplacian.laplacian_dense(g.row_ptr, g.col))
    lam, steps, trace, conv, mu = eigencount.estimate_lambda_k_kpm(A, 5, 50, 400, 0)
    assert conv and ev[4] - 1e-9 <= lam < ev[5]
    # the first tested point is the plain dichotomy's first pass, count for count
    plam, psteps, ptrace, pconv = eigencount.estimate_lambda_k(A, 5, 50, 400, 0)
    assert abs(trace[0][1] - ptrace[0][1]) <= 1e-9 * max(1.0, abs(ptrace[0][1]))
    # every count is the Hutchinson count of the pass's signals at that lambda
    R = philox.gaussian_block(0, g.n, 400, 1, philox.COUNT)
    for lt, ct in trace[:4]:
        assert abs(eigencount.eigencount(A, lt, 50, R) - ct) <= 1e-9 * max(1.0, abs(ct))


def test_chebyshev_doubling_identities_for_moments():
    """The GPU's eigencount pass forms mu_0..mu_p from T_0..T_ceil(p/2) by
    T_{2j} = 2 T_j^2 - 1 and T_{2j+1} = 2 T_j T_{j+1} - T_1 (A symmetric, so
    <R, T_{2j} R> = 2 <T_j R, T_j R> - <R, R> and likewise for odd orders);
    check the identities on the oracle's own terms."""
    gr = synth.sbm_config(300, 3, seed=5)
    A, _ = laplacian.normalized_adjacency(gr.row_ptr, gr.col)
    R = philox.gaussian_block(3, gr.n, 6, 1, philox.COUNT)
    p = 21
    T = list(cheb.chebyshev_terms(A, R, p))
    mu = cheb.moments(A, R, p)
    dot = lambda X, Y: float(np.sum(X * Y))
    for m in range(p + 1):
        j = m // 2
        est = (2 * dot(T[j], T[j]) - dot(T[0], T[0])) if m % 2 == 0 and m > 0 else \
              (2 * dot(T[j], T[j + 1]) - dot(T[0], T[1])) if m % 2 == 1 and m > 1 else mu[m]
        assert abs(est - mu[m]) <= 1e-12 * mu[0], (m, est, mu[m])
