"""Pins of variable-density sampling and the weighted decoder (oracle)."""
import math

import numpy as np
import pytest
import scipy.stats as st

import synth
from oracle import csc, interp, jackson, laplacian, metrics, sampling


def test_keys_are_an_exponential_race():
    # key_i = E_i / w_i with E_i ~ Exp(1): P(node i has the smallest key) = w_i / sum(w)
    w = np.array([1.0, 2.0, 3.0, 4.0])
    first = np.array([np.argmin(sampling.density_keys(w, s)) for s in range(4000)])
    obs = np.bincount(first, minlength=4)
    chi2 = st.chisquare(obs, 4000 * w / w.sum())
    assert chi2.pvalue > 1e-3


def test_inclusion_probabilities_of_successive_sampling():
    # n = 2 of N = 4: P(i in Omega) = sum over ordered pairs, drawn successively
    w = np.array([1.0, 2.0, 3.0, 6.0])
    W = w.sum()
    incl = np.zeros(4)
    for a in range(4):
        for b in range(4):
            if a != b:
                pr = w[a] / W * w[b] / (W - w[a])
                incl[a] += pr
                incl[b] += pr
    trials = 6000
    cnt = np.zeros(4)
    for s in range(trials):
        om, _ = sampling.sample_density(w, 2, s)
        cnt[om] += 1
    np.testing.assert_allclose(cnt / trials, incl, atol=0.025)


def test_equal_weights_sample_uniformly():
    N, n = 50, 5
    first = np.array([sampling.sample_density(np.ones(N), n, s)[0][0] for s in range(3000)])
    assert st.chisquare(np.bincount(first, minlength=N)).pvalue > 1e-3
    om, dw = sampling.sample_density(np.full(N, 7.0), n, 3)
    assert len(set(om.tolist())) == n and np.all(dw == 1.0)


def test_zero_weights_come_last():
    w = np.array([0.0, 1.0, 0.0, 2.0, 0.0])
    om, dw = sampling.sample_density(w, 4, 1)
    assert set(om[:2].tolist()) == {1, 3}
    assert om[2:].tolist() == [0, 2]  # +inf keys, index order
    assert np.all(dw[2:] == 0.0)


def test_decoder_weights_are_inverse_scaled_probabilities():
    w = np.array([1.0, 2.0, 5.0, 0.5, 1.5])
    om, dw = sampling.sample_density(w, 3, 2)
    p = w / w.sum()
    np.testing.assert_allclose(dw, 1.0 / (w.size * p[om]), rtol=1e-15)


def test_weighted_decoder_solves_the_weighted_normal_equations():
    g = synth.sbm_config(300, 4, seed=1)
    A, _ = laplacian.normalized_adjacency(g.row_ptr, g.col)
    N, k, lam, p, gamma = g.n, 4, 0.3, 30, 1e-2
    rng = np.random.default_rng(0)
    omega = rng.choice(N, 20, replace=False)
    lab_r = rng.integers(0, k, 20)
    wts = rng.uniform(0.5, 3.0, 20)
    X, _, _, _ = interp.interpolate(A, lam, p, gamma, omega, lab_r, k, tol=1e-12, weights=wts)
    # dense solve: (M^T W M + gamma (I - h~(L))) X = M^T W C
    a = jackson.lowpass_coeffs(lam, p)
    Hd = laplacian.chebyshev_dense(A, a) if hasattr(laplacian, "chebyshev_dense") else None
    from oracle import cheb
    H = cheb.filter_block(A, np.eye(N), a)
    Mw = np.diag(interp.sample_mask(N, omega, wts)) + gamma * (np.eye(N) - H)
    Xd = np.linalg.solve(Mw, interp.rhs(N, omega, lab_r, k, wts))
    assert np.linalg.norm(X - Xd) <= 1e-8 * np.linalg.norm(Xd)
    # unit weights are the unweighted decoder exactly
    X1, _, _, _ = interp.interpolate(A, lam, p, gamma, omega, lab_r, k, tol=1e-12, weights=np.ones(20))
    X0, _, _, _ = interp.interpolate(A, lam, p, gamma, omega, lab_r, k, tol=1e-12)
    assert np.array_equal(X1, X0)


def _regular_blocks(sizes, degree=6):
    """Disconnected random regular blocks of the given sizes (expanders: a clear gap above 0)."""
    rows, cols, truth, off = [], [], [], 0
    for b, m in enumerate(sizes):
        g = synth.disconnected_regular(1, m, degree, seed=b)
        deg = np.diff(g.row_ptr)
        rows.append(np.repeat(np.arange(m), deg) + off)
        cols.append(g.col + off)
        truth += [b] * m
        off += m
    row_ptr, col = synth.csr_from_edges(off, np.concatenate(rows), np.concatenate(cols))
    return row_ptr, col, np.array(truth)


def test_density_sampling_follows_the_coherence_on_heterogeneous_blocks():
    # disconnected blocks of very different sizes: v_k(i)^2 = 1 / |block(i)|
    # (Sec. 3.2.3), so density sampling gives every block about the same share
    sizes = [20, 40, 80, 160, 320]
    row_ptr, col, truth = _regular_blocks(sizes)
    A, _ = laplacian.normalized_adjacency(row_ptr, col)
    F, sq = csc.features(A, 0.1, 50, 40, 0, with_norms=True)
    per_block = np.array([sq[truth == b].mean() for b in range(5)]) * np.array(sizes)
    assert per_block.max() / per_block.min() < 1.6  # mean squared norm ~ 1 / block size
    counts = np.zeros(5)
    for s in range(30):
        om, _ = sampling.sample_density(sq, 15, s)
        counts += np.bincount(truth[om], minlength=5)
    assert counts.min() >= 0.5 * counts.mean()  # uniform sampling would give 20 : 320


def test_end_to_end_density_on_disconnected_blocks():
    gr = synth.disconnected_regular(6, 80, 6, seed=3)
    d = int(math.ceil(4 * math.log(gr.n)))
    res = csc.run(gr.row_ptr, gr.col, 6, d, 3, replicates=5, sampling="density")
    assert metrics.adjusted_rand_index(res.labels, gr.truth) == 1.0
