"""Precision form: float32 recurrences and SpMM, float64 only for the
eigencount moments and the CG inner products and norms.  Reports the error of
every result of Alg. 2 against the float64 oracle on the same seeded inputs
(printed with -s) and bounds it."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import cheb, eigencount, interp, jackson, kmeans, laplacian, metrics, philox, sampling
from oracle import csc as ocsc

pytestmark = pytest.mark.gpu


def test_per_result_error_against_float64():
    from paper_1602_02018_amd import api

    gr = synth.sbm_config(1000, 10, seed=0)
    A, _ = laplacian.normalized_adjacency(gr.row_ptr, gr.col)
    g = api.Graph(gr.row_ptr, gr.col)
    k, p, seed = 10, 50, 0
    d = int(math.ceil(4 * math.log(gr.n)))
    n_c = eigencount.count_signals(gr.n)
    rep = {}

    # eigencount moments and counts
    _, mom = api.eigencount(g, 0.5, p, n_c, seed, 1)
    mref = cheb.moments(A, philox.gaussian_block(seed, gr.n, n_c, 1, philox.COUNT), p)
    rep["moments max |err| / mu_0"] = float(np.max(np.abs(mom - mref)) / mref[0])
    counts = [(lam, float(np.dot(jackson.lowpass_coeffs(lam, p), mom)),
               float(np.dot(jackson.lowpass_coeffs(lam, p), mref))) for lam in (0.25, 0.4, 0.5, 1.0)]
    rep["count max |err|"] = max(abs(a - b) for _, a, b in counts)

    # dichotomy
    bis = api.estimate_lambda_k(g, k, p, n_c, seed)
    lam_ref, steps_ref, _, _ = eigencount.estimate_lambda_k(A, k, p, n_c, seed)
    rep["lambda_k |err|"] = abs(bis.lam - lam_ref)

    # features (unit rows, all nodes)
    F = api.filter(g, lam_ref, p, d, seed).cpu().numpy()
    Fref = ocsc.features(A, lam_ref, p, d, seed)
    rep["features rel Frobenius err"] = float(np.linalg.norm(F - Fref) / np.linalg.norm(Fref))

    # k-means labels from the float32 features vs from the float64 features
    omega = sampling.sample(gr.n, ocsc.default_n(k), seed)
    lab32, _ = api.kmeans_reduced(F[omega].astype(np.float64), k, seed)
    lab64, _, _ = kmeans.kmeans(Fref[omega], k, seed)
    rep["sampled labels ARI (f32 vs f64 features)"] = metrics.adjusted_rand_index(lab32, lab64)

    # interpolation: the side-by-side CGs against the oracle's (same iteration),
    # the block CG against the solution the oracle reaches at tolerance 1e-12
    res = api.interpolate(g, lam_ref, p, 1e-3, omega, lab64, k, method=0)
    X, lab, _, _ = interp.interpolate(A, lam_ref, p, 1e-3, omega, lab64, k)
    Xg = res.X.cpu().numpy()
    rep["X rel Frobenius err"] = float(np.linalg.norm(Xg - X) / np.linalg.norm(X))
    rep["labels ARI vs float64"] = metrics.adjusted_rand_index(res.labels.cpu().numpy(), lab)
    rb = api.interpolate(g, lam_ref, p, 1e-3, omega, lab64, k, method=1)
    Xt, _, _, _ = interp.interpolate(A, lam_ref, p, 1e-3, omega, lab64, k, tol=1e-12)
    rep["block CG X rel err vs tight solve"] = float(np.linalg.norm(rb.X.cpu().numpy() - Xt)
                                                     / np.linalg.norm(Xt))
    rep["side-by-side CG X rel err vs tight solve"] = float(np.linalg.norm(Xg - Xt) / np.linalg.norm(Xt))
    rep["block CG labels ARI vs float64"] = metrics.adjusted_rand_index(rb.labels.cpu().numpy(), lab)

    for key, val in rep.items():
        print(f"{key:45s} {val:.3e}")
    assert rep["moments max |err| / mu_0"] <= 1e-5
    assert rep["count max |err|"] <= 1e-2
    assert rep["lambda_k |err|"] <= 2.0 / 2 ** min(bis.steps, steps_ref)
    assert rep["features rel Frobenius err"] <= 1e-4
    assert rep["sampled labels ARI (f32 vs f64 features)"] >= 0.99
    assert rep["X rel Frobenius err"] <= 1e-3
    assert rep["labels ARI vs float64"] >= 0.99
    assert rep["block CG X rel err vs tight solve"] <= 1e-3
    assert rep["block CG labels ARI vs float64"] >= 0.99


@pytest.mark.parametrize("N,k,seed", [(1000, 10, 0), (20000, 40, 3)])
def test_block_products_float32_against_float64(N, k, seed):
    """The block CG's residual update with float32 sums (CSC_TUNE_BLOCK_PRODUCT
    = 1) against float64 sums (0; the other right products sum in float32
    either way) and against the oracle's solution at
    tolerance 1e-12: both meet the tolerance on the recursive residual, the
    float64 true residual stays below 1e-4, X lies within 1e-3 of the tight
    solve and the labels agree.  Also reports what float32 row norms would
    change in the unit-norm features."""
    from paper_1602_02018_amd import _lib, api

    gr = synth.sbm_config(N, k, seed=seed)
    A, _ = laplacian.normalized_adjacency(gr.row_ptr, gr.col)
    g = api.Graph(gr.row_ptr, gr.col)
    p, d = 50, int(math.ceil(4 * math.log(gr.n)))
    n_c = eigencount.count_signals(gr.n)
    lam, _, _, _ = eigencount.estimate_lambda_k(A, k, p, n_c, seed)
    omega = sampling.sample(gr.n, ocsc.default_n(k), seed)
    lab_r, _, _ = kmeans.kmeans(ocsc.features(A, lam, p, d, seed)[omega], k, seed)
    Xt, lab_t, _, _ = interp.interpolate(A, lam, p, 1e-3, omega, lab_r, k, tol=1e-12)
    mask = interp.sample_mask(gr.n, omega)
    a = jackson.lowpass_coeffs(lam, p)
    B = interp.rhs(gr.n, omega, lab_r, k)
    rep = {}
    out = {}
    saved = api.get_tuning(_lib.TUNE_BLOCK_PRODUCT)
    try:
        for f32 in (0, 1):
            api.set_tuning(_lib.TUNE_BLOCK_PRODUCT, f32)
            res = api.interpolate(g, lam, p, 1e-3, omega, lab_r, k)
            X = res.X.cpu().numpy().astype(np.float64)
            true = np.linalg.norm(B - interp.apply_operator(A, mask, 1e-3, a, X), axis=0) \
                / np.linalg.norm(B, axis=0)
            tag = "f32" if f32 else "f64"
            rep[f"{tag} products: iterations"] = float(res.iters.max())
            rep[f"{tag} products: max recursive relres"] = float(res.relres.max())
            rep[f"{tag} products: max true relres"] = float(true.max())
            rep[f"{tag} products: X rel err vs tight solve"] = float(np.linalg.norm(X - Xt) / np.linalg.norm(Xt))
            rep[f"{tag} products: labels ARI vs tight solve"] = metrics.adjusted_rand_index(
                res.labels.cpu().numpy(), lab_t)
            out[tag] = (res, X, true)
    finally:
        api.set_tuning(_lib.TUNE_BLOCK_PRODUCT, saved)
    # float32 row norms of the same unnormalized features
    Y = api.filter(g, lam, p, d, seed, normalize=False).cpu().numpy()
    F64 = api.filter(g, lam, p, d, seed, normalize=True).cpu().numpy()
    nrm32 = np.sqrt(np.sum(Y * Y, axis=1, dtype=np.float32), dtype=np.float32)
    F32 = np.where(nrm32[:, None] > 0, Y / np.maximum(nrm32, np.float32(1e-30))[:, None], 0).astype(np.float32)
    rep["features: float32 vs float64 row norms, rel Frobenius"] = float(
        np.linalg.norm(F32.astype(np.float64) - F64) / np.linalg.norm(F64))
    for key, val in rep.items():
        print(f"{key:55s} {val:.3e}")
    for tag in ("f64", "f32"):
        res, X, true = out[tag]
        assert res.status == 0 and np.all(res.relres <= 1e-6), tag
        assert true.max() <= 1e-4, tag
        assert rep[f"{tag} products: X rel err vs tight solve"] <= 1e-3, tag
        assert rep[f"{tag} products: labels ARI vs tight solve"] >= 0.99, tag
    assert rep["features: float32 vs float64 row norms, rel Frobenius"] <= 1e-6
