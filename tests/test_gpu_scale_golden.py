"""The library against the float64 oracle's stored results at full size.

The files in tests/golden/ are written by tests/golden/make_scale_goldens.py,
which runs only the oracle (Alg. 2 step by step) on the seeded workloads:

* the 1e5-node SBM (k = 100, p = 50): every step of Alg. 2 and the end-to-end
  labels;
* the 1e6-node Chung-Lu graph (k = 250, p = 60): the dichotomy, the first
  pass's moments, sampling, the features of the sampled nodes and two columns
  of the interpolation (the float64 oracle cannot afford all 250);
* 8 graphs of the batch of 64 SBMs, smallest to largest: the plain and the
  learned-bracket pipelines, run here through the batched calls and the
  single calls.

Tolerances (float32 recurrences against float64): moments 1e-5 mu_0; counts
1e-3 (1 + |count|), and each dichotomy decision equal unless the oracle's count
lies within twice that margin of k - 1/2, k + 1/2 or k (then the estimates
stay within the interval of that test); sampled nodes bit-exact; features
1e-4 relative Frobenius; interpolated columns within 1e-3 of the oracle's
solution to 1e-10 (relative, on the stored rows); labels ARI >= 0.99 against
the labels of the oracle's solve to 1e-10 whenever the two estimates of
lambda_k agree (the side-by-side CGs, the oracle's own algorithm, against
the oracle's CG at 1e-6).
"""
import os
import math

import numpy as np
import pytest
import torch

import search_compare
import synth
from oracle.metrics import adjusted_rand_index

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    path = os.path.join(GOLD, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not written (tests/golden/make_scale_goldens.py)")
    return np.load(path)


@pytest.fixture(scope="module")
def api():
    from paper_1602_02018_amd import api as a

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return a


def compare_search(trace, lam, steps, gold, prefix, k, mid_tol=0.0, tol=1e-3):
    """The library's search against the stored oracle search (tests/search_compare.py)."""
    return search_compare.compare_search(
        trace, lam, steps, gold[prefix + "trace"], gold[prefix + "intervals"],
        float(gold[prefix + "lam"]), int(gold[prefix + "steps"]), k,
        bool(gold[prefix + "missed"]), mid_tol, tol)


def rel_cols(X_gpu_rows, X_ref_rows):
    return np.linalg.norm(X_gpu_rows - X_ref_rows, axis=0) / np.linalg.norm(X_ref_rows, axis=0)


# ------------------------------------------------------ SBM N = 1e5 -----

@pytest.fixture(scope="module")
def sbm():
    gold = _load("scale_sbm_1e5.npz")
    gr = synth.sbm_config(int(gold["N"]), int(gold["k"]), seed=int(gold["seed"]))
    assert gr.nnz == int(gold["nnz"])
    return gr, gold


def test_sbm_1e5_dichotomy_and_moments(api, sbm):
    gr, gold = sbm
    g = api.Graph(gr.row_ptr, gr.col)
    k, p, nc, seed = int(gold["k"]), int(gold["p"]), int(gold["n_c"]), int(gold["seed"])
    res = api.estimate_lambda_k(g, k, p, nc, seed)
    compare_search(res.trace, res.lam, res.steps, gold, "", k)
    mu = gold["moments1"]
    assert np.max(np.abs(res.moments - mu)) <= 1e-5 * mu[0]


def test_sbm_1e5_sampling_features_kmeans(api, sbm):
    gr, gold = sbm
    g = api.Graph(gr.row_ptr, gr.col)
    k, p, d, seed, lam = int(gold["k"]), int(gold["p"]), int(gold["d"]), int(gold["seed"]), float(gold["lam"])
    omega = api.sample(gr.n, api.default_n(k), seed)
    assert np.array_equal(omega.cpu().numpy(), gold["omega"])
    F = api.filter(g, lam, p, d, seed, rows=omega)
    Fr = gold["features_sampled"]
    err = np.linalg.norm(F.cpu().numpy() - Fr) / np.linalg.norm(Fr)
    assert err <= 1e-4, err
    lab, _ = api.kmeans_reduced_device(F.contiguous(), k, seed)
    assert adjusted_rand_index(lab, gold["labels_r"]) >= 0.99


def test_sbm_1e5_interpolation_columns(api, sbm):
    gr, gold = sbm
    g = api.Graph(gr.row_ptr, gr.col)
    k, p, lam = int(gold["k"]), int(gold["p"]), float(gold["lam"])
    it = api.interpolate(g, lam, p, 1e-3, gold["omega"], gold["labels_r"], k)
    assert it.status == 0 and np.all(it.relres <= 1e-6)
    rows, cols = gold["x_rows"], gold["x_cols"]
    X = it.X.cpu().numpy().astype(np.float64)[rows][:, cols]
    err = rel_cols(X, gold["X_exact_at_rows"])
    assert np.all(err <= 1e-3), err
    # the labels of Eq. (5)'s solution against the oracle's, from the same
    # inputs: the block CG against the oracle's solve to 1e-10, the
    # side-by-side CGs (the oracle's own algorithm) against its CG at 1e-6
    assert adjusted_rand_index(it.labels.cpu().numpy(), gold["labels_tight"]) >= 0.99
    itc = api.interpolate(g, lam, p, 1e-3, gold["omega"], gold["labels_r"], k, method=api.CG_COLUMNS)
    assert adjusted_rand_index(itc.labels.cpu().numpy(), gold["labels"]) >= 0.99


def test_sbm_1e5_end_to_end(api, sbm):
    gr, gold = sbm
    g = api.Graph(gr.row_ptr, gr.col)
    k, p, d, seed = int(gold["k"]), int(gold["p"]), int(gold["d"]), int(gold["seed"])
    res = api.run(g, k, d, seed, p=p)
    same = compare_search(res.bisection.trace, res.lam, res.bisection.steps, gold, "", k)
    assert np.array_equal(res.omega.cpu().numpy(), gold["omega"])
    if same:
        assert adjusted_rand_index(res.labels.cpu().numpy(), gold["labels_tight"]) >= 0.99


# ------------------------------------------------- Chung-Lu N = 1e6 -----

@pytest.fixture(scope="module")
def chunglu():
    gold = _load("scale_chunglu_1e6.npz")
    gr = synth.chung_lu_blocks(int(gold["N"]), int(gold["k"]), seed=int(gold["seed"]))
    assert gr.nnz == int(gold["nnz"])
    return gr, gold


@pytest.mark.slow
def test_chunglu_1e6_dichotomy_and_moments(api, chunglu):
    gr, gold = chunglu
    g = api.Graph(gr.row_ptr, gr.col)
    k, p, nc, seed = int(gold["k"]), int(gold["p"]), int(gold["n_c"]), int(gold["seed"])
    res = api.estimate_lambda_k(g, k, p, nc, seed)
    compare_search(res.trace, res.lam, res.steps, gold, "", k)
    mu = gold["moments1"]
    assert np.max(np.abs(res.moments - mu)) <= 1e-5 * mu[0]


@pytest.mark.slow
def test_chunglu_1e6_sampling_and_features(api, chunglu):
    gr, gold = chunglu
    g = api.Graph(gr.row_ptr, gr.col)
    k, p, d, seed, lam = int(gold["k"]), int(gold["p"]), int(gold["d"]), int(gold["seed"]), float(gold["lam"])
    omega = api.sample(gr.n, api.default_n(k), seed)
    assert np.array_equal(omega.cpu().numpy(), gold["omega"])
    F = api.filter(g, lam, p, d, seed, rows=omega)
    Fr = gold["features_sampled"]
    err = np.linalg.norm(F.cpu().numpy() - Fr) / np.linalg.norm(Fr)
    assert err <= 1e-4, err
    # the all-row (Clenshaw) feature pass the pipeline runs, at the same rows
    Fa = api.filter(g, lam, p, d, seed, rows=None)
    Fa = Fa[omega.long()].cpu().numpy()
    err = np.linalg.norm(Fa - Fr) / np.linalg.norm(Fr)
    assert err <= 1e-4, err


@pytest.mark.slow
def test_chunglu_1e6_interpolation_columns(api, chunglu):
    gr, gold = chunglu
    g = api.Graph(gr.row_ptr, gr.col)
    k, p, lam = int(gold["k"]), int(gold["p"]), float(gold["lam"])
    it = api.interpolate(g, lam, p, 1e-3, gold["omega"], gold["labels_r"], k)
    assert it.status == 0 and np.all(it.relres <= 1e-6)
    rows, cols = gold["x_rows"], gold["x_cols"]
    X = it.X.cpu().numpy().astype(np.float64)[rows][:, cols]
    err = rel_cols(X, gold["X_at_rows"])
    assert np.all(err <= 1e-3), err


# ---------------------------------------- 8 graphs of the batch of 64 -----

@pytest.fixture(scope="module")
def batch8():
    gold = _load("scale_batch8.npz")
    pos = [int(x) for x in gold["positions"]]
    if f"g{pos[0]}_plain_labels_tight" not in gold.files:
        pytest.skip("scale_batch8.npz predates the solves to 1e-10 (tests/golden/make_scale_goldens.py)")
    gs = synth.sbm_batch(only=pos)
    for gi, gr in zip(pos, gs):
        assert gr.n == int(gold[f"g{gi}_N"]) and gr.nnz == int(gold[f"g{gi}_nnz"])
    return pos, gs, gold


def _batch_inputs(api, batch8):
    pos, gs, gold = batch8
    G = [api.Graph(gr.row_ptr, gr.col) for gr in gs]
    ks = [gr.k for gr in gs]
    ds = [int(math.ceil(4 * math.log(gr.n))) for gr in gs]
    return pos, gs, gold, G, ks, ds, pos  # graph g of the batch is seeded g


def _check_pipeline(api, g, res, gold, gi, prefix, k, mid_tol):
    """One graph's pipeline against the oracle's: the search; the samples;
    and, when the two estimates agree, the k-means labels of the sampled
    nodes, the interpolation from the oracle's own inputs and the final
    labels, both against the labels of the oracle's solve to 1e-10 (the block
    CG meets 1e-6 by another path than the oracle's CG, and on graphs with
    many nearly tied nodes two 1e-6 solutions can label a few percent of the
    nodes differently)."""
    same = compare_search(res.bisection.trace, res.lam, res.bisection.steps, gold, f"g{gi}_{prefix}",
                          k, mid_tol=mid_tol)
    assert np.array_equal(res.omega.cpu().numpy(), gold[f"g{gi}_plain_omega"])
    if not same:
        return False
    lab_r = gold[f"g{gi}_{prefix}labels_r"]
    tight = gold[f"g{gi}_{prefix}labels_tight"]
    assert adjusted_rand_index(res.labels_r, lab_r) >= 0.99, (gi, prefix)
    it = api.interpolate(g, res.lam, 50, 1e-3, gold[f"g{gi}_plain_omega"], lab_r, k)
    ari_i = adjusted_rand_index(it.labels.cpu().numpy(), tight)
    ari = adjusted_rand_index(res.labels.cpu().numpy(), tight)
    print(f"graph {gi} {prefix}: interpolation from the oracle's inputs ARI {ari_i:.4f}, end to end {ari:.4f}")
    assert ari_i >= 0.99, (gi, prefix, ari_i)
    assert ari >= 0.99, (gi, prefix, ari)
    return True


def test_batch8_plain_batched_and_single(api, batch8):
    pos, gs, gold, G, ks, ds, seeds = _batch_inputs(api, batch8)
    out = api.run_batched(G, ks, ds, seeds, p=50)
    for gi, g, k, res in zip(pos, G, ks, out):
        _check_pipeline(api, g, res, gold, gi, "plain_", k, 0.0)
    for gi, g, k, d, s in zip(pos, G, ks, ds, seeds):
        _check_pipeline(api, g, api.run(g, k, d, s, p=50), gold, gi, "plain_", k, 0.0)


def test_batch8_learned_batched_and_single(api, batch8):
    from paper_1602_02018_amd import learned

    pos, gs, gold, G, ks, ds, seeds = _batch_inputs(api, batch8)
    mlp = learned.load_params("cuda")
    out = api.run_batched(G, ks, ds, seeds, p=50, mlp_params=mlp)
    agree = 0
    for gi, g, k, res in zip(pos, G, ks, out):
        agree += _check_pipeline(api, g, res, gold, gi, "learned_", k, 2e-5)
    for gi, g, k, d, s in zip(pos, G, ks, ds, seeds):
        _check_pipeline(api, g, api.run(g, k, d, s, p=50, mlp_params=mlp), gold, gi, "learned_", k, 2e-5)
    assert agree >= 6  # a near-tie may part at most a few searches
