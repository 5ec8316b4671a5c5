"""A reduced parameter sweep (the trends of Fig. 1): perfect recovery without
inter-community edges, recovery falling as eps grows, order p = 50 at least as
good as p = 10, and the undamped series run against the float64 oracle."""
import numpy as np
import pytest
import torch

import synth
from oracle import cheb, jackson, laplacian

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_1602_02018_amd import api as a

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    yield a
    a.set_damping(0)


def test_reduced_sweep_trends(api):
    from paper_1602_02018_amd import sweeps

    rows = sweeps.sweep(api, [0.0, 0.5], 2, grid={"p": [10, 50], "damping": [0, 1]})
    get = {(r["eps_frac"], r["param"], r["value"]): r for r in rows}
    assert get[(0.0, "p", 50)]["ari_mean"] >= 0.99
    assert get[(0.5, "p", 50)]["ari_mean"] <= get[(0.0, "p", 50)]["ari_mean"] + 1e-9
    assert get[(0.5, "p", 50)]["ari_mean"] >= get[(0.5, "p", 10)]["ari_mean"] - 0.02
    # Fig. 1 e: the estimate sits between lambda_k and lambda_k+1 when the gap is clear
    r0 = get[(0.0, "p", 50)]
    assert r0["lam_k_mean"] - 1e-6 <= r0["lam_est_mean"] <= r0["lam_k1_mean"]


def test_undamped_filter_matches_oracle(api):
    gr = synth.sbm_config(1000, 10, seed=0)
    A, _ = laplacian.normalized_adjacency(gr.row_ptr, gr.col)
    g = api.Graph(gr.row_ptr, gr.col)
    X = api.gaussian_block(gr.n, 12, 3, 0, 2)
    a = jackson.lowpass_coeffs(0.4, 50, damping=False)
    Y = api.filter_block(g, a, X).cpu().numpy()
    ref = cheb.filter_block(A, X.cpu().numpy().astype(np.float64), a)
    assert np.linalg.norm(Y - ref) <= 1e-4 * np.linalg.norm(ref)
    api.set_damping(1)
    try:
        assert np.allclose(api.jackson_coeffs(0.4, 50), a, rtol=1e-13, atol=1e-15)
        cnt, mom = api.eigencount(g, 0.4, 50, 14, 0, 1)
        assert abs(cnt - float(np.dot(a, mom))) <= 1e-9 * max(1.0, abs(cnt))
    finally:
        api.set_damping(0)
