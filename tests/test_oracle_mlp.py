"""Pins of the float64 bracket-network oracle against torch (float64, CPU) and
finite differences, and of its input features against the exact spectral
density of a small graph."""
import math

import numpy as np
import torch

import synth
from oracle import cheb, eigencount, jackson, laplacian, mlp, philox


def _theta(seed=0, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.normal(scale=scale, size=mlp.N_PARAMS)


def _torch_net(theta):
    W1, b1, W2, b2, W3, b3 = [torch.tensor(a, dtype=torch.float64, requires_grad=True)
                              for a in mlp.unpack(theta)]
    params = [W1, b1, W2, b2, W3, b3]

    def f(X):
        h = torch.nn.functional.gelu(X @ W1 + b1)
        h = torch.nn.functional.gelu(h @ W2 + b2)
        return h @ W3 + b3

    return f, params


def _torch_pinball(Y, t):
    L = 0.0
    for j, tau in enumerate(mlp.TAUS):
        u = t - Y[:, j]
        L = L + torch.sum(u * (tau - (u < 0).double()))
    return L / Y.shape[0]


def test_parameter_count():
    assert mlp.N_PARAMS == 23554


def test_forward_matches_torch():
    theta = _theta()
    X = np.random.default_rng(1).normal(size=(33, mlp.D_IN))
    f, _ = _torch_net(theta)
    Y, _ = mlp.forward(theta, X)
    np.testing.assert_allclose(Y, f(torch.tensor(X)).detach().numpy(), rtol=1e-12, atol=1e-12)


def test_gradients_match_torch_autograd():
    theta = _theta(2)
    X = np.random.default_rng(3).normal(size=(40, mlp.D_IN))
    t = np.random.default_rng(4).uniform(0, 1, size=40)
    L, g = mlp.loss_and_grad(theta, X, t)
    f, params = _torch_net(theta)
    Lt = _torch_pinball(f(torch.tensor(X)), torch.tensor(t))
    Lt.backward()
    gt = np.concatenate([p.grad.numpy().ravel() for p in params])
    assert abs(L - Lt.item()) < 1e-12
    np.testing.assert_allclose(g, gt, rtol=1e-10, atol=1e-13)


def test_gradients_match_finite_differences():
    theta = _theta(5)
    X = np.random.default_rng(6).normal(size=(20, mlp.D_IN))
    t = np.random.default_rng(7).uniform(0, 1, size=20)
    _, g = mlp.loss_and_grad(theta, X, t)
    rng = np.random.default_rng(8)
    h = 1e-6
    for i in rng.choice(mlp.N_PARAMS, 40, replace=False):
        e = np.zeros(mlp.N_PARAMS)
        e[i] = h
        fd = (mlp.loss_and_grad(theta + e, X, t)[0] - mlp.loss_and_grad(theta - e, X, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i]))


def test_adam_matches_torch():
    theta = _theta(9)
    X = np.random.default_rng(10).normal(size=(16, mlp.D_IN))
    t = np.random.default_rng(11).uniform(0, 1, size=16)
    f, params = _torch_net(theta)
    opt = torch.optim.Adam(params, lr=1e-3)
    m = np.zeros(mlp.N_PARAMS)
    v = np.zeros(mlp.N_PARAMS)
    th = theta.copy()
    for step in range(1, 4):
        opt.zero_grad()
        _torch_pinball(f(torch.tensor(X)), torch.tensor(t)).backward()
        opt.step()
        _, g = mlp.loss_and_grad(th, X, t)
        th, m, v = mlp.adam_step(th, g, m, v, step, 1e-3)
    np.testing.assert_allclose(th, np.concatenate([p.detach().numpy().ravel() for p in params]),
                               rtol=1e-10, atol=1e-12)


def test_features_estimate_the_damped_spectral_moments():
    # E[mu_m] / E[mu_0] = (1/N) sum_l T_m(lambda_l - 1): the KPM density moments
    g = synth.sbm_config(500, 5, s=10.0, seed=3)
    A, _ = laplacian.normalized_adjacency(g.row_ptr, g.col)
    ev = np.linalg.eigvalsh(laplacian.laplacian_dense(g.row_ptr, g.col))
    n_c = 200
    R = philox.gaussian_block(1, g.n, n_c, 1, philox.COUNT)
    mu = cheb.moments(A, R, 50)
    x = mlp.features(mu, g.n, 5)
    t = np.arccos(np.clip(ev - 1.0, -1, 1))
    exact = jackson.jackson_factors(50)[1:51] * np.array([np.mean(np.cos(m * t)) for m in range(1, 51)])
    assert x.shape == (52,)
    assert np.max(np.abs(x[:50] - exact)) < 0.02
    assert abs(x[50] - math.log(500) / 10) < 1e-15 and abs(x[51] - 5 / 500) < 1e-15


def test_bracket_is_ordered_and_clipped():
    theta = np.zeros(mlp.N_PARAMS)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(theta)
    b3[:] = [2.0, -1.0]
    th = mlp.pack([W1, b1, W2, b2, W3, b3])
    assert mlp.bracket(th, np.zeros(mlp.D_IN), 0.5, 0.1) == (0.4, 0.7)
    assert mlp.bracket(th, np.zeros(mlp.D_IN), 1.9, 0.5) == (1.4, 2.0)


def test_count_root_recovers_the_eigenvalue_crossing():
    # with many signals the count curve is close to tr h~, whose k crossing lies
    # between lambda_k and lambda_{k+1} of a graph with a clear gap
    g = synth.disconnected_regular(5, 60, 6, seed=2)
    A, _ = laplacian.normalized_adjacency(g.row_ptr, g.col)
    ev = np.linalg.eigvalsh(laplacian.laplacian_dense(g.row_ptr, g.col))
    R = philox.gaussian_block(0, g.n, 400, 1, philox.COUNT)
    mu = cheb.moments(A, R, 50)
    lam0, s = mlp.count_root(mu, 50, 5, 400)
    assert ev[4] - 0.05 <= lam0 <= ev[5] + 0.05
    c = float(np.dot(jackson.lowpass_coeffs(lam0, 50), mu))
    assert abs(c - 5) < 1e-6
    assert 1e-4 <= s <= 0.5
