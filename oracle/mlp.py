"""float64 reference of the lambda_k bracket network (oracle; test only).

A multilayer perceptron 52 -> 128 -> 128 -> 2 with GELU activations maps a
graph's spectral summary to a bracket [lo, hi] for the dichotomy of Sec. 4.3.
The paper only notes that a better estimate of lambda_k would help (Sec. 5.2);
the network, its inputs and its loss are this build's.

Parameters are one flat vector in the order W1 (52 x 128, row = input),
b1 (128), W2 (128 x 128), b2 (128), W3 (128 x 2), b3 (2): 23,554 values.

Inputs (``features``): the Jackson-damped Chebyshev moments
g_m mu_m / mu_0, m = 1..50, of the first eigencount pass (mu_m = <R, T_m R>,
the kernel polynomial estimate of the spectral density), ln N / 10 and k / N.

Outputs are offsets in a scale-free unit around the root of the first pass's
own count curve: with c(lambda) = sum_m a_m(lambda) mu_m (the count those
signals give at any lambda), lambda_0 solves c(lambda_0) = k and
s = sqrt(2k / n_c) / c'(lambda_0) is the spread of lambda implied by the
count's standard deviation; the bracket is [lambda_0 + s y_lo, lambda_0 + s y_hi].

Loss: quantile (pinball) loss of output 0 at tau = 0.02 and of output 1 at
tau = 0.98 against (lambda_k - lambda_0) / s, lambda_k from the plain
dichotomy, averaged over the batch: rho_tau(u) = u (tau - 1[u < 0]),
u = target - output.

Optimiser: Adam (Kingma & Ba) with bias correction.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

D_IN, H, D_OUT = 52, 128, 2
TAUS = (0.02, 0.98)
SHAPES = [(D_IN, H), (H,), (H, H), (H,), (H, D_OUT), (D_OUT,)]
N_PARAMS = sum(int(np.prod(s)) for s in SHAPES)  # 23554


def unpack(theta):
    out, off = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(np.asarray(theta[off:off + n], dtype=np.float64).reshape(s))
        off += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def forward(theta, X):
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    Z1 = X @ W1 + b1
    A1 = gelu(Z1)
    Z2 = A1 @ W2 + b2
    A2 = gelu(Z2)
    Y = A2 @ W3 + b3
    return Y, (X, Z1, A1, Z2, A2)


def pinball(Y, t):
    B = Y.shape[0]
    L = 0.0
    dY = np.zeros_like(Y)
    for j, tau in enumerate(TAUS):
        u = t - Y[:, j]
        ind = (u < 0.0).astype(np.float64)
        L += np.sum(u * (tau - ind))
        dY[:, j] = -(tau - ind) / B
    return L / B, dY


def loss_and_grad(theta, X, t):
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    Y, (X, Z1, A1, Z2, A2) = forward(theta, X)
    L, dY = pinball(Y, t)
    gW3 = A2.T @ dY
    gb3 = dY.sum(axis=0)
    dA2 = dY @ W3.T
    dZ2 = dA2 * gelu_grad(Z2)
    gW2 = A1.T @ dZ2
    gb2 = dZ2.sum(axis=0)
    dA1 = dZ2 @ W2.T
    dZ1 = dA1 * gelu_grad(Z1)
    gW1 = X.T @ dZ1
    gb1 = dZ1.sum(axis=0)
    return L, pack([gW1, gb1, gW2, gb2, gW3, gb3])


def adam_step(theta, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def features(moments, N, k, p=50):
    """52 inputs: Jackson-damped moments g_m mu_m / mu_0 (m = 1..50), ln N / 10, k / N."""
    from .jackson import jackson_factors

    mu = np.asarray(moments, dtype=np.float64)
    g = jackson_factors(p)
    x = np.empty(D_IN)
    x[:50] = g[1:51] * mu[1:51] / mu[0]
    x[50] = math.log(N) / 10.0
    x[51] = k / N
    return x


def count_root(moments, p, k, n_c):
    """(lambda_0, s): root of the first pass's count curve and the lambda spread."""
    from .jackson import lowpass_coeffs

    mu = np.asarray(moments, dtype=np.float64)

    def c(lam):
        return float(np.dot(lowpass_coeffs(lam, p), mu))

    lo, hi = 0.0, 2.0
    for _ in range(50):
        mid = 0.5 * (lo + hi)
        if c(mid) < k:
            lo = mid
        else:
            hi = mid
    lam0 = 0.5 * (lo + hi)
    h = 1e-3
    slope = (c(min(2.0, lam0 + h)) - c(max(0.0, lam0 - h))) / (min(2.0, lam0 + h) - max(0.0, lam0 - h))
    s = math.sqrt(2.0 * k / n_c) / max(slope, 1e-9)
    return lam0, min(max(s, 1e-4), 0.5)


def bracket(theta, x, lam0, s):
    """[lo, hi] = lambda_0 + s * sorted outputs, clipped to [0, 2]."""
    y, _ = forward(theta, np.asarray(x, dtype=np.float64).reshape(1, -1))
    a, b = sorted((float(y[0, 0]), float(y[0, 1])))
    return max(0.0, min(2.0, lam0 + s * a)), max(0.0, min(2.0, lam0 + s * b))
