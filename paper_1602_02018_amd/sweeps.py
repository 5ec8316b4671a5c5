"""Parameter sweeps of the method on synthetic SBMs (the trends of Fig. 1 a-e
and of the heterogeneous-size experiment of the supplementary material).

For N = 1000, k = 20, mean degree s = 16 and eps = c eps_c (eps_c =
(s - sqrt s)/(s + sqrt s (k - 1))), the recovery (ARI against the planted
communities, averaged over realisations) is measured while one parameter moves
away from Alg. 2's defaults: n (sampled nodes), d (random signals), p
(polynomial order), gamma (regularisation), and the damping of the Chebyshev
series.  Fig. 1 e's comparison of the lambda_k estimate with the true
lambda_k and lambda_{k+1} is reported beside it (true values from a dense
eigendecomposition of the 1000-node Laplacian, as a reference only).

    python -m paper_1602_02018_amd.sweeps --realizations 5 --out DIR

writes DIR/sweeps_report.json and prints one line per (parameter, value, eps).
Every step of the method runs through libcsc; the graphs are generated on the
host.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def _paths():
    sys.path.insert(0, os.path.dirname(HERE))


def ari(a, b):
    """Adjusted Rand index of two labelings (Hubert & Arabie)."""
    a = np.asarray(a)
    b = np.asarray(b)
    _, ai = np.unique(a, return_inverse=True)
    _, bi = np.unique(b, return_inverse=True)
    M = np.zeros((ai.max() + 1, bi.max() + 1))
    np.add.at(M, (ai, bi), 1)
    comb = lambda x: x * (x - 1) / 2.0
    s_ij = comb(M).sum()
    s_a = comb(M.sum(axis=1)).sum()
    s_b = comb(M.sum(axis=0)).sum()
    tot = comb(len(a))
    exp = s_a * s_b / tot
    mx = 0.5 * (s_a + s_b)
    return 1.0 if mx == exp else float((s_ij - exp) / (mx - exp))


def sbm_graph(N, k, s, eps_frac, seed, sizes=None):
    _paths()
    import synth

    eps = eps_frac * synth.eps_critical(s, k)
    return synth.sbm(N, k, s, eps, seed, sizes=sizes)


def true_lambdas(gr, k):
    """(lambda_k, lambda_{k+1}) of the normalized Laplacian, dense (reference only)."""
    deg = np.diff(gr.row_ptr).astype(np.float64)
    N = gr.n
    W = np.zeros((N, N))
    rows = np.repeat(np.arange(N), np.diff(gr.row_ptr))
    W[rows, gr.col] = 1.0
    dinv = np.where(deg > 0, 1.0 / np.sqrt(np.maximum(deg, 1e-300)), 0.0)
    Lap = np.eye(N) - dinv[:, None] * W * dinv[None, :]
    ev = np.linalg.eigvalsh(Lap)
    return float(ev[k - 1]), float(ev[k])


def run_point(api, gr, k, seed, n=None, d=None, p=50, gamma=1e-3, damping=0, sampling="uniform"):
    g = api.Graph(gr.row_ptr, gr.col)
    nn = api.default_n(k) if n is None else n
    dd = int(math.ceil(4 * math.log(nn))) if d is None else d  # Fig. 1 default d = 4 log n
    api.set_damping(damping)
    try:
        r = api.run(g, k, dd, seed, p=p, n=nn, gamma=gamma, replicates=10, sampling=sampling)
    finally:
        api.set_damping(0)
    return dict(ari=ari(r.labels.cpu().numpy(), gr.truth), lam=r.lam,
                cg_status=int(r.interp.status), steps=r.bisection.steps)


def sweep(api, eps_fracs, realizations, k=20, N=1000, s=16.0, sizes=None, log=print,
          grid=None):
    base_n = api.default_n(k)
    grid = grid or {
        "n": [int(math.ceil(k * math.log(k))), base_n, 3 * int(math.ceil(k * math.log(k)))],
        "d": [int(math.ceil(2 * math.log(base_n))), int(math.ceil(4 * math.log(base_n))),
              int(math.ceil(8 * math.log(base_n)))],
        "p": [10, 20, 50, 100],
        "gamma": [1e-5, 1e-3, 1e-1],
        "damping": [0, 1],
    }
    rows = []
    for ef in eps_fracs:
        graphs = [sbm_graph(N, k, s, ef, 1000 * r + 7, sizes) for r in range(realizations)]
        lams = [true_lambdas(gr, k) for gr in graphs]
        for param, values in grid.items():
            for v in values:
                kw = {param: v}
                res = [run_point(api, gr, k, r, **kw) for r, gr in enumerate(graphs)]
                row = dict(eps_frac=ef, param=param, value=v,
                           ari_mean=float(np.mean([x["ari"] for x in res])),
                           ari_min=float(np.min([x["ari"] for x in res])),
                           lam_est_mean=float(np.mean([x["lam"] for x in res])),
                           lam_k_mean=float(np.mean([l[0] for l in lams])),
                           lam_k1_mean=float(np.mean([l[1] for l in lams])),
                           cg_not_converged=int(sum(x["cg_status"] != 0 for x in res)))
                rows.append(row)
                log(f"eps={ef:.2f} eps_c {param}={v}: ARI {row['ari_mean']:.4f} "
                    f"(min {row['ari_min']:.4f}), lambda est {row['lam_est_mean']:.4f} vs "
                    f"lambda_k {row['lam_k_mean']:.4f}, lambda_k+1 {row['lam_k1_mean']:.4f}")
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--realizations", type=int, default=5)
    ap.add_argument("--eps", type=float, nargs="+", default=[0.0, 0.25, 0.5, 0.75, 1.0])
    ap.add_argument("--out", default=os.path.join(HERE, "data"))
    args = ap.parse_args()
    from . import api

    os.makedirs(args.out, exist_ok=True)
    t0 = time.time()
    hom = sweep(api, args.eps, args.realizations, log=lambda m: print("[homogeneous] " + m, flush=True))
    sizes = [5, 10, 15, 20, 25, 30, 35, 40, 45, 50, 50, 55, 60, 65, 70, 75, 80, 85, 90, 95]
    het = sweep(api, args.eps, args.realizations, sizes=sizes,
                grid={"sampling": ["uniform", "density"], "damping": [0, 1]},
                log=lambda m: print("[heterogeneous] " + m, flush=True))
    with open(os.path.join(args.out, "sweeps_report.json"), "w") as f:
        json.dump(dict(N=1000, k=20, s=16, realizations=args.realizations,
                       homogeneous=hom, heterogeneous=het, seconds=time.time() - t0), f, indent=1)


if __name__ == "__main__":
    main()
