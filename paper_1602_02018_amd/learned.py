"""Training and evaluation of the lambda_k bracket network.

The dichotomy of Sec. 4.3 tests lambda = 1 first; the network maps the
moments of that first eigencount pass (plus ln N and k/N) to a bracket for
the rest of the search.  Everything runs through libcsc:

* ``label``     the plain dichotomy (batched) gives each training graph its
                target lambda_k and the first pass's moments;
* ``train``     float32 Adam on the pinball loss with the library's forward /
                backward / Adam kernels (csc_mlp_loss_grad, csc_mlp_adam_step);
                targets are (lambda_k - lambda_0) / s with lambda_0, s from the
                first pass's count curve (csc_count_root);
* ``evaluate``  plain vs learned dichotomy on held-out graphs: passes used,
                and |count(lambda) - k| from an independent eigencount pass
                (fresh signals, sub-stream 1000) as the referee of each lambda;
                the one-pass KPM root of the first pass's count curve is
                reported beside them.

    python -m paper_1602_02018_amd.learned --n-train 2000 --n-test 200 --out DIR

writes DIR/lambda_bracket_mlp.npy (float32[23554]) and DIR/report.json.
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "data", "lambda_bracket_mlp.npy")


# ------------------------------------------------------------- workloads ---

def graph_spec(i: int, seed: int, n_range):
    """Random workload i: SBM or Chung-Lu (alternating), N log-uniform in n_range,
    k uniform in [10, 100] capped at N / 20."""
    rng = np.random.default_rng([seed, i])
    N = int(round(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
    k = int(rng.integers(10, 101))
    k = max(2, min(k, N // 20))
    kind = "sbm" if i % 2 == 0 else "chunglu"
    s = float(rng.uniform(8.0, 32.0))
    return dict(i=i, seed=seed * 100003 + i, N=N, k=k, kind=kind, s=s)


def make_graph(spec):
    sys.path.insert(0, os.path.dirname(HERE))
    import synth

    if spec["kind"] == "sbm":
        eps = 0.25 * synth.eps_critical(spec["s"], spec["k"])
        g = synth.sbm(spec["N"], spec["k"], spec["s"], eps, spec["seed"])
    else:
        g = synth.chung_lu_blocks(spec["N"], spec["k"], mean_deg=spec["s"],
                                  max_deg=min(2000.0, spec["N"] / 10.0), seed=spec["seed"])
    return spec, g.row_ptr, g.col


def make_pool(processes: int = 16):
    """Host worker pool for graph generation.  Create it before the process
    touches the GPU: workers are forked and only run numpy."""
    return mp.get_context("fork").Pool(processes)


def generate(specs, pool=None):
    """Yield (spec, row_ptr, col) in order, from the pool or in this process."""
    if pool is None:
        for sp in specs:
            yield make_graph(sp)
    else:
        yield from pool.imap(make_graph, specs, chunksize=1)


# ---------------------------------------------------------------- labels ---

def label(specs, device="cuda", p: int = 50, chunk: int = 64, pool=None, log=None):
    """Plain dichotomy on every graph: features of the first pass, lambda_k, passes."""
    from . import api

    X, y, steps, meta = [], [], [], []
    buf = []

    def flush():
        gs = [api.Graph(rp, c, device) for _, rp, c in buf]
        ks = [s["k"] for s, _, _ in buf]
        ncs = [api.count_signals(g.n) for g in gs]
        seeds = [s["seed"] for s, _, _ in buf]
        res = api.estimate_lambda_k_batched(gs, ks, p, ncs, seeds)
        for (s, _, _), g, r, nc in zip(buf, gs, res, ncs):
            X.append(api.mlp_features(r.moments, g.n, s["k"]))
            lam0, sc = api.count_root(r.moments, s["k"], nc)
            y.append((r.lam - lam0) / sc)
            steps.append(r.steps)
            meta.append(s)
        buf.clear()
        if log:
            log(f"labelled {len(y)} graphs")

    for item in generate(specs, pool):
        buf.append(item)
        if len(buf) == chunk:
            flush()
    if buf:
        flush()
    return np.array(X, dtype=np.float32), np.array(y, dtype=np.float32), np.array(steps), meta


# --------------------------------------------------------------- training --

def init_params(seed: int = 0):
    """He-scaled Gaussian weights, zero biases (float32[23554])."""
    rng = np.random.default_rng(seed)
    parts = []
    for din, dout in ((52, 128), (128, 128), (128, 2)):
        parts.append(rng.normal(scale=math.sqrt(2.0 / din), size=(din, dout)))
        parts.append(np.zeros(dout))
    b3 = parts[-1]
    b3[:] = [-2.0, 2.0]  # first guess: two count standard deviations either side
    return np.concatenate([q.ravel() for q in parts]).astype(np.float32)


def train(X, y, steps: int = 3000, lr: float = 2e-3, seed: int = 0, device="cuda", log=None):
    import torch

    from . import api

    params = torch.tensor(init_params(seed), device=device)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    Xd = torch.tensor(X, device=device)
    yd = torch.tensor(y, device=device)
    hist = []
    for t in range(1, steps + 1):
        step_lr = lr * (0.1 ** (t / steps))
        loss, grad = api.mlp_loss_grad(params, Xd, yd)
        api.mlp_adam_step(params, grad, m, v, t, step_lr)
        if t == 1 or t % 250 == 0 or t == steps:
            hist.append((t, loss))
            if log:
                log(f"step {t} loss {loss:.5f}")
    return params, hist


# ------------------------------------------------------------- evaluation --



def evaluate(specs, params, device="cuda", p: int = 50, pool=None, chunk: int = 16, log=None):
    """Plain vs learned dichotomy (batched) on held-out graphs."""
    from . import api

    rows = []
    buf = []

    def flush():
        gs = [api.Graph(rp, c, device) for _, rp, c in buf]
        ks = [s["k"] for s, _, _ in buf]
        ncs = [api.count_signals(g.n) for g in gs]
        seeds = [s["seed"] for s, _, _ in buf]
        plain = api.estimate_lambda_k_batched(gs, ks, p, ncs, seeds)
        learned = api.estimate_lambda_k_batched(gs, ks, p, ncs, seeds, mlp_params=params)
        for (s, _, _), g, a, b, nc in zip(buf, gs, plain, learned, ncs):
            lk, _ = api.count_root(a.moments, s["k"], nc)
            referee = {}
            for name, lam in (("plain", a.lam), ("learned", b.lam), ("kpm", lk)):
                cnt, _ = api.eigencount(g, lam, p, nc, s["seed"], 1000)
                referee[name] = abs(cnt - s["k"])
            rows.append(dict(N=g.n, k=s["k"], kind=s["kind"], plain_steps=a.steps,
                             learned_steps=b.steps, plain_lambda=a.lam, learned_lambda=b.lam,
                             kpm_lambda=lk, learned_status=b.status, plain_status=a.status,
                             err_plain=referee["plain"], err_learned=referee["learned"],
                             err_kpm=referee["kpm"]))
        buf.clear()
        if log:
            log(f"evaluated {len(rows)} graphs")

    for item in generate(specs, pool):
        buf.append(item)
        if len(buf) == chunk:
            flush()
    if buf:
        flush()
    return rows


def summarize(rows):
    a = np.array([r["plain_steps"] for r in rows], dtype=float)
    b = np.array([r["learned_steps"] for r in rows], dtype=float)
    return dict(
        graphs=len(rows),
        plain_passes_mean=float(a.mean()), learned_passes_mean=float(b.mean()),
        passes_saved_mean=float((a - b).mean()), passes_saved_frac=float(1 - b.sum() / a.sum()),
        learned_misses=int(sum(r["learned_status"] == 7 for r in rows)),
        plain_exhausted=int(sum(r["plain_status"] == 6 for r in rows)),
        learned_exhausted=int(sum(r["learned_status"] == 6 for r in rows)),
        err_plain_mean=float(np.mean([r["err_plain"] for r in rows])),
        err_learned_mean=float(np.mean([r["err_learned"] for r in rows])),
        err_kpm_mean=float(np.mean([r["err_kpm"] for r in rows])),
    )


def load_params(device="cuda", path: str = WEIGHTS):
    import torch

    w = np.load(path, allow_pickle=False)
    if w.dtype != np.float32 or w.shape != (23554,):
        raise ValueError(f"{path}: expected float32[23554], got {w.dtype}{w.shape}")
    return torch.tensor(w, device=device)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-train", type=int, default=2000)
    ap.add_argument("--n-test", type=int, default=200)
    ap.add_argument("--train-range", type=float, nargs=2, default=(1e3, 1e5))
    ap.add_argument("--test-range", type=float, nargs=2, default=(1e5, 1e6))
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--processes", type=int, default=16)
    ap.add_argument("--out", default=os.path.join(HERE, "data"))
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)

    def log(msg):
        print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)

    pool = make_pool(args.processes)  # before any GPU work
    t0 = time.time()
    specs = [graph_spec(i, args.seed, args.train_range) for i in range(args.n_train)]
    X, y, steps, _ = label(specs, pool=pool, log=log)
    log(f"labelled {len(y)} training graphs in {time.time() - t0:.1f} s "
        f"(plain passes mean {steps.mean():.2f}, target range {y.min():.3f}..{y.max():.3f})")
    t1 = time.time()
    params, hist = train(X, y, steps=args.steps, seed=args.seed, log=log)
    log(f"trained in {time.time() - t1:.1f} s")
    w = params.cpu().numpy().astype(np.float32)
    np.save(os.path.join(args.out, "lambda_bracket_mlp.npy"), w)
    tspecs = [graph_spec(i, args.seed + 1, args.test_range) for i in range(args.n_test)]
    t2 = time.time()
    rows = evaluate(tspecs, params, pool=pool, log=log)
    pool.close()
    summ = summarize(rows)
    log(f"evaluated {len(rows)} held-out graphs in {time.time() - t2:.1f} s: {summ}")
    with open(os.path.join(args.out, "report.json"), "w") as f:
        json.dump(dict(train=dict(graphs=int(len(y)), range=list(args.train_range),
                                  plain_passes_mean=float(steps.mean()), loss=hist),
                       test=dict(range=list(args.test_range), summary=summ, rows=rows)), f)


if __name__ == "__main__":
    main()
