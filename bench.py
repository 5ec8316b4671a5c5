"""Benchmark of the compressive spectral clustering hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload sbm-1e5]

A step is one pass of the whole path over one synthetic graph already
resident in HBM: lambda_k dichotomy (eigencount passes), feature pass,
sampling, k-means on the sampled features, interpolation by CG and the hard
labels.  Prints one JSON line:

* value: whole-job throughput in GB/s, the algorithmic bytes of every
  Chebyshev step, random block and CG update in the step divided by the wall
  time of the step;
* roofline: the dominant kernel of the step, the Chebyshev-step kernel with
  the largest launches x time: the moment step of the eigencount passes (the
  dichotomy runs 4 tests side by side, width 4 x n_c rounded to a multiple of
  4 each, natural node order) or the Clenshaw step of the CG operator at
  width k (graph in community order), each timed per launch with HIP events on
  the stream it runs on, against the MI355X HBM peak (8 TB/s); its HBM traffic
  comes from rocprofv3 FETCH_SIZE / WRITE_SIZE counters recorded in profiles/
  and is null when the kernel source changed since they were taken (the other
  kernel is reported beside it);
* cpu_baseline: the float64 CPU oracle's filter pass (p products of the CSR
  matrix with an N x k block) on the same graph, in the same unit.
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
KERNEL_SRC = [os.path.join(ROOT, "paper_1602_02018_amd", "csrc", f)
              for f in ("kernels.hip", "device.hpp", "kernels.hpp", "common.hpp")]
# rocprofv3 counter summaries of the two candidate dominant kernels
COUNTERS = {
    "count": os.path.join(ROOT, "profiles", "cheb_step_count_sbm_N1e5_4x24_counters.txt"),
    "cg": os.path.join(ROOT, "profiles", "cheb_step_cg_sbm_N1e5_k100_counters.txt"),
    "cl_count_step": os.path.join(ROOT, "profiles", "cheb_step_count_chunglu_N1e6_4x28_counters.txt"),
    "cl_filter_step": os.path.join(ROOT, "profiles", "cheb_step_filter_chunglu_N1e6_w56_counters.txt"),
    "cl_cg_step": os.path.join(ROOT, "profiles", "cheb_step_cg_chunglu_N1e6_k250_counters.txt"),
}

WORKLOADS = {
    # SBM N = 1e5, k = 100, mean degree 16, eps = eps_c / 4; d = ceil(4 ln N), p = 50
    "sbm-1e5": dict(N=100000, k=100, s=16.0, p=50, model="sbm"),
    # Chung-Lu N = 1e6, power-law degrees (exponent 2.5, mean 20, max 2000), k = 250 blocks
    "chunglu-1e6": dict(N=1000000, k=250, p=60, model="chunglu"),
    # SBM N = 1000, k = 10 (oracle-sized)
    "sbm-1e3": dict(N=1000, k=10, s=16.0, p=50, model="sbm"),
    # 64 SBMs, N ~ U[2e3, 2e5], k ~ U[10, 100], s ~ U[8, 32], eps = eps_c / 4
    "batch64": dict(G=64, p=50, model="sbm_batch"),
}


def step_bytes(N, nnz, w, kind):
    """Algorithmic bytes of one Chebyshev step (float32 blocks, int32 indices).

    CSR read once (4(N+1) + 8 nnz) plus, per node and column, 4 bytes for each
    block touched: forward recurrence with a running sum, gathered T_m,
    T_{m-1}, T_{m+1} and the sum read + write (kind "y": 20); the moment step
    touches T_m (gathered, and its own row for the products), T_{m-1} and
    T_{m+1} ("mom": 12); Clenshaw's step reads the gathered b_{m+1}, b_{m+2}
    and R and writes b_m ("clen": 16).
    """
    csr = 4 * (N + 1) + 8 * nnz
    per = {"y": 20, "mom": 12, "ys": 12, "clen": 16}[kind]
    return csr + per * N * w


# block CG per iteration besides the pass, in N x k blocks touched: Gram Z^T Z
# (1), P = Z T (2), Grams P^T Q and P^T R (4), X and R updates (6), column
# norms of R (1), Jacobi scaling Z = D^-1 R (2), Gram Q^T Z (2), Z = Z + P beta (3)
BLOCK_CG_BLOCKS = 21


def moment_steps(p):
    """Steps of an eigencount pass of order p: the doubling identities give
    p + 1 moments from T_0 .. T_ceil(p/2)."""
    return (p + 1) // 2


def job_bytes(N, nnz, k, d, n_c, p, bis_steps, cg_iters):
    gauss = 4 * N
    count = bis_steps * (gauss * n_c + moment_steps(p) * step_bytes(N, nnz, n_c, "mom"))
    feat = gauss * d + p * step_bytes(N, nnz, d, "clen") + 8 * N * d
    cg = cg_iters * (p * step_bytes(N, nnz, k, "clen") + BLOCK_CG_BLOCKS * 4 * N * k)
    return count + feat + cg


def kernel_hash():
    """Hash of the sources the Chebyshev-step kernel is compiled from."""
    h = hashlib.sha256()
    for f in KERNEL_SRC:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def permuted_csr(gr, order):
    """CSR of the graph listed in `order` (row r = node order[r]), neighbours
    relabelled and kept in CSR order: the graph the ordered CG runs on."""
    import numpy as np

    order = np.asarray(order, dtype=np.int64)
    inv = np.empty_like(order)
    inv[order] = np.arange(order.size)
    deg = np.diff(gr.row_ptr).astype(np.int64)[order]
    rp = np.zeros(order.size + 1, np.int64)
    np.cumsum(deg, out=rp[1:])
    src = np.repeat(gr.row_ptr[order].astype(np.int64) - rp[:-1], deg) + np.arange(rp[-1])
    return rp.astype(np.int32), inv[gr.col[src]].astype(np.int32)


def read_traffic(which):
    """HBM bytes per launch from the committed counter summary, or None."""
    path = COUNTERS[which]
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if line.startswith("#") or "=" not in line:
            continue
        key, val = line.split("=", 1)
        rec[key.strip()] = val.strip()
    if rec.get("kernel_source_sha256_16") != kernel_hash():
        return None
    try:
        return float(rec["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def make_graph(wl, seed):
    import synth

    if wl["model"] == "sbm":
        return synth.sbm_config(wl["N"], wl["k"], s=wl["s"], seed=seed)
    return synth.chung_lu_blocks(wl["N"], wl["k"], seed=seed)


def cpu_baseline(gr, k, p, budget_s=30.0):
    """Oracle filter pass on an N x k block; fewer columns if it would run long."""
    import numpy as np

    from oracle import cheb, jackson, laplacian, philox

    A, _ = laplacian.normalized_adjacency(gr.row_ptr, gr.col)
    a = jackson.lowpass_coeffs(0.4, p)
    # time one product to bound the sample at ~budget_s of CPU work
    X1 = philox.gaussian_block(0, gr.n, k, 0, philox.FEAT)
    t0 = time.perf_counter()
    _ = A @ X1
    one = time.perf_counter() - t0
    w = k
    if one * p > budget_s:
        w = max(1, int(k * budget_s / (one * p)))
    X = X1[:, :w].copy()
    t0 = time.perf_counter()
    cheb.filter_block(A, X, a)
    t = time.perf_counter() - t0
    by = p * step_bytes(gr.n, gr.nnz, w, "y")
    return {
        "value": round(by / t / 1e9, 3),
        "unit": "GB/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"float64 oracle filter pass, p={p} products of the {gr.n}-node CSR matrix "
                  f"with an N x {w} block (the CG operator's filter), {t:.1f} s; scipy's CSR "
                  f"product runs on one thread; host reports {os.cpu_count()} CPUs",
    }


def quiet_gc():
    """Collect once and move every object alive after set-up out of the
    collector's reach, so that a full collection (tens of ms with torch
    loaded) does not land inside a timed run."""
    gc.collect()
    gc.freeze()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sbm-1e5", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 1e6-node Chung-Lu run and its step timings")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain 256 MiB device copy (for scaling memory counters)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch

        x = torch.ones(64 * 2**20, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 4, "copy_bytes_written": y.numel() * 4,
                          "dispatches": 3}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the path shards by columns across GPUs, which this build does not run)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from oracle.metrics import adjusted_rand_index  # ARI of the labels only
    from paper_1602_02018_amd import api

    wl = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    if args.workload == "batch64":
        return bench_batch(args, wl, dev)
    gr = make_graph(wl, args.seed)
    N, nnz, k, p = gr.n, gr.nnz, wl["k"], wl["p"]
    d = int(math.ceil(4 * math.log(N)))
    n_c = api.count_signals(N)
    g = api.Graph(gr.row_ptr, gr.col, dev)
    torch.cuda.synchronize()

    quiet_gc()
    for _ in range(args.warmup):
        api.run(g, k, d, args.seed, p=p)
    torch.cuda.synchronize()
    results = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        results.append(api.run(g, k, d, args.seed, p=p))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed / args.steps * 1e3

    total = 0.0
    for r in results:
        total += job_bytes(N, nnz, k, d, n_c, p, r.bisection.steps, int(r.interp.iters.max()))
    value = total / elapsed / 1e9
    last = results[-1]
    ari = adjusted_rand_index(last.labels.cpu().numpy(), gr.truth)

    # the same graph with the learned lambda_k bracket
    from paper_1602_02018_amd import learned

    mlp = learned.load_params(dev)
    api.run(g, k, d, args.seed, p=p, mlp_params=mlp)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lres = [api.run(g, k, d, args.seed, p=p, mlp_params=mlp) for _ in range(args.steps)]
    torch.cuda.synchronize()
    ms_learned = (time.perf_counter() - t0) / args.steps * 1e3
    ari_lp = adjusted_rand_index(lres[-1].labels.cpu().numpy(), last.labels.cpu().numpy())

    # the same graph with the one-pass KPM dichotomy
    api.run(g, k, d, args.seed, p=p, lambda_method="kpm")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kres = [api.run(g, k, d, args.seed, p=p, lambda_method="kpm") for _ in range(args.steps)]
    torch.cuda.synchronize()
    ms_kpm = (time.perf_counter() - t0) / args.steps * 1e3

    # candidate dominant kernels, per-launch times: the moment step of the
    # eigencount passes (width n_c, natural order) and the Clenshaw step of the
    # CG operator (width k, on the graph in the order the interpolation used)
    # (the dichotomy runs `group` tests' passes side by side, each test's
    # n_c columns rounded up to a multiple of 4)
    group, count_w, count_kind = count_shape(api, n_c)
    cands = {}
    for which, w, order, kind, bkind, launches in (
            ("count", count_w, None, count_kind, "mom",
             -(-last.bisection.steps // group) * moment_steps(p)),
            ("cg", k, last.order, 3, "clen", int(last.interp.iters.max()) * p)):
        avg_s = step_time(api, gr, order, w, p, args.kernel_reps, dev, kind=kind)
        per_launch = step_bytes(N, nnz, w, bkind)
        achieved = per_launch / avg_s / 1e9
        name = (f"k_cheb_step<EPI_MOM> (moment step of the eigencount passes, {group} tests of "
                f"{n_c} signals side by side" if which == "count"
                else "k_cheb_step<EPI_CLEN> (Clenshaw step of the CG operator pass")
        traffic = read_traffic(which)
        cands[which] = {
            "kernel": f"{name}, w={w}, panel width {api.panel_width(N, w, nnz)}"
                      f"{', community order' if order is not None else ', natural order'})",
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": traffic,
            # bytes below L2 per launch (counters) over the launch time
            "traffic_GBs": None if traffic is None else round(traffic / avg_s / 1e9, 1),
            "alg_bytes_per_launch": per_launch,
            "avg_launch_us": round(avg_s * 1e6, 2),
            "launches_per_step": launches,
            "ms_per_step": round(launches * avg_s * 1e3, 3),
        }
    dom = max(cands, key=lambda c: cands[c]["ms_per_step"])
    other = "cg" if dom == "count" else "count"
    large = None if args.no_large else large_shapes(api, args, dev)

    out = {
        "metric": "filter SpMM HBM GB/s (% peak) + end-to-end CSC s/graph vs plain at ARI>=0.99",
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {wl['model']} N={N} nnz={nnz} k={k} d={d} p={p} "
                        f"n={api.default_n(k)} n_c={n_c} gamma=1e-3 tol=1e-6",
            "plain": True,
        },
        "s_per_graph": round(ms_per_step / 1e3, 4),
        "phases_s": {kk: round(v, 4) for kk, v in last.timings.items()},
        "bisection_steps": last.bisection.steps,
        "lambda_k": last.lam,
        "cg_iters_max": int(last.interp.iters.max()),
        "ari_vs_truth": round(float(ari), 4),
        "learned": {
            "s_per_graph": round(ms_learned / 1e3, 4),
            "bisection_steps": lres[-1].bisection.steps,
            "lambda_k": lres[-1].lam,
            "ari_vs_plain": round(float(ari_lp), 4),
            "ari_vs_truth": round(float(adjusted_rand_index(lres[-1].labels.cpu().numpy(),
                                                            gr.truth)), 4),
        },
        "kpm": {
            "s_per_graph": round(ms_kpm / 1e3, 4),
            "moment_passes": 1,
            "tested_points": kres[-1].bisection.steps,
            "lambda_k": kres[-1].lam,
            "ari_vs_plain": round(float(adjusted_rand_index(kres[-1].labels.cpu().numpy(),
                                                            last.labels.cpu().numpy())), 4),
            "ari_vs_truth": round(float(adjusted_rand_index(kres[-1].labels.cpu().numpy(),
                                                            gr.truth)), 4),
        },
        "roofline": cands[dom],
        f"roofline_{other}_step": cands[other],
    }
    if large is not None:
        out["chunglu_1e6"] = large
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(gr, k, p)
    print(json.dumps(out), flush=True)


def count_shape(api, n_c):
    """(group size, block width, measurement-hook kind) of the dichotomy's
    moment step: `group` tests of n_c signals side by side, each rounded up to
    a multiple of 4 columns (one test: width n_c, kind 1)."""
    from paper_1602_02018_amd import _lib

    group = api.get_tuning(_lib.TUNE_COUNT_GROUP)
    if group <= 1:
        return 1, n_c, 1
    return group, group * (-(-n_c // 4) * 4), 4


def step_time(api, gr, order, w, p, reps, dev, kind=3):
    """Average seconds per launch of the Chebyshev step (kind 3: Clenshaw) at
    width w, on the graph in `order` (None: as given), timed with HIP events on
    the current stream, which the library launches on."""
    import torch

    if order is not None:
        rp, cl = permuted_csr(gr, order.cpu().numpy())
        g_run = api.Graph(rp, cl, dev)
    else:
        g_run = api.Graph(gr.row_ptr, gr.col, dev)
    st = api.StepTimer(g_run, w, kind)
    st.launch(10)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        st.launch(p)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / (reps * p)


def large_shapes(api, args, dev):
    """The 1e6-node Chung-Lu configuration (k = 250, d = 56, p = 60): one
    end-to-end run and the per-launch step kernels: the moment step at the
    count width n_c, the Clenshaw step at the filter width d (natural order)
    and at the CG width k (in the order that run's interpolation used)."""
    import torch

    from oracle.metrics import adjusted_rand_index  # ARI of the labels only

    wl = WORKLOADS["chunglu-1e6"]
    gr = make_graph(wl, args.seed)
    N, nnz, k, p = gr.n, gr.nnz, wl["k"], wl["p"]
    d = int(math.ceil(4 * math.log(N)))
    g = api.Graph(gr.row_ptr, gr.col, dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = api.run(g, k, d, args.seed, p=p)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    out = {"workload": f"chunglu N={N} nnz={nnz} k={k} d={d} p={p} n={api.default_n(k)}",
           "s_per_graph": round(secs, 3),
           "phases_s": {kk: round(v, 4) for kk, v in r.timings.items()},
           "bisection_steps": r.bisection.steps,
           "cg_iters_max": int(r.interp.iters.max()),
           "ari_vs_truth": round(float(adjusted_rand_index(r.labels.cpu().numpy(), gr.truth)), 4)}
    n_c = api.count_signals(N)
    group, count_w, count_kind = count_shape(api, n_c)
    for name, w, order, kind, bkind in (("count_step", count_w, None, count_kind, "mom"),
                                        ("filter_step", d, None, 3, "clen"),
                                        ("cg_step", k, r.order, 3, "clen")):
        avg = step_time(api, gr, order, w, p, max(2, args.kernel_reps // 5), dev, kind=kind)
        by = step_bytes(N, nnz, w, bkind)
        traffic = read_traffic("cl_" + name)
        out[name] = {"w": w, "panel_width": api.panel_width(N, w, nnz),
                     "order": "community" if order is not None else "natural",
                     "avg_launch_us": round(avg * 1e6, 1), "alg_bytes_per_launch": by,
                     "achieved_GBs": round(by / avg / 1e9, 1),
                     "frac": round(by / avg / 1e9 / PEAK_HBM_GBS, 4),
                     "traffic": traffic,
                     "traffic_GBs": None if traffic is None else round(traffic / avg / 1e9, 1)}
    return out


def bench_batch(args, wl, dev):
    """64 SBMs: plain form graph by graph vs batched vs batched + learned bracket."""
    import numpy as np
    import torch

    import synth
    from oracle.metrics import adjusted_rand_index
    from paper_1602_02018_amd import api, learned

    gs = synth.sbm_batch(wl["G"], seed=args.seed)
    p = wl["p"]
    G = [api.Graph(g.row_ptr, g.col, dev) for g in gs]
    ks = [g.k for g in gs]
    ds = [int(math.ceil(4 * math.log(g.n))) for g in gs]
    seeds = [args.seed + i for i in range(len(gs))]
    mlp = learned.load_params(dev)
    api.run_batched(G[:4], ks[:4], ds[:4], seeds[:4], p=p, mlp_params=mlp)  # warm-up
    api.run(G[0], ks[0], ds[0], seeds[0], p=p)
    torch.cuda.synchronize()
    quiet_gc()

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    plain, t_plain = timed(lambda: [api.run(g, k, d, s, p=p) for g, k, d, s in zip(G, ks, ds, seeds)])
    batched, t_batched = timed(lambda: api.run_batched(G, ks, ds, seeds, p=p))
    both, t_both = timed(lambda: api.run_batched(G, ks, ds, seeds, p=p, mlp_params=mlp))

    def ari_truth(res):
        return [adjusted_rand_index(r.labels.cpu().numpy(), g.truth) for r, g in zip(res, gs)]

    a_plain, a_both = ari_truth(plain), ari_truth(both)
    a_pair = [adjusted_rand_index(x.labels.cpu().numpy(), y.labels.cpu().numpy())
              for x, y in zip(both, plain)]
    total = sum(job_bytes(g.n, g.nnz, k, d, api.count_signals(g.n), p, r.bisection.steps,
                          int(r.interp.iters.max())) for g, k, d, r in zip(gs, ks, ds, both))
    out = {
        "metric": "filter SpMM HBM GB/s (% peak) + end-to-end CSC s/graph vs plain at ARI>=0.99",
        "value": round(total / t_both / 1e9, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": round(t_both * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batch64: {len(gs)} SBMs, sum N={sum(g.n for g in gs)}, "
                               f"sum nnz={sum(g.nnz for g in gs)}, k in [10,100], p={p}",
                   "form": "batched + learned"},
        "s_per_graph": {"plain": round(t_plain / len(gs), 4), "batched": round(t_batched / len(gs), 4),
                        "batched_learned": round(t_both / len(gs), 4)},
        "speedup_vs_plain": round(t_plain / t_both, 3),
        "phases_s": {
            "plain_sum": {kk: round(sum(r.timings[kk] for r in plain), 4) for kk in plain[0].timings},
            "batched": {kk: round(v, 4) for kk, v in batched[0].timings.items()},
            "batched_learned": {kk: round(v, 4) for kk, v in both[0].timings.items()},
        },
        "cg_iters_sum": {"plain": int(sum(r.interp.iters.max() for r in plain)),
                         "batched": int(sum(r.interp.iters.max() for r in batched))},
        "bisection_passes": {"plain": int(sum(r.bisection.steps for r in plain)),
                             "batched_learned": int(sum(r.bisection.steps for r in both))},
        "ari_vs_truth_mean": {"plain": round(float(np.mean(a_plain)), 4),
                              "batched_learned": round(float(np.mean(a_both)), 4)},
        "ari_batched_learned_vs_plain": {"median": round(float(np.median(a_pair)), 4),
                                         "frac_ge_0.99": round(float(np.mean(np.array(a_pair) >= 0.99)), 4)},
        "batched_identical_to_plain": int(sum(torch.equal(x.labels, y.labels)
                                              for x, y in zip(batched, plain))),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
