"""Benchmark of the compressive spectral clustering hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload chunglu-1e6]

A step is one pass of the whole path (Alg. 2) over one synthetic graph already
resident in HBM: lambda_k dichotomy (eigencount passes), feature pass,
sampling, k-means on the sampled features, interpolation by block CG and the
hard labels.  The default workload is the largest single-GPU configuration:
a Chung-Lu graph with N = 1e6 nodes, power-law expected degrees (exponent
2.5, mean 20, maximum 2000), k = 250 planted blocks, d = 56, p = 60.

Prints one JSON line:

* value: whole-job throughput in GB/s: the algorithmic bytes of every
  Chebyshev step, random block and CG update of the timed steps divided by
  their wall time (a whole-pipeline rate, not the rate of one SpMM kernel);
* roofline: the dominant step kernel of the pipeline (the largest launches x
  time per launch among the eigencount moment step, the feature step and the
  Clenshaw step of the CG operator), timed per launch with HIP events on the
  stream it runs on, against the MI355X HBM peak (8 TB/s); its traffic comes
  from rocprofv3 FETCH_SIZE / WRITE_SIZE counters recorded in profiles/ and is
  null when the kernel sources changed since they were taken; the other two
  step kernels are reported beside it;
* sbm_1e5 / batch64 (secondary workloads, unless --no-secondary): the
  1e5-node SBM (plain, learned bracket, one-pass KPM) and the batch of 64 SBMs
  (plain graph by graph, batched, batched + learned bracket) with the
  agreement of their labels;
* cpu_baseline: the float64 CPU oracle timed on the host: the filter pass on
  the headline graph (bounded sample, one core and all cores over column
  panels) and, per phase of Alg. 2, the 1e5-node SBM (bounded samples scaled
  to one graph).
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
METRIC = "filter SpMM HBM GB/s (% peak) + end-to-end CSC s/graph vs plain at ARI>=0.99"
KERNEL_SRC = [os.path.join(ROOT, "paper_1602_02018_amd", "csrc", f)
              for f in ("kernels.hip", "device.hpp", "kernels.hpp", "common.hpp")]
PROF = os.path.join(ROOT, "profiles")
# rocprofv3 counter summaries of the step kernels, per workload
COUNTERS = {
    ("sbm-1e5", "count"): os.path.join(PROF, "cheb_step_count_sbm_N1e5_4x24_counters.txt"),
    ("sbm-1e5", "cg"): os.path.join(PROF, "cheb_step_cg_sbm_N1e5_k100_counters.txt"),
    ("sbm-1e5", "filter"): os.path.join(PROF, "cheb_step_filter_sbm_N1e5_w47_counters.txt"),
    ("chunglu-1e6", "count"): os.path.join(PROF, "cheb_step_count_chunglu_N1e6_4x28_counters.txt"),
    ("chunglu-1e6", "filter"): os.path.join(PROF, "cheb_step_filter_chunglu_N1e6_w56_counters.txt"),
    ("chunglu-1e6", "cg"): os.path.join(PROF, "cheb_step_cg_chunglu_N1e6_k250_counters.txt"),
}
GOLDEN_BATCH = os.path.join(ROOT, "tests", "golden", "scale_batch8.npz")

WORKLOADS = {
    # Chung-Lu N = 1e6, power-law degrees (exponent 2.5, mean 20, max 2000), k = 250 blocks
    "chunglu-1e6": dict(N=1000000, k=250, p=60, model="chunglu"),
    # SBM N = 1e5, k = 100, mean degree 16, eps = eps_c / 4; d = ceil(4 ln N), p = 50
    "sbm-1e5": dict(N=100000, k=100, s=16.0, p=50, model="sbm"),
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


def live_widths(iters):
    """Columns still iterating at each block-CG iteration t = 1, 2, ... (a
    column leaves the block once it meets the tolerance; iters[j] is the
    iteration at which it did, 0 for a zero right-hand side)."""
    import numpy as np

    it = np.asarray(iters)
    return [int(np.sum(it >= t)) for t in range(1, int(it.max(initial=0)) + 1)]


def job_bytes(N, nnz, k, d, n_c, p, bis_steps, cg_iters):
    """Algorithmic bytes of one pipeline run; cg_iters: the per-column
    iteration counts of the interpolation (each CG iteration counts its live
    columns)."""
    gauss = 4 * N
    count = bis_steps * (gauss * n_c + moment_steps(p) * step_bytes(N, nnz, n_c, "mom"))
    feat = gauss * d + p * step_bytes(N, nnz, d, "clen") + 8 * N * d
    cg = sum(p * step_bytes(N, nnz, w, "clen") + BLOCK_CG_BLOCKS * 4 * N * w
             for w in live_widths(cg_iters))
    return count + feat + cg


def cg_pass_share(iters, k):
    """The block CG's operator passes in units of one pass at the full width
    k: the library runs each pass on a compact copy of the live columns, and
    a step's time follows its gathered lines, ceil(w / 32) per row."""
    return sum(math.ceil(w / 32) for w in live_widths(iters)) / math.ceil(k / 32)


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


def read_traffic(workload, which):
    """Bytes below L2 per launch from the committed counter summary, or None
    (no summary, or the kernel sources changed since it was taken)."""
    path = COUNTERS.get((workload, which))
    if path is None or not os.path.exists(path):
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


def quiet_gc():
    """Collect once and move every object alive after set-up out of the
    collector's reach, so that a full collection (tens of ms with torch
    loaded) does not land inside a timed run."""
    gc.collect()
    gc.freeze()


# ------------------------------------------------------------ CPU oracle ---
# The float64 oracle timed on the host, before the GPU is touched (the
# process pool forks).  Every column of a block is independent in every
# phase, so the all-core form splits the columns into panels over a pool.

_POOL = {}


def _pool_filter(task):
    """One panel of a filter pass in a pool worker: `steps` products of the
    shared CSR matrix with an N x w block (the oracle's recurrence)."""
    import numpy as np

    from oracle import cheb

    w, steps, salt = task
    A, a = _POOL["A"], _POOL["coeffs"][: steps + 1]
    X = np.random.default_rng(salt).standard_normal((A.shape[0], w))
    Y = cheb.filter_block(A, X, a)
    return float(Y[0, 0])


def _pool_kmeans(task):
    from oracle import kmeans

    Fr, k, seed, r = _POOL["km"]
    lab, C, inertia = kmeans.lloyd(Fr, kmeans.seed_plusplus(Fr, k, seed, task), 100)
    return inertia


def _timed_pool_map(pool, fn, tasks):
    t0 = time.perf_counter()
    pool.map(fn, tasks, chunksize=1)
    return time.perf_counter() - t0


def _panels(w, parts):
    base, extra = divmod(w, parts)
    return [base + (1 if i < extra else 0) for i in range(parts) if base + (1 if i < extra else 0) > 0]


def cpu_baseline(head_gr, head_wl, sbm_gr, sbm_wl, workers):
    """The oracle on the host: the headline graph's filter pass (sample: a few
    of its p products, scaled to the pass) on 1 core and on `workers` cores,
    and the 1e5-node SBM per phase of Alg. 2 (bounded samples scaled to one
    graph: one dichotomy test, the feature pass, sampling, k-means replicates,
    one CG iteration on a column panel, labels)."""
    import multiprocessing as mp

    import numpy as np

    from oracle import cheb, eigencount, interp, jackson, kmeans, laplacian, philox, sampling
    from oracle import csc as ocsc

    out = {"kind": "oracle", "unit": "GB/s", "host_cpus": os.cpu_count()}
    # headline graph: filter pass at d columns, `hsteps` of its p products
    A, _ = laplacian.normalized_adjacency(head_gr.row_ptr, head_gr.col)
    N, nnz, p = head_gr.n, head_gr.nnz, head_wl["p"]
    d = int(math.ceil(4 * math.log(N)))
    a = jackson.lowpass_coeffs(0.4, p)
    hsteps = 2
    X = philox.gaussian_block(0, N, d, 0, philox.FEAT)
    t0 = time.perf_counter()
    cheb.filter_block(A, X, a[: hsteps + 1])
    t1 = time.perf_counter() - t0
    del X
    by = hsteps * step_bytes(N, nnz, d, "y")
    # SBM phases
    As, _ = laplacian.normalized_adjacency(sbm_gr.row_ptr, sbm_gr.col)
    Ns, ks, ps = sbm_gr.n, sbm_wl["k"], sbm_wl["p"]
    ds, ncs, ns = int(math.ceil(4 * math.log(Ns))), eigencount.count_signals(Ns), ocsc.default_n(ks)
    one = {}
    t0 = time.perf_counter()
    R = philox.gaussian_block(0, Ns, ncs, 1, philox.COUNT)
    eigencount.eigencount(As, 0.5, ps, R)
    one["dichotomy_per_test"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    F = ocsc.features(As, 0.4, ps, ds, 0)
    one["features"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    omega = sampling.sample(Ns, ns, 0)
    one["sampling"] = time.perf_counter() - t0
    Fr = F[omega]
    km_reps = 2
    t0 = time.perf_counter()
    for r in range(km_reps):
        kmeans.lloyd(Fr, kmeans.seed_plusplus(Fr, ks, 0, r), 100)
    one["kmeans_per_replicate"] = (time.perf_counter() - t0) / km_reps
    labels_r = kmeans.lloyd(Fr, kmeans.seed_plusplus(Fr, ks, 0, 0), 100)[0]
    cg_cols = 10
    mask = interp.sample_mask(Ns, omega)
    B = interp.rhs(Ns, omega, labels_r, ks)[:, :cg_cols]
    t0 = time.perf_counter()
    interp.cg(As, mask, 1e-3, jackson.lowpass_coeffs(0.4, ps), B, tol=0.0, max_iter=1)
    one["cg_iteration_per_column"] = (time.perf_counter() - t0) / cg_cols
    Xl = np.random.default_rng(0).standard_normal((Ns, ks))
    t0 = time.perf_counter()
    interp.hard_labels(Xl)
    one["labels"] = time.perf_counter() - t0

    # all cores: the same samples with the columns (replicates) over a pool
    ctx = mp.get_context("fork")
    _POOL.update(A=A, coeffs=a)
    with ctx.Pool(workers) as pool:
        pool.map(abs, range(workers))  # start every worker before timing
        tN = _timed_pool_map(pool, _pool_filter, [(w, hsteps, i) for i, w in enumerate(_panels(d, workers))])
    _POOL.update(A=As, coeffs=jackson.lowpass_coeffs(0.5, ps), km=(Fr, ks, 0, 0))
    allc = {}
    with ctx.Pool(workers) as pool:
        pool.map(abs, range(workers))
        allc["dichotomy_per_test"] = _timed_pool_map(
            pool, _pool_filter, [(w, ps, i) for i, w in enumerate(_panels(ncs, workers))])
        allc["features"] = _timed_pool_map(
            pool, _pool_filter, [(w, ps, i) for i, w in enumerate(_panels(ds, workers))])
        allc["kmeans_20_replicates"] = _timed_pool_map(pool, _pool_kmeans, list(range(20)))
        allc["cg_iteration_all_columns"] = _timed_pool_map(
            pool, _pool_filter, [(w, ps, i) for i, w in enumerate(_panels(ks, workers))])
    _POOL.clear()

    tests, cg_iters = 9, 13  # the oracle's dichotomy tests and CG iterations on this graph
    if os.path.exists(os.path.join(ROOT, "tests", "golden", "scale_sbm_1e5.npz")):
        g = np.load(os.path.join(ROOT, "tests", "golden", "scale_sbm_1e5.npz"))
        tests, cg_iters = int(g["steps"]), int(g["cg_iters"].max())
    per_graph_1 = {
        "dichotomy": one["dichotomy_per_test"] * tests,
        "features": one["features"],
        "sampling": one["sampling"],
        "kmeans": one["kmeans_per_replicate"] * 20,
        "interpolation": one["cg_iteration_per_column"] * ks * cg_iters,
        "labels": one["labels"],
    }
    per_graph_n = {
        "dichotomy": allc["dichotomy_per_test"] * tests,
        "features": allc["features"],
        "sampling": one["sampling"],
        "kmeans": allc["kmeans_20_replicates"],
        "interpolation": allc["cg_iteration_all_columns"] * cg_iters,
        "labels": one["labels"],
    }
    out.update({
        "value": round(by / tN / 1e9, 3),
        "cores": workers,
        "sample": (f"float64 oracle filter pass on the {N}-node headline graph at d={d} columns: "
                   f"{hsteps} of its p={p} CSR products, columns split over {workers} worker "
                   f"processes ({tN:.2f} s); the host reports {os.cpu_count()} CPUs"),
        "one_core": {"value": round(by / t1 / 1e9, 3), "cores": 1,
                     "sample": f"the same {hsteps} products on one core ({t1:.2f} s)"},
        "sbm_1e5_s_per_graph": {
            "one_core": {kk: round(v, 3) for kk, v in per_graph_1.items()},
            "all_cores": {kk: round(v, 3) for kk, v in per_graph_n.items()},
            "total_one_core": round(sum(per_graph_1.values()), 2),
            "total_all_cores": round(sum(per_graph_n.values()), 2),
            "sample": (f"N={Ns}, k={ks}, d={ds}, n_c={ncs}, p={ps}: one dichotomy test x {tests} "
                       f"tests, one feature pass, sampling, k-means replicates (2 on one core, "
                       f"x10; 20 over the pool), one CG iteration ({cg_cols} columns on one "
                       f"core, x{ks // cg_cols}; all {ks} over the pool) x {cg_iters} iterations "
                       f"(the oracle's counts on this graph), labels; graph generation "
                       f"excluded"),
        },
    })
    return out


# ------------------------------------------------------------ GPU timing ---

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


def step_kernels(api, name, gr, wl, last, reps, dev):
    """Per-launch figures of the three step kernels of the pipeline run
    `last`: the eigencount moment step (natural order), the feature step
    (Clenshaw at width d, natural order) and the CG operator's Clenshaw step
    at width k (in the order the interpolation used)."""
    N, nnz, k, p = gr.n, gr.nnz, wl["k"], wl["p"]
    d = int(math.ceil(4 * math.log(N)))
    n_c = api.count_signals(N)
    group, count_w, count_kind = count_shape(api, n_c)
    out = {}
    for which, w, order, kind, bkind, launches, label in (
            ("count", count_w, None, count_kind, "mom",
             -(-last.bisection.steps // group) * moment_steps(p),
             f"k_cheb_step<EPI_MOMG> (moment step of the eigencount passes, {group} tests of "
             f"{n_c} signals side by side" if group > 1 else
             f"k_cheb_step<EPI_MOM> (moment step of the eigencount passes, {n_c} signals"),
            ("filter", d, None, 3, "clen", p, "k_cheb_step<EPI_CLEN> (Clenshaw step of the feature pass"),
            ("cg", k, last.order, 3, "clen", len(live_widths(last.interp.iters)) * p,
             "k_cheb_step<EPI_CLEN> (Clenshaw step of the CG operator pass")):
        avg_s = step_time(api, gr, order, w, p, reps, dev, kind=kind)
        # the sparse product alone at this width and order (CSR read, gathered
        # rows, one block written): the floor under any step of this shape
        floor_s = step_time(api, gr, order, w, p, reps, dev, kind=5)
        per_launch = step_bytes(N, nnz, w, bkind)
        achieved = per_launch / avg_s / 1e9
        traffic = read_traffic(name, which)
        out[which] = {
            "kernel": f"{label}, w={w}, panel width {api.panel_width(N, w, nnz)}"
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
            "spmm_floor_us": round(floor_s * 1e6, 2),
            "launches_per_step": launches,
            "ms_per_step": round(launches * avg_s * 1e3, 3),
        }
    # the CG passes run at their live widths: time in full-width passes
    share = cg_pass_share(last.interp.iters, k)
    out["cg"]["ms_per_step"] = round(share * p * out["cg"]["avg_launch_us"] / 1e3, 3)
    out["cg"]["kernel"] += (f"; {len(live_widths(last.interp.iters))} iterations with "
                            f"{live_widths(last.interp.iters)} live columns, passes on compact "
                            f"copies of them: ms_per_step counts {share:.2f} full-width passes")
    return out


def timed_runs(api, g, k, d, seed, p, steps, warmup, **kw):
    import torch

    for _ in range(warmup):
        api.run(g, k, d, seed, p=p, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [api.run(g, k, d, seed, p=p, **kw) for _ in range(steps)]
    torch.cuda.synchronize()
    return res, time.perf_counter() - t0


def bench_single(api, name, gr, wl, args, dev, variants):
    """Timed steps of the plain pipeline on one graph; with `variants`, the
    learned-bracket and one-pass KPM forms beside it."""
    import torch

    from oracle.metrics import adjusted_rand_index  # ARI of the labels only

    N, nnz, k, p = gr.n, gr.nnz, wl["k"], wl["p"]
    d = int(math.ceil(4 * math.log(N)))
    n_c = api.count_signals(N)
    g = api.Graph(gr.row_ptr, gr.col, dev)
    torch.cuda.synchronize()
    results, elapsed = timed_runs(api, g, k, d, args.seed, p, args.steps, args.warmup)
    total = sum(job_bytes(N, nnz, k, d, n_c, p, r.bisection.steps, r.interp.iters)
                for r in results)
    last = results[-1]
    lab = last.labels.cpu().numpy()
    out = {
        "workload": f"{name}: {wl['model']} N={N} nnz={nnz} k={k} d={d} p={p} "
                    f"n={api.default_n(k)} n_c={n_c} gamma=1e-3 tol=1e-6",
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "value": round(total / elapsed / 1e9, 3),
        "s_per_graph": round(elapsed / args.steps, 4),
        "phases_s": {kk: round(v, 4) for kk, v in last.timings.items()},
        "bisection_steps": last.bisection.steps,
        "lambda_k": last.lam,
        "cg_iters_max": int(last.interp.iters.max()),
        "cg_live_columns_per_iteration": live_widths(last.interp.iters),
        "ari_vs_truth": round(float(adjusted_rand_index(lab, gr.truth)), 4),
    }
    if variants:
        from paper_1602_02018_amd import learned

        mlp = learned.load_params(dev)
        for key, kw in (("learned", dict(mlp_params=mlp)), ("kpm", dict(lambda_method="kpm"))):
            res, el = timed_runs(api, g, k, d, args.seed, p, args.steps, 1, **kw)
            lv = res[-1].labels.cpu().numpy()
            out[key] = {
                "s_per_graph": round(el / args.steps, 4),
                "tested_points": res[-1].bisection.steps,
                "lambda_k": res[-1].lam,
                "ari_vs_plain": round(float(adjusted_rand_index(lv, lab)), 4),
                "ari_vs_truth": round(float(adjusted_rand_index(lv, gr.truth)), 4),
            }
    steps_k = step_kernels(api, name, gr, wl, last, args.kernel_reps, dev)
    dom = max(steps_k, key=lambda c: steps_k[c]["ms_per_step"])
    out["roofline"] = steps_k[dom]
    for other in steps_k:
        if other != dom:
            out[f"roofline_{other}_step"] = steps_k[other]
    del g
    torch.cuda.empty_cache()
    return out


def bench_batch(api, wl, args, dev):
    """64 SBMs: plain form graph by graph vs batched vs batched + learned
    bracket, and the agreement of their labels (with each other, with the
    planted communities and, on the graphs the oracle's results are stored
    for, with the oracle)."""
    import numpy as np
    import torch

    import synth
    from oracle.metrics import adjusted_rand_index
    from paper_1602_02018_amd import learned

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

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    plain, t_plain = timed(lambda: [api.run(g, k, d, s, p=p) for g, k, d, s in zip(G, ks, ds, seeds)])
    batched, t_batched = timed(lambda: api.run_batched(G, ks, ds, seeds, p=p))
    both, t_both = timed(lambda: api.run_batched(G, ks, ds, seeds, p=p, mlp_params=mlp))
    # the method's own spread: the plain form with other random signals
    other = api.run_batched(G, ks, ds, [s + 1000 for s in seeds], p=p)
    lab = {key: [r.labels.cpu().numpy() for r in res]
           for key, res in (("plain", plain), ("batched", batched), ("both", both), ("other", other))}

    def ari_list(xs, ys):
        return np.array([adjusted_rand_index(x, y) for x, y in zip(xs, ys)])

    a_plain = ari_list(lab["plain"], [g.truth for g in gs])
    a_both = ari_list(lab["both"], [g.truth for g in gs])
    a_pair = ari_list(lab["both"], lab["plain"])
    a_self = ari_list(lab["other"], lab["plain"])
    a_other = ari_list(lab["other"], [g.truth for g in gs])
    same_lam = np.array([x.lam == y.lam for x, y in zip(both, plain)])
    total = sum(job_bytes(g.n, g.nnz, k, d, api.count_signals(g.n), p, r.bisection.steps,
                          r.interp.iters) for g, k, d, r in zip(gs, ks, ds, both))
    out = {
        "workload": (f"batch64: {len(gs)} SBMs, sum N={sum(g.n for g in gs)}, "
                     f"sum nnz={sum(g.nnz for g in gs)}, k in [10,100], p={p}"),
        "value_batched_learned": round(total / t_both / 1e9, 3),
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
        "batched_labels_identical_to_plain": int(sum(np.array_equal(x, y)
                                                     for x, y in zip(lab["batched"], lab["plain"]))),
        # equal-ARI criterion of the speed-up: the learned search stops at another
        # point of the interval where the count rounds to k, so its labels move
        # against the plain ones; what must not move is the recovery
        "ari_vs_truth_mean": {"plain": round(float(a_plain.mean()), 4),
                              "batched_learned": round(float(a_both.mean()), 4)},
        "ari_vs_truth_delta": {"median": round(float(np.median(a_both - a_plain)), 4),
                               "min": round(float((a_both - a_plain).min()), 4),
                               "frac_within_0.01": round(float(np.mean(np.abs(a_both - a_plain) <= 0.01)), 4)},
        # two plain runs differing only in the random signals (seed + 1000)
        "ari_plain_other_signals_vs_plain": {
            "median": round(float(np.median(a_self)), 4),
            "frac_ge_0.99": round(float(np.mean(a_self >= 0.99)), 4),
            "ari_vs_truth_mean": round(float(a_other.mean()), 4)},
        "ari_batched_learned_vs_plain": {
            "median": round(float(np.median(a_pair)), 4),
            "frac_ge_0.99": round(float(np.mean(a_pair >= 0.99)), 4),
            "same_lambda": int(same_lam.sum()),
            "frac_ge_0.99_same_lambda": (round(float(np.mean(a_pair[same_lam] >= 0.99)), 4)
                                         if same_lam.any() else None),
        },
    }
    if os.path.exists(GOLDEN_BATCH):
        gold = np.load(GOLDEN_BATCH)
        # against the labels of the oracle's interpolation solved to 1e-10 (two
        # solutions that both meet 1e-6 can label nearly tied nodes differently)
        vs = {"plain": [], "batched": [], "batched_learned": []}
        tight = "_labels_tight" if f"g{int(gold['positions'][0])}_plain_labels_tight" in gold.files else "_labels"
        for gi in gold["positions"]:
            gi = int(gi)
            vs["plain"].append(adjusted_rand_index(lab["plain"][gi], gold[f"g{gi}_plain{tight}"]))
            vs["batched"].append(adjusted_rand_index(lab["batched"][gi], gold[f"g{gi}_plain{tight}"]))
            vs["batched_learned"].append(adjusted_rand_index(lab["both"][gi], gold[f"g{gi}_learned{tight}"]))
        out["ari_vs_oracle_8_graphs"] = {kk: {"min": round(float(min(v)), 4),
                                              "frac_ge_0.99": round(float(np.mean(np.array(v) >= 0.99)), 4)}
                                         for kk, v in vs.items()}
    del G
    torch.cuda.empty_cache()
    return out


def gather_ceiling(dev, reps=20):
    """The rate at which the GPU serves gathered rows: the sparse product alone
    (csc_cheb_steps kind 5: CSR read, every neighbour row gathered, one block
    written) on random graphs of mean degree 20 (uniform endpoints, random
    node order), for gathered blocks from L2-sized to far beyond the
    Infinity Cache.  Reported as 128-byte cache lines of gathered rows per
    second: a row of w float32 values spans 4w/128 lines (w a multiple of
    32), so this is the ceiling any step kernel of that width meets when its
    gathers miss."""
    import numpy as np
    import torch

    import synth
    from paper_1602_02018_amd import api

    rows = []
    for logn in (16, 18, 20, 21):
        N = 1 << logn
        rng = np.random.default_rng(logn)
        u = rng.integers(0, N, size=10 * N)
        v = rng.integers(0, N, size=10 * N)
        rp, cl = synth.csr_from_edges(N, u, v)
        g = api.Graph(rp, cl, dev)
        for w in (32, 64, 256):
            st = api.StepTimer(g, w, 5)
            st.launch(5)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            st.launch(reps)
            e1.record()
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) / 1e3 / reps
            lines = len(cl) * (4 * w // 128)
            rows.append({"N": N, "nnz": int(len(cl)), "w": w, "gathered_block_MB": round(N * w * 4 / 2**20, 1),
                         "us": round(t * 1e6, 2), "G_lines_per_s": round(lines / t / 1e9, 2),
                         "gathered_GBs": round(lines * 128 / t / 1e9, 1)})
            print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
            del st
        del g
        torch.cuda.empty_cache()
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="chunglu-1e6", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the secondary workloads (1e5-node SBM forms, batch of 64)")
    ap.add_argument("--kernel-reps", type=int, default=4)
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1),
                    help="processes of the all-core CPU baseline")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain 256 MiB device copy (for scaling memory counters)")
    ap.add_argument("--gather-ceiling", action="store_true",
                    help="run only the gathered-row rate of the sparse product on random graphs")
    args = ap.parse_args()
    if args.gather_ceiling:
        import torch

        print(json.dumps({"gather_ceiling": gather_ceiling(torch.device("cuda:0"))}), flush=True)
        return
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
              f"(the path would shard by columns across GPUs; no multi-GPU form is implemented)",
              file=sys.stderr)
        sys.exit(2)

    wl = WORKLOADS[args.workload]
    head_gr = None if args.workload == "batch64" else make_graph(wl, args.seed)
    sbm_wl = WORKLOADS["sbm-1e5"]
    sbm_gr = head_gr if args.workload == "sbm-1e5" else None
    if sbm_gr is None and not (args.no_secondary and args.no_cpu_baseline):
        sbm_gr = make_graph(sbm_wl, args.seed)
    cpu = None
    if not args.no_cpu_baseline and head_gr is not None:
        print(f"cpu baseline ({args.workers} workers) ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(head_gr, wl, sbm_gr, sbm_wl, args.workers)

    import torch

    from paper_1602_02018_amd import api

    dev = torch.device("cuda:0")
    quiet_gc()
    out = {"metric": METRIC}
    if args.workload == "batch64":
        b = bench_batch(api, wl, args, dev)
        out.update(value=b.pop("value_batched_learned"), unit="GB/s", n_gpus=1, steps=1, warmup=1,
                   ms_per_step=round(b["s_per_graph"]["batched_learned"] * 64e3, 3),
                   higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
                   data="synthetic", config={"workload": b.pop("workload"), "form": "batched + learned"})
        out.update(b)
        print(json.dumps(out), flush=True)
        return
    print(f"headline {args.workload} ...", file=sys.stderr, flush=True)
    head = bench_single(api, args.workload, head_gr, wl, args, dev,
                        variants=args.workload != "chunglu-1e6")
    out.update({
        "value": head.pop("value"),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": head.pop("workload"), "form": "plain",
                   "value_is": "whole-pipeline algorithmic bytes / wall time; the SpMM kernel "
                               "rate is roofline.achieved"},
    })
    out.update(head)
    if not args.no_secondary:
        if args.workload != "sbm-1e5":
            print("secondary sbm-1e5 ...", file=sys.stderr, flush=True)
            out["sbm_1e5"] = bench_single(api, "sbm-1e5", sbm_gr, sbm_wl, args, dev, variants=True)
        print("secondary batch64 ...", file=sys.stderr, flush=True)
        out["batch64"] = bench_batch(api, WORKLOADS["batch64"], args, dev)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
