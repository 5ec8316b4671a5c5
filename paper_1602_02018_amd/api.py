"""Python binding of libcsc: argument marshalling only.

PyTorch supplies device memory and the current HIP stream; every step on
graph-sized data runs in the library's kernels (k-means on the n sampled
features runs on the host inside the library).  The functions mirror the C
calls of include/csc.h; ``run`` chains them into Alg. 2.
"""
from __future__ import annotations

import ctypes as C
import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib
from ._lib import CscGraph, check, lib


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _ws(nbytes: int, device):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def _i32_device(x, device):
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=torch.int32).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.int32), device=device)


# degree skew (csc_row_schedule) from which the row schedule is attached:
# about 1.4 on the Poisson-degree SBMs, where it costs a few percent, 3.4 on
# the 1e6-node Chung-Lu graph, where the moment step gains 19%
SCHED_MIN_SKEW = 2.0


class Graph:
    """A = D^-1/2 W D^-1/2 on the GPU, built by csc_laplacian_from_adjacency."""

    def __init__(self, row_ptr, col, device="cuda", weights=None, check_csr: int = 1):
        """check_csr: 0 no check, 1 CSR form, 2 also no self-loops, sorted rows, symmetric W."""
        self.device = torch.device(device)
        self.row_ptr = _i32_device(row_ptr, self.device)
        self.col = _i32_device(col, self.device)
        self.n = int(self.row_ptr.numel() - 1)
        self.nnz = int(self.col.numel())
        w = None
        if weights is not None:
            w = torch.as_tensor(np.asarray(weights, dtype=np.float32), device=self.device)
        self.val = torch.empty(max(self.nnz, 1), dtype=torch.float32, device=self.device)
        self.dinv_sqrt = torch.empty(self.n, dtype=torch.float32, device=self.device)
        check(lib().csc_laplacian_from_adjacency(self.n, self.nnz, _ptr(self.row_ptr),
                                                 _ptr(self.col), _ptr(w), _ptr(self.val),
                                                 _ptr(self.dinv_sqrt), int(check_csr),
                                                 _stream()), "csc_laplacian_from_adjacency")
        # the step kernels' row walk (rows of similar degree share a wave),
        # attached when the degrees are skewed enough for it to pay
        self.sched = torch.empty(self.n, dtype=torch.int32, device=self.device)
        skew = C.c_double(1.0)
        ws = _ws(256, self.device)
        check(lib().csc_row_schedule(self.n, _ptr(self.row_ptr), _ptr(self.sched), C.byref(skew),
                                     _ptr(ws), ws.numel(), _stream()), "csc_row_schedule")
        self.skew = skew.value
        use = self.skew >= SCHED_MIN_SKEW
        self.c = CscGraph(self.n, self.nnz, self.row_ptr.data_ptr(), self.col.data_ptr(),
                          self.val.data_ptr(), self.dinv_sqrt.data_ptr(),
                          self.sched.data_ptr() if use else None)

    def use_schedule(self, on: bool) -> None:
        """Attach (or detach) the row schedule regardless of the skew."""
        self.c.sched = self.sched.data_ptr() if on else None

    @property
    def ref(self):
        return C.byref(self.c)


def version() -> int:
    return int(lib().csc_version())


def set_panel_width(pw: int) -> None:
    check(lib().csc_set_panel_width(int(pw)), "csc_set_panel_width")


def set_tuning(key: int, value: int) -> None:
    check(lib().csc_set_tuning(int(key), int(value)), "csc_set_tuning")


def set_damping(damping: int) -> None:
    """Jackson-damped (0, default) or plain truncated (1) Chebyshev low-pass."""
    check(lib().csc_set_damping(int(damping)), "csc_set_damping")


def get_damping() -> int:
    return int(lib().csc_get_damping())


def set_filter_form(form: int) -> None:
    """Forward recurrence (0) or Clenshaw (1, default) for accumulated filters."""
    check(lib().csc_set_filter_form(int(form)), "csc_set_filter_form")


def get_filter_form() -> int:
    return int(lib().csc_get_filter_form())


def get_tuning(key: int) -> int:
    return int(lib().csc_get_tuning(int(key)))


def autotune(g: Graph, w: int, kind: int = 0, reps: int = 20):
    """Times candidate panel widths for (g, w); the winner is used for this shape from now on."""
    pw, xcd, us = C.c_int32(0), C.c_int32(0), C.c_double(0.0)
    ws = _ws(lib().csc_cheb_steps_workspace_bytes(g.n, w), g.device)
    check(lib().csc_autotune(g.ref, int(w), int(kind), int(reps), C.byref(pw), C.byref(xcd),
                             C.byref(us), _ptr(ws), ws.numel(), _stream()), "csc_autotune")
    return pw.value, xcd.value, us.value


def autotune_clear() -> None:
    lib().csc_autotune_clear()


def panel_width(n: int, w: int, nnz: int = 0) -> int:
    return int(lib().csc_get_panel_width(int(n), int(nnz) if nnz else 16 * int(n), int(w)))


def jackson_coeffs(lam: float, p: int) -> np.ndarray:
    a = np.zeros(p + 1)
    check(lib().csc_jackson_coeffs(float(lam), int(p), a.ctypes.data_as(_lib.pd)), "csc_jackson_coeffs")
    return a


def gaussian_block(n_rows: int, w: int, seed: int, t: int, stream_id: int, device="cuda"):
    R = torch.empty((n_rows, w), dtype=torch.float32, device=device)
    check(lib().csc_gaussian_block(n_rows, w, seed, t, stream_id, _ptr(R), w, _stream()),
          "csc_gaussian_block")
    return R


def filter_block(g: Graph, coeffs, X: torch.Tensor) -> torch.Tensor:
    coeffs = np.ascontiguousarray(coeffs, dtype=np.float64)
    X = X.contiguous()
    n, w = X.shape
    Y = torch.empty_like(X)
    ws = _ws(lib().csc_filter_workspace_bytes(n, w), X.device)
    check(lib().csc_filter_block(g.ref, coeffs.ctypes.data_as(_lib.pd), len(coeffs) - 1, _ptr(X),
                                 w, w, _ptr(Y), _ptr(ws), ws.numel(), _stream()), "csc_filter_block")
    return Y


def filter(g: Graph, lam: float, p: int, d: int, seed: int, rows=None, normalize: bool = True):
    """Alg. 2 steps 2-4 (and the row selection of step 5 when ``rows`` is given)."""
    rows_t = None if rows is None else _i32_device(rows, g.device)
    n_rows = g.n if rows_t is None else int(rows_t.numel())
    Y = torch.empty((n_rows, d), dtype=torch.float32, device=g.device)
    ws = _ws(lib().csc_filter_workspace_bytes(g.n, d), g.device)
    check(lib().csc_filter(g.ref, float(lam), p, d, seed, _ptr(rows_t), n_rows if rows_t is not None else 0,
                           1 if normalize else 0, _ptr(Y), d, _ptr(ws), ws.numel(), _stream()),
          "csc_filter")
    return Y


def eigencount(g: Graph, lam: float, p: int, n_signals: int, seed: int, t: int = 1):
    cnt = C.c_double(0.0)
    mom = np.zeros(p + 1)
    ws = _ws(lib().csc_estimate_workspace_bytes(g.n, n_signals, p), g.device)
    check(lib().csc_eigencount(g.ref, float(lam), p, n_signals, seed, t, C.byref(cnt),
                               mom.ctypes.data_as(_lib.pd), _ptr(ws), ws.numel(), _stream()),
          "csc_eigencount")
    return cnt.value, mom


@dataclass
class Bisection:
    lam: float
    steps: int
    trace: list
    moments: np.ndarray
    status: int


def estimate_lambda_k(g: Graph, k: int, p: int, n_signals: int, seed: int, max_steps: int = 30,
                      bracket=None) -> Bisection:
    lam = C.c_double(0.0)
    steps = C.c_int32(0)
    trace = np.zeros(2 * max_steps * 2)
    mom = np.zeros(p + 1)
    br = None
    if bracket is not None:
        br_arr = np.ascontiguousarray(bracket, dtype=np.float64)
        br = br_arr.ctypes.data_as(_lib.pd)
    ws = _ws(lib().csc_estimate_workspace_bytes(g.n, n_signals, p), g.device)
    st = check(lib().csc_estimate_lambda_k(g.ref, k, p, n_signals, seed, max_steps, br,
                                           C.byref(lam), C.byref(steps),
                                           trace.ctypes.data_as(_lib.pd),
                                           mom.ctypes.data_as(_lib.pd), _ptr(ws), ws.numel(),
                                           _stream()), "csc_estimate_lambda_k")
    tr = [(trace[2 * i], trace[2 * i + 1]) for i in range(steps.value)]
    return Bisection(lam.value, steps.value, tr, mom, st)


def estimate_lambda_k_kpm(g: Graph, k: int, p: int, n_signals: int, seed: int,
                          max_steps: int = 30) -> Bisection:
    """One moment pass, then the dichotomy on its count curve (csc_estimate_lambda_k_kpm).
    ``steps`` counts tested points; the GPU ran one pass."""
    lam = C.c_double(0.0)
    steps = C.c_int32(0)
    trace = np.zeros(2 * max_steps)
    mom = np.zeros(p + 1)
    ws = _ws(lib().csc_estimate_workspace_bytes(g.n, n_signals, p), g.device)
    st = check(lib().csc_estimate_lambda_k_kpm(g.ref, k, p, n_signals, seed, max_steps,
                                               C.byref(lam), C.byref(steps),
                                               trace.ctypes.data_as(_lib.pd),
                                               mom.ctypes.data_as(_lib.pd), _ptr(ws), ws.numel(),
                                               _stream()), "csc_estimate_lambda_k_kpm")
    tr = [(trace[2 * i], trace[2 * i + 1]) for i in range(steps.value)]
    return Bisection(lam.value, steps.value, tr, mom, st)


def sample(N: int, n: int, seed: int, device="cuda") -> torch.Tensor:
    idx = torch.empty(n, dtype=torch.int32, device=device)
    ws = _ws(lib().csc_sample_workspace_bytes(N, n), device)
    check(lib().csc_sample(N, n, seed, _ptr(idx), _ptr(ws), ws.numel(), _stream()), "csc_sample")
    return idx


def kmeans_reduced(F, k: int, seed: int, replicates: int = 20, max_iter: int = 100):
    """Host k-means of the library on an n x d float32 or float64 matrix."""
    if isinstance(F, torch.Tensor):
        F = F.detach().cpu().numpy()
    F = np.ascontiguousarray(F)
    n, d = F.shape
    labels = np.zeros(n, dtype=np.int32)
    inertia = C.c_double(0.0)
    if F.dtype == np.float64:
        fn, name = lib().csc_kmeans_reduced_f64, "csc_kmeans_reduced_f64"
    else:
        F = F.astype(np.float32, copy=False)
        fn, name = lib().csc_kmeans_reduced, "csc_kmeans_reduced"
    check(fn(C.c_void_p(F.ctypes.data), n, d, d, k, replicates, max_iter, seed,
             labels.ctypes.data_as(_lib.pi), C.byref(inertia)), name)
    return labels, inertia.value


def kmeans_reduced_device(F: torch.Tensor, k: int, seed: int, replicates: int = 20,
                          max_iter: int = 100):
    """csc_kmeans_reduced_device: the host k-means, bit for bit, on the GPU."""
    assert F.is_cuda and F.dtype == torch.float32 and F.dim() == 2 and F.stride(1) == 1
    n, d = F.shape
    labels = np.zeros(n, dtype=np.int32)
    inertia = C.c_double()
    ws = _ws(lib().csc_kmeans_device_workspace_bytes(n, d, k, replicates), F.device)
    check(lib().csc_kmeans_reduced_device(_ptr(F), n, d, F.stride(0), k, replicates, max_iter,
                                          seed, labels.ctypes.data_as(_lib.pi), C.byref(inertia),
                                          _ptr(ws), ws.numel(), _stream()),
          "csc_kmeans_reduced_device")
    return labels, inertia.value


def kmeans_seeds(F, k: int, seed: int, replicates: int = 20) -> np.ndarray:
    """csc_kmeans_seeds: the host k-means++ picks, replicates x k point indices."""
    if isinstance(F, torch.Tensor):
        F = F.detach().cpu().numpy()
    F = np.ascontiguousarray(F, dtype=np.float64)
    n, d = F.shape
    picks = np.zeros((replicates, k), dtype=np.int32)
    check(lib().csc_kmeans_seeds(C.c_void_p(F.ctypes.data), n, d, d, k, replicates, seed,
                                 picks.ctypes.data_as(_lib.pi)), "csc_kmeans_seeds")
    return picks


def kmeans_seeds_device(F: torch.Tensor, k: int, seed: int, replicates: int = 20) -> np.ndarray:
    """csc_kmeans_seeds_device: the GPU k-means++ picks, replicates x k point indices."""
    assert F.is_cuda and F.dtype == torch.float32 and F.dim() == 2 and F.stride(1) == 1
    n, d = F.shape
    picks = np.zeros((replicates, k), dtype=np.int32)
    ws = _ws(lib().csc_kmeans_device_workspace_bytes(n, d, k, replicates), F.device)
    check(lib().csc_kmeans_seeds_device(_ptr(F), n, d, F.stride(0), k, replicates, seed,
                                        picks.ctypes.data_as(_lib.pi), _ptr(ws), ws.numel(),
                                        _stream()), "csc_kmeans_seeds_device")
    return picks


GOLDEN = 0x9E3779B97F4A7C15


def run_seed(seed: int, t: int) -> int:
    """Seed of run t of the community-core repetitions (run 0 is the plain run)."""
    return (int(seed) + t * GOLDEN) % (1 << 64)


def community_cores(labels_runs, k: int) -> np.ndarray:
    """csc_community_cores: labels_runs is T x n; returns int32[n] (-1 outside the cores)."""
    L = np.ascontiguousarray(labels_runs, dtype=np.int32)
    T, n = L.shape
    out = np.zeros(n, dtype=np.int32)
    check(lib().csc_community_cores(n, T, k, L.ctypes.data_as(_lib.pi), out.ctypes.data_as(_lib.pi)),
          "csc_community_cores")
    return out


@dataclass
class Interpolation:
    X: torch.Tensor
    labels: torch.Tensor
    iters: np.ndarray
    relres: np.ndarray
    status: int


CG_COLUMNS, CG_BLOCK, CG_BLOCK_JACOBI = 0, 1, 2


def interpolate(g: Graph, lam: float, p: int, gamma: float, idx, labels_r, k: int,
                tol: float = 1e-6, max_iter: int = 1000, want_X: bool = True,
                order: torch.Tensor | None = None, method: int = CG_BLOCK_JACOBI,
                weights: torch.Tensor | None = None) -> Interpolation:
    """Eq. (5) by CG (``method``: CG_BLOCK, one block CG over the k columns,
    CG_BLOCK_JACOBI, the same preconditioned by diag(mask) + gamma I, or
    CG_COLUMNS, k side-by-side CGs); with ``order`` (a permutation, see
    community_order) the solve runs on the graph listed in that order,
    outputs in node order."""
    idx_t = _i32_device(idx, g.device)
    lab_t = _i32_device(labels_r, g.device)
    ord_t = None if order is None else _i32_device(order, g.device)
    w_t = None if weights is None else torch.as_tensor(weights, dtype=torch.float32, device=g.device).contiguous()
    n = int(idx_t.numel())
    X = torch.empty((g.n, k), dtype=torch.float32, device=g.device) if want_X else None
    labels = torch.empty(g.n, dtype=torch.int32, device=g.device)
    iters = np.zeros(k, dtype=np.int32)
    relres = np.zeros(k)
    ws = _ws(lib().csc_interpolate_workspace_bytes(g.n, g.nnz, k, n), g.device)
    st = check(lib().csc_interpolate(g.ref, _ptr(ord_t), int(method), float(lam), p, float(gamma),
                                     _ptr(idx_t),
                                     _ptr(lab_t), _ptr(w_t), n, k, float(tol), max_iter, _ptr(X), k,
                                     _ptr(labels), iters.ctypes.data_as(_lib.pi),
                                     relres.ctypes.data_as(_lib.pd), _ptr(ws), ws.numel(),
                                     _stream()), "csc_interpolate")
    return Interpolation(X, labels, iters, relres, st)


# the community order pays off when most gathers stay inside a community
ORDER_MIN_SAME_LABEL = 0.25


def community_order(g: Graph, F: torch.Tensor, idx, labels_r, k: int, want_labels: bool = False,
                    want_frac: bool = False):
    """Node order by nearest k-means centroid (csc_community_order).

    F: device N x d features of every node; idx: sampled nodes; labels_r: their
    k-means labels.  Returns the order (device int32[N]), then, with
    ``want_labels``, every node's nearest-centroid label and, with
    ``want_frac``, the fraction of edges whose ends share a label."""
    assert F.is_cuda and F.dtype == torch.float32 and F.dim() == 2 and F.stride(1) == 1
    N, d = F.shape
    assert N == g.n
    idx_t = _i32_device(idx, F.device)
    lab = np.ascontiguousarray(labels_r, dtype=np.int32)
    n = int(idx_t.numel())
    order = torch.empty(N, dtype=torch.int32, device=F.device)
    nl = torch.empty(N, dtype=torch.int32, device=F.device) if want_labels else None
    frac = C.c_double(0.0)
    ws = _ws(lib().csc_community_order_workspace_bytes(N, d, k, n), F.device)
    check(lib().csc_community_order(g.ref, _ptr(F), F.stride(0), d, _ptr(idx_t),
                                    lab.ctypes.data_as(_lib.pi), n, k, _ptr(order), _ptr(nl),
                                    C.byref(frac), _ptr(ws), ws.numel(), _stream()),
          "csc_community_order")
    out = (order,)
    if want_labels:
        out += (nl,)
    if want_frac:
        out += (frac.value,)
    return out if len(out) > 1 else order


def normalize_rows(Y: torch.Tensor) -> torch.Tensor:
    """Unit rows in place (csc_normalize_rows); returns the float64 squared norms."""
    assert Y.is_cuda and Y.dtype == torch.float32 and Y.dim() == 2 and Y.stride(1) == 1
    sq = torch.empty(Y.shape[0], dtype=torch.float64, device=Y.device)
    check(lib().csc_normalize_rows(_ptr(Y), Y.stride(0), Y.shape[0], Y.shape[1], _ptr(sq),
                                   _stream()), "csc_normalize_rows")
    return sq


def sample_density(w: torch.Tensor, n: int, seed: int, decoder_weights: bool = True):
    """Variable-density sampling on weights w (device float64[N]); returns
    (omega, decoder weights or None)."""
    assert w.is_cuda and w.dtype == torch.float64 and w.dim() == 1
    N = w.numel()
    idx = torch.empty(n, dtype=torch.int32, device=w.device)
    dw = torch.empty(n, dtype=torch.float32, device=w.device) if decoder_weights else None
    ws = _ws(lib().csc_sample_density_workspace_bytes(N), w.device)
    check(lib().csc_sample_density(N, n, seed, _ptr(w), _ptr(idx), _ptr(dw), _ptr(ws), ws.numel(),
                                   _stream()), "csc_sample_density")
    return idx, dw


def gather_rows(F: torch.Tensor, rows) -> torch.Tensor:
    """F[rows] through csc_gather_rows."""
    assert F.is_cuda and F.dtype == torch.float32 and F.dim() == 2 and F.stride(1) == 1
    N, d = F.shape
    rows_t = _i32_device(rows, F.device)
    n = int(rows_t.numel())
    out = torch.empty((n, d), dtype=torch.float32, device=F.device)
    ws = _ws(256, F.device)
    check(lib().csc_gather_rows(_ptr(F), F.stride(0), N, d, _ptr(rows_t), n, _ptr(out), d,
                                _ptr(ws), ws.numel(), _stream()), "csc_gather_rows")
    return out


class StepTimer:
    """Launches Chebyshev-step kernels through csc_cheb_steps (measurement hook)."""

    def __init__(self, g: Graph, w: int, kind: int = 0):
        self.g, self.w, self.kind = g, w, kind
        self.ws = _ws(lib().csc_cheb_steps_workspace_bytes(g.n, w), g.device)
        self.launch(0, prepare=True)

    def launch(self, steps: int, prepare: bool = False):
        check(lib().csc_cheb_steps(self.g.ref, self.w, self.kind, 1 if prepare else 0, steps,
                                   _ptr(self.ws), self.ws.numel(), _stream()), "csc_cheb_steps")


# ------------------------------------------------------------ Alg. 2 ---------

def default_n(k: int) -> int:
    """n = ceil(2 k ln k) sampled nodes (Alg. 2), at least k."""
    return max(k, int(math.ceil(2.0 * k * math.log(k))))


def count_signals(N: int) -> int:
    """n_c = ceil(2 ln N) eigencount signals (Sec. 4.3), at least one."""
    return max(1, int(math.ceil(2.0 * math.log(N))))


@dataclass
class Result:
    lam: float
    bisection: Bisection
    omega: torch.Tensor
    features: torch.Tensor
    labels_r: np.ndarray
    inertia: float
    interp: Interpolation
    timings: dict = field(default_factory=dict)
    order: torch.Tensor | None = None  # node order of the interpolation, if any

    @property
    def labels(self) -> torch.Tensor:
        return self.interp.labels


def run(g: Graph, k: int, d: int, seed: int, p: int = 50, n: int | None = None,
        gamma: float = 1e-3, n_c: int | None = None, tol: float = 1e-6, max_iter: int = 1000,
        max_steps: int = 30, replicates: int = 20, kmeans_iter: int = 100, lam: float | None = None,
        bracket=None, want_X: bool = False, mlp_params: torch.Tensor | None = None,
        reorder: bool = True, cg: int = CG_BLOCK_JACOBI, kmeans_on_gpu: bool = True,
        sampling: str = "uniform", lambda_method: str = "dichotomy", cores: int = 1) -> Result:
    """Compressive spectral clustering (Alg. 2) with every graph-sized step on the GPU.

    With ``mlp_params`` the dichotomy starts from the learned bracket.  With
    ``reorder`` the feature pass keeps every node's features, and the
    interpolation runs on the graph listed community by community
    (community_order); the sampled features, and so the k-means, are the same
    either way.
    """
    n = default_n(k) if n is None else n
    n_c = count_signals(g.n) if n_c is None else n_c
    tm = {}
    t0 = time.perf_counter()
    if lam is None and lambda_method == "kpm":
        bis = estimate_lambda_k_kpm(g, k, p, n_c, seed, max_steps)
        lam = bis.lam
    elif lam is None and mlp_params is not None:
        lb = estimate_lambda_k_learned(g, k, p, n_c, seed, mlp_params, max_steps)
        bis = Bisection(lb.lam, lb.steps, lb.trace, np.zeros(p + 1), lb.status)
        lam = lb.lam
    elif lam is None:
        bis = estimate_lambda_k(g, k, p, n_c, seed, max_steps, bracket)
        lam = bis.lam
    else:
        bis = Bisection(lam, 0, [], np.zeros(p + 1), 0)
    t1 = time.perf_counter()
    reorder = reorder and d <= 128
    density = sampling == "density"
    dec_w = None
    if reorder or density:
        F_all = filter(g, lam, p, d, seed, rows=None, normalize=False)
        sq = normalize_rows(F_all)
        if density:
            omega, dec_w = sample_density(sq, n, seed)
        else:
            omega = sample(g.n, n, seed, g.device)
        F = gather_rows(F_all, omega)
    else:
        omega = sample(g.n, n, seed, g.device)
        F = filter(g, lam, p, d, seed, rows=omega, normalize=True)
    t2 = time.perf_counter()
    if kmeans_on_gpu:
        labels_r, inertia = kmeans_reduced_device(F, k, seed, replicates, kmeans_iter)
    else:
        labels_r, inertia = kmeans_reduced(F.cpu().numpy(), k, seed, replicates, kmeans_iter)
    t3 = time.perf_counter()
    order = None
    if reorder:
        order, frac = community_order(g, F_all, omega, labels_r, k, want_frac=True)
        if frac < ORDER_MIN_SAME_LABEL:
            order = None
    omega_i, labels_i, w_i = omega, labels_r, dec_w
    if cores > 1:  # community cores: T - 1 more filterings and clusterings
        runs = [labels_r]
        for t in range(1, cores):
            Ft = filter(g, lam, p, d, run_seed(seed, t), rows=omega, normalize=True)
            lt, _ = (kmeans_reduced_device(Ft, k, seed, replicates, kmeans_iter) if kmeans_on_gpu
                     else kmeans_reduced(Ft.cpu().numpy(), k, seed, replicates, kmeans_iter))
            runs.append(lt)
        cl = community_cores(np.stack(runs), k)
        keep = np.nonzero(cl >= 0)[0]
        keep_t = torch.as_tensor(keep, device=g.device)
        omega_i = omega[keep_t]
        labels_i = cl[keep]
        w_i = None if dec_w is None else dec_w[keep_t]
    it = interpolate(g, lam, p, gamma, omega_i, labels_i, k, tol, max_iter, want_X=want_X,
                     order=order, method=cg, weights=w_i)
    torch.cuda.current_stream().synchronize()
    t4 = time.perf_counter()
    tm.update(bisection_s=t1 - t0, features_s=t2 - t1, kmeans_s=t3 - t2, interpolate_s=t4 - t3,
              total_s=t4 - t0)
    return Result(lam, bis, omega, F, labels_r, inertia, it, tm, order)


# ------------------------------------------------------------ batched --------

def _i32(xs):
    return np.ascontiguousarray(xs, dtype=np.int32)


def _pa(ptrs):
    """ctypes array of void pointers (device or host addresses)."""
    arr = (C.c_void_p * len(ptrs))(*[C.c_void_p(int(p) if p else 0) for p in ptrs])
    return arr


def _graphs(graphs):
    return (CscGraph * len(graphs))(*[g.c for g in graphs])


def estimate_lambda_k_batched(graphs, ks, p, n_signals, seeds, max_steps=30, brackets=None,
                              mlp_params=None):
    G = len(graphs)
    ga = _graphs(graphs)
    ks, ns = _i32(ks), _i32(n_signals)
    sd = np.ascontiguousarray(seeds, dtype=np.uint64)
    lam = np.zeros(G)
    steps = np.zeros(G, dtype=np.int32)
    status = np.zeros(G, dtype=np.int32)
    trace = np.zeros((G, 2 * max_steps, 2))
    mom = np.zeros((G, p + 1))
    br = None
    if brackets is not None:
        br_arr = np.ascontiguousarray(brackets, dtype=np.float64).reshape(G, 2)
        br = br_arr.ctypes.data_as(_lib.pd)
    dev = graphs[0].device
    ws = _ws(lib().csc_estimate_workspace_bytes_batched(ga, G, ns.ctypes.data_as(_lib.pi), p), dev)
    check(lib().csc_estimate_lambda_k_batched(
        ga, G, ks.ctypes.data_as(_lib.pi), p, ns.ctypes.data_as(_lib.pi), sd.ctypes.data_as(_lib.pu),
        max_steps, br, _ptr(mlp_params), lam.ctypes.data_as(_lib.pd), steps.ctypes.data_as(_lib.pi),
        trace.ctypes.data_as(_lib.pd), mom.ctypes.data_as(_lib.pd), status.ctypes.data_as(_lib.pi),
        _ptr(ws), ws.numel(), _stream()), "csc_estimate_lambda_k_batched")
    return [Bisection(float(lam[g]), int(steps[g]),
                      [(trace[g, i, 0], trace[g, i, 1]) for i in range(steps[g])], mom[g].copy(),
                      int(status[g])) for g in range(G)]


def filter_batched(graphs, lams, p, ds, seeds, rows, normalize=True):
    """csc_filter_batched; rows[g] None keeps all N_g rows."""
    G = len(graphs)
    ga = _graphs(graphs)
    dev = graphs[0].device
    rows_t = [None if r is None else _i32_device(r, dev) for r in rows]
    n_rows = _i32([g.n if r is None else r.numel() for g, r in zip(graphs, rows_t)])
    ds = _i32(ds)
    Ys = [torch.empty((int(n_rows[g]), int(ds[g])), dtype=torch.float32, device=dev) for g in range(G)]
    lam = np.ascontiguousarray(lams, dtype=np.float64)
    sd = np.ascontiguousarray(seeds, dtype=np.uint64)
    ws = _ws(lib().csc_filter_workspace_bytes_batched(ga, G, ds.ctypes.data_as(_lib.pi), p), dev)
    check(lib().csc_filter_batched(ga, G, lam.ctypes.data_as(_lib.pd), p, ds.ctypes.data_as(_lib.pi),
                                   sd.ctypes.data_as(_lib.pu),
                                   _pa([0 if r is None else r.data_ptr() for r in rows_t]),
                                   n_rows.ctypes.data_as(_lib.pi), 1 if normalize else 0,
                                   _pa([y.data_ptr() for y in Ys]), ds.ctypes.data_as(_lib.pi),
                                   _ptr(ws), ws.numel(), _stream()), "csc_filter_batched")
    return Ys


def interpolate_batched(graphs, lams, p, gamma, idx, labels_r, ks, tol=1e-6, max_iter=1000,
                        want_X=True, orders=None, method=CG_BLOCK_JACOBI, weights=None):
    G = len(graphs)
    ga = _graphs(graphs)
    dev = graphs[0].device
    idx_t = [_i32_device(x, dev) for x in idx]
    lab_t = [_i32_device(x, dev) for x in labels_r]
    ns = _i32([x.numel() for x in idx_t])
    ks = _i32(ks)
    Xs = [torch.empty((g.n, int(ks[i])), dtype=torch.float32, device=dev) if want_X else None
          for i, g in enumerate(graphs)]
    labels = [torch.empty(g.n, dtype=torch.int32, device=dev) for g in graphs]
    iters = np.zeros(int(ks.sum()), dtype=np.int32)
    relres = np.zeros(int(ks.sum()))
    status = np.zeros(G, dtype=np.int32)
    lam = np.ascontiguousarray(lams, dtype=np.float64)
    ws = _ws(lib().csc_interpolate_workspace_bytes_batched(ga, G, ks.ctypes.data_as(_lib.pi), p), dev)
    ord_t = None if orders is None else [None if o is None else _i32_device(o, dev) for o in orders]
    st = check(lib().csc_interpolate_batched(
        ga, G, None if ord_t is None else _pa([0 if o is None else o.data_ptr() for o in ord_t]),
        int(method), lam.ctypes.data_as(_lib.pd), p, float(gamma), _pa([x.data_ptr() for x in idx_t]),
        _pa([x.data_ptr() for x in lab_t]),
        None if weights is None else _pa([0 if w is None else w.data_ptr() for w in weights]), ns.ctypes.data_as(_lib.pi), ks.ctypes.data_as(_lib.pi),
        float(tol), max_iter, _pa([x.data_ptr() if x is not None else 0 for x in Xs]) if want_X else None,
        ks.ctypes.data_as(_lib.pi), _pa([x.data_ptr() for x in labels]),
        iters.ctypes.data_as(_lib.pi), relres.ctypes.data_as(_lib.pd), status.ctypes.data_as(_lib.pi),
        _ptr(ws), ws.numel(), _stream()), "csc_interpolate_batched")
    out, off = [], 0
    for g in range(G):
        kg = int(ks[g])
        out.append(Interpolation(Xs[g], labels[g], iters[off:off + kg].copy(),
                                 relres[off:off + kg].copy(), int(status[g])))
        off += kg
    return out


def kmeans_reduced_batched(Fs, ks, seeds, replicates=20, max_iter=100):
    G = len(Fs)
    Fs = [np.ascontiguousarray(f.detach().cpu().numpy() if isinstance(f, torch.Tensor) else f,
                               dtype=np.float32) for f in Fs]
    ns = _i32([f.shape[0] for f in Fs])
    ds = _i32([f.shape[1] for f in Fs])
    ks = _i32(ks)
    sd = np.ascontiguousarray(seeds, dtype=np.uint64)
    labels = [np.zeros(f.shape[0], dtype=np.int32) for f in Fs]
    inertia = np.zeros(G)
    check(lib().csc_kmeans_reduced_batched(G, _pa([f.ctypes.data for f in Fs]), ns.ctypes.data_as(_lib.pi),
                                           ds.ctypes.data_as(_lib.pi), ks.ctypes.data_as(_lib.pi),
                                           replicates, max_iter, sd.ctypes.data_as(_lib.pu),
                                           _pa([l.ctypes.data for l in labels]),
                                           inertia.ctypes.data_as(_lib.pd)), "csc_kmeans_reduced_batched")
    return labels, inertia


def kmeans_reduced_device_batched(Fs, ks, seeds, replicates=20, max_iter=100):
    G = len(Fs)
    for f in Fs:
        assert f.is_cuda and f.dtype == torch.float32 and f.dim() == 2 and f.is_contiguous()
    ns = _i32([f.shape[0] for f in Fs])
    ds = _i32([f.shape[1] for f in Fs])
    ks = _i32(ks)
    sd = np.ascontiguousarray(seeds, dtype=np.uint64)
    labels = [np.zeros(f.shape[0], dtype=np.int32) for f in Fs]
    inertia = np.zeros(G)
    pi_ = _lib.pi
    ws = _ws(lib().csc_kmeans_device_workspace_bytes_batched(G, ns.ctypes.data_as(pi_),
                                                            ds.ctypes.data_as(pi_),
                                                            ks.ctypes.data_as(pi_), replicates),
             Fs[0].device)
    check(lib().csc_kmeans_reduced_device_batched(
        G, _pa([f.data_ptr() for f in Fs]), ns.ctypes.data_as(pi_), ds.ctypes.data_as(pi_),
        ks.ctypes.data_as(pi_), replicates, max_iter, sd.ctypes.data_as(_lib.pu),
        _pa([l.ctypes.data for l in labels]), inertia.ctypes.data_as(_lib.pd), _ptr(ws), ws.numel(),
        _stream()), "csc_kmeans_reduced_device_batched")
    return labels, inertia


def run_batched(graphs, ks, ds, seeds, p=50, ns=None, gamma=1e-3, n_cs=None, tol=1e-6,
                max_iter=1000, max_steps=30, replicates=20, kmeans_iter=100, brackets=None,
                lams=None, want_X=False, mlp_params=None, reorder=True, cg=CG_BLOCK_JACOBI,
                kmeans_on_gpu=True, sampling="uniform"):
    """Alg. 2 for G graphs at once with the batched calls; graph g matches run(graphs[g], ...)."""
    G = len(graphs)
    ns = [default_n(k) for k in ks] if ns is None else list(ns)
    n_cs = [count_signals(g.n) for g in graphs] if n_cs is None else list(n_cs)
    tm = {}
    t0 = time.perf_counter()
    if lams is None:
        bis = estimate_lambda_k_batched(graphs, ks, p, n_cs, seeds, max_steps, brackets, mlp_params)
        lams = [b.lam for b in bis]
    else:
        bis = [Bisection(l, 0, [], np.zeros(p + 1), 0) for l in lams]
    t1 = time.perf_counter()
    density = sampling == "density"
    re = [reorder and d <= 128 for d in ds]
    full = [r or density for r in re]
    dec_ws = None
    if any(full):
        omegas = [None if f else sample(g.n, n, sd, g.device)
                  for g, n, sd, f in zip(graphs, ns, seeds, full)]
        F_all = filter_batched(graphs, lams, p, ds, seeds, omegas, normalize=False)
        dec_ws = [None] * G
        for i in range(G):
            if not full[i]:
                normalize_rows(F_all[i])
                continue
            sq = normalize_rows(F_all[i])
            if density:
                omegas[i], dec_ws[i] = sample_density(sq, ns[i], seeds[i])
            else:
                omegas[i] = sample(graphs[i].n, ns[i], seeds[i], graphs[i].device)
        Fs = [gather_rows(f, o) if fl else f for f, o, fl in zip(F_all, omegas, full)]
    else:
        omegas = [sample(g.n, n, sd, g.device) for g, n, sd in zip(graphs, ns, seeds)]
        Fs = filter_batched(graphs, lams, p, ds, seeds, omegas, normalize=True)
    t2 = time.perf_counter()
    if kmeans_on_gpu:
        labels_r, inertia = kmeans_reduced_device_batched([f.contiguous() for f in Fs], ks, seeds,
                                                          replicates, kmeans_iter)
    else:
        labels_r, inertia = kmeans_reduced_batched([f.cpu().numpy() for f in Fs], ks, seeds,
                                                   replicates, kmeans_iter)
    t3 = time.perf_counter()
    orders = None
    if any(re):
        orders = [None] * G
        for i in range(G):
            if re[i]:
                o, frac = community_order(graphs[i], F_all[i], omegas[i], labels_r[i], ks[i],
                                          want_frac=True)
                orders[i] = o if frac >= ORDER_MIN_SAME_LABEL else None
    its = interpolate_batched(graphs, lams, p, gamma, omegas, labels_r, ks, tol, max_iter, want_X,
                              orders, cg, dec_ws)
    torch.cuda.current_stream().synchronize()
    t4 = time.perf_counter()
    tm.update(bisection_s=t1 - t0, features_s=t2 - t1, kmeans_s=t3 - t2, interpolate_s=t4 - t3,
              total_s=t4 - t0)
    return [Result(lams[g], bis[g], omegas[g], Fs[g], labels_r[g], float(inertia[g]), its[g], dict(tm),
                   orders[g] if orders is not None else None) for g in range(G)]


# ------------------------------------------------ learned lambda_k bracket ---

def mlp_param_count() -> int:
    return int(lib().csc_mlp_param_count())


def mlp_features(moments, N: int, k: int) -> np.ndarray:
    mom = np.ascontiguousarray(moments, dtype=np.float64)
    x = np.zeros(52, dtype=np.float32)
    check(lib().csc_mlp_features(mom.ctypes.data_as(_lib.pd), len(mom) - 1, int(N), int(k),
                                 x.ctypes.data_as(C.POINTER(C.c_float))), "csc_mlp_features")
    return x


def count_root(moments, k: int, n_signals: int):
    mom = np.ascontiguousarray(moments, dtype=np.float64)
    l0, sc = C.c_double(0.0), C.c_double(0.0)
    check(lib().csc_count_root(mom.ctypes.data_as(_lib.pd), len(mom) - 1, int(k), int(n_signals),
                               C.byref(l0), C.byref(sc)), "csc_count_root")
    return l0.value, sc.value


def mlp_forward(params: torch.Tensor, X: torch.Tensor) -> torch.Tensor:
    X = X.contiguous()
    B = X.shape[0]
    Y = torch.empty((B, 2), dtype=torch.float32, device=X.device)
    ws = _ws(lib().csc_mlp_workspace_bytes(B), X.device)
    check(lib().csc_mlp_forward(_ptr(params), _ptr(X), B, _ptr(Y), _ptr(ws), ws.numel(), _stream()),
          "csc_mlp_forward")
    return Y


def mlp_loss_grad(params: torch.Tensor, X: torch.Tensor, target: torch.Tensor, ws=None):
    X = X.contiguous()
    B = X.shape[0]
    grad = torch.empty_like(params)
    loss = C.c_double(0.0)
    if ws is None:
        ws = _ws(lib().csc_mlp_workspace_bytes(B), X.device)
    check(lib().csc_mlp_loss_grad(_ptr(params), _ptr(X), _ptr(target.contiguous()), B, _ptr(grad),
                                  C.byref(loss), _ptr(ws), ws.numel(), _stream()), "csc_mlp_loss_grad")
    return loss.value, grad


def mlp_adam_step(params, grad, m, v, step: int, lr: float) -> None:
    check(lib().csc_mlp_adam_step(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(step), float(lr),
                                  _stream()), "csc_mlp_adam_step")


@dataclass
class LearnedBisection:
    lam: float
    steps: int
    trace: list
    bracket: tuple
    status: int


def estimate_lambda_k_learned(g: Graph, k: int, p: int, n_signals: int, seed: int,
                              params: torch.Tensor, max_steps: int = 30) -> LearnedBisection:
    lam = C.c_double(0.0)
    steps = C.c_int32(0)
    trace = np.zeros(2 * max_steps)
    br = np.zeros(2)
    ws = _ws(lib().csc_estimate_workspace_bytes_learned(g.n, n_signals, p), g.device)
    st = check(lib().csc_estimate_lambda_k_learned(g.ref, k, p, n_signals, seed, max_steps, _ptr(params),
                                                   C.byref(lam), C.byref(steps),
                                                   trace.ctypes.data_as(_lib.pd),
                                                   br.ctypes.data_as(_lib.pd), _ptr(ws), ws.numel(),
                                                   _stream()), "csc_estimate_lambda_k_learned")
    tr = [(trace[2 * i], trace[2 * i + 1]) for i in range(steps.value)]
    return LearnedBisection(lam.value, steps.value, tr, (br[0], br[1]), st)
