"""CPU checks of the C ABI: the library loads, exports what include/csc.h
declares, rejects bad arguments before touching the GPU, and its host-side
k-means matches the oracle exactly on identical float64 inputs."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1602_02018_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(csc_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_five_calls():
    names = declared_functions()
    for n in ("csc_estimate_lambda_k", "csc_filter", "csc_sample", "csc_kmeans_reduced",
              "csc_interpolate"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(_lib.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(_lib.PROTOTYPES) == set(declared_functions())


def test_version_and_panel_width_validation():
    lib = _lib.lib()
    assert lib.csc_version() >= 100
    assert lib.csc_set_panel_width(3) == _lib.CSC_E_INVALID_ARG
    assert b"panel width" in lib.csc_last_error()
    assert lib.csc_set_panel_width(8) == _lib.CSC_OK
    assert lib.csc_get_panel_width(1000, 16000, 47) == 8
    assert lib.csc_set_panel_width(0) == _lib.CSC_OK
    # built-in choice follows gathered cache lines: 128-byte aligned rows when padding is cheap
    widths = [lib.csc_get_panel_width(100000, 1600000, w) for w in (1, 24, 28, 47, 56, 100, 250)]
    assert widths == [4, 32, 32, 48, 64, 100, 256], widths


def test_argument_errors_are_reported_without_gpu_work():
    lib = _lib.lib()
    assert lib.csc_sample(10, 0, 0, None, None, 0, None) == _lib.CSC_E_INVALID_ARG
    assert lib.csc_sample(10, 11, 0, None, None, 0, None) == _lib.CSC_E_INVALID_ARG
    assert lib.csc_filter(None, 0.5, 50, 4, 0, None, 0, 1, None, 4, None, 0, None) == _lib.CSC_E_INVALID_ARG
    assert lib.csc_laplacian_from_adjacency(0, 0, None, None, None, None, None, 0, None) == _lib.CSC_E_INVALID_ARG
    g = _lib.CscGraph(10, 0, 0, 0, 0, 0)
    assert lib.csc_filter(C.byref(g), 0.5, 50, 4, 0, None, 0, 1, None, 4, None, 0, None) == _lib.CSC_E_INVALID_ARG
    assert b"row_ptr" in lib.csc_last_error()
    g = _lib.CscGraph(10, 0, 16, 0, 0, 0)
    assert lib.csc_filter(C.byref(g), 2.5, 50, 4, 0, None, 0, 1, C.c_void_p(16), 4, None, 0, None) == _lib.CSC_E_INVALID_ARG
    assert b"lambda_c" in lib.csc_last_error()
    # workspace too small is caught before any launch
    assert lib.csc_filter(C.byref(g), 0.5, 50, 4, 0, None, 0, 1, C.c_void_p(16), 4,
                          C.c_void_p(256), 8, None) == _lib.CSC_E_INVALID_ARG
    assert b"workspace too small" in lib.csc_last_error()
    lam = C.c_double()
    st = C.c_int32()
    assert lib.csc_estimate_lambda_k(C.byref(g), 11, 50, 4, 0, 30, None, C.byref(lam), C.byref(st),
                                     None, None, None, 0, None) == _lib.CSC_E_INVALID_ARG
    assert lib.csc_estimate_lambda_k_kpm(C.byref(g), 11, 50, 4, 0, 30, C.byref(lam), C.byref(st),
                                         None, None, None, 0, None) == _lib.CSC_E_INVALID_ARG
    assert lib.csc_interpolate(C.byref(g), None, 1, 0.5, 50, 0.0, C.c_void_p(16), C.c_void_p(16),
                               None, 2, 2, 1e-6, 10, None, 2, C.c_void_p(16), None, None, None, 0,
                               None) == _lib.CSC_E_INVALID_ARG
    assert lib.csc_interpolate(C.byref(g), None, 3, 0.5, 50, 1e-3, C.c_void_p(16), C.c_void_p(16),
                               None, 2, 2, 1e-6, 10, None, 2, C.c_void_p(16), None, None, None, 0,
                               None) == _lib.CSC_E_INVALID_ARG
    assert b"method" in lib.csc_last_error()
    # community order: d above the register-resident limit, labels outside [0, k)
    lab = (C.c_int32 * 3)(0, 1, 2)
    assert lib.csc_community_order(C.byref(g), C.c_void_p(16), 200, 200, C.c_void_p(16), lab, 3, 3,
                                   C.c_void_p(16), None, None, None, 0,
                                   None) == _lib.CSC_E_INVALID_ARG
    assert b"d <= 128" in lib.csc_last_error()
    assert lib.csc_community_order(C.byref(g), C.c_void_p(16), 8, 8, C.c_void_p(16), lab, 3, 2,
                                   C.c_void_p(16), None, None, None, 0,
                                   None) == _lib.CSC_E_INVALID_ARG
    assert b"labels_r" in lib.csc_last_error()
    assert lib.csc_gather_rows(C.c_void_p(16), 4, 10, 8, C.c_void_p(16), 2, C.c_void_p(16), 8,
                               None, 0, None) == _lib.CSC_E_INVALID_ARG
    assert b"ldf" in lib.csc_last_error()
    assert lib.csc_sample_density(10, 11, 0, C.c_void_p(16), C.c_void_p(16), None, None, 0,
                                  None) == _lib.CSC_E_INVALID_ARG
    assert lib.csc_normalize_rows(C.c_void_p(16), 2, 4, 3, None, None) == _lib.CSC_E_INVALID_ARG


def test_filter_form_setting():
    lib = _lib.lib()
    assert lib.csc_get_filter_form() == _lib.FORM_CLENSHAW
    assert lib.csc_set_filter_form(5) == _lib.CSC_E_INVALID_ARG
    assert lib.csc_set_filter_form(_lib.FORM_FORWARD) == _lib.CSC_OK
    assert lib.csc_get_filter_form() == _lib.FORM_FORWARD
    assert lib.csc_set_filter_form(_lib.FORM_CLENSHAW) == _lib.CSC_OK


def test_workspace_sizes_grow_with_problem():
    lib = _lib.lib()
    a = lib.csc_filter_workspace_bytes(1000, 28)
    b = lib.csc_filter_workspace_bytes(100000, 47)
    assert 0 < a < b
    assert lib.csc_filter_workspace_bytes(0, 4) == 0
    assert lib.csc_estimate_workspace_bytes(1000, 14, 50) > 3 * 1000 * 14 * 4
    assert lib.csc_interpolate_workspace_bytes(1000, 16000, 10, 47) > 6 * 1000 * 10 * 4 + 8 * 16000
    assert lib.csc_community_order_workspace_bytes(1000, 28, 10, 47) > 4 * 1000 * 4
    assert lib.csc_sample_workspace_bytes(1000, 47) > 1000 * 24


def test_jackson_coefficients_host_call_matches_oracle():
    from oracle import jackson
    from paper_1602_02018_amd import api

    for lc, p in ((0.3, 50), (1.7, 60), (0.0, 10), (2.0, 10), (1.0, 0)):
        np.testing.assert_allclose(api.jackson_coeffs(lc, p), jackson.lowpass_coeffs(lc, p),
                                   rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("seed,n,d,k", [(0, 47, 28, 10), (3, 300, 12, 25), (5, 922, 47, 100),
                                        (7, 2761, 56, 250)])
def test_host_kmeans_matches_oracle(seed, n, d, k):
    """Seeding picks equal the oracle's (plain prefix sums) up to near-ties of
    the running sums; Lloyd and the replicate choice from the library's picks
    give its labels and inertia exactly."""
    from kmeans_parity import check_kmeans
    from paper_1602_02018_amd import api

    rng = np.random.default_rng(seed)
    centers = rng.normal(size=(k, d))
    X = centers[rng.integers(0, k, n)] + 0.3 * rng.normal(size=(n, d))
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    reps = 20 if n < 500 else 4
    picks = api.kmeans_seeds(X, k, seed, replicates=reps)
    lab, inertia = api.kmeans_reduced(X, k, seed, replicates=reps)
    same = check_kmeans(X, k, seed, picks, lab, inertia)
    assert sum(same) >= len(same) - 1  # near-ties are rare


def test_kmeans_parity_check_rejects_a_planted_wrong_pick():
    """The rounding-aware check is not vacuous: a pick moved by one point where
    no running sum is near the target fails it, and so does a wrong label."""
    from kmeans_parity import check_lloyd, check_seeding
    from oracle import kmeans

    rng = np.random.default_rng(1)
    X = rng.normal(size=(200, 5))
    picks = np.array([[rec[0] for rec in _record(kmeans, X, 8, 3, r)] for r in range(3)], np.int32)
    assert check_seeding(X, 8, 3, picks) == [True, True, True]
    bad = picks.copy()
    bad[1, 4] = (bad[1, 4] + 1) % 200
    with pytest.raises(AssertionError):
        check_seeding(X, 8, 3, bad)
    lab, _, inertia = kmeans.best_of(X, [X[picks[r]] for r in range(3)])
    check_lloyd(X, picks, lab, inertia)
    lab2 = lab.copy()
    lab2[0] = (lab2[0] + 1) % 8
    with pytest.raises(AssertionError):
        check_lloyd(X, picks, lab2, inertia)


def _record(kmeans, X, k, seed, r):
    rec = []
    kmeans.seed_plusplus(X, k, seed, r, record=rec)
    return rec


def test_host_kmeans_float32_input_and_errors():
    from paper_1602_02018_amd import api

    X = np.random.default_rng(0).normal(size=(50, 4)).astype(np.float32)
    lab, inertia = api.kmeans_reduced(X, 3, 0)
    assert lab.min() >= 0 and lab.max() < 3 and inertia > 0
    with pytest.raises(_lib.CscError):
        api.kmeans_reduced(X, 51, 0)


def test_count_root_host_call_matches_oracle():
    from oracle import mlp
    from paper_1602_02018_amd import api

    rng = np.random.default_rng(0)
    for k, nc in ((10, 14), (100, 24), (250, 28)):
        # a monotone synthetic count curve: moments of a spectrum with 3k eigenvalues in [0, 2]
        lam = np.sort(rng.uniform(0, 2, 3 * k))
        t = np.arccos(lam - 1.0)
        mu = np.array([np.sum(np.cos(m * t)) for m in range(51)])
        l0, s = api.count_root(mu, k, nc)
        r0, rs = mlp.count_root(mu, 50, k, nc)
        assert abs(l0 - r0) < 1e-12 and abs(s - rs) <= 1e-9 * rs


def test_argument_checks_from_two_threads_keep_their_own_errors():
    """Calls are reentrant on the host side: two threads hitting different
    argument errors at once each get their own status and csc_last_error
    message (the message is per thread)."""
    import threading

    lib = _lib.lib()
    g = _lib.CscGraph(10, 0, 16, 0, 0, 0)
    F = np.ones((4, 3))
    lab = np.zeros(4, dtype=np.int32)
    errors = []
    barrier = threading.Barrier(2)

    def panel():
        barrier.wait()
        for _ in range(2000):
            if lib.csc_set_panel_width(3) != _lib.CSC_E_INVALID_ARG or b"panel width" not in lib.csc_last_error():
                errors.append("panel")
                return

    def filt():
        barrier.wait()
        for _ in range(2000):
            st = lib.csc_filter(C.byref(g), 2.5, 50, 4, 0, None, 0, 1, C.c_void_p(16), 4, None, 0, None)
            if st != _lib.CSC_E_INVALID_ARG or b"lambda_c" not in lib.csc_last_error():
                errors.append("filter")
                return

    def kmeans():
        barrier.wait()
        for _ in range(2000):
            st = lib.csc_kmeans_reduced_f64(F.ctypes.data_as(_lib.pd), 4, 3, 3, 0, 1, 10, 0,
                                            lab.ctypes.data_as(_lib.pi), None)
            if st != _lib.CSC_E_INVALID_ARG or b"k must" not in lib.csc_last_error():
                errors.append("kmeans")
                return

    for pair in ((panel, filt), (filt, kmeans), (panel, kmeans)):
        barrier.reset()
        ts = [threading.Thread(target=f) for f in pair]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
    assert not errors, errors
    assert lib.csc_set_panel_width(0) == _lib.CSC_OK


def test_bench_accounting_of_block_cg_live_columns():
    """bench.py counts each block-CG iteration's live columns (a column leaves
    the block once it meets the tolerance; zero right-hand sides never enter)."""
    import bench

    it = np.array([1] * 33 + [3] * 216 + [4])
    assert bench.live_widths(it) == [250, 217, 217, 1]
    assert bench.live_widths(np.array([0, 0, 2])) == [1, 1]
    assert bench.live_widths(np.array([], dtype=int)) == []
    assert abs(bench.cg_pass_share(it, 250) - (8 + 7 + 7 + 1) / 8) < 1e-12
    full = bench.job_bytes(1000, 16000, 10, 28, 14, 50, 4, np.full(10, 3))
    part = bench.job_bytes(1000, 16000, 10, 28, 14, 50, 4, np.array([3] * 5 + [1] * 5))
    assert part < full
