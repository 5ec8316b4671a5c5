"""Host float64 algebra of the block CG (rank-revealing orthonormalisation,
Cholesky solves), checked against numpy on random and rank-deficient blocks."""
import ctypes as C
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


CLANG = "/opt/rocm/llvm/bin/clang++"  # the compiler the library's host code is built with


@pytest.fixture(scope="module", params=["g++", "clang++"])
def dense(request, tmp_path_factory):
    """The routines built with the system compiler and with the library's own
    host compiler and flags (the latter is what libcsc.so runs)."""
    if request.param == "g++":
        cxx, flags = shutil.which("g++"), ["-O2", "-ffp-contract=off", "-pthread"]
    else:
        cxx = CLANG if os.path.exists(CLANG) else None
        flags = ["-O3", "-std=c++17", "-Wall", "-ffp-contract=off"]
    if cxx is None:
        pytest.skip(f"no {request.param}")
    out = tmp_path_factory.mktemp("dense") / "libdense.so"
    subprocess.run([cxx, *flags, "-shared", "-fPIC", "-o", str(out),
                    os.path.join(HERE, "dense_host.cpp"),
                    os.path.join(HERE, "..", "paper_1602_02018_amd", "csrc", "dense.cpp")],
                   check=True)
    lib = C.CDLL(str(out))
    pd = C.POINTER(C.c_double)
    lib.dense_orth.argtypes = [pd, C.c_int, C.c_double, pd]
    lib.dense_orth.restype = C.c_int
    lib.dense_solve.argtypes = [pd, C.c_int, pd, C.c_int, C.c_double, C.c_int]
    lib.dense_solve.restype = C.c_int
    return lib


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _orth(lib, Z, rtol=1e-10):
    k = Z.shape[1]
    G = np.ascontiguousarray(Z.T @ Z)
    T = np.zeros((k, k))
    s = lib.dense_orth(_p(G), k, rtol, _p(T))
    return s, T[:, :s]


@pytest.mark.parametrize("seed", range(4))
def test_orth_of_full_rank_block(dense, seed):
    rng = np.random.default_rng(seed)
    Z = rng.normal(size=(300, 12)) * rng.uniform(1e-4, 10, size=12)  # widely scaled columns
    s, T = _orth(dense, Z)
    assert s == 12
    P = Z @ T
    np.testing.assert_allclose(P.T @ P, np.eye(s), atol=1e-10)
    # P spans Z: Z = P (P^T Z)
    np.testing.assert_allclose(P @ (P.T @ Z), Z, atol=1e-9 * np.abs(Z).max())


def test_orth_drops_dependent_and_zero_columns(dense):
    rng = np.random.default_rng(7)
    B = rng.normal(size=(200, 5))
    Z = np.concatenate([B, B[:, :2] @ rng.normal(size=(2, 3)), np.zeros((200, 2))], axis=1)
    s, T = _orth(dense, Z)
    assert s == 5
    P = Z @ T
    np.testing.assert_allclose(P.T @ P, np.eye(5), atol=1e-10)
    np.testing.assert_allclose(P @ (P.T @ Z), Z, atol=1e-9 * np.abs(Z).max())
    assert np.all(T[-2:] == 0.0)  # zero columns take no part


def test_orth_keeps_a_small_but_independent_column(dense):
    rng = np.random.default_rng(3)
    Z = rng.normal(size=(100, 4))
    Z[:, 2] *= 1e-9  # a nearly converged residual column is still a direction
    s, T = _orth(dense, Z)
    assert s == 4


@pytest.mark.parametrize("s,k", [(1, 3), (7, 7), (20, 5)])
def test_cholesky_solve(dense, s, k):
    rng = np.random.default_rng(s * 31 + k)
    M = rng.normal(size=(s, s))
    W = M @ M.T + s * np.eye(s)
    Cm = rng.normal(size=(s, k))
    out = Cm.copy()
    assert dense.dense_solve(_p(np.ascontiguousarray(W)), s, _p(out), k, -1.0, 1) == 1
    np.testing.assert_allclose(out, -np.linalg.solve(W, Cm), rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("s,k,threads", [(128, 256, 4), (250, 250, 8), (200, 257, 3), (64, 64, 8)])
def test_cholesky_solve_threads_bit_identical(dense, s, k, threads):
    """The column slices of a threaded solve take exactly the operations of
    the one-thread solve (a large solve splits, a small one does not).  Also
    the regression test of a crash: the library's compiler, given the address
    of the multi-versioned slice solver as a thread function, produced a
    pointer that faulted when called."""
    rng = np.random.default_rng(s + k)
    M = rng.normal(size=(s, s))
    W = np.ascontiguousarray(M @ M.T + s * np.eye(s))
    Cm = rng.normal(size=(s, k))
    one, many = Cm.copy(), Cm.copy()
    assert dense.dense_solve(_p(W), s, _p(one), k, -1.0, 1) == 1
    assert dense.dense_solve(_p(W), s, _p(many), k, -1.0, threads) == 1
    assert np.array_equal(one, many)
    np.testing.assert_allclose(one, -np.linalg.solve(W, Cm), rtol=1e-8, atol=1e-10)


def test_cholesky_rejects_indefinite(dense):
    W = np.array([[1.0, 2.0], [2.0, 1.0]])
    Cm = np.ones((2, 1))
    assert dense.dense_solve(_p(W), 2, _p(Cm), 1, 1.0, 1) == 0


def _plain(lib):
    pd = C.POINTER(C.c_double)
    lib.dense_orth_plain.argtypes = [pd, C.c_int, C.c_double, pd]
    lib.dense_orth_plain.restype = C.c_int
    lib.dense_subst_plain.argtypes = [pd, C.c_int, pd, C.c_int, C.c_double]
    lib.dense_subst_plain.restype = None
    lib.dense_factor.argtypes = [pd, C.c_int]
    lib.dense_factor.restype = C.c_int
    return lib


def _gram(rng, k, kind):
    m = k + 40
    if kind == "full":
        Z = rng.normal(size=(m, k)) * rng.uniform(1e-3, 10, size=k)
    elif kind == "low-rank":  # rank k/3: the remaining diagonal entries go to rounding noise
        Z = rng.normal(size=(m, k // 3 + 1)) @ rng.normal(size=(k // 3 + 1, k))
    elif kind == "zero-columns":
        Z = rng.normal(size=(m, k))
        Z[:, ::3] = 0.0
    elif kind == "near-duplicates":
        Z = rng.normal(size=(m, k))
        Z[:, 1::2] = Z[:, 0:k - 1:2][:, : Z[:, 1::2].shape[1]] + 1e-9 * rng.normal(size=(m, k // 2))
    else:  # exact combinations of earlier columns among independent ones: their remaining
        # diagonal entries fall to rounding noise, some below zero, while others are still O(1)
        Z = rng.normal(size=(m, k))
        for c in range(2, k, 3):
            Z[:, c] = Z[:, c - 2] - 0.5 * Z[:, c - 1]
    return np.ascontiguousarray(Z.T @ Z)


@pytest.mark.parametrize("k", [1, 2, 5, 16, 17, 31, 33, 64, 100, 129, 250])
@pytest.mark.parametrize("kind", ["full", "low-rank", "zero-columns", "near-duplicates",
                                  "combinations"])
def test_orth_equals_outer_product_form_bit_for_bit(dense, k, kind):
    """The library factors column by column over the columns still in the
    search (compacted positions, dependent columns squeezed out) and inverts
    with register tiles; every entry must still take the textbook outer-
    product form's operations in its order: T and s equal bit for bit."""
    lib = _plain(dense)
    G = _gram(np.random.default_rng(k * 7 + len(kind)), k, kind)
    T1, T2 = np.zeros((k, k)), np.zeros((k, k))
    s1 = lib.dense_orth(_p(G), k, 1e-10, _p(T1))
    s2 = lib.dense_orth_plain(_p(G), k, 1e-10, _p(T2))
    assert s1 == s2
    assert np.array_equal(T1, T2)
    if kind == "full":
        assert s1 == k


@pytest.mark.parametrize("s,k", [(1, 1), (5, 3), (6, 16), (7, 17), (13, 32), (100, 100),
                                 (101, 250), (250, 7)])
def test_solve_equals_plain_substitution_bit_for_bit(dense, s, k):
    """Forward substitution runs in register tiles of several rows sharing
    the loads of finished rows; each element's subtractions keep their
    order, so the solve equals row-by-row substitution bit for bit."""
    lib = _plain(dense)
    rng = np.random.default_rng(s * 13 + k)
    M = rng.normal(size=(s, s))
    W = np.ascontiguousarray(M @ M.T + s * np.eye(s))
    L = W.copy()
    assert lib.dense_factor(_p(L), s) == 1
    Cm = rng.normal(size=(s, k))
    lib_out, plain_out = Cm.copy(), Cm.copy()
    assert lib.dense_solve(_p(W), s, _p(lib_out), k, -1.0, 1) == 1
    lib.dense_subst_plain(_p(L), s, _p(plain_out), k, -1.0)
    assert np.array_equal(lib_out, plain_out)
