"""csc_filter_noalloc (the feature pass of Alg. 2 steps 2-4 on the library's
fixed scratch array) against csc_filter with a caller workspace: the same
kernels on the same inputs, so the outputs must be bit-identical, on two calls
in a row with the second one smaller (the array keeps the first call's
contents), and an oversized request must fail before any device work."""
import ctypes as C

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_1602_02018_amd import api as a

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return a


def _noalloc(api, g, lam, p, d, seed, rows=None, normalize=True):
    from paper_1602_02018_amd import _lib

    n_out = g.n if rows is None else rows.numel()
    Y = torch.full((n_out, d), float("nan"), dtype=torch.float32, device=g.device)
    st = api.lib().csc_filter_noalloc(
        g.ref, lam, p, d, seed, C.c_void_p(rows.data_ptr() if rows is not None else 0),
        0 if rows is None else rows.numel(), 1 if normalize else 0, C.c_void_p(Y.data_ptr()), d,
        C.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert st == _lib.CSC_OK, api.lib().csc_last_error()
    return Y


def test_noalloc_filter_matches_filter_on_two_calls(api):
    big = synth.sbm_config(5000, 20, seed=3)
    small = synth.sbm_config(1000, 10, seed=0)
    gb = api.Graph(big.row_ptr, big.col)
    gs = api.Graph(small.row_ptr, small.col)
    # first call: every row of the larger graph, unit rows
    y1 = _noalloc(api, gb, 0.41, 50, 36, 5)
    r1 = api.filter(gb, 0.41, 50, 36, 5)
    assert torch.equal(y1, r1)
    # second call: smaller graph and width, sampled rows, no normalisation
    rows = api.sample(small.n, 47, 0)
    y2 = _noalloc(api, gs, 0.46875, 50, 28, 0, rows=rows, normalize=False)
    r2 = api.filter(gs, 0.46875, 50, 28, 0, rows=rows, normalize=False)
    assert torch.equal(y2, r2)
    # and the larger one again after the smaller one
    assert torch.equal(_noalloc(api, gb, 0.41, 50, 36, 5), r1)


def test_noalloc_filter_rejects_requests_beyond_its_scratch(api):
    from paper_1602_02018_amd import _lib

    assert api.lib().csc_filter_noalloc_max_bytes() == 128 << 20
    n = 600_000  # a path: 4 blocks of n x 64 floats need 614 MB
    rp = np.concatenate([[0], np.cumsum([1] + [2] * (n - 2) + [1])]).astype(np.int32)
    inner = np.stack([np.arange(0, n - 2), np.arange(2, n)], axis=1).ravel()
    col = np.concatenate([[1], inner, [n - 2]]).astype(np.int32)
    g = api.Graph(rp, col)
    Y = torch.zeros((n, 56), dtype=torch.float32, device="cuda")
    st = api.lib().csc_filter_noalloc(g.ref, 0.5, 50, 56, 0, None, 0, 1, C.c_void_p(Y.data_ptr()),
                                      56, C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == _lib.CSC_E_INVALID_ARG
    assert b"scratch" in api.lib().csc_last_error()
    assert torch.count_nonzero(Y).item() == 0
