"""ctypes declarations of the libcsc C ABI (include/csc.h).

Loading fails loudly when the shared library has not been built: there is no
fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcsc.so")

CSC_OK = 0
CSC_E_INVALID_ARG = 1
CSC_E_GRAPH = 2
CSC_E_HIP = 3
CSC_E_OOM = 4
CSC_W_NOT_CONVERGED = 5
CSC_W_BISECT_EXHAUSTED = 6
CSC_W_BRACKET_MISS = 7
WARNINGS = (CSC_W_NOT_CONVERGED, CSC_W_BISECT_EXHAUSTED, CSC_W_BRACKET_MISS)

STREAM_COUNT, STREAM_FEAT, STREAM_SAMPLE, STREAM_KMEANS = 1, 2, 3, 4
TUNE_PANEL_WIDTH, TUNE_XCD_ORDER, TUNE_NONTEMPORAL, TUNE_HIP_GRAPHS, TUNE_ROW_SCHED = 0, 1, 2, 3, 4
TUNE_COUNT_GROUP = 5
TUNE_BATCH_COUNT_GROUP = 6
TUNE_BLOCK_PRODUCT = 7
FORM_FORWARD, FORM_CLENSHAW = 0, 1
DAMP_JACKSON, DAMP_NONE = 0, 1


class CscGraph(C.Structure):
    _fields_ = [
        ("n", C.c_int32),
        ("nnz", C.c_int32),
        ("row_ptr", C.c_void_p),
        ("col", C.c_void_p),
        ("val", C.c_void_p),
        ("dinv_sqrt", C.c_void_p),
        ("sched", C.c_void_p),
    ]


i32, u32, u64, f64, vp, sz = C.c_int32, C.c_uint32, C.c_uint64, C.c_double, C.c_void_p, C.c_size_t
i64 = C.c_int64
pg = C.POINTER(CscGraph)
pd = C.POINTER(C.c_double)
pi = C.POINTER(C.c_int32)
pu = C.POINTER(C.c_uint64)

# name: (restype, argtypes)
PROTOTYPES = {
    "csc_last_error": (C.c_char_p, []),
    "csc_version": (i32, []),
    "csc_set_panel_width": (i32, [i32]),
    "csc_get_panel_width": (i32, [i32, C.c_int64, i32]),
    "csc_set_tuning": (i32, [i32, i32]),
    "csc_autotune": (i32, [pg, i32, i32, i32, pi, pi, pd, vp, sz, vp]),
    "csc_autotune_clear": (None, []),
    "csc_get_tuning": (i32, [i32]),
    "csc_laplacian_from_adjacency": (i32, [i32, i32, vp, vp, vp, vp, vp, i32, vp]),
    "csc_row_schedule": (i32, [i32, vp, vp, pd, vp, sz, vp]),
    "csc_jackson_coeffs": (i32, [f64, i32, pd]),
    "csc_gaussian_block": (i32, [i32, i32, u64, u32, u32, vp, i32, vp]),
    "csc_filter_workspace_bytes": (sz, [i32, i32]),
    "csc_filter_block": (i32, [pg, pd, i32, vp, i32, i32, vp, vp, sz, vp]),
    "csc_filter": (i32, [pg, f64, i32, i32, u64, vp, i32, i32, vp, i32, vp, sz, vp]),
    "csc_filter_noalloc_max_bytes": (sz, []),
    "csc_filter_noalloc": (i32, [pg, f64, i32, i32, u64, vp, i32, i32, vp, i32, vp]),
    "csc_estimate_workspace_bytes": (sz, [i32, i32, i32]),
    "csc_eigencount": (i32, [pg, f64, i32, i32, u64, u32, pd, pd, vp, sz, vp]),
    "csc_estimate_lambda_k": (i32, [pg, i32, i32, i32, u64, i32, pd, pd, pi, pd, pd, vp, sz, vp]),
    "csc_estimate_lambda_k_kpm": (i32, [pg, i32, i32, i32, u64, i32, pd, pi, pd, pd, vp, sz, vp]),
    "csc_sample_workspace_bytes": (sz, [i32, i32]),
    "csc_sample": (i32, [i32, i32, u64, vp, vp, sz, vp]),
    "csc_kmeans_reduced": (i32, [vp, i32, i32, i32, i32, i32, i32, u64, pi, pd]),
    "csc_kmeans_reduced_f64": (i32, [vp, i32, i32, i32, i32, i32, i32, u64, pi, pd]),
    "csc_kmeans_seeds": (i32, [vp, i32, i32, i32, i32, i32, u64, pi]),
    "csc_kmeans_seeds_device": (i32, [vp, i32, i32, i32, i32, i32, u64, pi, vp, sz, vp]),
    "csc_interpolate_workspace_bytes": (sz, [i32, i64, i32, i32]),
    "csc_interpolate": (i32, [pg, vp, i32, f64, i32, f64, vp, vp, vp, i32, i32, f64, i32, vp, i32,
                              vp, pi, pd, vp, sz, vp]),
    "csc_sample_density_workspace_bytes": (sz, [i32]),
    "csc_sample_density": (i32, [i32, i32, u64, vp, vp, vp, vp, sz, vp]),
    "csc_normalize_rows": (i32, [vp, i64, i32, i32, vp, vp]),
    "csc_community_order_workspace_bytes": (sz, [i32, i32, i32, i32]),
    "csc_community_order": (i32, [pg, vp, i64, i32, vp, pi, i32, i32, vp, vp, pd, vp, sz, vp]),
    "csc_gather_rows": (i32, [vp, i64, i32, i32, vp, i32, vp, i32, vp, sz, vp]),
    "csc_estimate_workspace_bytes_batched": (sz, [pg, i32, pi, i32]),
    "csc_estimate_lambda_k_batched": (i32, [pg, i32, pi, i32, pi, pu, i32, pd, vp, pd, pi, pd, pd,
                                            pi, vp, sz, vp]),
    "csc_filter_workspace_bytes_batched": (sz, [pg, i32, pi, i32]),
    "csc_filter_batched": (i32, [pg, i32, pd, i32, pi, pu, vp, pi, i32, vp, pi, vp, sz, vp]),
    "csc_interpolate_workspace_bytes_batched": (sz, [pg, i32, pi, i32]),
    "csc_interpolate_batched": (i32, [pg, i32, vp, i32, pd, i32, f64, vp, vp, vp, pi, pi, f64, i32,
                                      vp, pi, vp, pi, pd, pi, vp, sz, vp]),
    "csc_kmeans_reduced_batched": (i32, [i32, vp, pi, pi, pi, i32, i32, pu, vp, pd]),
    "csc_kmeans_device_workspace_bytes": (sz, [i32, i32, i32, i32]),
    "csc_community_cores": (i32, [i32, i32, i32, pi, pi]),
    "csc_kmeans_reduced_device": (i32, [vp, i32, i32, i32, i32, i32, i32, u64, pi, pd, vp, sz, vp]),
    "csc_kmeans_device_workspace_bytes_batched": (sz, [i32, pi, pi, pi, i32]),
    "csc_kmeans_reduced_device_batched": (i32, [i32, vp, pi, pi, pi, i32, i32, pu, vp, pd, vp, sz,
                                                vp]),
    "csc_mlp_param_count": (i32, []),
    "csc_mlp_workspace_bytes": (sz, [i32]),
    "csc_mlp_features": (i32, [pd, i32, i32, i32, C.POINTER(C.c_float)]),
    "csc_count_root": (i32, [pd, i32, i32, i32, pd, pd]),
    "csc_mlp_forward": (i32, [vp, vp, i32, vp, vp, sz, vp]),
    "csc_mlp_loss_grad": (i32, [vp, vp, vp, i32, vp, pd, vp, sz, vp]),
    "csc_mlp_adam_step": (i32, [vp, vp, vp, vp, i32, C.c_float, vp]),
    "csc_estimate_workspace_bytes_learned": (sz, [i32, i32, i32]),
    "csc_estimate_lambda_k_learned": (i32, [pg, i32, i32, i32, u64, i32, vp, pd, pi, pd, pd, vp,
                                            sz, vp]),
    "csc_cheb_steps_workspace_bytes": (sz, [i32, i32]),
    "csc_cheb_steps": (i32, [pg, i32, i32, i32, i32, vp, sz, vp]),
    "csc_set_filter_form": (i32, [i32]),
    "csc_set_damping": (i32, [i32]),
    "csc_get_damping": (i32, []),
    "csc_get_filter_form": (i32, []),
}


class CscError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """The loaded libcsc with prototypes set (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1602_02018_amd.build`")
        handle = C.CDLL(LIB_PATH)
        for name, (res, args) in PROTOTYPES.items():
            f = getattr(handle, name)
            f.restype = res
            f.argtypes = args
        _lib = handle
    return _lib


def check(status: int, where: str, allow_warnings: bool = True) -> int:
    if status == CSC_OK or (allow_warnings and status in WARNINGS):
        return status
    msg = lib().csc_last_error().decode(errors="replace")
    raise CscError(status, where, msg)
