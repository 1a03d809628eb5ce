"""ctypes binding of libdeann.so: argument marshalling only.

Every computation happens in the HIP library; this module converts Python
values into the C ABI declared in include/deann.h and raises on a non-OK status.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# DEANN_LIB selects another build of the library (the host-AddressSanitizer
# build of the ABI tests, for instance)
LIB_PATH = os.environ.get("DEANN_LIB") or os.path.join(_HERE, "libdeann.so")

OK, EINVAL, EWORKSPACE, EHIP, EUNSUPPORTED = 0, 1, 2, 3, 4
NOALLOC_MAX_Q = 1 << 20   # DEANN_NOALLOC_MAX_Q
GAUSSIAN, EXPONENTIAL = 0, 1
FP32, BF16, FP16, FP32_SPLIT = 0, 1, 2, 3

EXPORTS = (
    "kde_exact_workspace", "kde_exact",
    "deann_query_workspace", "deann_query",
    "deann_query_with_grad_workspace", "deann_query_with_grad",
    "deann_prepared_bytes", "deann_prepare", "kde_exact_prepared", "kde_exact_backward_prepared",
    "kde_exact_with_grad_prepared",
    "deann_query_prepared", "deann_query_with_grad_prepared",
    "deann_query_permuted_workspace", "deann_query_permuted",
    "deann_perm_index_bytes", "deann_perm_index_create", "deann_query_permuted_index",
    "deann_query_backward_workspace", "deann_query_backward", "deann_query_backward_noalloc",
    "kde_exact_backward_workspace", "kde_exact_backward",
    "kde_exact_with_grad_workspace", "kde_exact_with_grad", "mean_shift_update",
    "kde_hybrid_workspace", "kde_hybrid",
    "ivf_build_workspace", "ivf_build", "ivf_index_bytes", "ivf_index_create_workspace",
    "ivf_index_create", "deann_ivf_query_workspace", "deann_ivf_query",
    "deann_last_error", "deann_default_options", "deann_get_options", "deann_set_options",
    "deann_last_stats",
    "deann_kernel_timing", "deann_kernel_times",
)


class Options(ctypes.Structure):
    """deann_options (include/deann.h)."""
    _fields_ = [("rel_tol", ctypes.c_double), ("value_floor", ctypes.c_double),
                ("knn_slack", ctypes.c_int64), ("knn_cap2", ctypes.c_int64),
                ("center", ctypes.c_int32), ("knn_seed_stride", ctypes.c_int32)]


class Stats(ctypes.Structure):
    """deann_stats (include/deann.h)."""
    _fields_ = [("exact_refined", ctypes.c_int64), ("knn_second_pass", ctypes.c_int64),
                ("knn_exhaustive", ctypes.c_int64)]


class DeannError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"deann status {status}: {message}")
        self.status = status


_lib = None

_i64, _u64, _int, _dbl, _sz, _vp = (ctypes.c_int64, ctypes.c_uint64, ctypes.c_int,
                                      ctypes.c_double, ctypes.c_size_t, ctypes.c_void_p)


def load(path: str = LIB_PATH):
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build the HIP library first "
            "(python -m paper_2107_02736_amd.build)")
    lib = ctypes.CDLL(path)
    lib.deann_last_error.restype = ctypes.c_char_p
    lib.deann_last_error.argtypes = []
    lib.kde_exact_workspace.restype = _sz
    lib.kde_exact_workspace.argtypes = [_i64, _i64, _i64, _int]
    lib.kde_exact.restype = _int
    lib.kde_exact.argtypes = [_vp, _i64, _vp, _i64, _i64, _dbl, _int, _int, _vp, _vp, _sz, _vp]
    lib.deann_query_workspace.restype = _sz
    lib.deann_query_workspace.argtypes = [_i64, _i64, _i64, _i64, _i64, _int]
    lib.deann_query.restype = _int
    lib.deann_query.argtypes = [_vp, _i64, _vp, _i64, _i64, _dbl, _int, _i64, _i64, _u64, _u64,
                                _u64, _int, _vp, _vp, _vp, _vp, _sz, _vp]
    lib.deann_query_with_grad_workspace.restype = _sz
    lib.deann_query_with_grad_workspace.argtypes = [_i64, _i64, _i64, _i64, _i64, _int]
    lib.deann_query_with_grad.restype = _int
    lib.deann_query_with_grad.argtypes = [_vp, _i64, _vp, _i64, _i64, _dbl, _int, _i64, _i64,
                                          _u64, _u64, _u64, _int, _vp, _vp, _vp, _vp, _vp, _vp,
                                          _sz, _vp]
    lib.deann_query_permuted_workspace.restype = _sz
    lib.deann_query_permuted_workspace.argtypes = [_i64, _i64, _i64, _i64, _i64, _int]
    lib.deann_query_permuted.restype = _int
    lib.deann_query_permuted.argtypes = [_vp, _i64, _vp, _i64, _i64, _dbl, _int, _i64, _i64, _u64,
                                         _u64, _int, _vp, _vp, _vp, _vp, _sz, _vp]
    lib.deann_perm_index_bytes.restype = _sz
    lib.deann_perm_index_bytes.argtypes = [_i64, _i64]
    lib.deann_perm_index_create.restype = _int
    lib.deann_perm_index_create.argtypes = [_vp, _i64, _i64, _u64, _vp, _sz, _vp]
    lib.deann_query_permuted_index.restype = _int
    lib.deann_query_permuted_index.argtypes = [_vp, _i64, _vp, _i64, _i64, _dbl, _int, _i64, _i64,
                                               _vp, _sz, _u64, _int, _vp, _vp, _vp, _vp, _sz, _vp]
    lib.deann_query_backward_workspace.restype = _sz
    lib.deann_query_backward_workspace.argtypes = [_i64, _i64, _i64, _i64, _i64]
    lib.deann_query_backward.restype = _int
    lib.deann_query_backward.argtypes = [_vp, _i64, _vp, _i64, _i64, _dbl, _int, _i64, _i64, _vp,
                                         _vp, _vp, _vp, _vp, _vp, _sz, _vp]
    lib.deann_query_backward_noalloc.restype = _int
    lib.deann_query_backward_noalloc.argtypes = [_vp, _i64, _vp, _i64, _i64, _dbl, _int, _i64,
                                                 _i64, _vp, _vp, _vp, _vp, _vp, _vp]
    lib.kde_exact_backward_workspace.restype = _sz
    lib.kde_exact_backward_workspace.argtypes = [_i64, _i64, _i64, _int]
    lib.kde_exact_backward.restype = _int
    lib.kde_exact_backward.argtypes = [_vp, _i64, _vp, _i64, _i64, _dbl, _int, _int, _vp, _vp, _vp,
                                       _vp,
                                       _sz, _vp]
    lib.kde_hybrid_workspace.restype = _sz
    lib.kde_hybrid_workspace.argtypes = [_i64, _i64, _i64, _i64, _int]
    lib.kde_hybrid.restype = _int
    lib.kde_hybrid.argtypes = [_vp, _i64, _vp, _i64, _i64, _dbl, _int, _i64, _int, _vp, _vp, _vp,
                               _vp, _sz, _vp]
    lib.kde_exact_with_grad_workspace.restype = _sz
    lib.kde_exact_with_grad_workspace.argtypes = [_i64, _i64, _i64, _int]
    lib.kde_exact_with_grad.restype = _int
    lib.kde_exact_with_grad.argtypes = [_vp, _i64, _vp, _i64, _i64, _dbl, _int, _int, _vp, _vp,
                                        _vp, _vp,
                                        _sz, _vp]
    lib.mean_shift_update.restype = _int
    lib.mean_shift_update.argtypes = [_vp, _vp, _vp, _i64, _i64, _dbl, _vp, _vp]
    lib.ivf_build_workspace.restype = _sz
    lib.ivf_build_workspace.argtypes = [_i64, _i64, _i64]
    lib.ivf_build.restype = _int
    lib.ivf_build.argtypes = [_vp, _i64, _i64, _i64, _int, _vp, _vp, _vp, _sz, _vp]
    lib.ivf_index_bytes.restype = _sz
    lib.ivf_index_bytes.argtypes = [_i64, _i64, _i64]
    lib.ivf_index_create_workspace.restype = _sz
    lib.ivf_index_create_workspace.argtypes = [_i64, _i64, _i64]
    lib.ivf_index_create.restype = _int
    lib.ivf_index_create.argtypes = [_vp, _i64, _i64, _vp, _i64, _vp, _sz, _vp, _sz, _vp]
    lib.deann_ivf_query_workspace.restype = _sz
    lib.deann_ivf_query_workspace.argtypes = [_i64, _i64, _i64, _i64, _i64, _i64, _i64]
    lib.deann_ivf_query.restype = _int
    lib.deann_ivf_query.argtypes = [_vp, _i64, _vp, _i64, _i64, _vp, _vp, _i64, _i64, _dbl, _int,
                                    _i64, _i64, _u64, _u64, _vp, _vp, _vp, _vp, _sz, _vp]
    lib.deann_default_options.restype = None
    lib.deann_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.deann_get_options.restype = _int
    lib.deann_get_options.argtypes = [ctypes.POINTER(Options)]
    lib.deann_set_options.restype = _int
    lib.deann_set_options.argtypes = [ctypes.POINTER(Options)]
    lib.deann_last_stats.restype = _int
    lib.deann_last_stats.argtypes = [ctypes.POINTER(Stats), _vp]
    lib.deann_kernel_timing.restype = _int
    lib.deann_kernel_timing.argtypes = [_int]
    lib.deann_kernel_times.restype = _int
    lib.deann_kernel_times.argtypes = [_int, ctypes.POINTER(ctypes.c_float), _int]
    # prepared-set variants: the plain call's arguments after (prepared, bytes)
    lib.deann_prepared_bytes.restype = _sz
    lib.deann_prepared_bytes.argtypes = [_i64, _i64, _int]
    lib.deann_prepare.restype = _int
    lib.deann_prepare.argtypes = [_vp, _i64, _i64, _int, _vp, _sz, _vp]
    lib.kde_exact_prepared.restype = _int
    lib.kde_exact_prepared.argtypes = [_vp, _sz] + lib.kde_exact.argtypes
    lib.kde_exact_backward_prepared.restype = _int
    lib.kde_exact_backward_prepared.argtypes = [_vp, _sz] + lib.kde_exact_backward.argtypes
    lib.kde_exact_with_grad_prepared.restype = _int
    lib.kde_exact_with_grad_prepared.argtypes = [_vp, _sz] + lib.kde_exact_with_grad.argtypes
    lib.deann_query_prepared.restype = _int
    lib.deann_query_prepared.argtypes = [_vp, _sz] + lib.deann_query.argtypes
    lib.deann_query_with_grad_prepared.restype = _int
    lib.deann_query_with_grad_prepared.argtypes = [_vp, _sz] + lib.deann_query_with_grad.argtypes
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != OK:
        msg = load().deann_last_error().decode(errors="replace")
        raise DeannError(status, msg)
