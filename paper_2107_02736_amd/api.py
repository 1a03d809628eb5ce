"""Torch-facing wrappers of the C ABI (device memory and streams from PyTorch).

Each function checks shapes and dtypes, allocates outputs and the workspace
with torch, and calls the HIP library on torch's current stream.  No value is
computed here.
"""
from __future__ import annotations

import torch

from . import _lib

_KERNELS = {"gaussian": _lib.GAUSSIAN, "exponential": _lib.EXPONENTIAL}
_PRECS = {"fp32": _lib.FP32, "bf16": _lib.BF16, "fp16": _lib.FP16, "fp32_split": _lib.FP32_SPLIT}


def kernel_id(kernel) -> int:
    if isinstance(kernel, int):
        return kernel
    return _KERNELS[kernel]


def precision_id(precision) -> int:
    if isinstance(precision, int):
        return precision
    return _PRECS[precision]


def _ptr(t):
    return None if t is None else t.data_ptr()


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _check_xy(X: torch.Tensor, Y: torch.Tensor):
    if not (X.is_cuda and Y.is_cuda):
        raise ValueError("X and Y must be device tensors (the HIP library has no CPU path)")
    if X.dtype != torch.float32 or Y.dtype != torch.float32:
        raise TypeError("X and Y must be float32")
    if X.dim() != 2 or Y.dim() != 2 or X.shape[1] != Y.shape[1]:
        raise ValueError("X must be [n, d] and Y [q, d]")
    if not (X.is_contiguous() and Y.is_contiguous()):
        raise ValueError("X and Y must be contiguous")
    if X.device != Y.device:
        raise ValueError("X and Y must be on the same device")


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


class Prepared:
    """A prepared data set (deann_prepare): X centred and stored in the scan
    precision with its norms, computed once; pass it as `prepared=` to
    kde_exact, deann_query and deann_query_with_grad with the same X."""

    def __init__(self, X: torch.Tensor, precision="fp32"):
        _check_xy(X, X[:0])
        lib = _lib.load()
        self.n, self.d = X.shape
        self.precision = precision_id(precision)
        self.device = X.device
        self.x_ptr = X.data_ptr()
        nbytes = lib.deann_prepared_bytes(self.n, self.d, self.precision)
        if nbytes == 0:
            raise ValueError("invalid size or precision for a prepared data set")
        self.buf = _workspace(nbytes, X.device)
        _lib.check(lib.deann_prepare(X.data_ptr(), self.n, self.d, self.precision,
                                     self.buf.data_ptr(), self.buf.numel(), _stream(X.device)))

    def args(self, X: torch.Tensor, precision: int):
        """(pointer, bytes) after checking that the call matches this set."""
        if (X.data_ptr() != self.x_ptr or tuple(X.shape) != (self.n, self.d)
                or X.device != self.device or precision != self.precision):
            raise ValueError("the prepared data set was made from another X or precision")
        return self.buf.data_ptr(), self.buf.numel()


def prepare(X: torch.Tensor, precision="fp32") -> Prepared:
    """Prepare X once for repeated calls (deann_prepare)."""
    return Prepared(X, precision)


def kde_exact(X: torch.Tensor, Y: torch.Tensor, h: float, kernel="gaussian",
              precision="fp32", out: torch.Tensor | None = None,
              prepared: Prepared | None = None) -> torch.Tensor:
    """Exact KDE of every query row (float64 [q]); `prepared` (made with the
    same X, in FP32 for the "fp32_split" precision) skips preparing X."""
    _check_xy(X, Y)
    lib = _lib.load()
    n, d = X.shape
    q = Y.shape[0]
    p = precision_id(precision)
    if out is None:
        out = torch.empty(q, dtype=torch.float64, device=X.device)
    ws = _workspace(lib.kde_exact_workspace(n, q, d, p), X.device)
    args = (X.data_ptr(), n, Y.data_ptr(), q, d, float(h), kernel_id(kernel), p,
            out.data_ptr(), ws.data_ptr(), ws.numel(), _stream(X.device))
    if prepared is None:
        _lib.check(lib.kde_exact(*args))
    else:
        pp = prepared.args(X, _lib.FP32 if p == _lib.FP32_SPLIT else p)
        _lib.check(lib.kde_exact_prepared(*pp, *args))
    return out


def deann_query(X: torch.Tensor, Y: torch.Tensor, h: float, k: int, m: int, kernel="gaussian",
                seed: int = 0, query_offset: int = 0, word2: int = 0, precision="fp32",
                return_indices: bool = True, prepared: Prepared | None = None):
    """DEANN estimate of every query: (out float64 [q], nn_idx int32 [q,k], sample_idx int32 [q,m]);
    `prepared` (made with the same X and precision) skips preparing X."""
    _check_xy(X, Y)
    lib = _lib.load()
    n, d = X.shape
    q = Y.shape[0]
    p = precision_id(precision)
    dev = X.device
    out = torch.empty(q, dtype=torch.float64, device=dev)
    nn = torch.empty((q, k), dtype=torch.int32, device=dev) if return_indices else None
    sm = torch.empty((q, m), dtype=torch.int32, device=dev) if return_indices else None
    ws = _workspace(lib.deann_query_workspace(n, q, d, k, m, p), dev)
    args = (X.data_ptr(), n, Y.data_ptr(), q, d, float(h), kernel_id(kernel), int(k), int(m),
            int(seed), int(query_offset), int(word2), p, out.data_ptr(), _ptr(nn), _ptr(sm),
            ws.data_ptr(), ws.numel(), _stream(dev))
    if prepared is None:
        _lib.check(lib.deann_query(*args))
    else:
        _lib.check(lib.deann_query_prepared(*prepared.args(X, p), *args))
    return out, nn, sm


def deann_query_with_grad(X: torch.Tensor, Y: torch.Tensor, h: float, k: int, m: int,
                          kernel="gaussian", seed: int = 0, query_offset: int = 0, word2: int = 0,
                          precision="fp32", need_grad_y: bool = True, need_grad_h: bool = True,
                          return_indices: bool = True, prepared: Prepared | None = None):
    """DEANN estimates with their gradients from one gather of each query's rows:
    (out float64 [q], grad_Y float32 [q,d] = d out_j / d y_j or None, grad_h
    float64 [q] = d out_j / d h or None, nn_idx int32 [q,k], sample_idx int32
    [q,m]); the same neighbours and draws as deann_query."""
    _check_xy(X, Y)
    lib = _lib.load()
    n, d = X.shape
    q = Y.shape[0]
    p = precision_id(precision)
    dev = X.device
    out = torch.empty(q, dtype=torch.float64, device=dev)
    gy = torch.empty((q, d), dtype=torch.float32, device=dev) if need_grad_y else None
    gh = torch.empty(q, dtype=torch.float64, device=dev) if need_grad_h else None
    nn = torch.empty((q, k), dtype=torch.int32, device=dev) if return_indices else None
    sm = torch.empty((q, m), dtype=torch.int32, device=dev) if return_indices else None
    ws = _workspace(lib.deann_query_with_grad_workspace(n, q, d, k, m, p), dev)
    args = (X.data_ptr(), n, Y.data_ptr(), q, d, float(h), kernel_id(kernel), int(k), int(m),
            int(seed), int(query_offset), int(word2), p, out.data_ptr(), _ptr(gy), _ptr(gh),
            _ptr(nn), _ptr(sm), ws.data_ptr(), ws.numel(), _stream(dev))
    if prepared is None:
        _lib.check(lib.deann_query_with_grad(*args))
    else:
        _lib.check(lib.deann_query_with_grad_prepared(*prepared.args(X, p), *args))
    return out, gy, gh, nn, sm


def kde_hybrid(X: torch.Tensor, Y: torch.Tensor, h: float, k: int, kernel="gaussian",
               precision="bf16", nn_idx: torch.Tensor | None = None,
               return_indices: bool = False):
    """Near/far exact KDE (float64 [q]): the k nearest rows of each query summed
    exactly in FP64, the other rows by the 16-bit tile sweep.  nn_idx (int32
    [q, k]) supplies the neighbour lists instead of computing them; with
    return_indices the lists used are returned as well."""
    _check_xy(X, Y)
    lib = _lib.load()
    n, d = X.shape
    q = Y.shape[0]
    p = precision_id(precision)
    dev = X.device
    if nn_idx is not None:
        if (nn_idx.dtype != torch.int32 or nn_idx.device != dev or not nn_idx.is_contiguous()
                or tuple(nn_idx.shape) != (q, k)):
            raise ValueError("nn_idx must be a contiguous int32 [q, k] tensor on X's device")
    out = torch.empty(q, dtype=torch.float64, device=dev)
    nn_out = torch.empty((q, k), dtype=torch.int32, device=dev) if return_indices else None
    ws = _workspace(lib.kde_hybrid_workspace(n, q, d, int(k), p), dev)
    _lib.check(lib.kde_hybrid(X.data_ptr(), n, Y.data_ptr(), q, d, float(h), kernel_id(kernel),
                              int(k), p, _ptr(nn_idx), out.data_ptr(), _ptr(nn_out),
                              ws.data_ptr(), ws.numel(), _stream(dev)))
    return (out, nn_out) if return_indices else out


class PermutedIndex:
    """The permuted copy of X for permuted random sampling (Algorithm 2's
    preprocessing, App. G): the keyed permutation of the rows, its inverse and
    the rows in permuted order, in one device buffer owned by this object.
    X must stay unchanged while the index is used."""

    def __init__(self, X: torch.Tensor, seed: int = 0):
        _check_xy(X, X)
        lib = _lib.load()
        self.n, self.d = X.shape
        self.seed = int(seed)
        nbytes = lib.deann_perm_index_bytes(self.n, self.d)
        self.buffer = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=X.device)
        _lib.check(lib.deann_perm_index_create(X.data_ptr(), self.n, self.d, self.seed,
                                               self.buffer.data_ptr(), self.buffer.numel(),
                                               _stream(X.device)))

    def permutation(self) -> torch.Tensor:
        """pi (int32 [n]): the row of X at each position of the permuted order."""
        return self.buffer[: 4 * self.n].view(torch.int32)


def deann_query_permuted(X: torch.Tensor, Y: torch.Tensor, h: float, k: int, m: int,
                         kernel="gaussian", seed: int = 0, start: int = 0, precision="fp32",
                         return_indices: bool = True, index: PermutedIndex | None = None):
    """DEANN with permuted random sampling (query i reads the permuted rows from
    running index start + i m): (out float64 [q], nn_idx [q,k], sample_idx [q,m]).
    With `index` (a PermutedIndex of X) the rows come from its permuted copy and
    the permutation is the index's (its seed replaces `seed`)."""
    _check_xy(X, Y)
    lib = _lib.load()
    n, d = X.shape
    q = Y.shape[0]
    p = precision_id(precision)
    dev = X.device
    out = torch.empty(q, dtype=torch.float64, device=dev)
    nn = torch.empty((q, k), dtype=torch.int32, device=dev) if return_indices else None
    sm = torch.empty((q, m), dtype=torch.int32, device=dev) if return_indices else None
    ws = _workspace(lib.deann_query_permuted_workspace(n, q, d, k, m, p), dev)
    if index is not None:
        if (index.n, index.d) != (n, d) or index.buffer.device != dev:
            raise ValueError("the permuted index was made for another X")
        _lib.check(lib.deann_query_permuted_index(
            X.data_ptr(), n, Y.data_ptr(), q, d, float(h), kernel_id(kernel), int(k), int(m),
            index.buffer.data_ptr(), index.buffer.numel(), int(start), p, out.data_ptr(),
            _ptr(nn), _ptr(sm), ws.data_ptr(), ws.numel(), _stream(dev)))
        return out, nn, sm
    _lib.check(lib.deann_query_permuted(X.data_ptr(), n, Y.data_ptr(), q, d, float(h),
                                        kernel_id(kernel), int(k), int(m), int(seed), int(start),
                                        p, out.data_ptr(), _ptr(nn), _ptr(sm), ws.data_ptr(),
                                        ws.numel(), _stream(dev)))
    return out, nn, sm


def deann_query_backward(X, Y, h, k, m, nn_idx, sample_idx, grad_out, kernel="gaussian",
                         need_grad_y: bool = True, need_grad_h: bool = True):
    """(grad_Y float32 [q,d] or None, grad_h float64 [1] or None) of deann_query."""
    _check_xy(X, Y)
    lib = _lib.load()
    n, d = X.shape
    q = Y.shape[0]
    dev = X.device
    # the kernels use the entries as row indices of X: shapes, dtype and device
    # are checked here (values are those a forward call returned)
    for name, t, cols in (("nn_idx", nn_idx, k), ("sample_idx", sample_idx, m)):
        if t is None:
            continue
        if (t.dtype != torch.int32 or t.device != dev or not t.is_contiguous()
                or tuple(t.shape) != (q, cols)):
            raise ValueError(f"{name} must be a contiguous int32 [q, {cols}] tensor on X's device")
    if grad_out.numel() != q:
        raise ValueError("grad_out must hold one value per query")
    grad_out = grad_out.to(device=dev, dtype=torch.float64).contiguous()
    gy = torch.empty((q, d), dtype=torch.float32, device=dev) if need_grad_y else None
    gh = torch.empty(1, dtype=torch.float64, device=dev) if need_grad_h else None
    ws = _workspace(lib.deann_query_backward_workspace(n, q, d, k, m), dev)
    _lib.check(lib.deann_query_backward(
        X.data_ptr(), n, Y.data_ptr(), q, d, float(h), kernel_id(kernel), int(k), int(m),
        _ptr(nn_idx), _ptr(sample_idx), grad_out.data_ptr(), _ptr(gy), _ptr(gh), ws.data_ptr(),
        ws.numel(), _stream(dev)))
    return gy, gh


def kde_exact_backward(X, Y, h, grad_out, kernel="gaussian", need_grad_y: bool = True,
                       need_grad_h: bool = True, precision="fp32",
                       prepared: Prepared | None = None):
    """(grad_Y float32 [q,d] or None, grad_h float64 [1] or None) of kde_exact;
    precision "fp32" or "fp32_split" (distance product from bfloat16 parts);
    `prepared`: an FP32 set of the same X."""
    _check_xy(X, Y)
    lib = _lib.load()
    n, d = X.shape
    q = Y.shape[0]
    dev = X.device
    grad_out = grad_out.to(device=dev, dtype=torch.float64).contiguous()
    gy = torch.empty((q, d), dtype=torch.float32, device=dev) if need_grad_y else None
    gh = torch.empty(1, dtype=torch.float64, device=dev) if need_grad_h else None
    p = precision_id(precision)
    ws = _workspace(lib.kde_exact_backward_workspace(n, q, d, p), dev)
    args = (X.data_ptr(), n, Y.data_ptr(), q, d, float(h), kernel_id(kernel), p,
            grad_out.data_ptr(), _ptr(gy), _ptr(gh), ws.data_ptr(), ws.numel(), _stream(dev))
    if prepared is None:
        _lib.check(lib.kde_exact_backward(*args))
    else:
        _lib.check(lib.kde_exact_backward_prepared(*prepared.args(X, _lib.FP32), *args))
    return gy, gh


def kde_exact_with_grad(X, Y, h, kernel="gaussian", need_grad_y: bool = True,
                        need_grad_h: bool = True, precision="fp32",
                        prepared: Prepared | None = None):
    """Exact KDE and its derivatives in one pass (d <= 128; precision "fp32" or
    "fp32_split"): (mu float64 [q], d mu/d y float32 [q,d] or None, d mu/d h
    float64 [q] or None); `prepared`: an FP32 set of the same X."""
    _check_xy(X, Y)
    lib = _lib.load()
    n, d = X.shape
    q = Y.shape[0]
    dev = X.device
    mu = torch.empty(q, dtype=torch.float64, device=dev)
    gy = torch.empty((q, d), dtype=torch.float32, device=dev) if need_grad_y else None
    gh = torch.empty(q, dtype=torch.float64, device=dev) if need_grad_h else None
    p = precision_id(precision)
    ws = _workspace(lib.kde_exact_with_grad_workspace(n, q, d, p), dev)
    args = (X.data_ptr(), n, Y.data_ptr(), q, d, float(h), kernel_id(kernel), p, mu.data_ptr(),
            _ptr(gy), _ptr(gh), ws.data_ptr(), ws.numel(), _stream(dev))
    if prepared is None:
        _lib.check(lib.kde_exact_with_grad(*args))
    else:
        _lib.check(lib.kde_exact_with_grad_prepared(*prepared.args(X, _lib.FP32), *args))
    return mu, gy, gh


def mean_shift_update(Y, grad_Y, density, h, out=None):
    """Gaussian mean-shift step y + h^2 grad / density (out may be Y)."""
    lib = _lib.load()
    q, d = Y.shape
    if out is None:
        out = torch.empty_like(Y)
    for t, dt in ((Y, torch.float32), (grad_Y, torch.float32), (density, torch.float64),
                  (out, torch.float32)):
        if t.dtype != dt or not t.is_contiguous() or t.device != Y.device:
            raise ValueError("mean_shift_update: contiguous tensors of the expected dtypes on one device")
    _lib.check(lib.mean_shift_update(Y.data_ptr(), grad_Y.data_ptr(), density.data_ptr(), q, d,
                                     float(h), out.data_ptr(), _stream(Y.device)))
    return out


def get_options() -> dict:
    """The options of this thread's calls (deann_options) as a dict."""
    o = _lib.Options()
    _lib.check(_lib.load().deann_get_options(o))
    return {name: getattr(o, name) for name, _ in _lib.Options._fields_}


def set_options(**kw) -> dict:
    """Change some options of this thread's calls (rel_tol, value_floor, knn_slack,
    knn_cap2, center, knn_seed_stride); returns the previous options."""
    prev = get_options()
    o = _lib.Options()
    _lib.check(_lib.load().deann_get_options(o))
    for name, v in kw.items():
        if name not in prev:
            raise KeyError(name)
        setattr(o, name, v)
    _lib.check(_lib.load().deann_set_options(o))
    return prev


def default_options() -> dict:
    o = _lib.Options()
    _lib.load().deann_default_options(o)
    return {name: getattr(o, name) for name, _ in _lib.Options._fields_}


def last_stats(device=None) -> dict:
    """Counts of the last call on this thread (synchronises the stream): queries
    re-evaluated exactly by the exact KDE, and the k-NN queries that needed the
    second pass or the exhaustive scan (-1: no such step)."""
    st = _lib.Stats()
    dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    _lib.check(_lib.load().deann_last_stats(st, _stream(dev)))
    return {name: int(getattr(st, name)) for name, _ in _lib.Stats._fields_}


TIMING_SITES = {"kde_exact": 0, "kde_exact_backward": 1, "kde_hybrid": 2}


def kernel_timing(capacity: int) -> None:
    """Record HIP events around the dense tile kernel of the next `capacity`
    kde_exact / kde_exact_backward calls on this thread (0 stops)."""
    _lib.check(_lib.load().deann_kernel_timing(int(capacity)))


def kernel_times(site: str, max_count: int = 4096) -> list:
    """Durations in ms of the recorded tile kernels of `site`, in call order
    (waits for them); frees the slots."""
    import ctypes
    buf = (ctypes.c_float * max_count)()
    n = _lib.load().deann_kernel_times(TIMING_SITES[site], buf, max_count)
    if n < 0:
        _lib.check(_lib.EHIP)
    return [float(buf[i]) for i in range(n)]


# ---- inverted-file neighbours (the ANN of the experiments, Sec. 5) ----------------
def ivf_build(X: torch.Tensor, n_clusters: int, iters: int = 10):
    """k-means over the rows of X: (centroids float32 [n_clusters, d],
    assign int32 [n], the closest final centroid of every row)."""
    if not X.is_cuda or X.dtype != torch.float32 or X.dim() != 2 or not X.is_contiguous():
        raise ValueError("X must be a contiguous float32 [n, d] device tensor")
    lib = _lib.load()
    n, d = X.shape
    dev = X.device
    C = torch.empty((n_clusters, d), dtype=torch.float32, device=dev)
    a = torch.empty(n, dtype=torch.int32, device=dev)
    ws = _workspace(lib.ivf_build_workspace(n, d, n_clusters), dev)
    _lib.check(lib.ivf_build(X.data_ptr(), n, d, int(n_clusters), int(iters), C.data_ptr(),
                             a.data_ptr(), ws.data_ptr(), ws.numel(), _stream(dev)))
    return C, a


class IvfIndex:
    """Rows of X laid out by cluster (an opaque device buffer) with the
    centroids they were assigned to."""

    def __init__(self, X: torch.Tensor, centroids: torch.Tensor, assign: torch.Tensor):
        if not X.is_cuda or X.dtype != torch.float32 or X.dim() != 2 or not X.is_contiguous():
            raise ValueError("X must be a contiguous float32 [n, d] device tensor")
        lib = _lib.load()
        n, d = X.shape
        dev = X.device
        self.centroids = centroids.to(device=dev, dtype=torch.float32).contiguous()
        if self.centroids.dim() != 2 or self.centroids.shape[1] != d:
            raise ValueError("centroids must be [n_clusters, d]")
        self.n_clusters = self.centroids.shape[0]
        self.n, self.d = n, d
        assign = assign.to(device=dev, dtype=torch.int32).contiguous()
        if assign.shape != (n,):
            raise ValueError("assign must be [n]")
        self.buffer = _workspace(lib.ivf_index_bytes(n, d, self.n_clusters), dev)
        ws = _workspace(lib.ivf_index_create_workspace(n, d, self.n_clusters), dev)
        _lib.check(lib.ivf_index_create(X.data_ptr(), n, d, assign.data_ptr(), self.n_clusters,
                                        self.buffer.data_ptr(), self.buffer.numel(),
                                        ws.data_ptr(), ws.numel(), _stream(dev)))


def deann_ivf_query(X: torch.Tensor, Y: torch.Tensor, index: IvfIndex, n_probe: int, h: float,
                    k: int, m: int, kernel="gaussian", seed: int = 0, query_offset: int = 0,
                    return_indices: bool = True):
    """DEANN with the inverted-file neighbours (the k nearest rows among the
    n_probe closest clusters): (out float64 [q], nn_idx [q,k], sample_idx [q,m])."""
    _check_xy(X, Y)
    if (index.n, index.d) != tuple(X.shape):
        raise ValueError("the index was made for another X")
    lib = _lib.load()
    n, d = X.shape
    q = Y.shape[0]
    dev = X.device
    out = torch.empty(q, dtype=torch.float64, device=dev)
    nn = torch.empty((q, k), dtype=torch.int32, device=dev) if return_indices else None
    sm = torch.empty((q, m), dtype=torch.int32, device=dev) if return_indices else None
    ws = _workspace(lib.deann_ivf_query_workspace(n, q, d, index.n_clusters, n_probe, k, m), dev)
    _lib.check(lib.deann_ivf_query(
        X.data_ptr(), n, Y.data_ptr(), q, d, index.buffer.data_ptr(), index.centroids.data_ptr(),
        index.n_clusters, int(n_probe), float(h), kernel_id(kernel), int(k), int(m), int(seed),
        int(query_offset), out.data_ptr(), _ptr(nn), _ptr(sm), ws.data_ptr(), ws.numel(),
        _stream(dev)))
    return out, nn, sm
