"""deann_query_backward_noalloc (the adjoint for callers that cannot allocate)
against deann_query_backward, through the C ABI: same gradients bit for bit on
two calls in a row, the second with a smaller input."""
import ctypes

import numpy as np
import pytest

import synth
from paper_2107_02736_amd import _lib
from tests.gpu_common import device, to_dev

pytestmark = pytest.mark.gpu


def _forward(torch, dev, n, q, d, k, m, seed):
    import paper_2107_02736_amd as dk
    spec, X, Y = synth.workload("mix10_n1e4_d16", n=n, q=q)
    if d != X.shape[1]:
        rng = np.random.default_rng(seed)
        X = rng.standard_normal((n, d)).astype(np.float32)
        Y = rng.standard_normal((q, d)).astype(np.float32)
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    h = 2.0
    out, nn, sm = dk.deann_query(Xd, Yd, h, k, m, "gaussian", seed=seed)
    return Xd, Yd, h, nn.contiguous(), sm.contiguous()


def _both(torch, lib, dev, Xd, Yd, h, k, m, nn, sm, kern):
    n, d = Xd.shape
    q = Yd.shape[0]
    g = torch.linspace(0.5, 1.5, q, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    gy_a = torch.full((q, d), float("nan"), dtype=torch.float32, device=dev)
    gh_a = torch.full((1,), float("nan"), dtype=torch.float64, device=dev)
    ws = torch.empty(max(int(lib.deann_query_backward_workspace(n, q, d, k, m)), 1),
                     dtype=torch.uint8, device=dev)
    _lib.check(lib.deann_query_backward(Xd.data_ptr(), n, Yd.data_ptr(), q, d, h, kern, k, m,
                                        nn.data_ptr(), sm.data_ptr(), g.data_ptr(),
                                        gy_a.data_ptr(), gh_a.data_ptr(), ws.data_ptr(),
                                        ws.numel(), stream))
    gy_b = torch.full((q, d), float("nan"), dtype=torch.float32, device=dev)
    gh_b = torch.full((1,), float("nan"), dtype=torch.float64, device=dev)
    _lib.check(lib.deann_query_backward_noalloc(Xd.data_ptr(), n, Yd.data_ptr(), q, d, h, kern,
                                                k, m, nn.data_ptr(), sm.data_ptr(),
                                                g.data_ptr(), gy_b.data_ptr(), gh_b.data_ptr(),
                                                stream))
    torch.cuda.synchronize()
    return gy_a.cpu().numpy(), gh_a.cpu().numpy(), gy_b.cpu().numpy(), gh_b.cpu().numpy()


@pytest.mark.parametrize("kern", [_lib.GAUSSIAN, _lib.EXPONENTIAL])
def test_noalloc_matches_workspace_entry(kern):
    torch = pytest.importorskip("torch")
    dev = device()
    lib = _lib.load()
    # first call larger, second smaller (fewer queries, other n and d): the
    # scratch keeps the first call's contents, which the second must not see
    for (n, q, d, k, m, seed) in ((3000, 700, 16, 20, 64, 3), (900, 37, 40, 7, 33, 4)):
        print(f"noalloc case n={n} q={q} d={d} k={k} m={m} kern={kern}", flush=True)
        Xd, Yd, h, nn, sm = _forward(torch, dev, n, q, d, k, m, seed)
        gy_a, gh_a, gy_b, gh_b = _both(torch, lib, dev, Xd, Yd, h, k, m, nn, sm, kern)
        assert np.isfinite(gy_a).all() and np.isfinite(gh_a).all()
        assert np.array_equal(gy_a, gy_b)
        assert np.array_equal(gh_a, gh_b)


def test_noalloc_rejects_too_many_queries():
    pytest.importorskip("torch")
    device()
    lib = _lib.load()
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: the size check fails first
    st = lib.deann_query_backward_noalloc(fake, 100, fake, _lib.NOALLOC_MAX_Q + 1, 3, 1.0, 0, 5,
                                          10, fake, fake, fake, fake, fake, None)
    assert st == _lib.EUNSUPPORTED
    assert "scratch" in lib.deann_last_error().decode()
