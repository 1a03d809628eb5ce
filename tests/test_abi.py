"""Host-side checks of the C ABI: the library loads, exports every declared
entry point, and rejects invalid arguments before launching anything."""
import ctypes
import os
import re

import pytest

from paper_2107_02736_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "deann.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"\b([a-z_]+)\s*\(", text)) - {"if", "sizeof"}


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libdeann.so not built")
    return _lib.load()


def test_header_and_exports_agree(lib):
    declared = _declared()
    assert declared == set(_lib.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


FAKE = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first


def _kde(lib, n=10, q=4, d=3, h=1.0, kernel=0, prec=0, out=FAKE, ws=FAKE, wsb=1 << 30, X=FAKE):
    return lib.kde_exact(X, n, FAKE, q, d, h, kernel, prec, out, ws, wsb, None)


@pytest.mark.parametrize("kw,status", [
    (dict(n=0), _lib.EINVAL), (dict(d=0), _lib.EINVAL), (dict(q=-1), _lib.EINVAL),
    (dict(h=0.0), _lib.EINVAL), (dict(h=float("nan")), _lib.EINVAL),
    (dict(h=float("inf")), _lib.EINVAL), (dict(kernel=7), _lib.EINVAL),
    (dict(prec=9), _lib.EINVAL), (dict(out=None), _lib.EINVAL), (dict(X=None), _lib.EINVAL),
    (dict(n=1 << 31), _lib.EINVAL), (dict(ws=None), _lib.EWORKSPACE), (dict(wsb=16), _lib.EWORKSPACE),
])
def test_kde_exact_validation(lib, kw, status):
    assert _kde(lib, **kw) == status
    assert lib.deann_last_error().decode()


def test_q_zero_is_a_noop(lib):
    assert _kde(lib, q=0, out=None, ws=None, wsb=0) == _lib.OK


def _dq(lib, n=100, q=4, d=3, h=1.0, kernel=0, k=5, m=10, prec=0, ws=FAKE, wsb=1 << 34):
    return lib.deann_query(FAKE, n, FAKE, q, d, h, kernel, k, m, 0, 0, 0, prec, FAKE, FAKE, FAKE,
                           ws, wsb, None)


@pytest.mark.parametrize("kw,status", [
    (dict(k=-1), _lib.EINVAL), (dict(k=101), _lib.EINVAL), (dict(m=-1), _lib.EINVAL),
    (dict(n=5000, k=2000), _lib.EUNSUPPORTED), (dict(prec=3), _lib.EINVAL),
    (dict(wsb=8), _lib.EWORKSPACE), (dict(h=-2.0), _lib.EINVAL),
])
def test_deann_query_validation(lib, kw, status):
    assert _dq(lib, **kw) == status


def test_backward_validation(lib):
    # grad_out missing
    st = lib.deann_query_backward(FAKE, 100, FAKE, 4, 3, 1.0, 0, 5, 10, FAKE, FAKE, None, FAKE,
                                  FAKE, FAKE, 1 << 20, None)
    assert st == _lib.EINVAL
    # exact backward beyond d = 128
    st = lib.kde_exact_backward(FAKE, 100, FAKE, 4, 200, 1.0, 0, 0, FAKE, FAKE, FAKE, FAKE,
                                1 << 30, None)
    assert st == _lib.EUNSUPPORTED
    # precisions other than FP32 and the float32 split
    for prec in (1, 2, 7):
        st = lib.kde_exact_backward(FAKE, 100, FAKE, 4, 8, 1.0, 0, prec, FAKE, FAKE, FAKE, FAKE,
                                    1 << 30, None)
        assert st == _lib.EINVAL
        st = lib.kde_exact_with_grad(FAKE, 100, FAKE, 4, 8, 1.0, 0, prec, FAKE, FAKE, FAKE, FAKE,
                                     1 << 30, None)
        assert st == _lib.EINVAL
    assert lib.kde_exact_with_grad_workspace(1000, 10, 64, 3) > lib.kde_exact_with_grad_workspace(
        1000, 10, 64, 0)


def test_workspace_sizes_grow(lib):
    a = lib.kde_exact_workspace(10_000, 1_000, 16, 0)
    b = lib.kde_exact_workspace(1_000_000, 10_000, 128, 0)
    assert 0 < a < b
    assert lib.deann_query_workspace(10_000, 1_000, 16, 50, 500, 1) > 0
    assert lib.kde_exact_workspace(0, 1, 1, 0) == 0


def _ivfq(lib, n=1000, q=4, d=3, L=10, np_=2, h=1.0, k=5, m=10, index=FAKE, C=FAKE, ws=FAKE,
          wsb=1 << 34):
    return lib.deann_ivf_query(FAKE, n, FAKE, q, d, index, C, L, np_, h, 0, k, m, 0, 0, FAKE,
                               FAKE, FAKE, ws, wsb, None)


@pytest.mark.parametrize("kw,status", [
    (dict(L=0), _lib.EINVAL), (dict(L=9000), _lib.EINVAL), (dict(np_=0), _lib.EINVAL),
    (dict(np_=11), _lib.EINVAL), (dict(L=600, np_=500), _lib.EINVAL), (dict(k=-1), _lib.EINVAL),
    (dict(k=1001), _lib.EINVAL), (dict(k=600), _lib.EUNSUPPORTED), (dict(m=-1), _lib.EINVAL),
    (dict(index=None), _lib.EINVAL), (dict(C=None), _lib.EINVAL), (dict(h=-1.0), _lib.EINVAL),
    (dict(ws=None), _lib.EWORKSPACE), (dict(wsb=64), _lib.EWORKSPACE),
])
def test_ivf_query_validation(lib, kw, status):
    assert _ivfq(lib, **kw) == status
    assert lib.deann_last_error().decode()


def test_ivf_build_and_index_validation(lib):
    def build(n=1000, d=3, L=10, iters=5, ws=FAKE, wsb=1 << 34):
        return lib.ivf_build(FAKE, n, d, L, iters, FAKE, FAKE, ws, wsb, None)
    assert build(L=0) == _lib.EINVAL
    assert build(L=1001) == _lib.EINVAL
    assert build(n=100000, L=9000) == _lib.EUNSUPPORTED
    assert build(iters=-1) == _lib.EINVAL
    assert build(d=5000) == _lib.EUNSUPPORTED
    assert build(ws=None) == _lib.EWORKSPACE

    def create(n=1000, d=3, L=10, index=FAKE, ib=1 << 34, ws=FAKE, wsb=1 << 34):
        return lib.ivf_index_create(FAKE, n, d, FAKE, L, index, ib, ws, wsb, None)
    assert create(L=0) == _lib.EINVAL
    assert create(L=9000) == _lib.EUNSUPPORTED
    assert create(index=None) == _lib.EINVAL
    assert create(ib=64) == _lib.EWORKSPACE
    assert create(wsb=64) == _lib.EWORKSPACE
    # sizes: positive, growing with n and with the cluster count
    assert lib.ivf_index_bytes(1000, 3, 10) > 0
    assert lib.ivf_index_bytes(2000, 3, 10) > lib.ivf_index_bytes(1000, 3, 10)
    assert lib.ivf_index_bytes(1000, 3, 20) > lib.ivf_index_bytes(1000, 3, 10)
    assert lib.ivf_build_workspace(1000, 3, 0) == 0
    assert lib.deann_ivf_query_workspace(1000, 4, 3, 10, 11, 5, 10) == 0


def _hyb(lib, n=1000, q=4, d=3, h=1.0, kernel=0, k=5, prec=1, nn_in=None, out=FAKE, ws=FAKE,
         wsb=1 << 34):
    return lib.kde_hybrid(FAKE, n, FAKE, q, d, h, kernel, k, prec, nn_in, out, None, ws, wsb, None)


@pytest.mark.parametrize("kw,status", [
    (dict(prec=0), _lib.EINVAL), (dict(prec=3), _lib.EINVAL), (dict(k=-1), _lib.EINVAL),
    (dict(k=1001), _lib.EINVAL), (dict(kernel=5), _lib.EINVAL), (dict(out=None), _lib.EINVAL),
    (dict(k=600), _lib.EUNSUPPORTED), (dict(d=5000), _lib.EUNSUPPORTED),
    (dict(n=1 << 30, q=1 << 24, k=200), _lib.EUNSUPPORTED), (dict(wsb=64), _lib.EWORKSPACE),
    (dict(ws=None), _lib.EWORKSPACE),
])
def test_kde_hybrid_validation(lib, kw, status):
    assert _hyb(lib, **kw) == status
    assert lib.deann_last_error().decode()


def test_kde_hybrid_given_neighbours_lift_the_knn_limits(lib):
    # with the lists supplied no k-NN runs, so k > 496 passes validation (and
    # fails only at the deliberately short workspace); d stays <= 4096
    assert _hyb(lib, k=600, nn_in=FAKE, wsb=64) == _lib.EWORKSPACE
    assert _hyb(lib, d=5000, nn_in=FAKE, wsb=64) == _lib.EUNSUPPORTED
    assert _hyb(lib, d=5000, k=0, wsb=64) == _lib.EWORKSPACE
    assert _hyb(lib, q=0, out=None, ws=None, wsb=0) == _lib.OK
    assert lib.kde_hybrid_workspace(1000, 4, 3, 5, 0) == 0
    assert lib.kde_hybrid_workspace(1000, 4, 3, 5, 1) > lib.kde_exact_workspace(1000, 4, 3, 1)


def test_options_roundtrip_and_validation(lib):
    d = _lib.Options()
    lib.deann_default_options(d)
    assert (d.rel_tol, d.value_floor, d.knn_slack, d.knn_cap2, d.center,
            d.knn_seed_stride) == (1e-5, 1e-16, 16, 4096, 1, 4)
    got = _lib.Options()
    assert lib.deann_get_options(got) == _lib.OK
    assert got.rel_tol == d.rel_tol and got.knn_cap2 == d.knn_cap2
    try:
        new = _lib.Options()
        lib.deann_default_options(new)
        new.knn_cap2, new.center, new.rel_tol = 8, 0, 1e-3
        assert lib.deann_set_options(new) == _lib.OK
        assert lib.deann_get_options(got) == _lib.OK
        assert (got.knn_cap2, got.center, got.rel_tol) == (8, 0, 1e-3)
        for field, bad in (("rel_tol", 0.0), ("rel_tol", 2.0), ("value_floor", -1.0),
                           ("value_floor", float("inf")), ("knn_slack", -1), ("knn_slack", 513),
                           ("knn_cap2", 0), ("knn_cap2", 4097), ("center", 2),
                           ("knn_seed_stride", 0), ("knn_seed_stride", 65)):
            o = _lib.Options()
            lib.deann_default_options(o)
            setattr(o, field, bad)
            assert lib.deann_set_options(o) == _lib.EINVAL, field
            assert lib.deann_last_error().decode()
        # a rejected call leaves the options as they were
        assert lib.deann_get_options(got) == _lib.OK
        assert (got.knn_cap2, got.center, got.rel_tol) == (8, 0, 1e-3)
        assert lib.deann_set_options(None) == _lib.EINVAL
    finally:
        assert lib.deann_set_options(d) == _lib.OK


def test_slack_enters_the_list_size_check(lib):
    # k + knn_slack beyond the 512 candidates of a list is refused before any launch
    d = _lib.Options()
    lib.deann_default_options(d)
    try:
        o = _lib.Options()
        lib.deann_default_options(o)
        o.knn_slack = 100
        assert lib.deann_set_options(o) == _lib.OK
        assert _dq(lib, n=5000, k=450) == _lib.EUNSUPPORTED
        assert "knn_slack" in lib.deann_last_error().decode()
        o.knn_slack = 0
        assert lib.deann_set_options(o) == _lib.OK
        assert _dq(lib, n=5000, k=496, wsb=8) == _lib.EWORKSPACE
    finally:
        lib.deann_set_options(d)



def test_prepared_sizes_and_validation(lib):
    # sizes: 0 for invalid arguments, growing with n and d, the float32 set
    # holding twice the 16-bit rows
    assert lib.deann_prepared_bytes(0, 8, 0) == 0
    assert lib.deann_prepared_bytes(10, 0, 0) == 0
    assert lib.deann_prepared_bytes(10, 8, 3) == 0          # the split form prepares in FP32
    small, big = lib.deann_prepared_bytes(1000, 64, 1), lib.deann_prepared_bytes(2000, 64, 1)
    assert 0 < small < big
    f32, b16 = lib.deann_prepared_bytes(100000, 960, 0), lib.deann_prepared_bytes(100000, 960, 1)
    assert f32 - b16 >= 100000 * 960 * 2
    # deann_prepare: host checks, nothing launched
    need = lib.deann_prepared_bytes(100, 3, 1)
    assert lib.deann_prepare(None, 100, 3, 1, FAKE, need, None) == _lib.EINVAL
    assert lib.deann_prepare(FAKE, 100, 3, 7, FAKE, need, None) == _lib.EINVAL
    assert lib.deann_prepare(FAKE, 100, 3, 1, None, need, None) == _lib.EINVAL
    assert lib.deann_prepare(FAKE, 100, 3, 1, FAKE, need - 1, None) == _lib.EWORKSPACE
    # the query calls check the set's size against their own n, d and precision
    st = lib.kde_exact_prepared(None, need, FAKE, 100, FAKE, 4, 3, 1.0, 0, 1, FAKE, FAKE, 1 << 30,
                                None)
    assert st == _lib.EINVAL
    need64 = lib.deann_prepared_bytes(100, 64, 1)
    st = lib.kde_exact_prepared(FAKE, need64, FAKE, 100, FAKE, 4, 64, 1.0, 0, 0, FAKE, FAKE,
                                1 << 30, None)
    assert st == _lib.EWORKSPACE          # an FP32 call needs the larger FP32 set
    st = lib.deann_query_prepared(FAKE, need, FAKE, 200, FAKE, 4, 3, 1.0, 0, 5, 10, 0, 0, 0, 1,
                                  FAKE, FAKE, FAKE, FAKE, 1 << 34, None)
    assert st == _lib.EWORKSPACE          # made for n = 100
    st = lib.deann_query_with_grad_prepared(None, need, FAKE, 100, FAKE, 4, 3, 1.0, 0, 5, 10, 0, 0,
                                            0, 1, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, 1 << 34, None)
    assert st == _lib.EINVAL
