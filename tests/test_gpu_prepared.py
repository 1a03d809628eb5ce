"""Prepared data sets (deann_prepare and the *_prepared calls): the same results,
bit for bit, as the calls that prepare X themselves, for several query batches
against one prepared set; and the oracle's values on a sample of queries."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import GAUSSIAN

from .gpu_common import bandwidth, device, to_dev

pytestmark = pytest.mark.gpu

WL = "mix10_n1e4_d16"


@pytest.fixture(scope="module")
def dev():
    return device()


@pytest.fixture(scope="module")
def data(dev):
    # 3000 rows of d = 100 (several tiles, a ragged last one, padded rows) and
    # two query batches of different sizes
    rng = np.random.default_rng(41)
    X = (rng.normal(size=(3000, 100)) * rng.uniform(0.5, 2.0, size=(3000, 1))).astype(np.float32)
    Y1 = (rng.normal(size=(300, 100)) * 1.2).astype(np.float32)
    Y2 = (rng.normal(size=(77, 100)) * 0.8).astype(np.float32)
    return X, Y1, Y2, to_dev(X, dev), to_dev(Y1, dev), to_dev(Y2, dev)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16", "fp32_split"])
def test_kde_exact_prepared_equals_unprepared(data, prec):
    import paper_2107_02736_amd as dk
    X, Y1, Y2, Xd, Y1d, Y2d = data
    pre = dk.prepare(Xd, "fp32" if prec == "fp32_split" else prec)
    for kern in ("gaussian", "exponential"):
        for Yd in (Y1d, Y2d, Y1d):
            a = dk.kde_exact(Xd, Yd, 9.0, kern, precision=prec)
            b = dk.kde_exact(Xd, Yd, 9.0, kern, precision=prec, prepared=pre)
            torch.cuda.synchronize()
            assert torch.equal(a, b), (prec, kern)


@pytest.mark.parametrize("prec", ["fp32", "fp32_split"])
def test_kde_exact_with_grad_prepared_equals_unprepared(data, prec):
    import paper_2107_02736_amd as dk
    X, Y1, Y2, Xd, Y1d, Y2d = data
    pre = dk.prepare(Xd, "fp32")
    for kern in ("gaussian", "exponential"):
        for Yd in (Y2d, Y1d):
            a = dk.kde_exact_with_grad(Xd, Yd, 9.0, kern, precision=prec)
            b = dk.kde_exact_with_grad(Xd, Yd, 9.0, kern, precision=prec, prepared=pre)
            for u, v in zip(a, b):
                assert torch.equal(u, v), (prec, kern)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_deann_prepared_equals_unprepared(data, prec):
    import paper_2107_02736_amd as dk
    X, Y1, Y2, Xd, Y1d, Y2d = data
    pre = dk.prepare(Xd, prec)
    for Yd in (Y2d, Y1d):
        a = dk.deann_query(Xd, Yd, 9.0, 40, 100, seed=3, precision=prec)
        b = dk.deann_query(Xd, Yd, 9.0, 40, 100, seed=3, precision=prec, prepared=pre)
        for u, v in zip(a, b):
            assert torch.equal(u, v), prec
        a = dk.deann_query_with_grad(Xd, Yd, 9.0, 40, 100, seed=3, precision=prec)
        b = dk.deann_query_with_grad(Xd, Yd, 9.0, 40, 100, seed=3, precision=prec, prepared=pre)
        for u, v in zip(a, b):
            assert torch.equal(u, v), prec


def test_prepared_small_mixture_matches_oracle(dev):
    # the small mixture: estimates, neighbours and draws of the prepared calls
    # against the oracle on sampled queries
    import paper_2107_02736_amd as dk
    spec, X, Y = synth.workload(WL)
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    h = bandwidth(WL, "gaussian")
    pre = dk.prepare(Xd, "bf16")
    out, nn, sm = (t.cpu().numpy() for t in
                   dk.deann_query(Xd, Yd, h, 50, 500, seed=0, precision="bf16", prepared=pre))
    for j in range(0, Y.shape[0], 97):
        est, nn_ref, s_ref = oracle.deann_estimate(X, Y[j], h, GAUSSIAN, 50, 500, 0, j)
        assert np.array_equal(nn[j], nn_ref), j
        assert np.array_equal(sm[j], s_ref), j
        assert abs(out[j] - est) <= 1e-12 * max(est, 1e-300), j
    pre32 = dk.prepare(Xd, "fp32")
    mu = dk.kde_exact(Xd, Yd, h, precision="fp32", prepared=pre32).cpu().numpy()
    ref = oracle.kde_exact(X, Y[::97], h, GAUSSIAN)
    assert np.max(np.abs(mu[::97] - ref) / ref) <= 1e-5


def test_prepared_mismatch_is_refused(data, dev):
    import paper_2107_02736_amd as dk
    X, Y1, Y2, Xd, Y1d, Y2d = data
    pre = dk.prepare(Xd, "bf16")
    other = Xd.clone()
    with pytest.raises(ValueError):
        dk.deann_query(other, Y1d, 9.0, 40, 100, precision="bf16", prepared=pre)
    with pytest.raises(ValueError):
        dk.deann_query(Xd, Y1d, 9.0, 40, 100, precision="fp32", prepared=pre)
    with pytest.raises(ValueError):
        dk.kde_exact(Xd, Y1d, 9.0, precision="fp32", prepared=pre)


def test_autograd_with_prepared_sets(data):
    # the autograd wrappers: values and gradients equal with and without a
    # prepared set of X
    import paper_2107_02736_amd as dk
    X, Y1, Y2, Xd, Y1d, Y2d = data
    pre32, pre16 = dk.prepare(Xd, "fp32"), dk.prepare(Xd, "bf16")
    res = []
    for p32, p16 in ((None, None), (pre32, pre16)):
        Y = Y2d.clone().requires_grad_(True)
        h = torch.tensor(9.0, dtype=torch.float64, requires_grad=True)
        v = dk.exact_kde(Y, h, Xd, prepared=p32).sum() + \
            dk.deann_kde(Y, h, Xd, 40, 100, precision="bf16", prepared=p16).sum()
        v.backward()
        res.append((v.detach(), Y.grad.clone(), h.grad.clone()))
    for u, w in zip(*res):
        assert torch.equal(u, w)


@pytest.mark.parametrize("kern", ["gaussian", "exponential"])
def test_prepared_degenerate_k_and_empty_batches(data, kern):
    # k = 0 (plain random sampling), k = n (exact sum) and q = 0 with a prepared
    # set: the same results as the unprepared calls
    import paper_2107_02736_amd as dk
    X, Y1, Y2, Xd, Y1d, Y2d = data
    n = X.shape[0]
    pre = dk.prepare(Xd, "bf16")
    for k, m in ((0, 64), (n, 0), (7, 0)):
        a = dk.deann_query_with_grad(Xd, Y2d, 9.0, k, m, kern, seed=5, precision="bf16")
        b = dk.deann_query_with_grad(Xd, Y2d, 9.0, k, m, kern, seed=5, precision="bf16",
                                     prepared=pre)
        for u, v in zip(a, b):
            assert (u is None and v is None) or torch.equal(u, v), (k, m)
    empty = Y2d[:0]
    out, _, _ = dk.deann_query(Xd, empty, 9.0, 7, 5, kern, precision="bf16", prepared=pre)
    assert out.numel() == 0
