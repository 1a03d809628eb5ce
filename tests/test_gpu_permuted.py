"""DEANN with permuted random sampling (App. G, Algorithm 2) on the GPU against
the oracle: neighbour sets and block rows bit-exact, estimates within 1e-12,
m = n - k equal to the exact KDE, batches that pass the running index
reproduce the whole call, the adjoint through autograd, and sampled queries
of the 100-cluster mixture at full size."""
import numpy as np
import pytest

import oracle
import synth
from oracle import GAUSSIAN, EXPONENTIAL

from .gpu_common import bandwidth, device, to_dev

pytestmark = pytest.mark.gpu

KNAME = {GAUSSIAN: "gaussian", EXPONENTIAL: "exponential"}


def _small(n, q, d, seed):
    rng = np.random.default_rng(seed)
    cen = rng.uniform(-3, 3, size=(5, d))
    X = (cen[rng.integers(0, 5, n)] + rng.normal(size=(n, d))).astype(np.float32)
    Y = (cen[rng.integers(0, 5, q)] + rng.normal(size=(q, d))).astype(np.float32)
    return X, Y


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("kern", [GAUSSIAN, EXPONENTIAL])
def test_permuted_matches_oracle(kern, prec):
    import paper_2107_02736_amd as dk
    dev = device()
    spec, X, Y = synth.workload("mix10_n1e4_d16")
    Y = Y[:120]
    h = bandwidth("mix10_n1e4_d16", KNAME[kern])
    k, m, seed, start = 50, 500, 3, 9_876
    out, nn, sm = (t.cpu().numpy() for t in dk.deann_query_permuted(
        to_dev(X, dev), to_dev(Y, dev), h, k, m, KNAME[kern], seed=seed, start=start,
        precision=prec))
    n = X.shape[0]
    for j in range(0, Y.shape[0], 7):
        est, nn_ref, s_ref = oracle.deann_estimate_permuted(X, Y[j], h, kern, k, m, seed,
                                                            (start + j * m) % n)
        assert np.array_equal(nn[j], nn_ref), j
        assert np.array_equal(sm[j], s_ref), j
        assert abs(out[j] - est) <= 1e-12 * max(est, 1e-300)
    # m distinct rows outside the neighbour set for every query
    for j in range(Y.shape[0]):
        assert len(np.unique(sm[j])) == m and not np.isin(sm[j], nn[j]).any()


@pytest.mark.parametrize("n,k", [(300, 20), (300, 0), (5, 1), (129, 128)])
def test_permuted_full_block_is_exact(n, k):
    import paper_2107_02736_amd as dk
    dev = device()
    X, Y = _small(n, 6, 4, seed=n + k)
    h = 1.2
    m = n - k
    out, nn, sm = (t.cpu().numpy() for t in dk.deann_query_permuted(
        to_dev(X, dev), to_dev(Y, dev), h, k, m, "gaussian", seed=1, start=3))
    ref = oracle.kde_exact(X, Y, h, GAUSSIAN)
    assert np.allclose(out, ref, rtol=1e-12, atol=0)
    for j in range(Y.shape[0]):
        assert sorted(sm[j].tolist()) == sorted(set(range(n)) - set(nn[j].tolist()))
    with pytest.raises(dk.DeannError):
        dk.deann_query_permuted(to_dev(X, dev), to_dev(Y, dev), h, k, m + 1, "gaussian")


def test_permuted_batches_pass_the_running_index():
    import paper_2107_02736_amd as dk
    dev = device()
    X, Y = _small(2000, 70, 8, seed=4)
    Xd = to_dev(X, dev)
    k, m, h, s0 = 10, 33, 1.5, 1_234_567
    whole = [t.cpu().numpy() for t in dk.deann_query_permuted(Xd, to_dev(Y, dev), h, k, m,
                                                             seed=6, start=s0, precision="bf16")]
    a = 29
    p1 = [t.cpu().numpy() for t in dk.deann_query_permuted(Xd, to_dev(Y[:a], dev), h, k, m,
                                                          seed=6, start=s0, precision="bf16")]
    p2 = [t.cpu().numpy() for t in dk.deann_query_permuted(Xd, to_dev(Y[a:], dev), h, k, m,
                                                          seed=6, start=s0 + a * m,
                                                          precision="bf16")]
    for w, x1, x2 in zip(whole, p1, p2):
        assert np.array_equal(w, np.concatenate([x1, x2]))


def test_permuted_adjoint_through_autograd():
    import torch
    import paper_2107_02736_amd as dk
    dev = device()
    X, Y = _small(3000, 25, 12, seed=8)
    Xd = to_dev(X, dev)
    Yd = to_dev(Y, dev).requires_grad_(True)
    h, k, m = 1.3, 16, 100
    out = dk.deann_kde(Yd, h, Xd, k, m, "gaussian", seed=2, start=77)
    g = torch.linspace(0.5, 1.5, 25, dtype=torch.float64, device=dev)
    (out * g).sum().backward()
    gy = Yd.grad.cpu().numpy()
    gn = g.cpu().numpy()
    for j in range(25):
        _, nn, s = oracle.deann_estimate_permuted(X, Y[j], h, GAUSSIAN, k, m, 2, 77 + j * m)
        _, gy_ref, _ = oracle.deann_grad(X, Y[j], h, GAUSSIAN, nn, s, m)
        assert np.linalg.norm(gy[j] - gn[j] * gy_ref) <= 1e-6 * np.linalg.norm(gn[j] * gy_ref)


def test_permuted_fullsize_sampled():
    import paper_2107_02736_amd as dk
    dev = device()
    wl = "mix100_n1e6_d128"
    spec, X, Y = synth.workload(wl)
    h = bandwidth(wl, "gaussian")
    k, m, start = 100, 1000, 5
    out, nn, sm = (t.cpu().numpy() for t in dk.deann_query_permuted(
        to_dev(X, dev), to_dev(Y, dev), h, k, m, "gaussian", seed=0, start=start,
        precision="bf16"))
    n = X.shape[0]
    for j in synth.query_subset(Y.shape[0], 3, seed=29):
        est, nn_ref, s_ref = oracle.deann_estimate_permuted(X, Y[j], h, GAUSSIAN, k, m, 0,
                                                            (start + int(j) * m) % n)
        assert np.array_equal(nn[j], nn_ref), j
        assert np.array_equal(sm[j], s_ref), j
        assert abs(out[j] - est) <= 1e-12 * max(est, 1e-300)


@pytest.mark.parametrize("n,d", [(10_000, 16), (300, 9), (129, 33), (5, 4), (4099, 128)])
def test_permuted_index_is_the_permutation(n, d):
    # Algorithm 2's preprocessing: pi is a permutation of [n] equal to the
    # oracle's keyed permutation, and the copy holds x_pi(i) at position i
    import torch

    import paper_2107_02736_amd as dk
    dev = device()
    X, _ = _small(n, 1, d, seed=n + d)
    Xd = to_dev(X, dev)
    idx = dk.PermutedIndex(Xd, seed=11)
    torch.cuda.synchronize()
    pi = idx.permutation().cpu().numpy()
    assert np.array_equal(np.sort(pi), np.arange(n))
    for pos in list(range(min(n, 40))) + list(range(max(0, n - 40), n)):
        assert pi[pos] == oracle.permutation(n, 11, pos), pos
    raw = idx.buffer.cpu().numpy()
    inv = raw[4 * n: 8 * n].view(np.int32)
    assert np.array_equal(inv[pi], np.arange(n))
    off = (8 * n + 255) // 256 * 256
    base = (256 - idx.buffer.data_ptr() % 256) % 256   # the library aligns the buffer start
    Xp = raw[base + off: base + off + 4 * n * d].view(np.float32).reshape(n, d)
    assert np.array_equal(Xp, X[pi])


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("kern", [GAUSSIAN, EXPONENTIAL])
def test_permuted_index_reproduces_the_evaluated_permutation(kern, prec):
    # with the permuted copy: the same neighbours, rows and estimates bit for
    # bit as the permutation evaluated per draw, and the oracle's
    import paper_2107_02736_amd as dk
    dev = device()
    spec, X, Y = synth.workload("mix10_n1e4_d16")
    Y = Y[:150]
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    h = bandwidth("mix10_n1e4_d16", KNAME[kern])
    n = X.shape[0]
    idx = dk.PermutedIndex(Xd, seed=5)
    for k, m, start in ((50, 500, 77), (0, 37, n - 10), (9, n - 9, 0)):
        a = [t.cpu().numpy() for t in dk.deann_query_permuted(Xd, Yd, h, k, m, KNAME[kern], seed=5,
                                                            start=start, precision=prec)]
        b = [t.cpu().numpy() for t in dk.deann_query_permuted(Xd, Yd, h, k, m, KNAME[kern],
                                                            start=start, precision=prec,
                                                            index=idx)]
        for u, v in zip(a, b):
            assert np.array_equal(u, v), (k, m)
        for j in range(0, Y.shape[0], 37):
            est, nn_ref, s_ref = oracle.deann_estimate_permuted(X, Y[j], h, kern, k, m, 5,
                                                                (start + j * m) % n)
            assert np.array_equal(b[1][j], nn_ref) and np.array_equal(b[2][j], s_ref)
            assert abs(b[0][j] - est) <= 1e-12 * max(est, 1e-300)


def test_permuted_index_fullsize_d960():
    # the large workload: the index's block rows against the evaluated
    # permutation on every query (bitwise), two queries against the oracle
    import torch

    import paper_2107_02736_amd as dk
    dev = device()
    wl = "mix200_n1e6_d960"
    spec, X, Y = synth.workload(wl, q=2000)
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    h = bandwidth(wl, "gaussian")
    idx = dk.PermutedIndex(Xd, seed=2)
    a = [t.cpu().numpy() for t in dk.deann_query_permuted(Xd, Yd, h, 200, 2000, seed=2, start=5,
                                                        precision="bf16")]
    b = [t.cpu().numpy() for t in dk.deann_query_permuted(Xd, Yd, h, 200, 2000, start=5,
                                                        precision="bf16", index=idx)]
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    del idx
    torch.cuda.empty_cache()
    n = X.shape[0]
    for j in (3, 1777):
        est, nn_ref, s_ref = oracle.deann_estimate_permuted(X, Y[j], h, GAUSSIAN, 200, 2000, 2,
                                                            (5 + j * 2000) % n)
        assert np.array_equal(b[1][j], nn_ref) and np.array_equal(b[2][j], s_ref)
        assert abs(b[0][j] - est) <= 1e-12 * est
