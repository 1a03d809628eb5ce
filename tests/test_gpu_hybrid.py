"""Near/far form of the exact KDE (kde_hybrid): the k nearest rows of a query
summed exactly in FP64, the remaining rows by the 16-bit tile sweep, which
leaves the neighbour pairs out of its sums.

Checked against the FP64 oracle: the neighbour lists equal the oracle's exact
k-NN, and every query's error against the exact KDE is within the bound of
tests/precision_bound.py with the neighbours' terms taken out (those are
exact).  Degenerate forms: k = 0 is kde_exact with the same precision (bit for
bit) and k = n the exact sum of deann_query with k = n.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import GAUSSIAN, EXPONENTIAL

from .gpu_common import bandwidth, device, rel_err, to_dev
from .precision_bound import exact_kde_bound, geometry as bound_geometry

pytestmark = pytest.mark.gpu

WL = "mix10_n1e4_d16"
KNAME = {GAUSSIAN: "gaussian", EXPONENTIAL: "exponential"}


@pytest.fixture(scope="module")
def dev():
    return device()


@pytest.fixture(scope="module")
def data(dev):
    _, X, Y = synth.workload(WL)
    return X, Y, to_dev(X, dev), to_dev(Y, dev)


@pytest.fixture(scope="module")
def geometry(data):
    X, Y, _, _ = data
    return bound_geometry(X, Y)


@pytest.fixture(scope="module")
def near50(data):
    X, Y, _, _ = data
    return np.stack([oracle.knn(X, Y[j], 50) for j in range(Y.shape[0])])


def _small(n, q, d, seed=0):
    rng = np.random.default_rng(seed)
    cen = rng.uniform(-3, 3, size=(5, d))
    X = (cen[rng.integers(0, 5, n)] + rng.normal(size=(n, d))).astype(np.float32)
    Y = (cen[rng.integers(0, 5, q)] + rng.normal(size=(q, d))).astype(np.float32)
    return X, Y


def _check_against_oracle(got, X, Y, h, kern, prec, near, label):
    ref = oracle.kde_exact(X, Y, h, kern)
    keep = ref >= 1e-16
    err = np.abs(got[keep] - ref[keep]) / ref[keep]
    bound = exact_kde_bound(bound_geometry(X, Y), X.shape[1], h, kern, prec, near=near)[keep]
    assert np.all(err <= bound), (label, err.max(), bound[np.argmax(err - bound)])
    return err, bound


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("kern", [GAUSSIAN, EXPONENTIAL])
def test_small_mixture_against_oracle(data, geometry, near50, kern, prec):
    import paper_2107_02736_amd as dk
    X, Y, Xd, Yd = data
    h = bandwidth(WL, KNAME[kern])
    got, nn = dk.kde_hybrid(Xd, Yd, h, 50, KNAME[kern], prec, return_indices=True)
    got, nn = got.cpu().numpy(), nn.cpu().numpy()
    assert np.array_equal(nn, near50)
    ref = oracle.kde_exact(X, Y, h, kern)
    keep = ref >= 1e-16
    err, _ = rel_err(got, ref)
    bound = exact_kde_bound(geometry, X.shape[1], h, kern, prec, near=near50)[keep]
    plain_bound = exact_kde_bound(geometry, X.shape[1], h, kern, prec)[keep]
    plain, _ = rel_err(dk.kde_exact(Xd, Yd, h, KNAME[kern], prec).cpu().numpy(), ref)
    print(f"{KNAME[kern]:11s} {prec} k=50: near/far rel err max {err.max():.2e} mean "
          f"{err.mean():.2e} (bound max {bound.max():.2e}); plain {prec} max {plain.max():.2e} "
          f"mean {plain.mean():.2e} (bound max {plain_bound.max():.2e})")
    assert np.all(err <= bound)
    assert np.all(bound <= plain_bound)


def test_degenerate_k(dev):
    import paper_2107_02736_amd as dk
    X, Y = _small(400, 37, 9, seed=4)
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    for prec in ("bf16", "fp16"):
        a = dk.kde_hybrid(Xd, Yd, 1.7, 0, "gaussian", prec).cpu().numpy()
        b = dk.kde_exact(Xd, Yd, 1.7, "gaussian", prec).cpu().numpy()
        assert np.array_equal(a, b)
    ref = oracle.kde_exact(X, Y, 1.7, GAUSSIAN)
    c, nn = dk.kde_hybrid(Xd, Yd, 1.7, 400, "gaussian", "bf16", return_indices=True)
    assert np.allclose(c.cpu().numpy(), ref, rtol=1e-12, atol=0)
    assert np.array_equal(nn.cpu().numpy(), np.tile(np.arange(400, dtype=np.int32), (37, 1)))
    e = dk.deann_query(Xd, Yd, 1.7, 400, 0, "gaussian", precision="bf16")[0]
    assert np.array_equal(c.cpu().numpy(), e.cpu().numpy())


@pytest.mark.parametrize("n,q,d", [(1000, 37, 9), (129, 1, 3), (300, 130, 33), (2500, 64, 64),
                                   (3000, 200, 100), (700, 20, 130)])
def test_edge_shapes(dev, n, q, d):
    # rows of 64, 128, 256 and 320 bytes in bfloat16 reach every tile engine
    import paper_2107_02736_amd as dk
    X, Y = _small(n, q, d, seed=n + d)
    k = min(20, n)
    h = 1.5 + 0.05 * d
    got, nn = dk.kde_hybrid(to_dev(X, dev), to_dev(Y, dev), h, k, "gaussian", "bf16",
                            return_indices=True)
    near = np.stack([oracle.knn(X, Y[j], k) for j in range(q)])
    assert np.array_equal(nn.cpu().numpy(), near)
    _check_against_oracle(got.cpu().numpy(), X, Y, h, GAUSSIAN, "bf16", near, (n, q, d))


def test_many_pairs_per_tile(dev):
    # 128 equal queries with k = 400 over 16 data tiles: most workgroups hold
    # more neighbour pairs than their LDS stage (read from global memory),
    # some fewer
    import paper_2107_02736_amd as dk
    X, _ = _small(2048, 1, 16, seed=9)
    Y = np.repeat(X[5:6] + np.float32(0.25), 128, axis=0)
    got = dk.kde_hybrid(to_dev(X, dev), to_dev(Y, dev), 1.2, 400, "exponential", "bf16")
    got = got.cpu().numpy()
    assert np.all(got == got[0])
    near = oracle.knn(X, Y[0], 400)[None, :]
    _check_against_oracle(got[:1], X, Y[:1], 1.2, EXPONENTIAL, "bf16", near, "many pairs")


def test_given_neighbour_lists(dev):
    import paper_2107_02736_amd as dk
    X, Y = _small(3000, 200, 33, seed=2)
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    h = 2.5
    # the lists of deann_query give the same result up to the FP64 order of Z1
    _, nn, _ = dk.deann_query(Xd, Yd, h, 40, 10, "gaussian", precision="bf16")
    a = dk.kde_hybrid(Xd, Yd, h, 40, "gaussian", "bf16", nn_idx=nn).cpu().numpy()
    b = dk.kde_hybrid(Xd, Yd, h, 40, "gaussian", "bf16").cpu().numpy()
    assert np.allclose(a, b, rtol=1e-13, atol=0)
    # any lists of distinct rows, also beyond the k-NN limit of 496
    rng = np.random.default_rng(5)
    rows = np.stack([rng.choice(3000, size=600, replace=False) for _ in range(200)])
    got, used = dk.kde_hybrid(Xd, Yd, h, 600, "gaussian", "bf16",
                              nn_idx=to_dev(rows.astype(np.int32), dev), return_indices=True)
    assert np.array_equal(used.cpu().numpy(), rows)
    _check_against_oracle(got.cpu().numpy(), X, Y, h, GAUSSIAN, "bf16", rows, "given lists")


def test_deann_with_every_row_near_at_large_n(dev):
    # k = n above the size of the sampler's shared-memory gap table
    import paper_2107_02736_amd as dk
    X, Y = _small(50_000, 3, 8, seed=6)
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    ref = oracle.kde_exact(X, Y, 1.5, GAUSSIAN)
    est = dk.deann_query(Xd, Yd, 1.5, 50_000, 10, "gaussian", precision="bf16",
                         return_indices=False)[0].cpu().numpy()
    assert np.allclose(est, ref, rtol=1e-12, atol=0)
    hyb = dk.kde_hybrid(Xd, Yd, 1.5, 50_000, "gaussian", "bf16").cpu().numpy()
    assert np.array_equal(hyb, est)
