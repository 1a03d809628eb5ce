"""Inverted-file neighbours (the ANN of the experiments, Sec. 5) on the GPU
against the oracle: k-means initial assignment bit-exact and one Lloyd step
within float32 rounding; with an index trained by the oracle, the inspected
clusters' k nearest rows, the draws and the DEANN estimates equal the
oracle's for several n_probe, k, widths and both kernels, including the
extension to further clusters and the fallback to the exact k-NN when the
inspected clusters are too small; every
cluster inspected reproduces deann_query; the adjoint takes the indices
unchanged."""
import numpy as np
import pytest

import oracle
from oracle import GAUSSIAN, EXPONENTIAL

from .gpu_common import device, to_dev

pytestmark = pytest.mark.gpu

KNAME = {GAUSSIAN: "gaussian", EXPONENTIAL: "exponential"}


def _mix(n, q, d, seed, centres=6):
    rng = np.random.default_rng(seed)
    cen = rng.uniform(-4, 4, size=(centres, d))
    X = (cen[rng.integers(0, centres, n)] + rng.normal(size=(n, d))).astype(np.float32)
    Y = (cen[rng.integers(0, centres, q)] + rng.normal(size=(q, d))).astype(np.float32)
    return X, Y


def _near_tie(X, C, i, a, b):
    """Rows whose two candidate centroids are too close to order reliably
    after a float32 rounding of the centroids."""
    da = float(((X[i].astype(np.float64) - C[a]) ** 2).sum())
    db = float(((X[i].astype(np.float64) - C[b]) ** 2).sum())
    return abs(da - db) <= 1e-5 * max(da, db, 1e-30)


@pytest.mark.parametrize("d", [16, 5])
def test_kmeans_initial_assignment_and_one_lloyd_step(d):
    import paper_2107_02736_amd as dk
    dev = device()
    X, _ = _mix(3000, 1, d, seed=1)
    Xd = to_dev(X, dev)
    C0, a0 = (t.cpu().numpy() for t in dk.ivf_build(Xd, 12, iters=0))
    C_init = oracle.kmeans_init(X, 12)
    assert np.array_equal(C0, C_init)
    assert np.array_equal(a0, oracle.kmeans_assign(X, C_init))
    C1, a1 = (t.cpu().numpy() for t in dk.ivf_build(Xd, 12, iters=1))
    C1_ref = oracle.kmeans_update(X, oracle.kmeans_assign(X, C_init), C_init)
    # FP64 row-order sum versus an exactly rounded sum: at most one float32 ulp
    assert np.all(np.abs(C1 - C1_ref) <= np.spacing(np.abs(C1_ref)) + 1e-30)
    a1_ref = oracle.kmeans_assign(X, C1_ref)
    for i in np.nonzero(a1 != a1_ref)[0]:
        assert _near_tie(X, C1_ref, i, a1[i], a1_ref[i])
    # the returned assignment is a closest centroid of the returned centroids
    assert np.array_equal(a1, oracle.kmeans_assign(X, C1))


def test_kmeans_iterations_give_a_valid_index():
    import paper_2107_02736_amd as dk
    dev = device()
    X, _ = _mix(4000, 1, 8, seed=2)
    C, a = (t.cpu().numpy() for t in dk.ivf_build(to_dev(X, dev), 20, iters=6))
    assert np.array_equal(a, oracle.kmeans_assign(X, C))
    C0 = oracle.kmeans_init(X, 20)
    a0 = oracle.kmeans_assign(X, C0)

    def sse(C, a):
        return float(((X.astype(np.float64) - C[a].astype(np.float64)) ** 2).sum())
    assert sse(C, a) < sse(C0, a0)


def _check_queries(X, Y, C, a, n_probe, k, m, kern, h, seed, out, nn, sm, rows):
    for j in rows:
        est, nn_ref, s_ref = oracle.deann_estimate_ivf(X, Y[j], h, kern, C, a, n_probe, k, m,
                                                       seed, j)
        assert np.array_equal(nn[j], nn_ref), (j, n_probe, k)
        assert np.array_equal(sm[j], s_ref), (j, n_probe, k)
        assert abs(out[j] - est) <= 1e-12 * max(est, 1e-300), (j, out[j], est)


@pytest.mark.parametrize("d", [16, 33])
@pytest.mark.parametrize("kern", [GAUSSIAN, EXPONENTIAL])
def test_ivf_query_matches_oracle(kern, d):
    import paper_2107_02736_amd as dk
    dev = device()
    X, Y = _mix(3000, 40, d, seed=3)
    C, a = oracle.ivf_train(X, 12, 2)
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    index = dk.IvfIndex(Xd, to_dev(C, dev), to_dev(a.astype(np.int32), dev))
    h = 3.0 if kern == GAUSSIAN else 2.0
    for n_probe, k, m in ((1, 5, 40), (3, 50, 200), (12, 20, 100), (2, 300, 60)):
        out, nn, sm = (t.cpu().numpy() for t in dk.deann_ivf_query(
            Xd, Yd, index, n_probe, h, k, m, KNAME[kern], seed=7))
        _check_queries(X, Y, C, a, n_probe, k, m, kern, h, 7, out, nn, sm, range(40))


def test_extension_to_further_clusters_and_the_fallback():
    import paper_2107_02736_amd as dk
    dev = device()
    # about 50 rows per cluster: k above the median size extends many queries
    X, Y = _mix(3000, 30, 6, seed=4, centres=30)
    C, a = oracle.ivf_train(X, 60, 1)
    sizes = np.bincount(a, minlength=60)
    k = int(np.sort(sizes)[len(sizes) // 2]) + 1
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    index = dk.IvfIndex(Xd, to_dev(C, dev), to_dev(a.astype(np.int32), dev))
    extended = 0
    for n_probe in (1, 2):
        out, nn, sm = (t.cpu().numpy() for t in dk.deann_ivf_query(
            Xd, Yd, index, n_probe, 2.0, k, 50, "gaussian", seed=1))
        _check_queries(X, Y, C, a, n_probe, k, 50, GAUSSIAN, 2.0, 1, out, nn, sm, range(30))
        extended += sum(len(oracle.ivf_probe(C, y, n_probe, sizes, k)) > n_probe for y in Y)
    assert extended > 0
    # about 5 rows per cluster: at most 65 clusters hold fewer than k = 400 rows,
    # so every query uses the exact k nearest rows of all of X
    C, a = oracle.ivf_train(X, 600, 1)
    index = dk.IvfIndex(Xd, to_dev(C, dev), to_dev(a.astype(np.int32), dev))
    out, nn, sm = (t.cpu().numpy() for t in dk.deann_ivf_query(Xd, Yd, index, 1, 2.0, 400, 50,
                                                               "gaussian", seed=1))
    sizes = np.bincount(a, minlength=600)
    assert all(oracle.ivf_probe(C, y, 1, sizes, 400).size == 0 for y in Y[:5])
    _check_queries(X, Y, C, a, 1, 400, 50, GAUSSIAN, 2.0, 1, out, nn, sm, range(0, 30, 3))


def test_every_cluster_inspected_is_deann_query_and_the_adjoint():
    import paper_2107_02736_amd as dk
    dev = device()
    X, Y = _mix(2500, 33, 12, seed=5)
    C, a = oracle.ivf_train(X, 7, 1)
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    index = dk.IvfIndex(Xd, to_dev(C, dev), to_dev(a.astype(np.int32), dev))
    r1 = [t.cpu().numpy() for t in dk.deann_ivf_query(Xd, Yd, index, 7, 2.5, 30, 120, seed=4)]
    r2 = [t.cpu().numpy() for t in dk.deann_query(Xd, Yd, 2.5, 30, 120, "gaussian", seed=4)]
    for u, v in zip(r1, r2):
        assert np.array_equal(u, v)
    # the adjoint of the estimate with the inverted-file index sets
    out, nn, sm = dk.deann_ivf_query(Xd, Yd, index, 2, 2.5, 30, 120, seed=4)
    g = np.linspace(0.5, 1.5, 33)
    gy, gh = dk.deann_query_backward(Xd, Yd, 2.5, 30, 120, nn, sm, to_dev(g, dev))
    gy, gh = gy.cpu().numpy(), float(gh.cpu().numpy()[0])
    nn, sm = nn.cpu().numpy(), sm.cpu().numpy()
    gh_ref = 0.0
    for j in range(33):
        _, gy_ref, ghj = oracle.deann_grad(X, Y[j], 2.5, GAUSSIAN, nn[j], sm[j], 120)
        assert np.linalg.norm(gy[j] - g[j] * gy_ref) <= 1e-5 * g[j] * np.linalg.norm(gy_ref) + 1e-12
        gh_ref += g[j] * ghj
    assert gh == pytest.approx(gh_ref, rel=1e-10)


def test_gpu_trained_index_and_recall():
    import paper_2107_02736_amd as dk
    dev = device()
    X, Y = _mix(6000, 25, 10, seed=6)
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    Cd, ad = dk.ivf_build(Xd, 24, iters=4)
    index = dk.IvfIndex(Xd, Cd, ad)
    C, a = Cd.cpu().numpy(), ad.cpu().numpy().astype(np.int64)
    out, nn, sm = (t.cpu().numpy() for t in dk.deann_ivf_query(Xd, Yd, index, 4, 2.0, 40, 100,
                                                               seed=2))
    _check_queries(X, Y, C, a, 4, 40, 100, GAUSSIAN, 2.0, 2, out, nn, sm, range(25))
    rec = [oracle.recall(oracle.knn(X, y, 40), nn[j]) for j, y in enumerate(Y)]
    print(f"recall at n_probe = 4 of 24 clusters: mean {np.mean(rec):.3f} min {np.min(rec):.3f}")
    assert np.mean(rec) > 0.5


def test_long_sweeps_in_parts():
    # uneven clusters (k-means gives about 4000, 4200, 2200 and 1100 rows, up
    # to 34 data tiles): the query tiles of the large clusters sweep them in
    # up to 4 parts, each with lists of its own, which the refinement merges
    import paper_2107_02736_amd as dk
    dev = device()
    rng = np.random.default_rng(8)
    d = 16
    cen = rng.uniform(-20, 20, size=(4, d))
    sizes = (8000, 2000, 1000, 500)
    X = np.concatenate([cen[i] + rng.normal(size=(c, d)) for i, c in enumerate(sizes)])
    X = X[rng.permutation(X.shape[0])].astype(np.float32)
    Y = (cen[rng.choice(4, size=300, p=[0.55, 0.25, 0.1, 0.1])] +
         rng.normal(size=(300, d))).astype(np.float32)
    C, a = oracle.ivf_train(X, 4, 2)
    assert np.bincount(a, minlength=4).max() >= 4000
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    index = dk.IvfIndex(Xd, to_dev(C, dev), to_dev(a.astype(np.int32), dev))
    for n_probe, k, m in ((1, 50, 100), (2, 200, 60)):
        out, nn, sm = (t.cpu().numpy() for t in dk.deann_ivf_query(
            Xd, Yd, index, n_probe, 2.0, k, m, "gaussian", seed=3))
        _check_queries(X, Y, C, a, n_probe, k, m, GAUSSIAN, 2.0, 3, out, nn, sm, range(0, 300, 4))
