"""Pins of the inverted-file (IVF) oracle (the ANN of the experiments, Sec. 5):
hand-computed Lloyd steps on one-dimensional data (including an empty
cluster and centroid ties), the reduction to the exact k-NN when every
cluster is inspected or there is one cluster, a brute force over exact
rational distances on tiny inputs, the fallback when the inspected clusters
hold fewer than k rows, the mean property of the update, the monotone k-means
objective, and the recall of Sec. 5."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import GAUSSIAN


def _mix(n, d, seed, centres=4):
    rng = np.random.default_rng(seed)
    cen = rng.uniform(-4, 4, size=(centres, d))
    X = (cen[rng.integers(0, centres, n)] + rng.normal(size=(n, d))).astype(np.float32)
    Y = (cen[rng.integers(0, centres, 6)] + rng.normal(size=(6, d))).astype(np.float32)
    return X, Y


def test_lloyd_steps_by_hand():
    X = np.array([[0], [1], [10], [11]], dtype=np.float32)
    C0 = oracle.kmeans_init(X, 2)                  # rows 0 and 2
    assert C0.ravel().tolist() == [0.0, 10.0]
    a1 = oracle.kmeans_assign(X, C0)
    assert a1.tolist() == [0, 0, 1, 1]
    C1 = oracle.kmeans_update(X, a1, C0)
    assert C1.ravel().tolist() == [0.5, 10.5]
    C, a = oracle.ivf_train(X, 2, 3)
    assert C.ravel().tolist() == [0.5, 10.5] and a.tolist() == [0, 0, 1, 1]


def test_empty_cluster_and_centroid_ties_by_hand():
    # both initial centroids are the point 0: ties go to cluster 0, so
    # cluster 1 is empty and keeps its centroid
    X = np.array([[0], [0], [0], [5]], dtype=np.float32)
    C0 = oracle.kmeans_init(X, 2)                  # rows 0 and 2
    a1 = oracle.kmeans_assign(X, C0)
    assert a1.tolist() == [0, 0, 0, 0]
    C1 = oracle.kmeans_update(X, a1, C0)
    assert C1.ravel().tolist() == [1.25, 0.0]
    # zeros are now closer to centroid 1 (distance 0), 5 to centroid 0
    assert oracle.kmeans_assign(X, C1).tolist() == [1, 1, 1, 0]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_update_is_the_mean_and_the_objective_never_grows(seed):
    X, _ = _mix(300, 3, seed)
    C = oracle.kmeans_init(X, 7)
    prev = np.inf
    for _ in range(5):
        a = oracle.kmeans_assign(X, C)
        sse = float(((X.astype(np.float64) - C[a].astype(np.float64)) ** 2).sum())
        assert sse <= prev * (1 + 1e-6)
        prev = sse
        C_new = oracle.kmeans_update(X, a, C)
        for l in range(7):
            rows = a == l
            if rows.any():
                mean = X[rows].astype(np.float64).mean(axis=0)
                assert np.allclose(C_new[l], mean, rtol=1e-6, atol=1e-6)
            else:
                assert np.array_equal(C_new[l], C[l])
        C = C_new


def test_assignment_is_a_closest_centroid():
    X, _ = _mix(200, 4, 5)
    C = oracle.kmeans_init(X, 9)
    a = oracle.kmeans_assign(X, C)
    D = np.stack([oracle.sq_dists(C, x) for x in X])
    assert np.all(D[np.arange(len(X)), a] <= D.min(axis=1))


@pytest.mark.parametrize("seed", range(4))
def test_every_cluster_or_one_cluster_is_the_exact_knn(seed):
    X, Y = _mix(400, 5, seed)
    C, a = oracle.ivf_train(X, 6, 2)
    C1, a1 = oracle.ivf_train(X, 1, 1)
    for y in Y:
        for k in (1, 7, 40):
            exact = oracle.knn(X, y, k)
            assert np.array_equal(oracle.ivf_knn(X, y, C, a, 6, k), exact)
            assert np.array_equal(oracle.ivf_knn(X, y, C1, a1, 1, k), exact)


def _exact(x, y):
    return sum((Fraction(float(p)) - Fraction(float(q))) ** 2 for p, q in zip(x, y))


def _probe_by_hand(C, y, n_probe, sizes, k):
    order = sorted(range(len(C)), key=lambda l: (_exact(C[l], y), l))
    cap = min(len(C), max(2 * n_probe, n_probe + 64), 496)
    p = n_probe
    while p < cap and sum(sizes[l] for l in order[:p]) < k:
        p += 1
    if sum(sizes[l] for l in order[:p]) < k:
        return None
    return order[:p]


@pytest.mark.parametrize("seed", range(6))
def test_brute_force_on_tiny_inputs(seed):
    rng = np.random.default_rng(100 + seed)
    X = rng.integers(-3, 4, size=(14, 2)).astype(np.float32)   # many exact ties
    C = rng.integers(-3, 4, size=(4, 2)).astype(np.float32)
    a = np.asarray([min(range(4), key=lambda l: (_exact(C[l], x), l)) for x in X])
    assert np.array_equal(a, oracle.kmeans_assign(X, C))
    sizes = np.bincount(a, minlength=4)
    for y in rng.integers(-3, 4, size=(5, 2)).astype(np.float32):
        want_order = sorted(range(4), key=lambda l: (_exact(C[l], y), l))
        assert oracle.cluster_order(C, y).tolist() == want_order
        for n_probe, k in itertools.product((1, 2, 3), (1, 3, 9)):
            probes = _probe_by_hand(C, y, n_probe, sizes, k)
            rows = list(range(14)) if probes is None else [i for i in range(14) if a[i] in probes]
            want = sorted(sorted(rows, key=lambda i: (_exact(X[i], y), i))[:k])
            got = oracle.ivf_knn(X, y, C, a, n_probe, k)
            assert got.tolist() == want


def test_cluster_order_is_the_exact_order():
    rng = np.random.default_rng(7)
    C = rng.normal(size=(40, 5)).astype(np.float32)
    C[7] = C[3]                       # an exact tie: the lower id first
    C[9] = np.nextafter(C[2], np.float32(np.inf))   # a near tie
    for y in rng.normal(size=(6, 5)).astype(np.float32):
        want = sorted(range(40), key=lambda l: (_exact(C[l], y), l))
        assert oracle.cluster_order(C, y).tolist() == want


def test_extension_to_further_clusters_and_the_fallback():
    X = np.array([[0], [1], [2], [50], [51], [52], [53]], dtype=np.float32)
    C = np.array([[1], [52]], dtype=np.float32)
    a = oracle.kmeans_assign(X, C)
    sizes = np.bincount(a, minlength=2)
    y = np.array([0.4], dtype=np.float32)
    # cluster 0 holds 3 rows: k = 3 stays inside it, k = 4 also inspects cluster 1
    assert oracle.ivf_probe(C, y, 1, sizes, 3).tolist() == [0]
    assert oracle.ivf_probe(C, y, 1, sizes, 4).tolist() == [0, 1]
    assert oracle.ivf_knn(X, y, C, a, 1, 3).tolist() == [0, 1, 2]
    assert oracle.ivf_knn(X, y, C, a, 1, 4).tolist() == [0, 1, 2, 3]
    # 70 single-row clusters: at most min(70, max(2, 1 + 64)) = 65 are inspected
    X = np.arange(70, dtype=np.float32).reshape(-1, 1)
    C, a = X.copy(), np.arange(70)
    sizes = np.ones(70, dtype=np.int64)
    y = np.array([0.0], dtype=np.float32)
    assert oracle.ivf_probe(C, y, 1, sizes, 65).tolist() == list(range(65))
    assert oracle.ivf_probe(C, y, 1, sizes, 66).size == 0          # exact fallback
    assert oracle.ivf_knn(X, y, C, a, 1, 66).tolist() == list(range(66))


def test_estimate_with_every_cluster_equals_deann_and_recall():
    X, Y = _mix(500, 4, 9)
    C, a = oracle.ivf_train(X, 5, 2)
    for j, y in enumerate(Y):
        e1, nn1, s1 = oracle.deann_estimate_ivf(X, y, 2.0, GAUSSIAN, C, a, 5, 20, 50, 3, j)
        e2, nn2, s2 = oracle.deann_estimate(X, y, 2.0, GAUSSIAN, 20, 50, 3, j)
        assert e1 == e2 and np.array_equal(nn1, nn2) and np.array_equal(s1, s2)
        assert oracle.recall(nn2, nn1) == 1.0
        part = oracle.ivf_knn(X, y, C, a, 1, 20)
        r = oracle.recall(nn2, part)
        assert 0.0 <= r <= 1.0 and r == len(set(nn2) & set(part)) / 20
    assert oracle.recall(np.array([1, 2]), np.array([3, 4])) == 0.0
