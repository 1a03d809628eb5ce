"""Pins of the permuted random sampling oracle (App. G, Algorithm 2): the keyed
permutation is a bijection with the stated inverse, the per-query block holds
m distinct rows outside the neighbour set, consecutive running indices
partition the permuted order, m = n - k reduces DEANN to the exact KDE, and the
estimate is unbiased with the variance of sampling without replacement."""
import math

import numpy as np
import pytest

import oracle
from oracle import GAUSSIAN, EXPONENTIAL


def _data(n, d=3, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, d)).astype(np.float32)
    Y = rng.normal(size=(8, d)).astype(np.float32)
    return X, Y


@pytest.mark.parametrize("b", [2, 4, 6])
def test_feistel_is_a_bijection_with_its_inverse(b):
    for seed in (0, 1, 12345):
        img = [oracle.feistel(x, b, seed) for x in range(1 << b)]
        assert sorted(img) == list(range(1 << b))
        assert all(oracle.feistel(img[x], b, seed, inverse=True) == x for x in range(1 << b))


@pytest.mark.parametrize("n", [1, 2, 3, 5, 17, 64, 100, 257])
def test_permutation_of_n_with_inverse(n):
    for seed in (0, 7):
        p = [oracle.permutation(n, seed, x) for x in range(n)]
        assert sorted(p) == list(range(n))
        assert all(oracle.permutation_inverse(n, seed, p[x]) == x for x in range(n))


def test_permutation_image_uniform_over_seeds():
    # pi(0) over many keys: chi-square against the uniform law on [n]
    n, S = 7, 3500
    counts = np.bincount([oracle.permutation(n, s, 0) for s in range(S)], minlength=n)
    chi2 = ((counts - S / n) ** 2 / (S / n)).sum()
    assert chi2 < 22.46   # 99.9% quantile, 6 degrees of freedom


def test_block_excludes_neighbours_and_has_distinct_rows():
    n, seed = 60, 3
    nn = np.array([2, 9, 10, 33, 59])
    for start in (0, 17, 59):
        for m in (1, 20, n - len(nn)):
            s = oracle.permuted_sample_indices(n, nn, m, seed, start)
            assert len(s) == m and len(set(s.tolist())) == m
            assert not np.isin(s, nn).any()
            assert s.min() >= 0 and s.max() < n
    full = oracle.permuted_sample_indices(n, nn, n - len(nn), seed, 11)
    assert sorted(full.tolist()) == sorted(set(range(n)) - set(nn.tolist()))
    with pytest.raises(ValueError):
        oracle.permuted_sample_indices(n, nn, n - len(nn) + 1, seed, 0)


def test_running_index_partitions_the_permuted_order():
    # without neighbours, queries with running indices 0, m, 2m, ... read
    # consecutive blocks of the permuted order: together every row once
    n, m, seed = 48, 8, 9
    empty = np.empty(0, dtype=np.int64)
    rows = np.concatenate([oracle.permuted_sample_indices(n, empty, m, seed, i * m)
                           for i in range(n // m)])
    assert sorted(rows.tolist()) == list(range(n))
    assert rows.tolist() == [oracle.permutation(n, seed, x) for x in range(n)]


@pytest.mark.parametrize("kernel", [GAUSSIAN, EXPONENTIAL])
def test_sampling_all_of_x2_is_exact(kernel):
    X, Y = _data(90)
    for j, k in ((0, 0), (1, 5), (2, 30)):
        mu = oracle.kde_exact(X, Y[j][None], 0.8, kernel)[0]
        est, nn, s = oracle.deann_estimate_permuted(X, Y[j], 0.8, kernel, k, 90 - k, seed=2,
                                                    start=13 * j)
        assert est == pytest.approx(mu, rel=1e-12, abs=0)


def test_unbiased_with_variance_of_sampling_without_replacement():
    X, Y = _data(120)
    y, h, k, m = Y[4], 0.9, 6, 10
    mu = oracle.kde_exact(X, y[None], h, GAUSSIAN)[0]
    nn = oracle.knn(X, y, k)
    rest = np.setdiff1d(np.arange(120), nn)
    Kr = oracle.kernel_values(oracle.sq_dists(X[rest], y), h, GAUSSIAN)
    N = 120 - k
    var = ((N / 120) ** 2) * Kr.var() / m * (N - m) / (N - 1)
    S = 3000
    ests = np.array([oracle.deann_estimate_permuted(X, y, h, GAUSSIAN, k, m, seed=s, start=s % 120,
                                                    nn=nn)[0] for s in range(S)])
    assert abs(ests.mean() - mu) < 4.5 * math.sqrt(var / S)
    assert 0.85 * var < ests.var(ddof=1) < 1.15 * var
