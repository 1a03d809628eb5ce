"""Pins for the oracle's exact k-NN, Philox4x64-10 and the X2 sampler."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle


def _brute_knn(X, y, k):
    keys = []
    for i in range(X.shape[0]):
        d2 = sum((Fraction(float(a)) - Fraction(float(b))) ** 2 for a, b in zip(X[i], y))
        keys.append((d2, i))
    keys.sort()
    return sorted(i for _, i in keys[:k])


@pytest.mark.parametrize("seed", range(4))
def test_knn_matches_exact_rational_brute_force(seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(60, 4)).astype(np.float32)
    y = rng.normal(size=4).astype(np.float32)
    for k in (0, 1, 7, 30, 59, 60):
        assert oracle.knn(X, y, k).tolist() == _brute_knn(X, y, k)


def test_knn_exact_ties_break_to_lower_index():
    # Integer lattice points: many exactly equal distances.
    rng = np.random.default_rng(5)
    X = rng.integers(-2, 3, size=(80, 3)).astype(np.float32)
    y = np.zeros(3, dtype=np.float32)
    for k in (1, 5, 13, 40):
        assert oracle.knn(X, y, k).tolist() == _brute_knn(X, y, k)


def test_knn_resolves_ties_fp64_cannot_see():
    # ||x_a||^2 = 1 + 2^-60 rounds to 1.0 in FP64, exactly the distance of
    # x_b = (0, 1).  Exact arithmetic puts x_b first although x_a has the
    # lower index.
    X = np.array([[2.0 ** -30, 1.0], [0.0, 1.0], [0.0, 3.0]], dtype=np.float32)
    y = np.zeros(2, dtype=np.float32)
    assert oracle.sq_dists(X, y)[0] == oracle.sq_dists(X, y)[1]
    assert oracle.knn(X, y, 1).tolist() == [1]
    assert oracle.knn(X, y, 2).tolist() == [0, 1]


def test_philox_known_answer(golden_dir):
    with open(os.path.join(golden_dir, "philox4x64_10_kat.json")) as f:
        kat = json.load(f)
    for v in kat["vectors"]:
        key = tuple(int(s, 16) for s in v["key"])
        ctr = tuple(int(s, 16) for s in v["counter"])
        assert oracle.philox4x64_10(key, ctr) == [int(s, 16) for s in v["out"]]


def test_philox_matches_numpy_bit_generator():
    # numpy's Philox (an independent Philox4x64-10) advances its counter
    # before producing a block, so counter c here is numpy's c - 1.
    rng = np.random.default_rng(11)
    for _ in range(25):
        key = [int(x) for x in rng.integers(0, 2 ** 63, size=2)]
        ctr = [int(x) for x in rng.integers(1, 2 ** 63, size=4)]
        g = np.random.Philox(key=np.array(key, dtype=np.uint64),
                             counter=np.array([ctr[0] - 1] + ctr[1:], dtype=np.uint64))
        assert oracle.philox4x64_10(tuple(key), tuple(ctr)) == [int(v) for v in g.random_raw(4)]


def test_rank_to_index_enumerates_complement():
    rng = np.random.default_rng(4)
    for n in (1, 2, 5, 17, 40):
        for k in range(0, n + 1, max(1, n // 5)):
            nn = np.sort(rng.choice(n, size=k, replace=False))
            comp = [i for i in range(n) if i not in set(nn.tolist())]
            assert [oracle.rank_to_index(nn, r) for r in range(n - k)] == comp


def test_sampler_draws_uniform_over_complement():
    n, k, m = 50, 12, 20000
    rng = np.random.default_rng(9)
    nn = np.sort(rng.choice(n, size=k, replace=False))
    s = oracle.sample_indices(n, nn, m, seed=3, stream=0)
    assert s.min() >= 0 and s.max() < n
    assert not np.isin(s, nn).any()
    counts = np.bincount(s, minlength=n)[np.setdiff1d(np.arange(n), nn)]
    expect = m / (n - k)
    chi2 = float(((counts - expect) ** 2 / expect).sum())
    # 37 degrees of freedom: the 0.999 quantile is about 69.3
    assert chi2 < 69.3


def test_sampler_counter_layout():
    # draw j of stream s with word2 w is word j%4 of block (j//4, s, w, 0)
    n, nn = 1000, np.array([3, 10, 500])
    s = oracle.sample_indices(n, nn, 9, seed=77, stream=5, word2=2)
    blk = oracle.philox4x64_10((77, 0), (2, 5, 2, 0))
    r = (blk[0] * (n - 3)) >> 64
    assert s[8] == oracle.rank_to_index(nn, r)
    # empty complement: no draws possible
    assert (oracle.sample_indices(4, np.arange(4), 3, 0, 0) == -1).all()
