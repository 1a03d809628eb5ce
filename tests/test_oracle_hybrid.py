"""Pins for the oracle's near/far split of the exact KDE (the split of
Algorithm 1 with the far part summed over all of X2 instead of sampled)."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import GAUSSIAN, EXPONENTIAL


def _data(n=60, d=3, seed=3):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, d)).astype(np.float32)
    Y = rng.normal(size=(4, d)).astype(np.float32)
    return X, Y


def _values_by_hand(X, y, h, kernel):
    """Kernel values with the distance summed as an exact rational per row."""
    out = []
    for row in X:
        d2 = float(sum((Fraction(float(a)) - Fraction(float(b))) ** 2 for a, b in zip(row, y)))
        out.append(math.exp(-d2 / (2 * h * h)) if kernel == GAUSSIAN else math.exp(-math.sqrt(d2) / h))
    return np.array(out)


@pytest.mark.parametrize("kernel", [GAUSSIAN, EXPONENTIAL])
@pytest.mark.parametrize("k", [1, 7, 30])
def test_near_is_the_k_largest_values(kernel, k):
    # the kernels decrease with the distance, so the k nearest rows carry the
    # k largest kernel values: a sort of the values, no k-NN involved
    X, Y = _data()
    n = X.shape[0]
    for y in Y:
        v = _values_by_hand(X, y, 0.8, kernel)
        nn, near, far = oracle.kde_near_far(X, y, 0.8, kernel, k)
        assert len(nn) == k and len(set(nn.tolist())) == k
        assert near * n == pytest.approx(math.fsum(np.sort(v)[::-1][:k]), rel=1e-13)
        assert (near + far) * n == pytest.approx(math.fsum(v), rel=1e-13)
        inside = np.zeros(n, bool)
        inside[nn] = True
        assert v[~inside].max() <= v[inside].min() * (1 + 1e-12)


@pytest.mark.parametrize("kernel", [GAUSSIAN, EXPONENTIAL])
def test_all_far_and_all_near(kernel):
    X, Y = _data()
    n = X.shape[0]
    for y in Y[:2]:
        exact = math.fsum(_values_by_hand(X, y, 1.3, kernel)) / n
        nn0, near0, far0 = oracle.kde_near_far(X, y, 1.3, kernel, 0)
        assert len(nn0) == 0 and near0 == 0.0 and far0 == pytest.approx(exact, rel=1e-13)
        nnn, nearn, farn = oracle.kde_near_far(X, y, 1.3, kernel, n)
        assert np.array_equal(nnn, np.arange(n)) and farn == 0.0
        assert nearn == pytest.approx(exact, rel=1e-13)


def test_given_rows_split_the_sum():
    X, Y = _data()
    n = X.shape[0]
    rng = np.random.default_rng(1)
    rows = rng.choice(n, size=11, replace=False)
    v = _values_by_hand(X, Y[0], 0.7, GAUSSIAN)
    nn, near, far = oracle.kde_near_far(X, Y[0], 0.7, GAUSSIAN, 11, nn=rows)
    assert np.array_equal(nn, np.sort(rows))
    assert near * n == pytest.approx(math.fsum(v[rows]), rel=1e-13)
    assert far * n == pytest.approx(math.fsum(np.delete(v, rows)), rel=1e-13)
