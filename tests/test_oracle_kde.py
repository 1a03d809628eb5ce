"""Pins for the oracle's distances, kernels and exact KDE (Eq. (1)-(2)).

Each check compares against something the oracle does not compute itself:
hand-worked values, the power-law construction of Lemma 4, limits, exact
rational arithmetic and the GEMM identity of App. F.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import GAUSSIAN, EXPONENTIAL


def test_single_point_worked_values():
    # x = (3, 4), y = 0: ||x - y|| = 5.  With h = 5 the Gaussian kernel is
    # exp(-25/50) = e^{-1/2} and the exponential kernel exp(-5/5) = e^{-1}.
    X = np.array([[3.0, 4.0]], dtype=np.float32)
    y = np.zeros((1, 2), dtype=np.float32)
    assert oracle.kde_exact(X, y, 5.0, GAUSSIAN)[0] == pytest.approx(0.6065306597126334, rel=1e-15)
    assert oracle.kde_exact(X, y, 5.0, EXPONENTIAL)[0] == pytest.approx(0.36787944117144233, rel=1e-15)
    # two points, one at the query: (1 + e^{-1/2}) / 2
    X2 = np.array([[0.0, 0.0], [3.0, 4.0]], dtype=np.float32)
    assert oracle.kde_exact(X2, y, 5.0, GAUSSIAN)[0] == pytest.approx(0.8032653298563167, rel=1e-15)


@pytest.mark.parametrize("kernel", [GAUSSIAN, EXPONENTIAL])
def test_range_and_limits(kernel):
    rng = np.random.default_rng(0)
    X = rng.normal(size=(300, 5)).astype(np.float32)
    Y = rng.normal(size=(20, 5)).astype(np.float32)
    v = oracle.kde_exact(X, Y, 0.7, kernel)
    assert np.all(v >= 0.0) and np.all(v <= 1.0)
    # h -> infinity: every term tends to 1
    assert np.allclose(oracle.kde_exact(X, Y, 1e9, kernel), 1.0, rtol=1e-9)
    # h -> 0: only coincident points survive; a query equal to row 7 gives 1/n
    Yc = X[7:8].copy()
    assert oracle.kde_exact(X, Yc, 1e-6, kernel)[0] == pytest.approx(1.0 / 300, rel=1e-12)
    # non-decreasing in h (radially decreasing kernel)
    hs = [0.1, 0.3, 1.0, 3.0]
    vals = [oracle.kde_exact(X, Y[:3], h, kernel) for h in hs]
    for a, b in zip(vals, vals[1:]):
        assert np.all(b >= a)


def _lemma4_points(n, d, alpha, beta):
    """Points x'_i with ||x'_i - y||^2 = alpha ((i+1)/n)^beta, y = 0 (Lemma 4).

    Each point lies on a random direction; coordinates are float64 so the
    squared norms hold to FP64 rounding.
    """
    rng = np.random.default_rng(3)
    dirs = rng.normal(size=(n, d))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    r = np.sqrt(alpha * ((np.arange(n) + 1) / n) ** beta)
    perm = rng.permutation(n)            # stored in random order
    X = np.empty((n, d))
    X[perm] = dirs * r[:, None]
    return X, perm


def test_lemma4_power_law_construction():
    # With h^2 = (alpha/2) n^-beta each kernel value is exp(-(i+1)^beta), so
    # the KDE is (1/n) sum_i exp(-(i+1)^beta) (proof of Lemma 4).
    n, d, alpha, beta = 2000, 6, 3.0, 0.5
    X, _ = _lemma4_points(n, d, alpha, beta)
    h = math.sqrt(alpha / 2.0 * n ** -beta)
    want = sum(math.exp(-((i + 1) ** beta)) for i in range(n)) / n
    got = oracle.kde_exact(X, np.zeros((1, d)), h, GAUSSIAN)[0]
    assert got == pytest.approx(want, rel=1e-12)
    # Reading of part (b): at h^2 = (alpha/2) n^-beta / ln(1/tau) the nearest
    # point contributes exactly tau, and the KDE is at most tau.
    tau = 0.05
    h_b = math.sqrt(alpha / 2.0 * n ** -beta / math.log(1 / tau))
    d2 = oracle.sq_dists(X, np.zeros(d))
    k0 = oracle.kernel_values(np.array([d2.min()]), h_b, GAUSSIAN)[0]
    assert k0 == pytest.approx(tau, rel=1e-12)
    assert oracle.kde_exact(X, np.zeros((1, d)), h_b, GAUSSIAN)[0] <= tau


def test_gemm_identity_matches_direct_distances():
    # App. F: ||x - y||^2 = ||x||^2 + ||y||^2 - 2 <x, y>
    rng = np.random.default_rng(1)
    X = rng.normal(size=(500, 9)).astype(np.float32)
    y = rng.normal(size=9).astype(np.float32)
    X64, y64 = X.astype(np.float64), y.astype(np.float64)
    gemm = (X64 ** 2).sum(1) + (y64 ** 2).sum() - 2.0 * (X64 @ y64)
    direct = oracle.sq_dists(X, y)
    scale = (X64 ** 2).sum(1) + (y64 ** 2).sum()
    assert np.all(np.abs(gemm - direct) <= 64 * 2.0 ** -52 * scale)


@pytest.mark.parametrize("kernel", [GAUSSIAN, EXPONENTIAL])
def test_exact_rational_brute_force(kernel):
    rng = np.random.default_rng(2)
    X = rng.normal(size=(40, 3)).astype(np.float32)
    Y = rng.normal(size=(5, 3)).astype(np.float32)
    h = 0.8
    got = oracle.kde_exact(X, Y, h, kernel)
    for j in range(Y.shape[0]):
        terms = []
        for i in range(X.shape[0]):
            d2 = sum((Fraction(float(a)) - Fraction(float(b))) ** 2 for a, b in zip(X[i], Y[j]))
            r2 = float(d2)   # correctly rounded exact squared distance
            if kernel == GAUSSIAN:
                terms.append(math.exp(-r2 / (2 * h * h)))
            else:
                terms.append(math.exp(-math.sqrt(r2) / h))
        assert got[j] == pytest.approx(math.fsum(terms) / X.shape[0], rel=1e-14)
