"""Pins for the oracle's DEANN estimate (Algorithm 1), gradients, mean shift
and bandwidth bisection."""
import math

import numpy as np
import pytest

import oracle
from oracle import GAUSSIAN, EXPONENTIAL


def _data(n=400, d=5, seed=0):
    rng = np.random.default_rng(seed)
    centers = rng.uniform(-3, 3, size=(4, d))
    X = (centers[rng.integers(0, 4, n)] + rng.normal(size=(n, d))).astype(np.float32)
    Y = (centers[rng.integers(0, 4, 6)] + rng.normal(size=(6, d))).astype(np.float32)
    return X, Y


@pytest.mark.parametrize("kernel", [GAUSSIAN, EXPONENTIAL])
def test_k_equals_n_is_exact(kernel):
    X, Y = _data()
    est, nn, s = oracle.deann_estimate(X, Y[0], 0.9, kernel, k=X.shape[0], m=50, seed=1, stream=0)
    assert est == pytest.approx(oracle.kde_exact(X, Y[:1], 0.9, kernel)[0], rel=1e-14)
    assert (s == -1).all()


def test_m_zero_keeps_only_neighbours():
    X, Y = _data()
    est, nn, _ = oracle.deann_estimate(X, Y[1], 0.9, GAUSSIAN, k=10, m=0, seed=1, stream=0)
    d2 = oracle.sq_dists(X, Y[1])
    assert est == pytest.approx(np.sort(np.exp(-d2 / (2 * 0.81)))[::-1][:10].sum() / X.shape[0],
                                rel=1e-12)


@pytest.mark.parametrize("kernel", [GAUSSIAN, EXPONENTIAL])
def test_unbiased_over_seeds_with_variance_formula(kernel):
    # Lemma 1 / Corollary 1: unbiased for any partition; with draws made with
    # repetition Var = ((n-k)/n)^2 sigma^2_{X2} / m.
    X, Y = _data(n=200)
    y, h, k, m = Y[2], 0.9, 8, 4
    mu = oracle.kde_exact(X, y[None], h, kernel)[0]
    nn = oracle.knn(X, y, k)
    rest = np.setdiff1d(np.arange(200), nn)
    Kr = oracle.kernel_values(oracle.sq_dists(X[rest], y), h, kernel)
    var = ((200 - k) / 200) ** 2 * Kr.var() / m
    S = 3000
    ests = np.array([oracle.deann_estimate(X, y, h, kernel, k, m, seed=s, stream=0, nn=nn)[0]
                     for s in range(S)])
    assert abs(ests.mean() - mu) < 4.5 * math.sqrt(var / S)
    # sample variance of S draws: within a wide chi-square band
    assert 0.85 * var < ests.var(ddof=1) < 1.15 * var


def test_unbiased_with_a_bad_neighbour_set():
    # Any X1 gives an unbiased estimate (the estimate does not need good neighbours).
    X, Y = _data(n=150)
    y, h, m = Y[3], 0.7, 6
    bad = np.arange(0, 150, 15)          # arbitrary rows, not the nearest ones
    mu = oracle.kde_exact(X, y[None], h, GAUSSIAN)[0]
    rest = np.setdiff1d(np.arange(150), bad)
    Kr = oracle.kernel_values(oracle.sq_dists(X[rest], y), h, GAUSSIAN)
    var = ((150 - 10) / 150) ** 2 * Kr.var() / m
    S = 3000
    ests = [oracle.deann_estimate(X, y, h, GAUSSIAN, 10, m, seed=s, stream=4, nn=bad)[0]
            for s in range(S)]
    assert abs(np.mean(ests) - mu) < 4.5 * math.sqrt(var / S)


def test_bernoulli_worst_case_input():
    # App. D: a tau-fraction of X sits at the query, the rest so far away that
    # the kernel underflows to exactly 0.  KDE = tau; with k >= tau n the
    # estimate is exact for every seed.
    n, tau = 400, 0.05
    X = np.zeros((n, 3), dtype=np.float32)
    X[int(tau * n):] = 1e4
    y = np.zeros(3, dtype=np.float32)
    h = 1.0
    assert oracle.kde_exact(X, y[None], h, GAUSSIAN)[0] == tau
    for s in range(5):
        est, _, _ = oracle.deann_estimate(X, y, h, GAUSSIAN, k=int(tau * n), m=30, seed=s, stream=0)
        assert est == tau
    # plain random sampling (k = 0): estimate = (#draws at y)/m, a binomial proportion
    est, _, draws = oracle.deann_estimate(X, y, h, GAUSSIAN, k=0, m=100, seed=2, stream=0)
    assert est == pytest.approx(np.sum(draws < tau * n) / 100, rel=1e-15)


@pytest.mark.parametrize("kernel", [GAUSSIAN, EXPONENTIAL])
def test_gradients_match_central_differences(kernel):
    X, Y = _data(n=120, d=4)
    y = Y[0].astype(np.float64)
    h = 1.1
    mu, gy, gh = oracle.kde_grad(X, y, h, kernel)
    eps = 1e-3 * h
    for t in range(4):
        e = np.zeros(4)
        e[t] = eps
        fd = (oracle.kde_grad(X, y + e, h, kernel)[0] - oracle.kde_grad(X, y - e, h, kernel)[0]) / (2 * eps)
        assert gy[t] == pytest.approx(fd, rel=2e-5, abs=1e-12)
    fdh = (oracle.kde_grad(X, y, h + eps, kernel)[0] - oracle.kde_grad(X, y, h - eps, kernel)[0]) / (2 * eps)
    assert gh == pytest.approx(fdh, rel=2e-5)
    # DEANN with frozen sets
    nn = oracle.knn(X, y.astype(np.float32), 9)
    s = oracle.sample_indices(120, nn, 17, seed=4, stream=1)
    est, dgy, dgh = oracle.deann_grad(X, y, h, kernel, nn, s, 17)

    def f(yy, hh):
        return oracle.deann_grad(X, yy, hh, kernel, nn, s, 17)[0]
    for t in range(4):
        e = np.zeros(4)
        e[t] = eps
        assert dgy[t] == pytest.approx((f(y + e, h) - f(y - e, h)) / (2 * eps), rel=2e-5, abs=1e-12)
    assert dgh == pytest.approx((f(y, h + eps) - f(y, h - eps)) / (2 * eps), rel=2e-5)
    assert est == pytest.approx(
        oracle.deann_estimate(X, y.astype(np.float32), h, kernel, 9, 17, 4, 1, nn=nn)[0], rel=1e-12)


def test_single_point_gradient_closed_form():
    # n = 1, Gaussian: d/dy exp(-||x-y||^2/2h^2) = K (x - y)/h^2; exponential at r = 0 is 0.
    X = np.array([[1.0, 2.0]], dtype=np.float32)
    y = np.array([0.0, 0.0])
    _, gy, gh = oracle.kde_grad(X, y, 2.0, GAUSSIAN)
    K = math.exp(-5.0 / 8.0)
    assert gy == pytest.approx([K * 1 / 4, K * 2 / 4], rel=1e-14)
    assert gh == pytest.approx(K * 5 / 8, rel=1e-14)
    _, gy0, _ = oracle.kde_grad(X, np.array([1.0, 2.0]), 2.0, EXPONENTIAL)
    assert np.all(gy0 == 0.0)


def test_mean_shift_pins():
    X = np.array([[1.5, -2.0, 0.25]], dtype=np.float32)
    y = np.array([4.0, 4.0, 4.0], dtype=np.float32)
    assert np.allclose(oracle.mean_shift_exact(X, y, 1.0, 1), X[0].astype(np.float64), rtol=0, atol=0)
    Xd, Yd = _data(n=300, d=3, seed=8)
    h = 0.8
    yy = Yd[0]
    prev = oracle.kde_exact(Xd, yy[None], h, GAUSSIAN)[0]
    for _ in range(6):
        yy = oracle.mean_shift_exact(Xd, yy, h, 1).astype(np.float32)
        cur = oracle.kde_exact(Xd, yy[None], h, GAUSSIAN)[0]
        assert cur >= prev * (1 - 1e-6)
        prev = cur
    # DEANN weights with k = n reduce to the exact step
    a = oracle.mean_shift_deann(Xd, Yd[1], h, k=300, m=5, seed=0, stream=0, steps=2)
    b = oracle.mean_shift_exact(Xd, Yd[1], h, 2)
    assert np.allclose(a, b, rtol=1e-6, atol=1e-6)


def test_mean_shift_deann_sampled_step_pins():
    # k < n: a DEANN mean-shift step is y + h^2 grad(est) / est with the
    # estimate and gradient of the same neighbour set and draws (Gaussian:
    # grad = (1/n) sum W (x - y) / h^2 with W = K times the Algorithm 1
    # weight), and step t draws with counter word 2 = t.
    Xd, Yd = _data(n=300, d=3, seed=8)
    n, h, k, m, seed, stream = 300, 0.8, 20, 40, 3, 2
    y0 = Yd[2]
    got = oracle.mean_shift_deann(Xd, y0, h, k, m, seed, stream, steps=2)

    def step(y, t):
        y32 = np.asarray(y, dtype=np.float32)
        nn = oracle.knn(Xd, y32, k)
        s = oracle.sample_indices(n, nn, m, seed, stream, word2=t)
        est, gy, _ = oracle.deann_grad(Xd, y32.astype(np.float64), h, GAUSSIAN, nn, s, m)
        return (y32.astype(np.float64) + h * h * gy / est).astype(np.float32), nn, s

    y1, nn0, s0 = step(y0, 0)
    y2, _, s1 = step(y1, 1)
    assert np.allclose(got, y2.astype(np.float64), rtol=0, atol=1e-6)
    assert not np.array_equal(s0, s1)            # the two steps draw different rows
    # the pin tells the sample weight apart: with weight 1 instead of (n-k)/m
    # (or with step 1 drawing word 2 = 0) the end point moves far beyond atol
    y1w = y1.astype(np.float64)
    rows = np.concatenate([nn0, s0])
    wts = np.concatenate([np.ones(k), np.ones(m)])
    R = Xd[rows].astype(np.float64)
    y0d = np.asarray(y0, dtype=np.float32).astype(np.float64)
    K = np.exp(-((R - y0d) ** 2).sum(1) / (2 * h * h)) * wts
    y1_wrong = (K[:, None] * R).sum(0) / K.sum()
    assert np.abs(y1_wrong - y1w).max() > 1e-3
    y2_same_draws = step(y1, 0)[0]
    assert np.abs(y2_same_draws.astype(np.float64) - y2.astype(np.float64)).max() > 1e-4


def test_bisect_bandwidth_hits_target():
    X, Y = _data(n=500, d=6)
    D2 = oracle.pairwise_sq_dists(X, Y)
    for target in (1e-2, 1e-3):
        h = oracle.bisect_h(D2, target, GAUSSIAN)
        got = oracle.kde_exact(X, Y, h, GAUSSIAN).mean()
        assert abs(got - target) <= 0.01 * target
