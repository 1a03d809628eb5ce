"""Plain FP64 CPU oracle for DEANN's query path.

TEST INFRASTRUCTURE ONLY.  This module is the slow, obviously correct
definition that the HIP path is checked against.  Only the test suite, the
smoke check and the benchmark's CPU-baseline leg may import it; the product
path never does, and it shares no code with the HIP library (the two meet only
in the seeded inputs of the ``synth`` package).

Everything is float64 NumPy with element-wise operations only (no BLAS GEMM),
single-threaded.  Inputs are the float32 bytes the GPU receives, upcast
exactly to float64.

Paper: Karppa, Aumueller, Pagh, "DEANN: Speeding up Kernel-Density Estimation
using Approximate Nearest Neighbor Search" (arXiv 2107.02736).

Parity status of each function (what pins it in tests/test_oracle_*.py):
  sq_dists, kernel_values, kde_exact  pinned: n=1 closed form, power-law
      construction of Lemma 4 (exact values), h -> inf limit, KDE in [0,1],
      exact rational brute force on tiny inputs, GEMM identity of App. F.
  knn        pinned: exact rational brute force (fractions) incl. exact ties.
  philox4x64_10  pinned: numpy's independent Philox4x64-10 and the SC'11 zero
      known-answer vector.
  sample_indices pinned: exhaustive rank->index enumeration on tiny n,
      chi-square uniformity over X minus NN, no draw inside NN.
  deann_estimate pinned: k=n gives kde_exact, unbiasedness over many seeds,
      variance formula of random sampling with repetition, Bernoulli worst
      case of App. D.
  kde_near_far pinned: the near part is the sum of the k largest kernel
      values (a sort of the values, independent of the k-NN), k = 0 and k = n
      give all-far and all-near, near + far equals the exact KDE computed by a
      fresh loop, every far value is at most the k-th nearest value.
  permutation, permutation_inverse pinned: bijection of [n] and mutual
      inverses (exhaustive on small n), uniformity of pi over seeds.
  permuted_sample_indices / deann_estimate_permuted pinned: m distinct rows
      outside NN; consecutive running indices partition the permuted order;
      m = n - k gives exactly X2, so the estimate equals kde_exact;
      unbiasedness over seeds.
  kde_grad / deann_grad pinned: central finite differences, n=1 closed form.
  mean_shift pinned: n=1 lands on the point in one step; density never
      decreases along exact Gaussian mean-shift steps; a DEANN step with
      k < n equals y + h^2 grad/est of deann_grad over the same neighbours and
      draws (counter word 2 = step), and a wrong sample weight or a repeated
      word 2 moves the end point detectably.
  bisect_h   pinned: monotonicity of KDE in h and the target tolerance.
  kmeans_init / kmeans_assign / kmeans_update / ivf_train pinned: Lloyd
      steps computed by hand on one-dimensional data (an empty cluster,
      centroid ties), the update equals the mean of the rows, the k-means
      objective never grows, exact-rational brute force of the assignment.
  cluster_order / ivf_probe / ivf_knn / deann_estimate_ivf pinned: every
      cluster inspected or a single cluster gives the exact k-NN (and then
      DEANN itself), exact-rational brute force on tiny inputs with ties
      (including the extension to further clusters and the cap), the
      extension and the fallback on hand-made clusters, the order against an
      exact-rational sort.
  recall     pinned: identical sets give 1, disjoint sets 0.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

GAUSSIAN = 0
EXPONENTIAL = 1

_ROW_CHUNK = 1 << 15
_U64 = (1 << 64) - 1


# --------------------------------------------------------------------------
# Distances and kernels (Eq. (1), Eq. (2), the exponential kernel of Sec. 1)
# --------------------------------------------------------------------------

def sq_dists(X: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Squared Euclidean distances ||x_i - y||^2 for every row of X, in FP64.

    Direct differences (not the GEMM identity of App. F), row chunks to bound
    memory.
    """
    y64 = np.asarray(y, dtype=np.float64)
    out = np.empty(X.shape[0], dtype=np.float64)
    for r0 in range(0, X.shape[0], _ROW_CHUNK):
        diff = X[r0:r0 + _ROW_CHUNK].astype(np.float64) - y64
        out[r0:r0 + _ROW_CHUNK] = np.einsum("ij,ij->i", diff, diff, optimize=False)
    return out


def kernel_values(d2: np.ndarray, h: float, kernel: int) -> np.ndarray:
    """K_h as a function of the squared distance.

    Gaussian (Eq. (2)): exp(-d^2 / (2 h^2)).  Exponential (Sec. 1):
    exp(-d / h).  Both are unnormalised, so every value lies in [0, 1].
    """
    d2 = np.maximum(np.asarray(d2, dtype=np.float64), 0.0)
    if kernel == GAUSSIAN:
        return np.exp(-d2 / (2.0 * h * h))
    if kernel == EXPONENTIAL:
        return np.exp(-np.sqrt(d2) / h)
    raise ValueError("unknown kernel")


def kde_exact(X: np.ndarray, Y: np.ndarray, h: float, kernel: int) -> np.ndarray:
    """Exact KDE of Eq. (1) for every query row: (1/n) sum_i K_h(x_i, y).

    The sum over i is math.fsum (correctly rounded), so the only rounding left
    is that of each distance and kernel value.
    """
    n = X.shape[0]
    Y = np.atleast_2d(Y)
    out = np.empty(Y.shape[0], dtype=np.float64)
    for j in range(Y.shape[0]):
        out[j] = math.fsum(kernel_values(sq_dists(X, Y[j]), h, kernel)) / n
    return out


# --------------------------------------------------------------------------
# Exact k nearest neighbours (the black-box ANN of Algorithm 1, made exact)
# --------------------------------------------------------------------------

def _exact_sq_dist(x_row: np.ndarray, y: np.ndarray) -> Fraction:
    """||x - y||^2 as an exact rational (every float32 value is dyadic)."""
    s = Fraction(0)
    for a, b in zip(x_row.tolist(), y.tolist()):
        t = Fraction(a) - Fraction(b)
        s += t * t
    return s


def knn(X: np.ndarray, y: np.ndarray, k: int) -> np.ndarray:
    """Indices of the k nearest rows of X to y, sorted ascending by index.

    The order is the lexicographic key (exact real ||x_i - y||^2, i): the
    sequence of points sorted by distance (Sec. 2) with ties broken towards
    the lower index.  Ranking is done in FP64; wherever the FP64 values near
    the k-th place are too close for FP64 rounding to decide, those points
    are compared again with exact rational arithmetic.
    """
    n, d = X.shape
    if k <= 0:
        return np.empty(0, dtype=np.int64)
    if k >= n:
        return np.arange(n, dtype=np.int64)
    d2 = sq_dists(X, y)
    order = np.lexsort((np.arange(n), d2))
    dk = d2[order[k - 1]]
    # Relative error of an FP64 sum of d squared differences (each difference
    # of two float32 values is exact in FP64 within this range of magnitudes).
    rel = 4.0 * (d + 2) * 2.0 ** -53
    lo, hi = dk * (1.0 - rel), dk * (1.0 + rel)
    if dk == 0.0:
        lo, hi = -1.0, 0.0
    sure = d2 < lo
    band = np.nonzero((d2 >= lo) & (d2 <= hi))[0]
    n_sure = int(sure.sum())
    need = k - n_sure
    if need == len(band):
        chosen = band
    else:
        keyed = sorted(band.tolist(), key=lambda i: (_exact_sq_dist(X[i], y), i))
        chosen = np.asarray(keyed[:need], dtype=np.int64)
    res = np.concatenate([np.nonzero(sure)[0], chosen]).astype(np.int64)
    res.sort()
    assert res.size == k
    return res


# --------------------------------------------------------------------------
# Counter-based random numbers: Philox4x64-10 (Salmon, Moraes, Dror, Shaw,
# "Parallel Random Numbers: As Easy as 1, 2, 3", SC'11)
# --------------------------------------------------------------------------

_PHILOX_M0 = 0xD2E7470EE14C6C93
_PHILOX_M1 = 0xCA5A826395121157
_PHILOX_W0 = 0x9E3779B97F4A7C15   # golden ratio
_PHILOX_W1 = 0xBB67AE8584CAA73B   # sqrt(3) - 1


def philox4x64_10(key: tuple[int, int], counter: tuple[int, int, int, int]) -> list[int]:
    """One 4x64-bit Philox block with 10 rounds, in Python integers."""
    k0, k1 = key[0] & _U64, key[1] & _U64
    c0, c1, c2, c3 = (c & _U64 for c in counter)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + _PHILOX_W0) & _U64
            k1 = (k1 + _PHILOX_W1) & _U64
        p0 = _PHILOX_M0 * c0
        p1 = _PHILOX_M1 * c2
        c0, c1, c2, c3 = ((p1 >> 64) ^ c1 ^ k0, p1 & _U64, (p0 >> 64) ^ c3 ^ k1, p0 & _U64)
    return [c0, c1, c2, c3]


def sample_indices(n: int, nn_sorted: np.ndarray, m: int, seed: int, stream: int,
                   word2: int = 0) -> np.ndarray:
    """The m uniform draws, with repetition, from X2 = [n] minus NN (Algorithm 1).

    Draw j uses u = word (j mod 4) of Philox4x64-10 with key (seed, 0) and
    counter (j div 4, stream, word2, 0); the rank r = floor(u (n-k) / 2^64)
    (multiply-shift, no rejection) selects the r-th smallest element of X2.
    With NN sorted e_0 < ... < e_{k-1}, that element is r + #{t : e_t - t <= r}.
    Returns int64 indices in draw order; all -1 when X2 is empty.
    """
    k = len(nn_sorted)
    size2 = n - k
    if m <= 0:
        return np.empty(0, dtype=np.int64)
    if size2 <= 0:
        return np.full(m, -1, dtype=np.int64)
    out = np.empty(m, dtype=np.int64)
    block = None
    for j in range(m):
        if j % 4 == 0:
            block = philox4x64_10((seed, 0), (j // 4, stream, word2, 0))
        u = block[j % 4]
        r = (u * size2) >> 64
        out[j] = rank_to_index(nn_sorted, r)
    return out


def rank_to_index(nn_sorted, r: int) -> int:
    """The r-th smallest (0-based) element of [n] minus the sorted set NN.

    e_t - t counts the elements of X2 below e_t, so e_t lies below the answer
    exactly when e_t - t <= r.
    """
    below = sum(1 for t, e in enumerate(nn_sorted) if int(e) - t <= r)
    return r + below


# --------------------------------------------------------------------------
# DEANN estimate (Algorithm 1) and its extremes
# --------------------------------------------------------------------------

def deann_estimate(X: np.ndarray, y: np.ndarray, h: float, kernel: int, k: int, m: int,
                   seed: int, stream: int, word2: int = 0, nn: np.ndarray | None = None):
    """DEANN for one query.  Returns (estimate, nn_sorted, sample_idx).

    X1 = the k nearest rows (exact k-NN unless ``nn`` is given), X2 = the rest,
    Z1 = sum over X1 of K, S = m draws from X2, Z2 = sum over S of K, and the
    estimate (k/n)(Z1/k) + ((n-k)/n)(Z2/m) written as (Z1 + ((n-k)/m) Z2)/n so
    that k = 0 (plain random sampling) and m = 0 (far points dropped) need no
    special case.  When k = n the estimate is the exact KDE and no draw is made.
    """
    n = X.shape[0]
    if nn is None:
        nn = knn(X, y, k)
    nn = np.sort(np.asarray(nn, dtype=np.int64))
    k = len(nn)
    s_idx = sample_indices(n, nn, m, seed, stream, word2)
    z1 = math.fsum(kernel_values(sq_dists(X[nn], y), h, kernel)) if k else 0.0
    if m > 0 and n - k > 0:
        z2 = math.fsum(kernel_values(sq_dists(X[s_idx], y), h, kernel))
        est = (z1 + (n - k) / m * z2) / n
    else:
        est = z1 / n
    return est, nn, s_idx


def kde_near_far(X: np.ndarray, y: np.ndarray, h: float, kernel: int, k: int,
                 nn: np.ndarray | None = None):
    """Near/far split of the exact KDE of one query: (nn_sorted, near, far).

    The split of Algorithm 1 into X1 = the k nearest rows (exact k-NN unless
    ``nn`` is given) and X2 = the rest, with both parts summed exactly:
    near = Z1 / n over X1, far = (1/n) sum over all of X2 (no sampling), so
    near + far is the exact KDE of Eq. (1) for any X1.  The 16-bit form of
    the library approximates only the far part.
    """
    n = X.shape[0]
    if nn is None:
        nn = knn(X, y, k)
    nn = np.sort(np.asarray(nn, dtype=np.int64))
    kv = kernel_values(sq_dists(X, y), h, kernel)
    inside = np.zeros(n, dtype=bool)
    inside[nn] = True
    return nn, math.fsum(kv[inside]) / n, math.fsum(kv[~inside]) / n


# --------------------------------------------------------------------------
# Permuted random sampling (App. G, Algorithm 2) for DEANN
# --------------------------------------------------------------------------
# The permutation pi of Algorithm 2 is a keyed pseudo-random permutation of
# [n]: a balanced 4-round Feistel network on b-bit words (b even, 2^b >= n)
# whose round function is word 0 of Philox4x64-10 with key (seed, 1) and
# counter (half, round, 0, 0), restricted to [n] by cycle walking (Black and
# Rogaway, CT-RSA 2002).  Query i reads the permuted rows starting at the
# running index l_i = (start + i m) mod n, as Algorithm 2 advances l by m per
# query; the neighbours of the query are skipped, so the sample is m distinct
# rows of X2 (m <= n - k).

PERM_ROUNDS = 4


def perm_bits(n: int) -> int:
    """Smallest even b >= 2 with 2^b >= n."""
    b = max(2, (n - 1).bit_length())
    return b + (b & 1)


def feistel(x: int, b: int, seed: int, inverse: bool = False) -> int:
    """One pass of the balanced Feistel network on [0, 2^b) (or its inverse)."""
    half = b // 2
    mask = (1 << half) - 1
    left, right = x >> half, x & mask
    if not inverse:
        for rnd in range(PERM_ROUNDS):
            f = philox4x64_10((seed, 1), (right, rnd, 0, 0))[0] & mask
            left, right = right, left ^ f
    else:
        for rnd in reversed(range(PERM_ROUNDS)):
            f = philox4x64_10((seed, 1), (left, rnd, 0, 0))[0] & mask
            left, right = right ^ f, left
    return (left << half) | right


def permutation(n: int, seed: int, x: int) -> int:
    """pi(x) for x in [n]: apply the network until the value falls in [n]."""
    b = perm_bits(n)
    y = feistel(x, b, seed)
    while y >= n:
        y = feistel(y, b, seed)
    return y


def permutation_inverse(n: int, seed: int, y: int) -> int:
    """pi^-1(y): the inverse network, walked the same way."""
    b = perm_bits(n)
    x = feistel(y, b, seed, inverse=True)
    while x >= n:
        x = feistel(x, b, seed, inverse=True)
    return x


def permuted_sample_indices(n: int, nn_sorted: np.ndarray, m: int, seed: int,
                            start: int) -> np.ndarray:
    """The m rows at permuted positions start, start + 1, ... (cyclic) that
    are not neighbours, in that order (Algorithm 2 with X1 skipped).

    With the neighbours' positions relative to start sorted, r_0 < ... <
    r_{k-1}, draw j takes relative position j + #{t : r_t - t <= j}, the j-th
    position not held by a neighbour.
    """
    k = len(nn_sorted)
    if m <= 0:
        return np.empty(0, dtype=np.int64)
    if m > n - k:
        raise ValueError("permuted sampling needs m <= n - k")
    rel = sorted((permutation_inverse(n, seed, int(e)) - start) % n for e in nn_sorted)
    out = np.empty(m, dtype=np.int64)
    for j in range(m):
        u = rank_to_index(rel, j)
        out[j] = permutation(n, seed, (start + u) % n)
    return out


def deann_estimate_permuted(X: np.ndarray, y: np.ndarray, h: float, kernel: int, k: int,
                            m: int, seed: int, start: int, nn: np.ndarray | None = None):
    """DEANN with permuted random sampling for one query whose running index is
    ``start``.  Returns (estimate, nn_sorted, sample_idx); the estimate has the
    same form as deann_estimate, (Z1 + ((n-k)/m) Z2) / n."""
    n = X.shape[0]
    if nn is None:
        nn = knn(X, y, k)
    nn = np.sort(np.asarray(nn, dtype=np.int64))
    k = len(nn)
    s_idx = permuted_sample_indices(n, nn, m, seed, start % n)
    z1 = math.fsum(kernel_values(sq_dists(X[nn], y), h, kernel)) if k else 0.0
    if m > 0:
        z2 = math.fsum(kernel_values(sq_dists(X[s_idx], y), h, kernel))
        est = (z1 + (n - k) / m * z2) / n
    else:
        est = z1 / n
    return est, nn, s_idx


# --------------------------------------------------------------------------
# Gradients (derived from Eq. (1)-(2); the paper gives none)
# --------------------------------------------------------------------------

def _kernel_and_grads(Xs: np.ndarray, y: np.ndarray, h: float, kernel: int):
    """K, dK/dy (rows) and dK/dh for the rows Xs against y, all FP64."""
    y64 = np.asarray(y, dtype=np.float64)
    diff = Xs.astype(np.float64) - y64            # x - y
    d2 = np.einsum("ij,ij->i", diff, diff, optimize=False)
    K = kernel_values(d2, h, kernel)
    if kernel == GAUSSIAN:
        w = K / (h * h)                           # dK/dy = K (x - y) / h^2
        dh = K * d2 / h ** 3                      # dK/dh = K d^2 / h^3
    else:
        r = np.sqrt(d2)
        with np.errstate(divide="ignore", invalid="ignore"):
            w = np.where(r > 0.0, K / (h * r), 0.0)   # dK/dy = K (x - y) / (h r), 0 at r = 0
        dh = K * r / (h * h)                      # dK/dh = K r / h^2
    return K, w[:, None] * diff, dh


def kde_grad(X: np.ndarray, y: np.ndarray, h: float, kernel: int):
    """(KDE, dKDE/dy [d], dKDE/dh) of Eq. (1) for one query, summing all n rows."""
    n, d = X.shape
    gy = np.zeros(d, dtype=np.float64)
    val, gh = [], []
    for r0 in range(0, n, _ROW_CHUNK):
        K, gK, dh = _kernel_and_grads(X[r0:r0 + _ROW_CHUNK], y, h, kernel)
        val.append(K)
        gh.append(dh)
        gy += gK.sum(axis=0)
    return (math.fsum(np.concatenate(val)) / n, gy / n, math.fsum(np.concatenate(gh)) / n)


def deann_grad(X: np.ndarray, y: np.ndarray, h: float, kernel: int, nn: np.ndarray,
               s_idx: np.ndarray, m: int):
    """(estimate, d/dy, d/dh) of the DEANN estimate with the index sets held fixed.

    The selected sets are piecewise constant in y and h, so this is the
    derivative almost everywhere: the weights of Algorithm 1 (1 for X1,
    (n-k)/m for each draw) times the kernel derivatives.
    """
    n = X.shape[0]
    nn = np.asarray(nn, dtype=np.int64)
    k = len(nn)
    d = X.shape[1]
    K1, g1, h1 = _kernel_and_grads(X[nn], y, h, kernel) if k else (
        np.zeros(0), np.zeros((0, d)), np.zeros(0))
    est, gy, gh = math.fsum(K1), g1.sum(axis=0), math.fsum(h1)
    if m > 0 and n - k > 0:
        c = (n - k) / m
        K2, g2, h2 = _kernel_and_grads(X[np.asarray(s_idx, dtype=np.int64)], y, h, kernel)
        est += c * math.fsum(K2)
        gy = gy + c * g2.sum(axis=0)
        gh += c * math.fsum(h2)
    return est / n, gy / n, gh / n


# --------------------------------------------------------------------------
# Mean shift (an application of density gradients, Sec. 1) and bandwidth
# selection by bisection (Sec. 5, "Bandwidth selection")
# --------------------------------------------------------------------------

def mean_shift_exact(X: np.ndarray, y: np.ndarray, h: float, steps: int) -> np.ndarray:
    """Gaussian-kernel mean shift: y <- sum_i K_i x_i / sum_i K_i, repeated.

    The point is kept in float32 between steps, as a query array would be.
    """
    y = np.asarray(y, dtype=np.float32).astype(np.float64)
    for _ in range(steps):
        num = np.zeros_like(y)
        den = []
        for r0 in range(0, X.shape[0], _ROW_CHUNK):
            Xs = X[r0:r0 + _ROW_CHUNK].astype(np.float64)
            diff = Xs - y
            K = kernel_values(np.einsum("ij,ij->i", diff, diff, optimize=False), h, GAUSSIAN)
            num += (K[:, None] * Xs).sum(axis=0)
            den.append(K)
        y = (num / math.fsum(np.concatenate(den))).astype(np.float32).astype(np.float64)
    return y


def mean_shift_deann(X: np.ndarray, y: np.ndarray, h: float, k: int, m: int, seed: int,
                     stream: int, steps: int) -> np.ndarray:
    """Mean shift with DEANN weights: NN rows weigh 1, each draw (n-k)/m.

    Step t re-selects the k-NN of the current point and draws with counter
    word 2 equal to t.  The point is kept in float32 between steps.
    """
    n = X.shape[0]
    y = np.asarray(y, dtype=np.float32).astype(np.float64)
    for t in range(steps):
        y32 = y.astype(np.float32)
        nn = knn(X, y32, k)
        s_idx = sample_indices(n, nn, m, seed, stream, word2=t)
        rows = [X[nn].astype(np.float64)]
        wts = [np.ones(len(nn))]
        if m > 0 and n - len(nn) > 0:
            rows.append(X[s_idx].astype(np.float64))
            wts.append(np.full(m, (n - len(nn)) / m))
        R = np.concatenate(rows)
        W = np.concatenate(wts)
        diff = R - y32.astype(np.float64)
        K = kernel_values(np.einsum("ij,ij->i", diff, diff, optimize=False), h, GAUSSIAN) * W
        y = ((K[:, None] * R).sum(axis=0) / math.fsum(K)).astype(np.float32).astype(np.float64)
    return y


def pairwise_sq_dists(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """All squared distances [q, n] in FP64 (for bisection over a fixed query set)."""
    Y = np.atleast_2d(Y)
    return np.stack([sq_dists(X, y) for y in Y])


def bisect_h(D2: np.ndarray, target: float, kernel: int, stat: str = "mean",
             rel_tol: float = 0.01, max_iter: int = 200) -> float:
    """Bandwidth h whose mean (or median) exact KDE over the queries is within
    ``rel_tol`` relative of ``target``, by bisection on log h.

    D2 holds the FP64 squared distances [q, n] of the query set.  The KDE is
    non-decreasing in h for a radially decreasing kernel, which the bisection
    relies on.
    """
    agg = np.mean if stat == "mean" else np.median

    def value(h):
        # a 1% target needs no correctly rounded sum: numpy's pairwise sum
        return float(agg([kernel_values(row, h, kernel).sum() / row.size for row in D2]))

    lo, hi = -20.0, 20.0
    for _ in range(max_iter):
        mid = 0.5 * (lo + hi)
        h = math.exp(mid)
        v = value(h)
        if abs(v - target) <= rel_tol * target:
            return h
        if v < target:
            lo = mid
        else:
            hi = mid
    raise RuntimeError("bisection did not converge")


# --------------------------------------------------------------------------
# Inverted-file index: the approximate nearest neighbours of the experiments
# (Sec. 5).  k-means over the data gives n_l centroids, each row belongs to
# its closest centroid, and a query inspects every row of the n_q closest
# centroids.  The estimate of Algorithm 1 stays unbiased for any neighbour
# set (only the split of X into X1 and X2 changes), so the returned set is
# used as X1 unchanged.
#
# Readings where the paper leaves the index unspecified:
#   * initial centroids are the rows floor(l n / n_l), l = 0..n_l-1;
#   * "closest" is the exact order (||c - x||^2, l) with ties towards the
#     lower centroid, like the k-NN order above;
#   * a Lloyd step replaces each centroid by the mean of its rows (an FP64
#     sum rounded once to float32); a centroid without rows stays;
#   * training runs `iters` Lloyd steps and then assigns every row to the
#     closest final centroid;
#   * a query whose n_q closest clusters hold fewer than k rows inspects the
#     next closest clusters too, one at a time, until they hold at least k
#     rows, but never more than probe_cap(n_l, n_q) = min(n_l, max(2 n_q,
#     n_q + 64), 496) clusters in all; if even those hold fewer than k rows,
#     the exact k nearest rows of all of X are used.
# --------------------------------------------------------------------------

def kmeans_init(X: np.ndarray, n_clusters: int) -> np.ndarray:
    """Initial centroids: the rows floor(l n / n_l) of X, as float32."""
    n = X.shape[0]
    rows = [(l * n) // n_clusters for l in range(n_clusters)]
    return np.asarray(X[rows], dtype=np.float32)


def kmeans_assign(X: np.ndarray, C: np.ndarray) -> np.ndarray:
    """Index of the closest centroid of every row (exact order, ties to the
    lower centroid)."""
    return np.asarray([knn(C, x, 1)[0] for x in X], dtype=np.int64)


def kmeans_update(X: np.ndarray, assign: np.ndarray, C_prev: np.ndarray) -> np.ndarray:
    """Lloyd step: each centroid becomes the mean of its rows, summed exactly
    (math.fsum per coordinate) and divided in FP64, then rounded to float32;
    a centroid without rows keeps its previous value."""
    C = np.array(C_prev, dtype=np.float32, copy=True)
    Xd = np.asarray(X, dtype=np.float64)
    for l in range(C.shape[0]):
        rows = np.nonzero(assign == l)[0]
        if rows.size == 0:
            continue
        sums = [math.fsum(Xd[rows, t].tolist()) for t in range(X.shape[1])]
        C[l] = np.asarray([s / rows.size for s in sums], dtype=np.float64).astype(np.float32)
    return C


def ivf_train(X: np.ndarray, n_clusters: int, iters: int):
    """(centroids float32 [n_l, d], assignment int64 [n]) after `iters`
    Lloyd steps from kmeans_init and a final assignment."""
    C = kmeans_init(X, n_clusters)
    for _ in range(iters):
        C = kmeans_update(X, kmeans_assign(X, C), C)
    return C, kmeans_assign(X, C)


def probe_cap(n_clusters: int, n_probe: int) -> int:
    """Most clusters one query may inspect."""
    return min(n_clusters, max(2 * n_probe, n_probe + 64), 496)


def cluster_order(C: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Every cluster id in the exact order (||c_l - y||^2, l): an FP64 sort,
    with runs of values too close for FP64 to decide re-sorted exactly."""
    L, d = C.shape
    d2 = sq_dists(C, y)
    order = list(np.lexsort((np.arange(L), d2)))
    rel = 4.0 * (d + 2) * 2.0 ** -53
    i = 0
    while i < L:
        j = i
        while j + 1 < L and d2[order[j + 1]] <= d2[order[j]] * (1.0 + 2.0 * rel) + 1e-300:
            j += 1
        if j > i:
            order[i:j + 1] = sorted(order[i:j + 1], key=lambda l: (_exact_sq_dist(C[l], y), l))
        i = j + 1
    return np.asarray(order, dtype=np.int64)


def ivf_probe(C: np.ndarray, y: np.ndarray, n_probe: int, sizes: np.ndarray | None = None,
              k: int = 0) -> np.ndarray:
    """The clusters a query inspects, ascending by id: the n_q closest, and
    with cluster sizes given, the next closest too while they hold fewer than
    k rows (at most probe_cap clusters).  Empty when even those hold fewer
    than k rows (the caller then uses the exact k-NN)."""
    order = cluster_order(C, y)
    p = n_probe
    if sizes is not None:
        cap = probe_cap(C.shape[0], n_probe)
        while p < cap and int(sizes[order[:p]].sum()) < k:
            p += 1
        if int(sizes[order[:p]].sum()) < k:
            return np.empty(0, dtype=np.int64)
    return np.sort(order[:p])


def ivf_knn(X: np.ndarray, y: np.ndarray, C: np.ndarray, assign: np.ndarray, n_probe: int,
            k: int) -> np.ndarray:
    """The k nearest rows among those of the inspected clusters (sorted by
    index); the exact k-NN of all of X when those hold fewer than k rows."""
    if k <= 0:
        return np.empty(0, dtype=np.int64)
    sizes = np.bincount(assign[(assign >= 0) & (assign < C.shape[0])], minlength=C.shape[0])
    probes = ivf_probe(C, y, n_probe, sizes, k)
    rows = np.nonzero(np.isin(assign, probes))[0]
    if rows.size < k:
        return knn(X, y, k)
    # the rows keep ascending order, so the lower position is the lower index
    return np.sort(rows[knn(X[rows], y, k)])


def deann_estimate_ivf(X: np.ndarray, y: np.ndarray, h: float, kernel: int, C: np.ndarray,
                       assign: np.ndarray, n_probe: int, k: int, m: int, seed: int,
                       stream: int):
    """DEANN (Algorithm 1) with the inverted-file neighbours as X1."""
    nn = ivf_knn(X, y, C, assign, n_probe, k)
    return deann_estimate(X, y, h, kernel, k, m, seed, stream, nn=nn)


def recall(nn_true: np.ndarray, nn_found: np.ndarray) -> float:
    """|NN_k(q) & NN~_k(q)| / |NN_k(q)| (the recall of Sec. 5)."""
    if len(nn_true) == 0:
        return 1.0
    return len(np.intersect1d(nn_true, nn_found)) / len(nn_true)
