"""Isotropic Gaussian-mixture datasets standing in for the paper's real datasets.

The paper measures on nine real datasets (n from 58k to 2.46M, d from 9 to
3072; Section 5, dataset table) that are not available here.  These seeded
mixtures have the same kind of shape: a training set X[n, d] and a query set
Y[q, d] drawn from the same distribution, optionally with a fraction of
queries spread uniformly over X's bounding box (outliers with tiny density).

Draw order (fixed, so a spec and seed define the bytes exactly):
means -> per-cluster std -> X labels -> X noise -> Y labels -> Y noise ->
uniform-box queries.  Everything is drawn in float64 with numpy's PCG64
``default_rng`` and cast to float32 once at the end.
"""
from __future__ import annotations

import dataclasses
import numpy as np

_CHUNK_ROWS = 1 << 16


@dataclasses.dataclass(frozen=True)
class MixtureSpec:
    name: str
    n: int
    q: int
    d: int
    clusters: int
    mean_lo: float
    mean_hi: float
    std_lo: float
    std_hi: float
    box_frac: float = 0.0      # fraction of queries uniform in X's bounding box
    absolute: bool = False     # pass X and Y through |.| after drawing
    seed: int = 0

    def scaled(self, n: int | None = None, q: int | None = None) -> "MixtureSpec":
        """Same distribution with fewer points or queries (for parity tests)."""
        return dataclasses.replace(self, n=self.n if n is None else int(n),
                                   q=self.q if q is None else int(q))


# The five workloads of the measurement plan.  Sizes follow the paper's
# dataset range (d=16..960, n up to 1e6).
WORKLOADS = {
    # small: 10 clusters, means U[-5,5]^16, unit std, all queries from the mixture
    "mix10_n1e4_d16": MixtureSpec("mix10_n1e4_d16", 10_000, 1_000, 16, 10, -5.0, 5.0, 1.0, 1.0,
                                  seed=1001),
    # full size: 100 clusters, means U[-10,10]^128, std U[0.5,2], 10% box queries
    "mix100_n1e6_d128": MixtureSpec("mix100_n1e6_d128", 1_000_000, 10_000, 128, 100, -10.0, 10.0,
                                    0.5, 2.0, box_frac=0.1, seed=1002),
    # differentiation workload: 50 clusters in d=64
    "mix50_n5e5_d64": MixtureSpec("mix50_n5e5_d64", 500_000, 4_096, 64, 50, -10.0, 10.0, 0.5, 2.0,
                                  seed=1004),
    # large high-dimensional, non-negative entries
    "mix200_n1e6_d960": MixtureSpec("mix200_n1e6_d960", 1_000_000, 10_000, 960, 200, -10.0, 10.0,
                                    0.5, 2.0, absolute=True, seed=1005),
}


def make_mixture(spec: MixtureSpec) -> tuple[np.ndarray, np.ndarray]:
    """Return (X[n,d], Y[q,d]) as C-contiguous float32 arrays."""
    rng = np.random.default_rng(spec.seed)
    means = rng.uniform(spec.mean_lo, spec.mean_hi, size=(spec.clusters, spec.d))
    stds = rng.uniform(spec.std_lo, spec.std_hi, size=spec.clusters)
    X = np.empty((spec.n, spec.d), dtype=np.float32)
    xl = rng.integers(0, spec.clusters, size=spec.n)
    for r0 in range(0, spec.n, _CHUNK_ROWS):
        r1 = min(spec.n, r0 + _CHUNK_ROWS)
        lab = xl[r0:r1]
        noise = rng.standard_normal((r1 - r0, spec.d))
        X[r0:r1] = means[lab] + stds[lab, None] * noise
    q_box = int(round(spec.q * spec.box_frac))
    q_mix = spec.q - q_box
    Y = np.empty((spec.q, spec.d), dtype=np.float32)
    yl = rng.integers(0, spec.clusters, size=q_mix)
    noise = rng.standard_normal((q_mix, spec.d))
    Y[:q_mix] = means[yl] + stds[yl, None] * noise
    if q_box:
        lo = X.min(axis=0).astype(np.float64)
        hi = X.max(axis=0).astype(np.float64)
        Y[q_mix:] = rng.uniform(lo, hi, size=(q_box, spec.d))
    if spec.absolute:
        np.abs(X, out=X)
        np.abs(Y, out=Y)
    return X, Y


def workload(name: str, n: int | None = None, q: int | None = None):
    """(spec, X, Y) for a named workload, optionally scaled down."""
    spec = WORKLOADS[name].scaled(n, q)
    X, Y = make_mixture(spec)
    return spec, X, Y


def query_subset(q: int, size: int, seed: int = 7) -> np.ndarray:
    """A fixed, sorted random subset of query rows (for sampled checks at full size)."""
    if size >= q:
        return np.arange(q, dtype=np.int64)
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(q, size=size, replace=False)).astype(np.int64)
