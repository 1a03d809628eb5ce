"""Full-size parity in the benchmark's launch configuration: the 100-cluster
mixture with n = 1,000,000, d = 128, q = 10,000 (k = 100, m = 1,000) and the
differentiation workload n = 500,000, d = 64, q = 4,096, and the large
high-dimensional workload n = 1,000,000, d = 960, q = 10,000.  Sampled queries are
checked against the oracle one by one; properties that hold at any size are
checked on every query."""
import numpy as np
import pytest

import oracle
import synth
from oracle import GAUSSIAN, EXPONENTIAL

from .gpu_common import bandwidth, device, rel_err, to_dev

pytestmark = pytest.mark.gpu

WL = "mix100_n1e6_d128"
KNAME = {GAUSSIAN: "gaussian", EXPONENTIAL: "exponential"}


@pytest.fixture(scope="module")
def big():
    dev = device()
    spec, X, Y = synth.workload(WL)
    return X, Y, to_dev(X, dev), to_dev(Y, dev)


def _check_indices(nn, sm, n, k):
    # sorted, distinct, in range; draws in range and outside the neighbour set
    assert nn.min() >= 0 and nn.max() < n
    assert np.all(np.diff(nn, axis=1) > 0)
    assert sm.min() >= 0 and sm.max() < n
    for j in range(0, nn.shape[0], 97):
        assert not np.isin(sm[j], nn[j]).any()


@pytest.mark.parametrize("kern", [GAUSSIAN, EXPONENTIAL])
def test_fullsize_deann_and_exact(big, kern):
    import paper_2107_02736_amd as dk
    X, Y, Xd, Yd = big
    h = bandwidth(WL, KNAME[kern])
    k, m = 100, 1000
    mu = dk.kde_exact(Xd, Yd, h, KNAME[kern], "fp32").cpu().numpy()
    res = {p: dk.deann_query(Xd, Yd, h, k, m, KNAME[kern], seed=0, precision=p)
           for p in ("bf16", "fp32")}
    out, nn, sm = (t.cpu().numpy() for t in res["bf16"])
    out32, nn32, sm32 = (t.cpu().numpy() for t in res["fp32"])
    # BF16 scan + refinement reproduces the FP32 result exactly
    assert np.array_equal(nn, nn32) and np.array_equal(sm, sm32)
    assert np.array_equal(out, out32)
    assert np.all((mu >= 0) & (mu <= 1)) and np.all(out >= 0)
    _check_indices(nn, sm, X.shape[0], k)
    for j in synth.query_subset(Y.shape[0], 5, seed=3):
        est, nn_ref, s_ref = oracle.deann_estimate(X, Y[j], h, kern, k, m, 0, int(j))
        assert np.array_equal(nn[j], nn_ref), j
        assert np.array_equal(sm[j], s_ref), j
        assert abs(out[j] - est) <= 1e-12 * max(est, 1e-300)
        ref = oracle.kde_exact(X, Y[j:j + 1], h, kern)[0]
        if ref >= 1e-16:
            print(f"query {j}: exact fp32 rel err {abs(mu[j] - ref) / ref:.2e}")
            assert abs(mu[j] - ref) <= 1e-5 * ref


@pytest.mark.parametrize("kern", [GAUSSIAN, EXPONENTIAL])
def test_fullsize_exact_with_grad(big, kern):
    # the benchmark step's exact part (kde_exact_with_grad) at n = 1e6, d = 128
    # on all 10,000 queries: values of sampled queries within 1e-5 and their
    # gradients within 1e-4 of the normwise scale; every query's value agrees
    # with kde_exact (both certified to 5e-6)
    import paper_2107_02736_amd as dk
    X, Y, Xd, Yd = big
    h = bandwidth(WL, KNAME[kern])
    mu, gy, gh = (t.cpu().numpy() for t in dk.kde_exact_with_grad(Xd, Yd, h, KNAME[kern]))
    st = dk.last_stats(Xd.device)
    mu_fwd = dk.kde_exact(Xd, Yd, h, KNAME[kern], "fp32").cpu().numpy()
    keep = mu_fwd >= 1e-16
    print(f"{KNAME[kern]}: queries re-evaluated {st['exact_refined']}, "
          f"kept {keep.sum()} of {keep.size}")
    assert np.all(np.abs(mu[keep] - mu_fwd[keep]) <= 1e-5 * mu_fwd[keep])
    for j in synth.query_subset(Y.shape[0], 4, seed=11):
        j = int(j)
        mu_ref, gy_ref, gh_ref = oracle.kde_grad(X, Y[j].astype(np.float64), h, kern)
        if mu_ref < 1e-16:
            continue
        assert abs(mu[j] - mu_ref) <= 1e-5 * mu_ref, j
        d2 = oracle.sq_dists(X, Y[j])
        K = oracle.kernel_values(d2, h, kern)
        r = np.sqrt(d2)
        scale = ((K * r).sum() / (X.shape[0] * h * h) if kern == GAUSSIAN
                 else K.sum() / (X.shape[0] * h))
        print(f"query {j}: value {abs(mu[j] - mu_ref) / mu_ref:.2e}, gradient "
              f"{np.linalg.norm(gy[j] - gy_ref) / scale:.2e} of the normwise scale")
        assert np.linalg.norm(gy[j] - gy_ref) <= 1e-4 * scale, j


def test_fullsize_near_far(big):
    # the near/far exact KDE in the benchmark's configuration (BF16, k = 100):
    # its neighbour lists are DEANN's on every query; sampled queries against
    # the oracle's k-NN and the exact KDE within the bound without the exact
    # neighbour terms
    import paper_2107_02736_amd as dk
    from .precision_bound import exact_kde_bound, geometry as bound_geometry
    X, Y, Xd, Yd = big
    h = bandwidth(WL, "gaussian")
    got, nn = dk.kde_hybrid(Xd, Yd, h, 100, "gaussian", "bf16", return_indices=True)
    got, nn = got.cpu().numpy(), nn.cpu().numpy()
    nn_deann = dk.deann_query(Xd, Yd, h, 100, 0, "gaussian", precision="bf16")[1].cpu().numpy()
    assert np.array_equal(nn, nn_deann)
    assert np.all((got >= 0) & (got <= 1))
    given = dk.kde_hybrid(Xd, Yd, h, 100, "gaussian", "bf16", nn_idx=to_dev(nn, Xd.device))
    assert np.allclose(given.cpu().numpy(), got, rtol=1e-13, atol=0)
    for j in synth.query_subset(Y.shape[0], 3, seed=11):
        near = oracle.knn(X, Y[j], 100)
        assert np.array_equal(nn[j], near), j
        ref = oracle.kde_exact(X, Y[j:j + 1], h, GAUSSIAN)[0]
        if ref < 1e-16:
            continue
        bound = exact_kde_bound(bound_geometry(X, Y[j:j + 1]), X.shape[1], h, GAUSSIAN, "bf16",
                                near=near[None, :])[0]
        err = abs(got[j] - ref) / ref
        print(f"query {j}: near/far bf16 rel err {err:.2e} (bound {bound:.2e})")
        assert err <= bound


def test_fullsize_exact_backward():
    import paper_2107_02736_amd as dk
    dev = device()
    wl = "mix50_n5e5_d64"
    spec, X, Y = synth.workload(wl)
    h = bandwidth(wl, "gaussian")
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    g = np.ones(Y.shape[0])
    gy, gh = dk.kde_exact_backward(Xd, Yd, h, to_dev(g, dev), "gaussian")
    gy = gy.cpu().numpy()
    assert np.all(np.isfinite(gy))
    for j in synth.query_subset(Y.shape[0], 3, seed=5):
        _, gy_ref, _ = oracle.kde_grad(X, Y[j].astype(np.float64), h, GAUSSIAN)
        d2 = oracle.sq_dists(X, Y[j])
        K = oracle.kernel_values(d2, h, GAUSSIAN)
        scale = (K * np.sqrt(d2)).sum() / (X.shape[0] * h * h)
        assert np.linalg.norm(gy[j] - gy_ref) <= 1e-4 * scale


def test_fullsize_d960_bf16_refine():
    """Large high-dimensional workload (200-cluster mixture through |.|,
    n = 1,000,000, d = 960, q = 10,000, k = 200, m = 2,000): the BF16 scan
    with refinement gives the FP32 scan's result exactly; sampled queries and
    the DEANN adjoint against the oracle."""
    import paper_2107_02736_amd as dk
    dev = device()
    wl = "mix200_n1e6_d960"
    spec, X, Y = synth.workload(wl)
    h = bandwidth(wl, "gaussian")
    k, m = 200, 2000
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    mu = dk.kde_exact(Xd, Yd, h, "gaussian", "fp32").cpu().numpy()
    res = {p: dk.deann_query(Xd, Yd, h, k, m, "gaussian", seed=0, precision=p)
           for p in ("bf16", "fp32")}
    out, nn, sm = (t.cpu().numpy() for t in res["bf16"])
    out32, nn32, sm32 = (t.cpu().numpy() for t in res["fp32"])
    assert np.array_equal(nn, nn32) and np.array_equal(sm, sm32)
    assert np.array_equal(out, out32)
    assert np.all((mu >= 0) & (mu <= 1)) and np.all(out >= 0)
    _check_indices(nn, sm, X.shape[0], k)
    g = np.linspace(0.5, 1.5, Y.shape[0])
    gy, gh = dk.deann_query_backward(Xd, Yd, h, k, m, res["bf16"][1], res["bf16"][2],
                                     to_dev(g, dev), "gaussian")
    gy = gy.cpu().numpy()
    for j in synth.query_subset(Y.shape[0], 2, seed=13):
        est, nn_ref, s_ref = oracle.deann_estimate(X, Y[j], h, GAUSSIAN, k, m, 0, int(j))
        assert np.array_equal(nn[j], nn_ref), j
        assert np.array_equal(sm[j], s_ref), j
        assert abs(out[j] - est) <= 1e-12 * max(est, 1e-300)
        ref = oracle.kde_exact(X, Y[j:j + 1], h, GAUSSIAN)[0]
        print(f"query {j}: exact {ref:.4e}, fp32 rel err {abs(mu[j] - ref) / ref:.2e}, "
              f"DEANN rel err {abs(out[j] - ref) / ref:.2e}")
        assert abs(mu[j] - ref) <= 1e-5 * ref
        _, gy_ref, _ = oracle.deann_grad(X, Y[j], h, GAUSSIAN, nn_ref, s_ref, m)
        assert np.linalg.norm(gy[j] - g[j] * gy_ref) <= 1e-6 * np.linalg.norm(g[j] * gy_ref)


def test_fullsize_mean_shift_d64():
    """Differentiation workload (50-cluster mixture, n = 500,000, d = 64,
    q = 4,096): 20 Gaussian mean-shift steps of every query through the
    autograd functions, exact (FP32 tiles) and DEANN (BF16 scan, k = 64,
    m = 512).  Exact trajectories of sampled queries against the oracle's;
    DEANN steps from the final points against the oracle's step."""
    import time
    import torch
    import paper_2107_02736_amd as dk
    dev = device()
    wl = "mix50_n5e5_d64"
    spec, X, Y = synth.workload(wl)
    h = bandwidth(wl, "gaussian")
    k, m, steps = 64, 512, 20
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    t0 = time.perf_counter()
    ye = dk.mean_shift(Xd, Yd, h, steps, "exact")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    yd = dk.mean_shift(Xd, Yd, h, steps, "deann", k=k, m=m, seed=2, precision="bf16")
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    print(f"20 mean-shift steps of 4096 queries: exact {t1 - t0:.3f} s, DEANN {t2 - t1:.3f} s")
    ye, yd = ye.cpu().numpy(), yd.cpu().numpy()
    assert np.all(np.isfinite(ye)) and np.all(np.isfinite(yd))
    sub = synth.query_subset(Y.shape[0], 2, seed=17)
    for j in sub:
        ref = oracle.mean_shift_exact(X, Y[j], h, steps)
        assert np.max(np.abs(ye[j] - ref)) <= 1e-3, j
    # one more DEANN step from the GPU's end points (streams 0 and 1 of the subset)
    y_end = np.ascontiguousarray(yd[sub])
    y1 = dk.mean_shift(Xd, to_dev(y_end, dev), h, 1, "deann", k=k, m=m, seed=2,
                       precision="bf16").cpu().numpy()
    for i in range(len(sub)):
        ref = oracle.mean_shift_deann(X, y_end[i], h, k, m, 2, i, 1)
        assert np.max(np.abs(y1[i] - ref)) <= 1e-4 * max(1.0, np.max(np.abs(ref)))


def test_fullsize_inverted_file(big):
    # an inverted-file configuration of the cluster-count sweep: 1000 clusters,
    # 4 Lloyd steps, 16 inspected clusters; sampled rows' clusters are their
    # closest centroids, sampled queries equal the oracle given that index
    import paper_2107_02736_amd as dk
    X, Y, Xd, Yd = big
    h = bandwidth(WL, "gaussian")
    k, m = 100, 1000
    Cd, ad = dk.ivf_build(Xd, 1000, iters=4)
    C, a = Cd.cpu().numpy(), ad.cpu().numpy().astype(np.int64)
    rows = synth.query_subset(X.shape[0], 1000, seed=5)
    assert np.array_equal(a[rows], oracle.kmeans_assign(X[rows], C))
    index = dk.IvfIndex(Xd, Cd, ad)
    out, nn, sm = (t.cpu().numpy() for t in dk.deann_ivf_query(Xd, Yd, index, 16, h, k, m,
                                                               seed=0))
    _check_indices(nn, sm, X.shape[0], k)
    for j in synth.query_subset(Y.shape[0], 4, seed=6):
        est, nn_ref, s_ref = oracle.deann_estimate_ivf(X, Y[j], h, GAUSSIAN, C, a, 16, k, m,
                                                       0, int(j))
        assert np.array_equal(nn[j], nn_ref), j
        assert np.array_equal(sm[j], s_ref), j
        assert abs(out[j] - est) <= 1e-12 * max(est, 1e-300)
        print(f"query {j}: recall {oracle.recall(oracle.knn(X, Y[j], k), nn[j]):.2f}")
