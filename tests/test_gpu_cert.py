"""The float32 exact KDE's accuracy certificate and the fallbacks it and the
k-NN certificate lead to, on small inputs where the oracle is cheap:

* at a quarter of the workload bandwidth a few rows carry each query's mass and
  the GEMM identity's rounding of ||x~||^2 + ||y~||^2 no longer averages out:
  the certificate sends those queries to the exact FP64 re-evaluation, and the
  values (kde_exact, kde_exact_with_grad, kde_exact_backward) stay within 1e-5
  of the oracle, the gradients within 1e-4 of the normwise scale;
* a second-pass capacity below k (the knn_cap2 option) sends every query that
  needs the second pass to the exhaustive FP64 scan, whose neighbours must
  equal the oracle's bit for bit, ties and duplicate rows included.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import GAUSSIAN, EXPONENTIAL

from .gpu_common import bandwidth, device, rel_err, to_dev

pytestmark = pytest.mark.gpu

WL = "mix10_n1e4_d16"
KNAME = {GAUSSIAN: "gaussian", EXPONENTIAL: "exponential"}


@pytest.fixture(scope="module")
def c1():
    dev = device()
    spec, X, Y = synth.workload(WL, q=300)
    return X, Y, to_dev(X, dev), to_dev(Y, dev)


@pytest.fixture
def options():
    import paper_2107_02736_amd as dk
    prev = dk.get_options()
    yield dk
    dk.set_options(**prev)


def _scale(X, y, h, kern):
    d2 = oracle.sq_dists(X, y)
    K = oracle.kernel_values(d2, h, kern)
    r = np.sqrt(d2)
    if kern == GAUSSIAN:
        return (K * r).sum() / (X.shape[0] * h * h), (K * d2).sum() / (X.shape[0] * h ** 3)
    return K.sum() / (X.shape[0] * h), (K * r).sum() / (X.shape[0] * h * h)


@pytest.mark.parametrize("prec", ["fp32", "fp32_split"])
@pytest.mark.parametrize("scale", [0.25, 1.0])
@pytest.mark.parametrize("kern", [GAUSSIAN, EXPONENTIAL])
def test_exact_small_bandwidth_values_and_gradients(c1, kern, scale, prec):
    import paper_2107_02736_amd as dk
    X, Y, Xd, Yd = c1
    q = Y.shape[0]
    h = scale * bandwidth(WL, KNAME[kern])
    got = dk.kde_exact(Xd, Yd, h, KNAME[kern], prec).cpu().numpy()
    st = dk.last_stats(Xd.device)
    mu, gy, gh = (t.cpu().numpy() for t in dk.kde_exact_with_grad(Xd, Yd, h, KNAME[kern],
                                                                   precision=prec))
    st_g = dk.last_stats(Xd.device)
    g = np.linspace(0.5, 1.5, q)
    gy_b, gh_b = dk.kde_exact_backward(Xd, Yd, h, to_dev(g, Xd.device), KNAME[kern],
                                       precision=prec)
    gy_b, gh_b = gy_b.cpu().numpy(), float(gh_b.cpu().numpy()[0])
    ref = np.empty(q)
    gh_ref = gh_abs = 0.0
    worst_g = 0.0
    for j in range(q):
        mu_ref, gy_ref, ghj = oracle.kde_grad(X, Y[j].astype(np.float64), h, kern)
        ref[j] = mu_ref
        sy, shh = _scale(X, Y[j], h, kern)
        gh_ref += g[j] * ghj
        gh_abs += g[j] * shh
        if mu_ref < 1e-16:
            continue
        worst_g = max(worst_g, np.linalg.norm(gy[j] - gy_ref) / sy)
        assert np.linalg.norm(gy[j] - gy_ref) <= 1e-4 * sy, j
        assert np.linalg.norm(gy_b[j] - g[j] * gy_ref) <= 1e-4 * g[j] * sy, j
        assert abs(gh[j] - ghj) <= 1e-4 * shh, j
    err, excluded = rel_err(got, ref)
    err_g, _ = rel_err(mu, ref)
    print(f"{KNAME[kern]} h x{scale} {prec}: re-evaluated {st['exact_refined']} (value) "
          f"{st_g['exact_refined']} (with gradient) of {q}; max rel err {err.max():.2e} / "
          f"{err_g.max():.2e}; gradient {worst_g:.2e} of the normwise scale; "
          f"{excluded} below 1e-16")
    assert err.max() <= 1e-5 and err_g.max() <= 1e-5
    assert abs(gh_b - gh_ref) <= 1e-4 * gh_abs
    if scale == 0.25 and kern == GAUSSIAN:
        assert st["exact_refined"] > 0   # this case does exercise the fallback


@pytest.mark.parametrize("prec", ["fp32", "fp32_split"])
@pytest.mark.parametrize("h", [2.5, 5.0])
@pytest.mark.parametrize("kern", [GAUSSIAN, EXPONENTIAL])
def test_exact_wide_rows_certificate(kern, h, prec):
    # rows wider than 128 floats take the generic tile kernel (float32 or
    # split operands), whose certificate uses each pair's own norm term; a few
    # far rows make the largest row norm much larger than the norms of the
    # pairs that matter
    import paper_2107_02736_amd as dk
    rng = np.random.default_rng(21)
    n, q, d = 4000, 200, 200
    cen = rng.uniform(-3, 3, size=(5, d))
    X = cen[rng.integers(0, 5, n)] + rng.normal(size=(n, d))
    X[:8] *= 6.0
    Y = cen[rng.integers(0, 5, q)] + rng.normal(size=(q, d))
    X, Y = X.astype(np.float32), Y.astype(np.float32)
    dev = device()
    got = dk.kde_exact(to_dev(X, dev), to_dev(Y, dev), h, KNAME[kern], prec).cpu().numpy()
    st = dk.last_stats(dev)
    ref = oracle.kde_exact(X, Y, h, kern)
    err, excluded = rel_err(got, ref)
    print(f"{KNAME[kern]} {prec} h={h}: re-evaluated {st['exact_refined']} of {q}, max rel err "
          f"{err.max():.2e}, {excluded} below 1e-16")
    assert err.max() <= 1e-5


def test_value_floor_zero_refines_tiny_values(c1, options):
    # with value_floor = 0 the queries below 1e-16 are certified or re-evaluated
    # too: every query is then within 1e-5 of the oracle, however small
    dk = options
    X, Y, Xd, Yd = c1
    Yf = Y.copy()
    Yf[:20] += 5.0   # away from the clusters: densities far below 1e-16
    Yfd = to_dev(Yf, Xd.device)
    h = 0.5 * bandwidth(WL, "gaussian")
    ref = oracle.kde_exact(X, Yf, h, GAUSSIAN)
    tiny = (ref < 1e-16) & (ref > 1e-280)
    assert tiny.sum() >= 5
    dk.set_options(value_floor=0.0)
    got = dk.kde_exact(Xd, Yfd, h, "gaussian", "fp32").cpu().numpy()
    st = dk.last_stats(Xd.device)
    print(f"re-evaluated {st['exact_refined']}, values below 1e-16: {tiny.sum()}")
    assert np.all(np.abs(got - ref) <= 1e-5 * ref)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_knn_exhaustive_fallback(options, prec):
    dk = options
    spec, X, Y = synth.workload(WL, n=3000, q=96)
    dev = device()
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    k, m = 64, 40
    # FP32: with no slack the list holds K1 = k = 64 keys, so the first-pass
    # certificate (the K1-th key above the k-th distance) cannot hold and every
    # query needs the second pass; 16-bit scans always take it.  A capacity of
    # 8 < k then overflows every second pass.
    dk.set_options(knn_slack=0, knn_cap2=8)
    out, nn, sm = (t.cpu().numpy() for t in dk.deann_query(Xd, Yd, 2.0, k, m, "gaussian",
                                                           seed=3, precision=prec))
    st = dk.last_stats(dev)
    print(f"{prec}: second pass {st['knn_second_pass']}, exhaustive {st['knn_exhaustive']} of 96")
    assert st["knn_exhaustive"] == 96 and st["knn_second_pass"] == 96
    for j in range(96):
        est, nn_ref, s_ref = oracle.deann_estimate(X, Y[j], 2.0, GAUSSIAN, k, m, 3, j)
        assert np.array_equal(nn[j], nn_ref), j
        assert np.array_equal(sm[j], s_ref), j
        assert abs(out[j] - est) <= 1e-12 * est


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_knn_exhaustive_fallback_ties(options, prec):
    # lattice data: many exactly equal distances and duplicate rows, every
    # query through the exhaustive scan's top-k buffer
    dk = options
    rng = np.random.default_rng(5)
    X = rng.integers(-2, 3, size=(900, 3)).astype(np.float32)
    Y = rng.integers(-2, 3, size=(40, 3)).astype(np.float32)
    dev = device()
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    dk.set_options(knn_slack=0, knn_cap2=1)
    for k in (1, 9, 64):
        _, nn, _ = dk.deann_query(Xd, Yd, 1.0, k, 0, precision=prec)
        nn = nn.cpu().numpy()
        st = dk.last_stats(dev)
        if k == 64 or prec != "fp32":   # no first-pass certificate without slack
            assert st["knn_exhaustive"] == 40, (k, st)
        for j in range(40):
            assert np.array_equal(nn[j], oracle.knn(X, Y[j], k)), (k, j)


def test_options_do_not_change_results(c1, options):
    # slack, capacity and centring change the path, not the result
    dk = options
    X, Y, Xd, Yd = c1
    h = bandwidth(WL, "gaussian")
    base = [t.cpu().numpy() for t in dk.deann_query(Xd, Yd, h, 20, 50, seed=1, precision="bf16")]
    mu0 = dk.kde_exact(Xd, Yd, h, "gaussian", "fp32").cpu().numpy()
    for kw in (dict(knn_slack=100), dict(knn_cap2=16), dict(center=0), dict(knn_seed_stride=1)):
        dk.set_options(**kw)
        got = [t.cpu().numpy() for t in dk.deann_query(Xd, Yd, h, 20, 50, seed=1,
                                                        precision="bf16")]
        for a, b in zip(got, base):
            assert np.array_equal(a, b), kw
        mu = dk.kde_exact(Xd, Yd, h, "gaussian", "fp32").cpu().numpy()
        assert np.all(np.abs(mu - mu0) <= 2e-5 * mu0), kw
        dk.set_options(**dk.default_options())


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_knn_seed_stride(options, prec):
    # the 16-bit candidate pass reads every ts-th data tile (782 tiles here, so
    # ts up to 48); the seeds only bound the second pass: the neighbours, draws
    # and estimates are the same for every stride, and the oracle's
    dk = options
    spec, X, Y = synth.workload(WL, n=100_000, q=200)
    dev = device()
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    h, k, m = bandwidth(WL, "gaussian"), 40, 60
    outs = {}
    for ts in (1, 4, 48):
        dk.set_options(knn_seed_stride=ts)
        outs[ts] = [t.cpu().numpy() for t in dk.deann_query(Xd, Yd, h, k, m, seed=2,
                                                             precision=prec)]
        st = dk.last_stats(dev)
        print(f"{prec} seed stride {ts}: exhaustive {st['knn_exhaustive']} of 200")
    for ts in (4, 48):
        for a, b in zip(outs[ts], outs[1]):
            assert np.array_equal(a, b), ts
    out, nn, sm = outs[48]
    for j in synth.query_subset(Y.shape[0], 12, seed=4):
        j = int(j)
        est, nn_ref, s_ref = oracle.deann_estimate(X, Y[j], h, GAUSSIAN, k, m, 2, j)
        assert np.array_equal(nn[j], nn_ref), j
        assert np.array_equal(sm[j], s_ref), j
        assert abs(out[j] - est) <= 1e-12 * est


def test_backward_rejects_bad_index_tensors(c1):
    # the adjoint uses the entries as row indices of X: the binding checks
    # dtype, shape and device before calling the library
    import torch

    import paper_2107_02736_amd as dk
    X, Y, Xd, Yd = c1
    _, nn, sm = dk.deann_query(Xd, Yd, 2.0, 5, 7)
    g = torch.ones(Y.shape[0], dtype=torch.float64, device=Xd.device)
    for bad_nn, bad_sm in ((nn.long(), sm), (nn, sm[:, :6].contiguous()), (nn.cpu(), sm),
                           (nn.t().contiguous(), sm)):
        with pytest.raises(ValueError):
            dk.deann_query_backward(Xd, Yd, 2.0, 5, 7, bad_nn, bad_sm, g)
    with pytest.raises(ValueError):
        dk.deann_query_backward(Xd, Yd, 2.0, 5, 7, nn, sm, g[:-1])


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_small_batch_with_capped_seed_splits(prec):
    # n = 200 000 rows and one query tile: the candidate pass's split count is
    # capped (128 splits, 4096 cells per query) below the second pass's; the
    # neighbours, draws and estimates equal the oracle's and those of the same
    # queries inside a batch of 1024
    import paper_2107_02736_amd as dk
    dev = device()
    spec, X, Y = synth.workload(WL, n=200_000, q=1024)
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    h, k, m = bandwidth(WL, "gaussian"), 50, 100
    big = [t.cpu().numpy() for t in dk.deann_query(Xd, Yd, h, k, m, seed=4, precision=prec)]
    small = [t.cpu().numpy() for t in dk.deann_query(Xd, Yd[:64].contiguous(), h, k, m, seed=4,
                                                     precision=prec)]
    for a, b in zip(small, big):
        assert np.array_equal(a, b[:64])
    out, nn, sm = small
    for j in range(0, 64, 9):
        est, nn_ref, s_ref = oracle.deann_estimate(X, Y[j], h, GAUSSIAN, k, m, 4, j)
        assert np.array_equal(nn[j], nn_ref), j
        assert np.array_equal(sm[j], s_ref), j
        assert abs(out[j] - est) <= 1e-12 * max(est, 1e-300), j
