"""Parity of the HIP path with the FP64 oracle on the small mixture workload
(n = 10,000, d = 16, q = 1,000, k = 50, m = 500) and on edge shapes."""
import numpy as np
import pytest

import oracle
import synth
from oracle import GAUSSIAN, EXPONENTIAL

from .precision_bound import exact_kde_bound, geometry as bound_geometry
from .gpu_common import bandwidth, device, rel_err, to_dev

pytestmark = pytest.mark.gpu

KNAME = {GAUSSIAN: "gaussian", EXPONENTIAL: "exponential"}
KIDS = {"gaussian": GAUSSIAN, "exponential": EXPONENTIAL}
WL = "mix10_n1e4_d16"


@pytest.fixture(scope="module")
def dev():
    return device()


@pytest.fixture(scope="module")
def c1(dev):
    spec, X, Y = synth.workload(WL)
    return X, Y, to_dev(X, dev), to_dev(Y, dev)


@pytest.fixture(scope="module")
def c1_exact():
    spec, X, Y = synth.workload(WL)
    return {kern: oracle.kde_exact(X, Y, bandwidth(WL, KNAME[kern]), kern)
            for kern in (GAUSSIAN, EXPONENTIAL)}


@pytest.mark.parametrize("prec", ["fp32", "fp32_split"])
@pytest.mark.parametrize("kern", [GAUSSIAN, EXPONENTIAL])
def test_exact_kde_fp32_within_1e5(c1, c1_exact, kern, prec):
    # fp32_split: float32-accurate dot products from three bfloat16 parts
    import paper_2107_02736_amd as dk
    X, Y, Xd, Yd = c1
    h = bandwidth(WL, KNAME[kern])
    got = dk.kde_exact(Xd, Yd, h, KNAME[kern], prec).cpu().numpy()
    err, excluded = rel_err(got, c1_exact[kern])
    print(f"exact {prec} {KNAME[kern]}: max rel {err.max():.3e} mean {err.mean():.3e} "
          f"excluded {excluded}")
    assert err.max() <= 1e-5


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("kern", [GAUSSIAN, EXPONENTIAL])
def test_exact_kde_low_precision_bound(c1, c1_exact, kern, prec):
    # Stated bound for 16-bit GEMM operands (8- or 11-bit significands):
    # mean relative error <= 1% at the workload bandwidth.
    import paper_2107_02736_amd as dk
    X, Y, Xd, Yd = c1
    h = bandwidth(WL, KNAME[kern])
    got = dk.kde_exact(Xd, Yd, h, KNAME[kern], prec).cpu().numpy()
    err, _ = rel_err(got, c1_exact[kern])
    print(f"exact {prec} {KNAME[kern]}: max rel {err.max():.3e} mean {err.mean():.3e}")
    assert err.mean() <= (1e-2 if prec == "bf16" else 2e-3)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_knn_bit_exact(c1, prec):
    import paper_2107_02736_amd as dk
    X, Y, Xd, Yd = c1
    k = 50
    _, nn, _ = dk.deann_query(Xd, Yd, 2.0, k, 0, "gaussian", precision=prec)
    nn = nn.cpu().numpy()
    for j in range(0, Y.shape[0], 3):
        assert np.array_equal(nn[j], oracle.knn(X, Y[j], k)), f"query {j}"


@pytest.mark.parametrize("kern", [GAUSSIAN, EXPONENTIAL])
def test_deann_estimate_and_samples(c1, kern):
    import paper_2107_02736_amd as dk
    X, Y, Xd, Yd = c1
    h = bandwidth(WL, KNAME[kern])
    k, m, seed = 50, 500, 0
    out, nn, sm = dk.deann_query(Xd, Yd, h, k, m, KNAME[kern], seed=seed)
    out, nn, sm = out.cpu().numpy(), nn.cpu().numpy(), sm.cpu().numpy()
    for j in range(0, Y.shape[0], 10):
        est, nn_ref, s_ref = oracle.deann_estimate(X, Y[j], h, kern, k, m, seed, j)
        assert np.array_equal(nn[j], nn_ref)
        assert np.array_equal(sm[j], s_ref)
        assert abs(out[j] - est) <= 1e-12 * est + 1e-300


def test_query_offset_reproduces_batch(c1):
    import paper_2107_02736_amd as dk
    X, Y, Xd, Yd = c1
    a = dk.deann_query(Xd, Yd[:300], 2.4, 50, 500, seed=9)
    b1 = dk.deann_query(Xd, Yd[:120].contiguous(), 2.4, 50, 500, seed=9)
    b2 = dk.deann_query(Xd, Yd[120:300].contiguous(), 2.4, 50, 500, seed=9, query_offset=120)
    for i in range(3):
        full = a[i].cpu()
        split = np.concatenate([b1[i].cpu().numpy(), b2[i].cpu().numpy()])
        assert np.array_equal(full.numpy(), split)


def test_determinism(c1):
    import paper_2107_02736_amd as dk
    X, Y, Xd, Yd = c1
    for prec in ("fp32", "bf16"):
        r1 = dk.deann_query(Xd, Yd, 2.4, 50, 500, seed=3, precision=prec)
        r2 = dk.deann_query(Xd, Yd, 2.4, 50, 500, seed=3, precision=prec)
        for a, b in zip(r1, r2):
            assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
        e1 = dk.kde_exact(Xd, Yd, 2.4, "gaussian", prec).cpu().numpy()
        e2 = dk.kde_exact(Xd, Yd, 2.4, "gaussian", prec).cpu().numpy()
        assert np.array_equal(e1, e2)


# --------------------------------------------------------------------------
# edge shapes and degenerate parameters
# --------------------------------------------------------------------------

def _small(n, q, d, seed=0):
    rng = np.random.default_rng(seed)
    cen = rng.uniform(-3, 3, size=(5, d))
    X = (cen[rng.integers(0, 5, n)] + rng.normal(size=(n, d))).astype(np.float32)
    Y = (cen[rng.integers(0, 5, q)] + rng.normal(size=(q, d))).astype(np.float32)
    return X, Y


@pytest.mark.parametrize("kern", [GAUSSIAN, EXPONENTIAL])
@pytest.mark.parametrize("n,q,d", [(1000, 37, 9), (129, 1, 3), (1, 5, 2), (300, 130, 33),
                                   (700, 50, 100), (500, 20, 128),
                                   # wider rows: the split engine of the generic tile kernel
                                   (300, 130, 129), (1000, 37, 300), (129, 3, 960),
                                   (2500, 140, 500), (1, 2, 200)])
def test_edge_shapes_split_exact(dev, n, q, d, kern):
    # the three-part bfloat16 form: every query within 1e-5, as the float32 path
    import paper_2107_02736_amd as dk
    X, Y = _small(n, q, d, seed=n + d)
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    h = 2.0 + 0.1 * d if kern == GAUSSIAN else 1.0 + 0.05 * d
    ref = oracle.kde_exact(X, Y, h, kern)
    got = dk.kde_exact(Xd, Yd, h, KNAME[kern], "fp32_split").cpu().numpy()
    err, _ = rel_err(got, ref)
    assert err.max() <= 1e-5, err.max()


def test_split_precision_width_limit(dev):
    # the split form of the adjoint and of the fused value + gradient pass
    # takes rows of at most 128 floats; kde_exact takes any width
    import paper_2107_02736_amd as dk
    X, Y = _small(200, 4, 129, seed=1)
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    with pytest.raises(dk.DeannError):
        dk.kde_exact_with_grad(Xd, Yd, 3.0, "gaussian", precision="fp32_split")
    got = dk.kde_exact(Xd, Yd, 3.0, "gaussian", "fp32_split").cpu().numpy()
    err, _ = rel_err(got, oracle.kde_exact(X, Y, 3.0, GAUSSIAN))
    assert err.max() <= 1e-5


@pytest.mark.parametrize("n,q,d", [(1000, 37, 9), (129, 1, 3), (1, 5, 2), (300, 130, 33),
                                   (2500, 64, 64), (3000, 200, 100)])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_edge_shapes_exact_and_knn(dev, n, q, d, prec):
    import paper_2107_02736_amd as dk
    X, Y = _small(n, q, d, seed=n + d)
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    h = 1.5
    ref = oracle.kde_exact(X, Y, h, GAUSSIAN)
    got = dk.kde_exact(Xd, Yd, h, "gaussian", prec).cpu().numpy()
    err, _ = rel_err(got, ref)
    keep = ref >= 1e-16
    if prec == "fp32":   # queries the certificate does not pass are re-evaluated exactly
        assert err.max() <= 1e-5, err.max()
    else:   # the derived per-query bound of the 16-bit operands
        assert np.all(err <= exact_kde_bound(bound_geometry(X, Y), d, h, GAUSSIAN, prec)[keep])
    k = min(n, 7)
    m = 11
    out, nn, sm = dk.deann_query(Xd, Yd, h, k, m, precision=prec, seed=1)
    out, nn, sm = out.cpu().numpy(), nn.cpu().numpy(), sm.cpu().numpy()
    for j in range(q):
        est, nn_ref, s_ref = oracle.deann_estimate(X, Y[j], h, GAUSSIAN, k, m, 1, j)
        assert np.array_equal(nn[j], nn_ref)
        assert np.array_equal(sm[j], s_ref)
        assert abs(out[j] - est) <= 1e-12 * max(est, 1e-300)


@pytest.mark.parametrize("k,m", [(0, 40), (10, 0), (0, 0), (400, 50), (395, 3000), (1, 1)])
def test_degenerate_k_m(dev, k, m):
    import paper_2107_02736_amd as dk
    X, Y = _small(400, 20, 5, seed=4)
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    h = 1.1
    out, nn, sm = dk.deann_query(Xd, Yd, h, k, m, "exponential", seed=2)
    out, nn, sm = out.cpu().numpy(), nn.cpu().numpy(), sm.cpu().numpy()
    for j in range(20):
        est, nn_ref, s_ref = oracle.deann_estimate(X, Y[j], h, EXPONENTIAL, k, m, 2, j)
        assert np.array_equal(nn[j], nn_ref)
        assert np.array_equal(sm[j], s_ref)
        assert abs(out[j] - est) <= 1e-12 * max(est, 1e-300)
    if k == 400:   # k = n is the exact KDE
        ref = oracle.kde_exact(X, Y, h, EXPONENTIAL)
        assert np.allclose(out, ref, rtol=1e-12, atol=0)


@pytest.mark.parametrize("d", [100])
@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_knn_bit_exact_256_byte_rows(dev, d, prec):
    # 16-bit rows of 256 bytes (64 < d <= 128) take the query-tile-in-LDS engine
    import paper_2107_02736_amd as dk
    X, Y = _small(5000, 150, d, seed=21)
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    k, m, h = 40, 50, 4.0
    out, nn, sm = (t.cpu().numpy() for t in dk.deann_query(Xd, Yd, h, k, m, "gaussian", seed=3,
                                                            precision=prec))
    for j in range(0, Y.shape[0], 7):
        est, nn_ref, s_ref = oracle.deann_estimate(X, Y[j], h, GAUSSIAN, k, m, 3, j)
        assert np.array_equal(nn[j], nn_ref), j
        assert np.array_equal(sm[j], s_ref), j
        assert abs(out[j] - est) <= 1e-12 * max(est, 1e-300)


@pytest.mark.parametrize("n,k", [(129, 100), (129, 128), (300, 120), (700, 250)])
@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_knn_more_neighbours_than_cells(dev, n, k, prec):
    # k above the number of 16-bit candidate cells (32 per data split): the
    # second pass runs with an infinite threshold and must still skip the
    # padding columns of the last data tile
    import paper_2107_02736_amd as dk
    X, Y = _small(n, 9, 5, seed=n + k)
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    h, m = 1.4, 37
    out, nn, sm = (t.cpu().numpy() for t in dk.deann_query(Xd, Yd, h, k, m, "gaussian", seed=5,
                                                            precision=prec))
    assert nn.max() < n and sm.max() < n
    for j in range(Y.shape[0]):
        est, nn_ref, s_ref = oracle.deann_estimate(X, Y[j], h, GAUSSIAN, k, m, 5, j)
        assert np.array_equal(nn[j], nn_ref), j
        assert np.array_equal(sm[j], s_ref), j
        assert abs(out[j] - est) <= 1e-12 * max(est, 1e-300)


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("nb", [1500, 2500])
def test_second_pass_heavy_and_light_queries(dev, prec, nb):
    # half the queries sit in a blob of nb nearly equal rows that 16-bit keys
    # cannot tell apart (every blob row passes the second-pass threshold, far
    # more hits per tile than a wave stages: the rest go straight to the
    # lists), the other half in sparse data with few hits; all must equal the
    # oracle's k-NN and estimate.  The second refinement's first launch takes
    # the light queries; the blob ones go to its full-capacity launch (1500:
    # the exact pairs exceed the first launch's 1024; 2500: the list exceeds
    # its 2048 keys)
    import paper_2107_02736_amd as dk
    rng = np.random.default_rng(31)
    d = 24
    P = rng.uniform(-1, 1, size=d)
    blob = P + 1e-3 * rng.normal(size=(nb, d))
    rest = 3.0 * rng.normal(size=(1500, d))
    X = np.concatenate([blob, rest])[rng.permutation(nb + 1500)].astype(np.float32)
    Y = np.concatenate([P + 1e-3 * rng.normal(size=(64, d)),
                        3.0 * rng.normal(size=(64, d))]).astype(np.float32)
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    k, m, h = 50, 40, 2.0
    out, nn, sm = (t.cpu().numpy() for t in dk.deann_query(Xd, Yd, h, k, m, "gaussian", seed=6,
                                                            precision=prec))
    for j in list(range(0, 64, 3)) + list(range(64, 128, 3)):
        est, nn_ref, s_ref = oracle.deann_estimate(X, Y[j], h, GAUSSIAN, k, m, 6, j)
        assert np.array_equal(nn[j], nn_ref), j
        assert np.array_equal(sm[j], s_ref), j
        assert abs(out[j] - est) <= 1e-12 * max(est, 1e-300)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_knn_exact_ties_and_duplicates(dev, prec):
    # integer lattice data: many exactly equal distances, duplicate rows
    import paper_2107_02736_amd as dk
    rng = np.random.default_rng(12)
    X = rng.integers(-2, 3, size=(700, 3)).astype(np.float32)
    Y = rng.integers(-2, 3, size=(30, 3)).astype(np.float32)
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    for k in (1, 9, 40):
        _, nn, _ = dk.deann_query(Xd, Yd, 1.0, k, 0, precision=prec)
        nn = nn.cpu().numpy()
        for j in range(30):
            assert np.array_equal(nn[j], oracle.knn(X, Y[j], k)), (k, j)


@pytest.mark.parametrize("kern", ["gaussian", "exponential"])
def test_extreme_bandwidths(dev, kern):
    # h -> infinity: every kernel value tends to 1 (both paths).  h -> 0: only
    # coincident points count, so a query equal to a data row gets 1/n: the
    # DEANN path evaluates its neighbours directly; the exact path's GEMM form
    # cannot resolve d^2 = 0 below its rounding of ||x||^2 + ||y||^2, so its
    # certificate sends that query to the exact re-evaluation.
    import paper_2107_02736_amd as dk
    X, Y = _small(500, 8, 4, seed=2)
    Y[0] = X[17]
    Y[3] = X[400]
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    big = dk.kde_exact(Xd, Yd, 1e6, kern).cpu().numpy()
    ref_big = oracle.kde_exact(X, Y, 1e6, KIDS[kern])   # 1 - O(r / h) for the exponential
    assert np.all(ref_big > 1.0 - 1e-5)
    assert np.allclose(big, ref_big, rtol=1e-6, atol=0)
    out, _, _ = dk.deann_query(Xd, Yd, 1e6, 3, 10, kern, seed=0)
    for j in range(Y.shape[0]):
        est, _, _ = oracle.deann_estimate(X, Y[j], 1e6, KIDS[kern], 3, 10, 0, j)
        assert out.cpu().numpy()[j] == pytest.approx(est, rel=1e-12)
    out, _, _ = dk.deann_query(Xd, Yd, 1e-4, 3, 10, kern, seed=0)
    assert out.cpu().numpy()[0] == pytest.approx(1.0 / 500, rel=1e-12)
    ref = oracle.kde_exact(X, Y, 1e-4, KIDS[kern])
    for prec in ("fp32", "fp32_split"):
        tiny = dk.kde_exact(Xd, Yd, 1e-4, kern, prec).cpu().numpy()
        assert tiny[0] == pytest.approx(1.0 / 500, rel=1e-6), prec
        assert tiny[3] == pytest.approx(1.0 / 500, rel=1e-6), prec
        # the other queries are far from every row: values far below 1e-16
        assert np.all(tiny[ref < 1e-16] < 1e-16)
        mu, gy, gh = dk.kde_exact_with_grad(Xd, Yd, 1e-4, kern, prec)
        assert mu.cpu().numpy()[0] == pytest.approx(1.0 / 500, rel=1e-6), prec
        # on a data row the gradient of that row's term is zero; the rest underflows
        assert np.all(np.abs(gy.cpu().numpy()[0]) <= 1e-30)


# --------------------------------------------------------------------------
# adjoints
# --------------------------------------------------------------------------

@pytest.mark.parametrize("d", [12, 300, 301])   # 16 lanes per row, a wave per row, generic
@pytest.mark.parametrize("kern", [GAUSSIAN, EXPONENTIAL])
def test_deann_backward_vs_oracle(dev, kern, d):
    import paper_2107_02736_amd as dk
    X, Y = _small(3000, 40, d, seed=7)
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    h, k, m = 1.3 * np.sqrt(d / 12), 16, 100   # comparable kernel values at every d
    out, nn, sm = dk.deann_query(Xd, Yd, h, k, m, KNAME[kern], seed=4)
    g = np.linspace(0.5, 1.5, 40)
    gy, gh = dk.deann_query_backward(Xd, Yd, h, k, m, nn, sm, to_dev(g, dev), KNAME[kern])
    gy, gh = gy.cpu().numpy(), float(gh.cpu().numpy()[0])
    nn, sm = nn.cpu().numpy(), sm.cpu().numpy()
    gh_ref = 0.0
    for j in range(40):
        _, gy_ref, ghj = oracle.deann_grad(X, Y[j], h, kern, nn[j], sm[j], m)
        assert np.linalg.norm(gy[j] - g[j] * gy_ref) <= 1e-6 * np.linalg.norm(g[j] * gy_ref) + 1e-30
        gh_ref += g[j] * ghj
    assert gh == pytest.approx(gh_ref, rel=1e-10)


@pytest.mark.parametrize("d", [12, 300, 301])   # fused (16 lanes, a wave per row), two gathers
@pytest.mark.parametrize("kern", [GAUSSIAN, EXPONENTIAL])
def test_deann_with_grad(dev, kern, d):
    # one gather for the estimate and its derivatives: the neighbours and draws
    # of deann_query, the gradient of deann_query_backward with unit upstream
    # gradient bit for bit, and the oracle's estimate and derivatives
    import paper_2107_02736_amd as dk
    X, Y = _small(3000, 40, d, seed=7)
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    h, k, m = 1.3 * np.sqrt(d / 12), 16, 100
    out, gy, gh, nn, sm = dk.deann_query_with_grad(Xd, Yd, h, k, m, KNAME[kern], seed=4,
                                                   query_offset=3, word2=5)
    out0, nn0, sm0 = dk.deann_query(Xd, Yd, h, k, m, KNAME[kern], seed=4, query_offset=3, word2=5)
    ones = to_dev(np.ones(40), dev)
    gy0, gh0 = dk.deann_query_backward(Xd, Yd, h, k, m, nn0, sm0, ones, KNAME[kern])
    assert np.array_equal(nn.cpu().numpy(), nn0.cpu().numpy())
    assert np.array_equal(sm.cpu().numpy(), sm0.cpu().numpy())
    assert np.array_equal(gy.cpu().numpy(), gy0.cpu().numpy())
    out, out0, gh = out.cpu().numpy(), out0.cpu().numpy(), gh.cpu().numpy()
    assert np.all(np.abs(out - out0) <= 1e-14 * out0)
    assert gh.sum() == pytest.approx(float(gh0.cpu().numpy()[0]), rel=1e-12)
    gy, nn, sm = gy.cpu().numpy(), nn.cpu().numpy(), sm.cpu().numpy()
    for j in range(40):
        est, gy_ref, gh_ref = oracle.deann_grad(X, Y[j], h, kern, nn[j], sm[j], m)
        assert abs(out[j] - est) <= 1e-12 * est, j
        assert np.linalg.norm(gy[j] - gy_ref) <= 1e-6 * np.linalg.norm(gy_ref) + 1e-30, j
        assert gh[j] == pytest.approx(gh_ref, rel=1e-10), j


@pytest.mark.parametrize("k,m", [(0, 64), (300, 64), (7, 0), (299, 64)])
def test_deann_with_grad_degenerate(dev, k, m):
    # plain random sampling (k = 0), the exact sum (k = n: no draws, sample
    # indices -1), neighbours only (m = 0), a single row left to draw from
    import paper_2107_02736_amd as dk
    X, Y = _small(300, 24, 32, seed=3)
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    h = 2.0
    out, gy, gh, nn, sm = dk.deann_query_with_grad(Xd, Yd, h, k, m, "gaussian", seed=9)
    out0, nn0, sm0 = dk.deann_query(Xd, Yd, h, k, m, "gaussian", seed=9)
    assert np.array_equal(nn.cpu().numpy(), nn0.cpu().numpy())
    assert np.array_equal(sm.cpu().numpy(), sm0.cpu().numpy())
    out, out0 = out.cpu().numpy(), out0.cpu().numpy()
    assert np.all(np.abs(out - out0) <= 1e-14 * out0)
    gy, gh, nn, sm = gy.cpu().numpy(), gh.cpu().numpy(), nn.cpu().numpy(), sm.cpu().numpy()
    for j in range(24):
        est, gy_ref, gh_ref = oracle.deann_grad(X, Y[j], h, GAUSSIAN, nn[j],
                                                sm[j] if k < 300 else sm[j][:0], m)
        assert abs(out[j] - est) <= 1e-12 * est, j
        assert np.linalg.norm(gy[j] - gy_ref) <= 1e-6 * np.linalg.norm(gy_ref) + 1e-30, j
        assert gh[j] == pytest.approx(gh_ref, rel=1e-10, abs=1e-300), j


@pytest.mark.parametrize("prec", ["fp32", "fp32_split"])
@pytest.mark.parametrize("kern", [GAUSSIAN, EXPONENTIAL])
def test_exact_backward_vs_oracle(dev, kern, prec):
    import paper_2107_02736_amd as dk
    X, Y = _small(6000, 70, 64, seed=9)
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    h = 6.0
    g = np.linspace(1.0, 2.0, 70)
    gy, gh = dk.kde_exact_backward(Xd, Yd, h, to_dev(g, dev), KNAME[kern], precision=prec)
    gy, gh = gy.cpu().numpy(), float(gh.cpu().numpy()[0])
    gh_ref, gh_scale = 0.0, 0.0
    for j in range(70):
        mu, gy_ref, ghj = oracle.kde_grad(X, Y[j].astype(np.float64), h, kern)
        d2 = oracle.sq_dists(X, Y[j])
        K = oracle.kernel_values(d2, h, kern)
        r = np.sqrt(d2)
        # normwise scale: the sum of the magnitudes of the terms of the gradient
        if kern == GAUSSIAN:
            scale = (K * r).sum() / (X.shape[0] * h * h)
        else:
            scale = K.sum() / (X.shape[0] * h)
        assert np.linalg.norm(gy[j] - g[j] * gy_ref) <= 1e-4 * g[j] * scale
        gh_ref += g[j] * ghj
        gh_scale += g[j] * abs(ghj)
    assert abs(gh - gh_ref) <= 1e-4 * gh_scale


@pytest.mark.parametrize("prec", ["fp32", "fp32_split"])
@pytest.mark.parametrize("d", [16, 64, 90, 128])
@pytest.mark.parametrize("kern", [GAUSSIAN, EXPONENTIAL])
def test_exact_value_and_gradient_in_one_pass(dev, kern, d, prec):
    # kde_exact_with_grad: the KDE, its y-gradient and its per-query h-derivative;
    # padded widths 32, 64, 96 and 128 (a trailing 32-coordinate block at 32 and
    # 96), with the distance product on float32 or three-part bfloat16 MFMAs
    import paper_2107_02736_amd as dk
    X, Y = _small(6000, 70, d, seed=9)
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    h = 6.0
    mu, gy, gh = (t.cpu().numpy() for t in dk.kde_exact_with_grad(Xd, Yd, h, KNAME[kern],
                                                                   precision=prec))
    mu_fwd = dk.kde_exact(Xd, Yd, h, KNAME[kern], prec).cpu().numpy()
    gy_bwd, _ = dk.kde_exact_backward(Xd, Yd, h, to_dev(np.ones(70), dev), KNAME[kern],
                                      precision=prec)
    assert np.allclose(gy, gy_bwd.cpu().numpy(), rtol=0, atol=0)   # same kernel, same order
    for j in range(70):
        mu_ref, gy_ref, gh_ref = oracle.kde_grad(X, Y[j].astype(np.float64), h, kern)
        assert abs(mu[j] - mu_ref) <= 1e-5 * mu_ref
        assert abs(mu[j] - mu_fwd[j]) <= 5e-6 * mu_ref
        d2 = oracle.sq_dists(X, Y[j])
        K = oracle.kernel_values(d2, h, kern)
        r = np.sqrt(d2)
        scale = (K * r).sum() / (X.shape[0] * h * h) if kern == GAUSSIAN else K.sum() / (X.shape[0] * h)
        assert np.linalg.norm(gy[j] - gy_ref) <= 1e-4 * scale
        hs = (K * d2).sum() / (X.shape[0] * h ** 3) if kern == GAUSSIAN else (K * r).sum() / (X.shape[0] * h * h)
        assert abs(gh[j] - gh_ref) <= 1e-4 * hs


def test_autograd_matches_finite_differences(dev):
    # DEANN with the index sets fixed: central differences of the GPU forward.
    import torch

    import paper_2107_02736_amd as dk
    X, Y = _small(2000, 6, 8, seed=3)
    Xd = to_dev(X, dev)
    h, k, m = 1.2, 12, 64
    Yr = to_dev(Y, dev).requires_grad_(True)
    hr = torch.tensor(h, dtype=torch.float64, requires_grad=True)
    out = dk.deann_kde(Yr, hr, Xd, k, m, seed=8)
    out.sum().backward()
    gy = Yr.grad.cpu().numpy()
    nn0 = dk.deann_query(Xd, to_dev(Y, dev), h, k, m, seed=8)[1].cpu().numpy()
    checked = 0
    for j in range(6):
        for t in range(8):
            step = 1e-3 * h
            yp, ym = Y.copy(), Y.copy()
            yp[j, t] += step
            ym[j, t] -= step
            dp = float(yp[j, t]) - float(Y[j, t])
            dm = float(Y[j, t]) - float(ym[j, t])
            rp = dk.deann_query(Xd, to_dev(yp, dev), h, k, m, seed=8)
            rm = dk.deann_query(Xd, to_dev(ym, dev), h, k, m, seed=8)
            if not (np.array_equal(rp[1].cpu().numpy()[j], nn0[j])
                    and np.array_equal(rm[1].cpu().numpy()[j], nn0[j])):
                continue   # the neighbour set moved: the estimate jumps there
            fd = (rp[0].cpu().numpy()[j] - rm[0].cpu().numpy()[j]) / (dp + dm)
            assert gy[j, t] == pytest.approx(fd, rel=2e-3, abs=1e-6 * abs(out[j].item()) / h)
            checked += 1
    assert checked >= 40
    fp = dk.deann_query(Xd, to_dev(Y, dev), h * (1 + 1e-4), k, m, seed=8)[0].cpu().numpy().sum()
    fm = dk.deann_query(Xd, to_dev(Y, dev), h * (1 - 1e-4), k, m, seed=8)[0].cpu().numpy().sum()
    assert hr.grad.item() == pytest.approx((fp - fm) / (2e-4 * h), rel=1e-4)


def test_mean_shift_matches_oracle(dev):
    import paper_2107_02736_amd as dk
    X, Y = _small(3000, 5, 6, seed=11)
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    h = 1.0
    ye = dk.mean_shift(Xd, Yd, h, 5, "exact").cpu().numpy()
    yd = dk.mean_shift(Xd, Yd, h, 5, "deann", k=20, m=100, seed=1).cpu().numpy()
    for j in range(5):
        ref_e = oracle.mean_shift_exact(X, Y[j], h, 5)
        assert np.allclose(ye[j], ref_e, rtol=1e-4, atol=1e-4)
        ref_d = oracle.mean_shift_deann(X, Y[j], h, 20, 100, 1, j, 5)
        assert np.allclose(yd[j], ref_d, rtol=1e-4, atol=1e-4)


# --------------------------------------------------------------------------
# largest supported shapes and empty batches
# --------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_maximum_k_and_d(dev, prec):
    # k = 496 (largest list size), d = 4096 (largest row for the query path),
    # the DEANN adjoint at its largest row (d = 2048), exact KDE at d = 4096
    import paper_2107_02736_amd as dk
    X, Y = _small(3000, 12, 4096, seed=41)
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    h, k, m = 40.0, 496, 64
    out, nn, sm = (t.cpu().numpy() for t in dk.deann_query(Xd, Yd, h, k, m, "gaussian", seed=9,
                                                            precision=prec))
    for j in range(0, 12, 3):
        est, nn_ref, s_ref = oracle.deann_estimate(X, Y[j], h, GAUSSIAN, k, m, 9, j)
        assert np.array_equal(nn[j], nn_ref), j
        assert np.array_equal(sm[j], s_ref), j
        assert abs(out[j] - est) <= 1e-12 * max(est, 1e-300)
    mu = dk.kde_exact(Xd, Yd, h, "gaussian", "fp32").cpu().numpy()
    ref = oracle.kde_exact(X, Y, h, GAUSSIAN)
    err, _ = rel_err(mu, ref)
    assert err.max() <= 1e-5, err.max()
    X2, Y2 = np.ascontiguousarray(X[:, :2048]), np.ascontiguousarray(Y[:, :2048])
    X2d, Y2d = to_dev(X2, dev), to_dev(Y2, dev)
    h2 = 28.0
    _, nn2, sm2 = dk.deann_query(X2d, Y2d, h2, 32, 100, "gaussian", seed=1, precision=prec)
    g = np.linspace(1.0, 2.0, 12)
    gy, _ = dk.deann_query_backward(X2d, Y2d, h2, 32, 100, nn2, sm2, to_dev(g, dev), "gaussian")
    gy, nn2, sm2 = gy.cpu().numpy(), nn2.cpu().numpy(), sm2.cpu().numpy()
    for j in range(0, 12, 4):
        _, gy_ref, _ = oracle.deann_grad(X2, Y2[j], h2, GAUSSIAN, nn2[j], sm2[j], 100)
        assert np.linalg.norm(gy[j] - g[j] * gy_ref) <= 1e-6 * np.linalg.norm(g[j] * gy_ref)


def test_empty_query_batches(dev):
    import torch
    import paper_2107_02736_amd as dk
    X, _ = _small(500, 1, 8, seed=2)
    Xd = to_dev(X, dev)
    Y0 = torch.empty((0, 8), dtype=torch.float32, device=dev)
    assert dk.kde_exact(Xd, Y0, 1.0, "gaussian").numel() == 0
    out, nn, sm = dk.deann_query(Xd, Y0, 1.0, 5, 7, precision="bf16")
    assert out.numel() == 0 and nn.shape == (0, 5) and sm.shape == (0, 7)
    out, nn, sm = dk.deann_query_permuted(Xd, Y0, 1.0, 5, 7)
    assert out.numel() == 0
    gy, _ = dk.deann_query_backward(Xd, Y0, 1.0, 5, 7, nn, sm,
                                    torch.empty(0, dtype=torch.float64, device=dev), "gaussian",
                                    True, False)
    assert gy.shape == (0, 8)
