"""Precision form of the small workload (10-cluster mixture, n = 10,000, d = 16,
q = 1,000): exact KDE with FP32, BF16 and FP16 operands of the distance GEMM
(FP32 accumulation), for both kernels at the workload bandwidth scaled by
0.25, 1 and 4, against the FP64 oracle; and DEANN with the 16-bit scans, whose
refined neighbour sets, draws and estimates must equal the FP32 scan's.

The error of every query is checked against a bound derived from the
arithmetic (first-order in the unit roundoffs, worst case over summation
orders):
  * operand rounding: x~ = fl_p(fl_32(x - c)) moves every point by at most
    e_x = (u_p + u_32) ||x - c||, so |d~ - d| <= E = e_x + e_y and
    |d~^2 - d^2| <= 2 d E + E^2;
  * dot product: FP32 accumulation of d_p products, at most
    2 gamma(d_p + 2) ||x~|| ||y~|| of d^2 (gamma(k) = k u / (1 - k u));
  * epilogue: 1.5 u_32 (||x~||^2 + ||y~||^2) of d^2 (norm term, add, FMA);
  * the kernel constant rounded to FP32 (and the square root of the
    exponential kernel): u_32 d^2 resp. 2 u_32 d in the exponent's units;
  * exp2 and the FP32 tile partial sums: 1e-6 relative.
With D the sum of the d^2 terms, a Gaussian term is off by at most a factor
exp((D + u_32 d^2) / (2 h^2)), an exponential one by
exp((min(sqrt(D), D / d) + 2 u_32 d) / h).  The
bound of a query is the kernel-weighted mean of those factors minus one, plus
the 1e-6.  The printed table is the precision report of this workload.
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
U32 = 2.0 ** -24
UNIT = {"fp32": 0.0, "bf16": 2.0 ** -8, "fp16": 2.0 ** -11}   # operand rounding beyond FP32
DPAD = {"fp32": 32, "bf16": 64, "fp16": 64}                   # padded row length
SCALES = (0.25, 1.0, 4.0)


@pytest.fixture(scope="module")
def data():
    dev = device()
    spec, X, Y = synth.workload(WL)
    return X, Y, to_dev(X, dev), to_dev(Y, dev)


@pytest.fixture(scope="module")
def geometry(data):
    X, Y, _, _ = data
    c = X.astype(np.float64).mean(axis=0)
    xn = np.sqrt(((X - c) ** 2).sum(1))              # ||x - c||
    yn = np.sqrt(((Y - c) ** 2).sum(1))
    d2 = np.stack([oracle.sq_dists(X, Y[j]) for j in range(Y.shape[0])])   # [q, n]
    return xn, yn, d2


def _bound(geometry, h, kern, prec):
    xn, yn, d2 = geometry
    up = UNIT[prec] + U32
    dp = DPAD[prec]
    gam = (dp + 2) * U32 / (1 - (dp + 2) * U32)
    xt, yt = xn * (1 + up), yn * (1 + up)              # bounds on ||x~||, ||y~||
    E = up * (xn[None, :] + yn[:, None])
    d = np.sqrt(d2)
    D = (2 * d * E + E * E + 2 * gam * xt[None, :] * yt[:, None]
         + 1.5 * U32 * (xt[None, :] ** 2 + yt[:, None] ** 2))
    if kern == GAUSSIAN:
        K = np.exp(-d2 / (2 * h * h))
        f = np.expm1((D + U32 * d2) / (2 * h * h))
    else:
        K = np.exp(-d / h)
        f = np.expm1((np.minimum(np.sqrt(D), D / np.maximum(d, 1e-300)) + 2 * U32 * d) / h)
    w = K.sum(1)
    with np.errstate(invalid="ignore", divide="ignore"):
        b = (K * f).sum(1) / w
    return b + 1e-6



@pytest.mark.parametrize("scale", SCALES)
@pytest.mark.parametrize("kern", [GAUSSIAN, EXPONENTIAL])
def test_precision_exact_and_deann(data, geometry, kern, scale):
    import paper_2107_02736_amd as dk
    X, Y, Xd, Yd = data
    h = scale * bandwidth(WL, KNAME[kern])
    ref = oracle.kde_exact(X, Y, h, kern)
    for prec in ("fp32", "bf16", "fp16"):
        got = dk.kde_exact(Xd, Yd, h, KNAME[kern], prec).cpu().numpy()
        err, excluded = rel_err(got, ref)
        keep = ref >= 1e-16
        bound = _bound(geometry, h, kern, prec)[keep]
        line = (f"{KNAME[kern]:11s} h x{scale:<4} {prec}: exact KDE rel err max {err.max():.2e} "
                f"mean {err.mean():.2e} (bound: max {bound.max():.2e} mean {bound.mean():.2e}; "
                f"{excluded} queries < 1e-16)")
        print(line)
        assert np.all(err <= bound), line
    # DEANN: the 16-bit scans reproduce the FP32 scan bit for bit
    k, m = 50, 500
    res = {p: [t.cpu().numpy() for t in dk.deann_query(Xd, Yd, h, k, m, KNAME[kern], seed=0,
                                                      precision=p)]
           for p in ("fp32", "bf16", "fp16")}
    for p in ("bf16", "fp16"):
        for a, b in zip(res[p], res["fp32"]):
            assert np.array_equal(a, b), p
    e, _ = rel_err(res["fp32"][0], ref)
    line = (f"{KNAME[kern]:11s} h x{scale:<4} DEANN k={k} m={m} (all precisions identical): "
            f"rel err vs exact mean {e.mean():.2e} median {np.median(e):.2e}")
    print(line)
    for j in range(0, Y.shape[0], 97):
        est, nn, s = oracle.deann_estimate(X, Y[j], h, kern, k, m, 0, j)
        assert np.array_equal(res["fp32"][1][j], nn) and np.array_equal(res["fp32"][2][j], s)
        assert abs(res["fp32"][0][j] - est) <= 1e-12 * max(est, 1e-300)
