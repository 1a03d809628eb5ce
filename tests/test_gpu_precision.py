"""Precision form of the small workload (10-cluster mixture, n = 10,000, d = 16,
q = 1,000): exact KDE with FP32, BF16 and FP16 operands of the distance GEMM
(FP32 accumulation) and with float32 operands split into three bfloat16 parts, for both kernels at the workload bandwidth scaled by
0.25, 1 and 4, against the FP64 oracle; and DEANN with the 16-bit scans, whose
refined neighbour sets, draws and estimates must equal the FP32 scan's.

The float32-operand forms (fp32, fp32_split) must be within 1e-5 of the
oracle for every query at every bandwidth: the queries their error
certificate does not pass are re-evaluated exactly.  The 16-bit forms are
checked against the bound derived from the arithmetic in
tests/precision_bound.py.  The printed table is the precision report of this
workload.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import GAUSSIAN, EXPONENTIAL

from .gpu_common import bandwidth, device, rel_err, to_dev
from .precision_bound import exact_kde_bound, geometry as bound_geometry

pytestmark = pytest.mark.gpu

WL = "mix10_n1e4_d16"
KNAME = {GAUSSIAN: "gaussian", EXPONENTIAL: "exponential"}
SCALES = (0.25, 1.0, 4.0)


@pytest.fixture(scope="module")
def data():
    dev = device()
    spec, X, Y = synth.workload(WL)
    return X, Y, to_dev(X, dev), to_dev(Y, dev)


@pytest.fixture(scope="module")
def geometry(data):
    X, Y, _, _ = data
    return bound_geometry(X, Y)


@pytest.mark.parametrize("scale", SCALES)
@pytest.mark.parametrize("kern", [GAUSSIAN, EXPONENTIAL])
def test_precision_exact_and_deann(data, geometry, kern, scale):
    import paper_2107_02736_amd as dk
    X, Y, Xd, Yd = data
    h = scale * bandwidth(WL, KNAME[kern])
    ref = oracle.kde_exact(X, Y, h, kern)
    for prec in ("fp32", "fp32_split", "bf16", "fp16"):
        got = dk.kde_exact(Xd, Yd, h, KNAME[kern], prec).cpu().numpy()
        err, excluded = rel_err(got, ref)
        keep = ref >= 1e-16
        bound = exact_kde_bound(geometry, X.shape[1], h, kern, prec)[keep]
        line = (f"{KNAME[kern]:11s} h x{scale:<4} {prec}: exact KDE rel err max {err.max():.2e} "
                f"mean {err.mean():.2e} (bound: max {bound.max():.2e} mean {bound.mean():.2e}; "
                f"{excluded} queries < 1e-16)")
        print(line)
        if prec in ("fp32", "fp32_split"):
            assert err.max() <= 1e-5, line
        else:
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
