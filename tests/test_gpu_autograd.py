"""torch.autograd paths of the exact KDE (ExactKDE: value, d/dy and d/dh,
Eq. (1)-(2) differentiated) against the oracle's analytic gradient and against
central differences (step 1e-3 h) of the GPU forward, and the bandwidth
bisection (Sec. 5) against the oracle's mean KDE."""
import numpy as np
import pytest

import oracle
import synth
from oracle import GAUSSIAN, EXPONENTIAL

from .gpu_common import bandwidth, device, to_dev

pytestmark = pytest.mark.gpu

KNAME = {GAUSSIAN: "gaussian", EXPONENTIAL: "exponential"}


@pytest.mark.parametrize("kern", [GAUSSIAN, EXPONENTIAL])
def test_exact_kde_autograd(kern):
    import torch

    import paper_2107_02736_amd as dk
    dev = device()
    spec, X, Y = synth.workload("mix50_n5e5_d64", n=20000, q=24)
    Xd = to_dev(X, dev)
    h0 = bandwidth("mix50_n5e5_d64", "gaussian") * (1.0 if kern == GAUSSIAN else 0.8)
    Yr = to_dev(Y, dev).requires_grad_(True)
    hr = torch.tensor(h0, dtype=torch.float64, requires_grad=True)
    w = torch.linspace(0.5, 1.5, Y.shape[0], dtype=torch.float64, device=dev)
    out = dk.exact_kde(Yr, hr, Xd, KNAME[kern])
    (out * w).sum().backward()
    gy = Yr.grad.cpu().numpy()
    gh = float(hr.grad)
    wn = w.cpu().numpy()
    mu = out.detach().cpu().numpy()
    gh_ref = gh_abs = 0.0
    for j in range(Y.shape[0]):
        mu_ref, gy_ref, ghj = oracle.kde_grad(X, Y[j].astype(np.float64), h0, kern)
        assert abs(mu[j] - mu_ref) <= 1e-5 * mu_ref, j
        d2 = oracle.sq_dists(X, Y[j])
        K = oracle.kernel_values(d2, h0, kern)
        r = np.sqrt(d2)
        if kern == GAUSSIAN:
            sy, sh = (K * r).sum() / (X.shape[0] * h0 ** 2), (K * d2).sum() / (X.shape[0] * h0 ** 3)
        else:
            sy, sh = K.sum() / (X.shape[0] * h0), (K * r).sum() / (X.shape[0] * h0 ** 2)
        assert np.linalg.norm(gy[j] - wn[j] * gy_ref) <= 1e-4 * wn[j] * sy, j
        gh_ref += wn[j] * ghj
        gh_abs += wn[j] * sh
    assert abs(gh - gh_ref) <= 1e-4 * gh_abs

    # central differences of the GPU forward: h, and y along a random direction
    eps = 1e-3 * h0
    with torch.no_grad():
        up = (dk.exact_kde(Yr.detach(), h0 + eps, Xd, KNAME[kern]) * w).sum().item()
        dn = (dk.exact_kde(Yr.detach(), h0 - eps, Xd, KNAME[kern]) * w).sum().item()
    fd_h = (up - dn) / (2 * eps)
    assert abs(fd_h - gh) <= 2e-3 * abs(gh)
    rng = np.random.default_rng(4)
    for j in range(0, Y.shape[0], 6):
        v = rng.standard_normal(Y.shape[1])
        v /= np.linalg.norm(v)
        yp = (Y[j] + eps * v).astype(np.float32)
        ym = (Y[j] - eps * v).astype(np.float32)
        step = (yp.astype(np.float64) - ym.astype(np.float64))   # the float32 step taken
        pair = to_dev(np.stack([yp, ym]), dev)
        with torch.no_grad():
            fp, fm = dk.exact_kde(pair, h0, Xd, KNAME[kern]).cpu().numpy()
        fd = fp - fm
        an = float(gy[j].astype(np.float64) @ step) / wn[j]
        assert abs(fd - an) <= 2e-3 * max(abs(an), 1e-3 * np.linalg.norm(gy[j]) / wn[j] *
                                          np.linalg.norm(step)), j


@pytest.mark.parametrize("kern", [GAUSSIAN, EXPONENTIAL])
def test_bisect_h_hits_the_target(kern):
    import paper_2107_02736_amd as dk
    dev = device()
    spec, X, Y = synth.workload("mix10_n1e4_d16", q=200)
    Xd, Yd = to_dev(X, dev), to_dev(Y, dev)
    target = 1e-2
    h = dk.bisect_h(Xd, Yd, target, KNAME[kern], rel_tol=0.01)
    mean = oracle.kde_exact(X, Y, h, kern).mean()
    print(f"{KNAME[kern]}: h = {h:.6g}, oracle mean KDE {mean:.6g}")
    assert abs(mean - target) <= 0.0101 * target
    # the median statistic (the paper's target) as well
    h_med = dk.bisect_h(Xd, Yd, target, KNAME[kern], stat="median", rel_tol=0.01)
    med = np.median(oracle.kde_exact(X, Y, h_med, kern))
    assert abs(med - target) <= 0.0101 * target
