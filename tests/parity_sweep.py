"""Large parity sweep (not collected by pytest; run on a GPU host):

    python tests/parity_sweep.py --workload mix100_n1e6_d128 --queries 500

Runs the GPU path once on the whole workload (exact KDE in FP32, for d <= 128
also the exact KDE with its gradient in one pass, DEANN with the given scan
precision, DEANN adjoint) and checks a fixed random subset of
queries against the FP64 oracle, computed in spawned processes (one per host
core, at most 16, fewer when the data is large).  Prints one JSON summary:
neighbour sets and draws must be bit-identical, DEANN estimates within 1e-12,
FP32 exact KDE within 1e-5, the DEANN adjoint within 1e-6 (normwise) and the
exact gradient within 1e-4 of the normwise scale sum K |x - y| / (n h^2)
(Gaussian) or sum K / (n h) (exponential).  For d <= 128 the float32-split
forms of both exact calls meet the same bars, and the near/far exact KDE
(BF16, the same k) has the oracle's neighbour sets and stays within the
16-bit bound of tests/precision_bound.py without the neighbours' terms."""
import argparse
import concurrent.futures as cf
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _oracle_queries(workload, kern, h, k, m, queries, with_grad):
    import numpy as np

    import oracle
    import synth
    from tests.precision_bound import exact_kde_bound
    spec, X, Y = synth.workload(workload)
    c = X.astype(np.float64).mean(axis=0)
    xn = np.sqrt(((X - c) ** 2).sum(1))
    out = []
    for j in queries:
        if with_grad:   # the exact KDE with its y-gradient and the normwise scale
            mu, gye, _ = oracle.kde_grad(X, Y[j].astype(np.float64), h, kern)
            d2 = oracle.sq_dists(X, Y[j])
            K = oracle.kernel_values(d2, h, kern)
            scale = ((K * np.sqrt(d2)).sum() / (X.shape[0] * h * h) if kern == oracle.GAUSSIAN
                     else K.sum() / (X.shape[0] * h))
        else:
            mu, gye, scale = oracle.kde_exact(X, Y[j:j + 1], h, kern)[0], None, None
        est, nn, s = oracle.deann_estimate(X, Y[j], h, kern, k, m, 0, int(j))
        _, gy, _ = oracle.deann_grad(X, Y[j], h, kern, nn, s, m)
        geo = (xn, np.sqrt(((Y[j:j + 1] - c) ** 2).sum(1)), oracle.sq_dists(X, Y[j])[None, :])
        hb = float(exact_kde_bound(geo, X.shape[1], h, kern, "bf16", near=[nn])[0])
        out.append((int(j), float(mu), float(est), np.asarray(nn), np.asarray(s), np.asarray(gy),
                    gye, scale, hb))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="mix100_n1e6_d128")
    ap.add_argument("--queries", type=int, default=500)
    ap.add_argument("--kernel", default="gaussian", choices=["gaussian", "exponential"])
    ap.add_argument("--k", type=int, default=100)
    ap.add_argument("--m", type=int, default=1000)
    ap.add_argument("--precision", default="bf16")
    args = ap.parse_args()

    import numpy as np
    import torch

    import oracle
    import paper_2107_02736_amd as dk
    import synth

    with open(os.path.join(ROOT, "tests", "golden", "bandwidths.json")) as f:
        h = float(json.load(f)[args.workload][args.kernel]["h"])
    kern = oracle.GAUSSIAN if args.kernel == "gaussian" else oracle.EXPONENTIAL
    spec, X, Y = synth.workload(args.workload)
    dev = torch.device("cuda:0")
    Xd, Yd = torch.from_numpy(X).to(dev), torch.from_numpy(Y).to(dev)
    mu = dk.kde_exact(Xd, Yd, h, args.kernel, "fp32").cpu().numpy()
    with_grad = X.shape[1] <= 128   # the fused exact value + gradient kernel
    if with_grad:
        mu_g, gy_e, _ = (t.cpu().numpy() for t in dk.kde_exact_with_grad(Xd, Yd, h, args.kernel))
        mu_s = dk.kde_exact(Xd, Yd, h, args.kernel, "fp32_split").cpu().numpy()
        mu_gs, gy_s, _ = (t.cpu().numpy() for t in dk.kde_exact_with_grad(
            Xd, Yd, h, args.kernel, precision="fp32_split"))
    mu_h, nn_h = (t.cpu().numpy() for t in dk.kde_hybrid(Xd, Yd, h, args.k, args.kernel, "bf16",
                                                          return_indices=True))
    est, nn, sm = dk.deann_query(Xd, Yd, h, args.k, args.m, args.kernel, seed=0,
                                 precision=args.precision)
    g = torch.ones(Y.shape[0], dtype=torch.float64, device=dev)
    gy, _ = dk.deann_query_backward(Xd, Yd, h, args.k, args.m, nn, sm, g, args.kernel)
    est, nn, sm, gy = (t.cpu().numpy() for t in (est, nn, sm, gy))

    sub = [int(j) for j in synth.query_subset(Y.shape[0], args.queries, seed=23)]
    workers = max(1, min(16, os.cpu_count() or 1, int(150e9 // (5 * X.nbytes))))
    shards = [sub[w::workers] for w in range(workers)]
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        parts = list(ex.map(_oracle_queries, [args.workload] * workers, [kern] * workers,
                            [h] * workers, [args.k] * workers, [args.m] * workers, shards,
                            [with_grad] * workers))
    t_oracle = time.perf_counter() - t0
    nn_bad, s_bad, e_exact, e_est, e_gy, excluded, gy_tiny, e_abs = 0, 0, [], [], [], 0, 0, 0.0
    e_fused, e_egrad, e_split, e_sgrad, hyb_nn_bad, hyb_over, e_hyb = [], [], [], [], 0, 0, []
    for part in parts:
        for j, mu_r, est_r, nn_r, s_r, gy_r, gye_r, scale, hb in part:
            # below a KDE of 1e-16 the FP32 kernel values underflow: such queries
            # are excluded from relative errors (as for the exact KDE)
            if with_grad and mu_r >= 1e-16:
                e_fused.append(abs(mu_g[j] - mu_r) / mu_r)
                e_egrad.append(float(np.linalg.norm(gy_e[j] - gye_r) / scale))
                e_split.append(max(abs(mu_s[j] - mu_r), abs(mu_gs[j] - mu_r)) / mu_r)
                e_sgrad.append(float(np.linalg.norm(gy_s[j] - gye_r) / scale))
            hyb_nn_bad += not np.array_equal(nn_h[j], nn_r)
            if mu_r >= 1e-16:
                eh = abs(mu_h[j] - mu_r) / mu_r
                e_hyb.append(eh)
                hyb_over += int(eh > hb)
            nn_bad += not np.array_equal(nn[j], nn_r)
            s_bad += not np.array_equal(sm[j], s_r)
            if mu_r >= 1e-16:
                e_exact.append(abs(mu[j] - mu_r) / mu_r)
            else:
                excluded += 1
            if est_r > 0:
                e_est.append(abs(est[j] - est_r) / est_r)
            nrm = np.linalg.norm(gy_r)
            if nrm >= 1e-30:   # grad_Y is float32: smaller gradients underflow
                e_gy.append(float(np.linalg.norm(gy[j] - gy_r) / nrm))
            else:
                gy_tiny += 1
                e_abs = max(e_abs, float(np.linalg.norm(gy[j] - gy_r)))
    res = {"workload": args.workload, "kernel": args.kernel, "k": args.k, "m": args.m,
           "scan_precision": args.precision, "queries": len(sub),
           "nn_mismatches": nn_bad, "sample_mismatches": s_bad,
           "exact_fp32_max_rel": max(e_exact) if e_exact else None,
           "exact_excluded_below_1e-16": excluded,
           "deann_max_rel": max(e_est) if e_est else None,
           "deann_grad_y_max_rel": max(e_gy) if e_gy else None,
           "deann_grad_y_below_1e-30": gy_tiny, "deann_grad_y_max_abs_there": e_abs,
           "exact_with_grad_value_max_rel": max(e_fused) if e_fused else None,
           "exact_grad_y_max_err_normwise": max(e_egrad) if e_egrad else None,
           "split_exact_max_rel": max(e_split) if e_split else None,
           "split_grad_y_max_err_normwise": max(e_sgrad) if e_sgrad else None,
           "near_far_nn_mismatches": hyb_nn_bad, "near_far_over_bound": hyb_over,
           "near_far_bf16_max_rel": max(e_hyb) if e_hyb else None,
           "oracle_processes": workers, "oracle_seconds": t_oracle}
    res["pass"] = bool(nn_bad == 0 and s_bad == 0 and (not e_exact or max(e_exact) <= 1e-5)
                       and (not e_est or max(e_est) <= 1e-12) and (not e_gy or max(e_gy) <= 1e-6)
                       and e_abs <= 1e-30 and (not e_fused or max(e_fused) <= 1e-5)
                       and (not e_egrad or max(e_egrad) <= 1e-4)
                       and (not e_split or max(e_split) <= 1e-5)
                       and (not e_sgrad or max(e_sgrad) <= 1e-4)
                       and hyb_nn_bad == 0 and hyb_over == 0)
    print(json.dumps(res), flush=True)
    sys.exit(0 if res["pass"] else 1)


if __name__ == "__main__":
    main()
