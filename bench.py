"""Benchmark of DEANN's query path on one MI355X.

One step = the whole hot path over one batch of queries:
  exact KDE (float32 MFMA tiles, certified per query)      kde_exact
    (d <= 128: with its gradient in one pass, d/dy, d/dh)   kde_exact_with_grad
  DEANN estimate with the BF16 scan + FP64 refinement,     deann_query_with_grad
    and its d/dy, d/dh from the same gather of the k + m rows
The headline workload is the large high-dimensional one: the 200-cluster
mixture with non-negative entries, n = 1,000,000, d = 960, q = 10,000,
Gaussian kernel, k = 200, m = 2,000; the 100-cluster mixture with n =
1,000,000, d = 128, q = 10,000 (k = 100, m = 1,000) follows as a secondary
block.  Inputs are resident in HBM before the timed region.  Also measured,
outside the step: the DEANN estimate alone with the BF16 scan and with the FP32
scan (the metric's comparison: same indices and estimates), the DEANN adjoint
alone (deann_query_backward), the exact KDE alone (its own roofline),
permuted-sampling and inverted-file DEANN, the BF16 exact KDE and the near/far
form.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-secondary]
                    [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("queries/s at ≤1% rel KDE err, BF16+refine vs FP32; exact KDE % MFMA peak")
WORKLOAD = "mix200_n1e6_d960"
SECONDARY = "mix100_n1e6_d128"
KERNEL = "gaussian"
MEAN_SHIFT_STEPS = 20
# (k, m) per workload; the default line is the 100-cluster mixture, the others
# are for separate runs with --workload
KM = {"mix100_n1e6_d128": (100, 1000), "mix10_n1e4_d16": (50, 500),
      "mix50_n5e5_d64": (64, 512), "mix200_n1e6_d960": (200, 2000)}
PEAK_FP32_MFMA = 157.3e12     # dense FP32 matrix, MI355X
PEAK_BF16_MFMA = 2.5e15
PEAK_HBM = 8.0e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=WORKLOAD)
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the secondary workload block")
    ap.add_argument("--step-only", action="store_true",
                    help="time the step and the exact KDE alone only (for profiler runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--all-cores", action="store_true",
                    help="also time the oracle in one process per host core")
    ap.add_argument("--cpu-sample", type=int, default=None,
                    help="queries in the oracle sample (default: about 20 s of oracle work)")
    ap.add_argument("--sweep-km", action="store_true",
                    help="only run DEANN (BF16 scan + refinement) over a (k, m) grid and print its "
                         "error against the exact KDE and its queries/s")
    ap.add_argument("--sweep-ivf", action="store_true",
                    help="print recall, error and queries/s of the inverted-file DEANN over "
                         "cluster counts and inspected clusters, then exit")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a device-to-device copy of 1 GiB (counter calibration)")
    ap.add_argument("--ceilings", action="store_true",
                    help="only measure the access patterns of the hot kernels without their "
                         "arithmetic (libdeann_ceiling.so) and a library BF16 GEMM, then exit")
    return ap.parse_args()


def calibrate_copy():
    """A plain copy of known size: 1 GiB read + 1 GiB written per launch, three
    launches.  Its FETCH_SIZE / WRITE_SIZE counters scale the hot kernels'."""
    import torch
    dev = torch.device("cuda:0")
    src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": src.numel() * 4, "launches": 3}))


def ceilings():
    """What the hot kernels' own data movement reaches with their arithmetic
    taken out, at the shapes of the two full-size workloads (random data):
    random-row gathers of k + m rows per query as in the DEANN gather, and the
    16-bit tile sweep of the k-NN passes with no epilogue; beside them a library
    BF16 GEMM (torch.matmul) at the same inner dimension."""
    import ctypes
    import torch
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2107_02736_amd", "libdeann_ceiling.so"))
    i64, vp = ctypes.c_int64, ctypes.c_void_p
    lib.ceiling_gather.restype = ctypes.c_int
    lib.ceiling_gather.argtypes = [vp, i64, i64, vp, i64, i64, vp, vp]
    lib.ceiling_tile_sweep.restype = ctypes.c_int
    lib.ceiling_tile_sweep.argtypes = [vp, i64, vp, i64, i64, i64, i64, vp, vp]
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev).cuda_stream
    gen = torch.Generator(device=dev)
    gen.manual_seed(0)
    n, q = 1_000_000, 10_000

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        b.synchronize()
        return a.elapsed_time(b) / reps

    res = {}
    for d, (k, m) in ((960, KM["mix200_n1e6_d960"]), (128, KM["mix100_n1e6_d128"])):
        X = torch.randn((n, d), device=dev, generator=gen)
        idx = torch.randint(0, n, (q, k + m), device=dev, dtype=torch.int32, generator=gen)
        out = torch.empty(q * 256, device=dev)

        def gather():
            st = lib.ceiling_gather(X.data_ptr(), n, d, idx.data_ptr(), q, k + m, out.data_ptr(),
                                    stream)
            if st != 0:
                raise RuntimeError(f"ceiling_gather: hipError {st}")
        ms = timed(gather)
        gb = q * (k + m) * d * 4
        res[f"gather_d{d}"] = {"rows_per_query": k + m, "ms": round(ms, 4),
                               "TB_per_s": round(gb / ms / 1e9, 3),
                               "frac_hbm": round(gb / ms / 1e9 / (PEAK_HBM / 1e12), 3)}
        del X, idx
        qp, np_, dp = (q + 127) // 128 * 128, (n + 127) // 128 * 128, (d + 63) // 64 * 64
        Ys = torch.randn((qp, dp), device=dev, generator=gen).to(torch.bfloat16)
        Xs = torch.randn((np_, dp), device=dev, generator=gen).to(torch.bfloat16)

        def sweep():
            st = lib.ceiling_tile_sweep(Ys.data_ptr(), qp, Xs.data_ptr(), np_, dp, 4096, 0,
                                        out.data_ptr(), stream)
            if st != 0:
                raise RuntimeError(f"ceiling_tile_sweep: hipError {st}")
        ms = timed(sweep, reps=3)
        fl = 2.0 * n * q * d
        res[f"bf16_tile_sweep_d{d}"] = {"ms": round(ms, 3), "TFLOP_per_s": round(fl / ms / 1e9, 1),
                                        "frac_bf16": round(fl / ms / 1e9 / (PEAK_BF16_MFMA / 1e12), 3)}
        del Xs
        B = torch.randn((262144, d), device=dev, generator=gen).to(torch.bfloat16)
        A = Ys[:q, :d].contiguous()
        ms = timed(lambda: torch.matmul(A, B.t()), reps=3)
        fl = 2.0 * q * 262144 * d
        res[f"library_bf16_gemm_k{d}"] = {"shape": [q, 262144, d], "ms": round(ms, 3),
                                          "TFLOP_per_s": round(fl / ms / 1e9, 1),
                                          "frac_bf16": round(fl / ms / 1e9 / (PEAK_BF16_MFMA / 1e12), 3)}
        del A, B, Ys
        torch.cuda.empty_cache()
    print(json.dumps({"ceilings": res, "n": n, "q": q, "data": "synthetic random"}))


def counters_path(workload):
    return os.path.join(ROOT, "profiles", f"counters_{workload}.json")


def kernel_sources_sha(names):
    import hashlib
    h = hashlib.sha256()
    for nm in names:
        with open(os.path.join(ROOT, "paper_2107_02736_amd", "csrc", nm), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    FETCH_SIZE / WRITE_SIZE counter runs, scaled by the same counters for a copy
    of known size; None when the kernel's sources changed after the counters
    were taken."""
    try:
        with open(counters_path(workload)) as f:
            rec = json.load(f)
        k = rec["kernels"][kernel]
        if kernel_sources_sha(k["sources"]) != k["sources_sha256"]:
            return None
        cal = rec["copy_calibration"]
        fetch = k["FETCH_SIZE_kb"] * cal["bytes_per_launch"] / cal["FETCH_SIZE_kb"]
        write = k["WRITE_SIZE_kb"] * cal["bytes_per_launch"] / cal["WRITE_SIZE_kb"]
        return fetch + write
    except (OSError, KeyError, ValueError):
        return None


def bandwidth(workload, kernel):
    with open(os.path.join(ROOT, "tests", "golden", "bandwidths.json")) as f:
        return float(json.load(f)[workload][kernel]["h"])


def ivf_config(n):
    """Inverted-file parameters: about sqrt(n)/4 clusters (256 at n = 10^6, the best
    recall per time of the cluster-count sweep there), 8 inspected, 4 Lloyd steps."""
    n_clusters = max(1, min(8192, int(round(math.sqrt(n) / 4))))
    return n_clusters, min(8, n_clusters), 4


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.ceilings:
        ceilings()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the query path needs no communication "
              "(queries shard with query_offset); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.sweep_km or args.sweep_ivf:
        import synth
        spec, X, Y = synth.workload(args.workload)
        h = bandwidth(args.workload, KERNEL)
        if args.sweep_km:
            sweep_km(args, X, Y, h)
        else:
            sweep_ivf(args, X, Y, h, *KM[args.workload])
        return
    import torch
    if args.step_only:
        print(json.dumps(run_workload(args, args.workload, with_cpu=False)), flush=True)
        return
    prim = run_workload(args, args.workload, with_cpu=not args.no_cpu_baseline)
    sec = None
    if not args.no_secondary and args.workload != SECONDARY:
        torch.cuda.empty_cache()
        sec = run_workload(args, SECONDARY, with_cpu=False)
    qps = prim["queries_per_s"]
    out = {
        "metric": METRIC,
        "value": qps["step"],
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": prim["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16 scan + f32 exact tiles + f64 refine/reductions",
        "data": "synthetic",
        "config": prim["config"],
        # the metric's comparison on the same workload: DEANN with the BF16 scan +
        # FP64 refinement against DEANN with the FP32 scan (identical indices,
        # hence estimates), and the exact KDE's fraction of the FP32 MFMA peak
        "deann_bf16_refine_queries_per_s": qps["deann_bf16_refine"],
        "deann_fp32_queries_per_s": qps["deann_fp32"],
        "deann_bf16_refine_speedup_vs_fp32": qps["deann_bf16_refine"] / qps["deann_fp32"],
        "deann_bf16_vs_fp32_same_indices": prim["accuracy"]["deann_bf16_vs_fp32_same_indices"],
        "deann_bf16_vs_fp32_max_rel": prim["accuracy"]["deann_bf16_vs_fp32_max_rel"],
        "exact_kde_mfma_frac": prim["roofline_exact_kde"]["frac"],
        "roofline": prim["roofline"],
    }
    for key in ("cpu_baseline", "cpu_baseline_all_cores", "parity_sample"):
        if key in prim:
            out[key] = prim.pop(key)
    for key in ("metric", "value", "ms_per_step", "config", "roofline"):
        prim.pop(key, None)
    out["detail"] = prim
    if sec is not None:
        out["secondary"] = sec
    print(json.dumps(out), flush=True)


def run_workload(args, workload, with_cpu):
    """One workload: the timed steps, the measurements outside the step and, with
    with_cpu, the oracle baseline and parity sample.  Returns a dict."""
    import numpy as np
    import torch

    import paper_2107_02736_amd as dk
    import synth

    dev = torch.device("cuda:0")
    t0 = time.time()
    spec, X, Y = synth.workload(workload)
    h = bandwidth(workload, KERNEL)
    K_NN, M_SAMPLES = KM[workload]
    n, d = X.shape
    q = Y.shape[0]
    Xd = torch.from_numpy(X).to(dev)
    Yd = torch.from_numpy(Y).to(dev)
    gout = torch.ones(q, dtype=torch.float64, device=dev)
    print(f"# {workload}: data {time.time() - t0:.1f}s  n={n} d={d} q={q} h={h:.6g}",
          file=sys.stderr, flush=True)

    def ev():
        return torch.cuda.Event(enable_timing=True)

    # exact KDE and its gradient from one pass over the distance tiles (the
    # fused entry point supports d <= 128; above, the step has the KDE only)
    fused = d <= 128
    comp = {"exact_kde_and_grad_fp32" if fused else "exact_kde_fp32": [],
            "deann_bf16_with_grad": []}

    def step(record):
        e = [ev() for _ in range(3)]
        e[0].record()
        if fused:
            mu, gye, ghe = dk.kde_exact_with_grad(Xd, Yd, h, KERNEL)
        else:
            mu, gye, ghe = dk.kde_exact(Xd, Yd, h, KERNEL, "fp32"), None, None
        e[1].record()
        est, gy, gh, nn, sm = dk.deann_query_with_grad(Xd, Yd, h, K_NN, M_SAMPLES, KERNEL, seed=0,
                                                       precision="bf16")
        e[2].record()
        if record is not None:
            record.append(e)
        return mu, est, nn, sm, gy, gh, gye, ghe

    for _ in range(args.warmup):
        step(None)
    torch.cuda.synchronize()
    events = []
    dk.kernel_timing(args.steps)     # events around the dense tile kernels
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        res = step(events)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    step_tile_ms = dk.kernel_times("kde_exact_backward" if fused else "kde_exact")
    dk.kernel_timing(0)
    names = list(comp)
    for e in events:
        for i, name in enumerate(names):
            comp[name].append(e[i].elapsed_time(e[i + 1]))
    ms_step = wall * 1e3 / args.steps
    comp_ms = {k: float(np.mean(v)) for k, v in comp.items()}

    # the exact KDE alone (forward tiles only), outside the step: its own roofline
    reps = max(2, args.steps // 2)
    dk.kde_exact(Xd, Yd, h, KERNEL, "fp32")
    torch.cuda.synchronize()
    dk.kernel_timing(reps)
    a, b = ev(), ev()
    a.record()
    for _ in range(reps):
        mu_fwd = dk.kde_exact(Xd, Yd, h, KERNEL, "fp32")
    b.record()
    torch.cuda.synchronize()
    ms_exact_fwd = a.elapsed_time(b) / reps
    tile_ms = dk.kernel_times("kde_exact")
    dk.kernel_timing(0)
    mu, est, nn, sm, gy, gh, gye, ghe = res
    if args.step_only:
        tile_avg = float(np.mean(tile_ms))
        return {"value": q / (ms_step * 1e-3), "ms_per_step": ms_step,
                "config": {"workload": workload, "n": n, "d": d, "q": q, "k": K_NN,
                           "m": M_SAMPLES},
                "components_ms": {k: float(np.mean(v)) for k, v in comp.items()},
                "exact_kde_tile_ms": tile_avg,
                "step_tile_ms": float(np.mean(step_tile_ms)) if step_tile_ms else None,
                "queries_per_s": {"step": q / (ms_step * 1e-3)}}

    # the DEANN estimate alone (BF16 scan + refinement) and its adjoint alone
    for _ in range(max(1, args.warmup)):
        est16, nn16, sm16 = dk.deann_query(Xd, Yd, h, K_NN, M_SAMPLES, KERNEL, seed=0,
                                           precision="bf16")
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        est16, nn16, sm16 = dk.deann_query(Xd, Yd, h, K_NN, M_SAMPLES, KERNEL, seed=0,
                                           precision="bf16")
    b.record()
    torch.cuda.synchronize()
    ms_deann16 = a.elapsed_time(b) / reps
    same_as_step = bool(torch.equal(nn16, nn) and torch.equal(sm16, sm))
    step_vs_alone = float(((est - est16).abs() / est16).max())
    dk.deann_query_backward(Xd, Yd, h, K_NN, M_SAMPLES, nn16, sm16, gout, KERNEL)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        gy16, _ = dk.deann_query_backward(Xd, Yd, h, K_NN, M_SAMPLES, nn16, sm16, gout, KERNEL)
    b.record()
    torch.cuda.synchronize()
    ms_bwd = a.elapsed_time(b) / reps
    same_grad_as_step = bool(torch.equal(gy16, gy))

    # FP32-scan DEANN for the BF16+refine vs FP32 comparison (same seed)
    for _ in range(max(1, args.warmup)):
        est32, nn32, sm32 = dk.deann_query(Xd, Yd, h, K_NN, M_SAMPLES, KERNEL, seed=0,
                                           precision="fp32")
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        est32, nn32, sm32 = dk.deann_query(Xd, Yd, h, K_NN, M_SAMPLES, KERNEL, seed=0,
                                           precision="fp32")
    b.record()
    torch.cuda.synchronize()
    ms_deann32 = a.elapsed_time(b) / reps

    # DEANN with permuted random sampling (App. G), BF16 scan (not part of the step)
    estp = dk.deann_query_permuted(Xd, Yd, h, K_NN, M_SAMPLES, KERNEL, seed=0, start=0,
                                   precision="bf16")[0]
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        estp = dk.deann_query_permuted(Xd, Yd, h, K_NN, M_SAMPLES, KERNEL, seed=0, start=0,
                                       precision="bf16")[0]
    b.record()
    torch.cuda.synchronize()
    ms_deannp = a.elapsed_time(b) / reps

    # the same with Algorithm 2's preprocessing: the permuted copy of X built
    # once, each query's block read contiguously from it (same rows, same estimates)
    torch.cuda.synchronize()
    t0p = time.perf_counter()
    pidx = dk.PermutedIndex(Xd, seed=0)
    torch.cuda.synchronize()
    perm_build_s = time.perf_counter() - t0p
    estpi = dk.deann_query_permuted(Xd, Yd, h, K_NN, M_SAMPLES, KERNEL, start=0,
                                    precision="bf16", index=pidx)[0]
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        estpi = dk.deann_query_permuted(Xd, Yd, h, K_NN, M_SAMPLES, KERNEL, start=0,
                                        precision="bf16", index=pidx)[0]
    b.record()
    torch.cuda.synchronize()
    ms_deannp_idx = a.elapsed_time(b) / reps
    perm_same = bool(torch.equal(estpi, estp))
    perm_bytes = int(pidx.buffer.numel())
    del pidx

    # DEANN with the inverted-file neighbours of the experiments (Sec. 5), not
    # part of the step: index build, query time, recall against the exact k-NN
    n_clusters, n_probe, ivf_iters = ivf_config(n)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    C_ivf, a_ivf = dk.ivf_build(Xd, n_clusters, iters=ivf_iters)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    index = dk.IvfIndex(Xd, C_ivf, a_ivf)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    esti, nni, _ = dk.deann_ivf_query(Xd, Yd, index, n_probe, h, K_NN, M_SAMPLES, KERNEL, seed=0)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        esti, nni, _ = dk.deann_ivf_query(Xd, Yd, index, n_probe, h, K_NN, M_SAMPLES, KERNEL,
                                          seed=0)
    b.record()
    torch.cuda.synchronize()
    ms_ivf = a.elapsed_time(b) / reps
    nn_h, nni_h = nn.cpu().numpy(), nni.cpu().numpy()
    recall = np.array([np.intersect1d(nn_h[j], nni_h[j]).size / max(K_NN, 1) for j in range(q)])
    del index, C_ivf, a_ivf

    # float32-accurate dot products from three-part bfloat16 MFMAs (not part of
    # the step): the exact KDE alone and with its gradient, speed and their
    # difference from the float32 MFMA path
    ms_split = ms_split_grad = ms_step_split = None
    musg_h = None
    flops_exact = 2.0 * n * d * q
    mus = dk.kde_exact(Xd, Yd, h, KERNEL, "fp32_split")
    torch.cuda.synchronize()
    dk.kernel_timing(reps)
    a.record()
    for _ in range(reps):
        mus = dk.kde_exact(Xd, Yd, h, KERNEL, "fp32_split")
    b.record()
    torch.cuda.synchronize()
    ms_split = a.elapsed_time(b) / reps
    split_tile_ms = float(np.mean(dk.kernel_times("kde_exact")))
    dk.kernel_timing(0)
    split_refined = dk.last_stats(dev)["exact_refined"]
    mus_h = mus.cpu().numpy()
    split_kernel = {
        "kernel": "kde_tile_kernel<float,gaussian,split engine>" if d > 128
                  else "kde_split_kernel<gaussian>",
        "kernel_avg_ms": split_tile_ms,
        "bf16_flops_per_launch": 6.0 * flops_exact,
        "frac_of_bf16_peak": 6.0 * flops_exact / (split_tile_ms * 1e-3) / PEAK_BF16_MFMA,
        "fp32_equivalent_tflops": flops_exact / (split_tile_ms * 1e-3) / 1e12,
        "note": "six bfloat16 products per element (12*n*d*q flops) on BF16 MFMAs; the "
                "FP32-equivalent rate counts the 2*n*d*q flops of the float32 product"}
    if d <= 128:
        musg = dk.kde_exact_with_grad(Xd, Yd, h, KERNEL, precision="fp32_split")[0]
        torch.cuda.synchronize()
        a.record()
        for _ in range(reps):
            musg = dk.kde_exact_with_grad(Xd, Yd, h, KERNEL, precision="fp32_split")[0]
        b.record()
        torch.cuda.synchronize()
        ms_split_grad = a.elapsed_time(b) / reps
        musg_h = musg.cpu().numpy()

        # the whole step with the split exact part (same work, same outputs); at
        # larger widths the split form's certificate re-evaluates too many
        # queries to compete (its kernel is still timed above)
        for _ in range(max(1, args.warmup)):
            dk.kde_exact_with_grad(Xd, Yd, h, KERNEL, precision="fp32_split")
            dk.deann_query_with_grad(Xd, Yd, h, K_NN, M_SAMPLES, KERNEL, seed=0, precision="bf16")
        torch.cuda.synchronize()
        t0s = time.perf_counter()
        for _ in range(args.steps):
            dk.kde_exact_with_grad(Xd, Yd, h, KERNEL, precision="fp32_split")
            dk.deann_query_with_grad(Xd, Yd, h, K_NN, M_SAMPLES, KERNEL, seed=0, precision="bf16")
        torch.cuda.synchronize()
        ms_step_split = (time.perf_counter() - t0s) * 1e3 / args.steps

    # the step with X prepared once (deann_prepare; the data set fixed across
    # calls, as when serving queries): the exact KDE (with its gradient for
    # d <= 128) and DEANN prepare only the queries.  Same outputs as the step.
    pre32 = dk.prepare(Xd, "fp32")
    pre16 = dk.prepare(Xd, "bf16")

    def step_prepared():
        if fused:
            mu_p = dk.kde_exact_with_grad(Xd, Yd, h, KERNEL, prepared=pre32)[0]
        else:
            mu_p = dk.kde_exact(Xd, Yd, h, KERNEL, "fp32", prepared=pre32)
        est_p = dk.deann_query_with_grad(Xd, Yd, h, K_NN, M_SAMPLES, KERNEL, seed=0,
                                         precision="bf16", prepared=pre16)[0]
        return mu_p, est_p

    for _ in range(max(1, args.warmup)):
        mu_p, est_p = step_prepared()
    torch.cuda.synchronize()
    t0p = time.perf_counter()
    for _ in range(args.steps):
        mu_p, est_p = step_prepared()
    torch.cuda.synchronize()
    ms_step_prepared = (time.perf_counter() - t0p) * 1e3 / args.steps
    prepared_same = bool(torch.equal(mu_p, mu) and torch.equal(est_p, est))

    # serving: small query batches against the fixed data set, DEANN (BF16
    # scan, estimate and gradient) per batch with and without the prepared set
    serving = {}
    for qb in (128, 1024):
        Yb = Yd[:qb].contiguous()
        for name, kw in (("prepared", {"prepared": pre16}), ("unprepared", {})):
            dk.deann_query_with_grad(Xd, Yb, h, K_NN, M_SAMPLES, KERNEL, seed=0, precision="bf16",
                                     **kw)
            torch.cuda.synchronize()
            a.record()
            for _ in range(10):
                dk.deann_query_with_grad(Xd, Yb, h, K_NN, M_SAMPLES, KERNEL, seed=0,
                                         precision="bf16", **kw)
            b.record()
            torch.cuda.synchronize()
            ms_b = a.elapsed_time(b) / 10
            serving[f"q{qb}_{name}"] = {"ms_per_batch": ms_b, "queries_per_s": qb / (ms_b * 1e-3)}
    del pre32, pre16

    # exact KDE with BF16 operands (not part of the step): speed and its error
    # against the FP32 exact path (itself within about 1e-6 of the FP64 oracle)
    mu16 = dk.kde_exact(Xd, Yd, h, KERNEL, "bf16")
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        mu16 = dk.kde_exact(Xd, Yd, h, KERNEL, "bf16")
    b.record()
    torch.cuda.synchronize()
    ms_exact16 = a.elapsed_time(b) / reps

    # near/far form (not part of the step): the k nearest rows exact, the rest
    # from the BF16 sweep; alone (its own k-NN) and with the step's neighbours
    muh = dk.kde_hybrid(Xd, Yd, h, K_NN, KERNEL, "bf16")
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        muh = dk.kde_hybrid(Xd, Yd, h, K_NN, KERNEL, "bf16")
    b.record()
    torch.cuda.synchronize()
    ms_hyb = a.elapsed_time(b) / reps
    muhn = dk.kde_hybrid(Xd, Yd, h, K_NN, KERNEL, "bf16", nn_idx=nn)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        muhn = dk.kde_hybrid(Xd, Yd, h, K_NN, KERNEL, "bf16", nn_idx=nn)
    b.record()
    torch.cuda.synchronize()
    ms_hyb_nn = a.elapsed_time(b) / reps

    # Gaussian mean shift of all queries (not part of the step): MEAN_SHIFT_STEPS
    # steps y <- y + h^2 grad(mu)/mu, with the exact density and gradient
    # (one fused pass per step, d <= 128) and with DEANN (BF16 scan) and its adjoint
    def time_mean_shift(method, **kw):
        dk.mean_shift(Xd, Yd, h, 1, method, **kw)   # workspaces allocated once
        torch.cuda.synchronize()
        a.record()
        y_end = dk.mean_shift(Xd, Yd, h, MEAN_SHIFT_STEPS, method, **kw)
        b.record()
        torch.cuda.synchronize()
        del y_end
        return a.elapsed_time(b)
    ms_shift_exact = time_mean_shift("exact") if fused else None
    ms_shift_deann = time_mean_shift("deann", k=K_NN, m=M_SAMPLES, seed=0, precision="bf16")

    mu_h = mu.cpu().numpy()
    mu_fwd_h = mu_fwd.cpu().numpy()
    mu16_h = mu16.cpu().numpy()
    muh_h, muhn_h = muh.cpu().numpy(), muhn.cpu().numpy()
    est_h, est16_h, est32_h = est.cpu().numpy(), est16.cpu().numpy(), est32.cpu().numpy()
    same_idx = bool(torch.equal(nn16, nn32) and torch.equal(sm16, sm32))
    keep = mu_h >= 1e-16
    rel_bf16_vs_fp32 = (float(np.max(np.abs(est16_h - est32_h)[keep] / est32_h[keep]))
                        if keep.any() else 0.0)
    rel_deann_vs_exact = np.abs(est_h[keep] - mu_h[keep]) / mu_h[keep]
    rel_exact16 = np.abs(mu16_h[keep] - mu_h[keep]) / mu_h[keep]
    rel_hyb = np.abs(muh_h[keep] - mu_h[keep]) / mu_h[keep]
    rel_hyb_nn = np.abs(muhn_h[keep] - mu_h[keep]) / mu_h[keep]
    estp_h = estp.cpu().numpy()
    rel_deannp = np.abs(estp_h[keep] - mu_h[keep]) / mu_h[keep]
    esti_h = esti.cpu().numpy()
    rel_ivf = np.abs(esti_h[keep] - mu_h[keep]) / mu_h[keep]

    tile_avg_ms = float(np.mean(tile_ms))
    fwd_achieved = flops_exact / (tile_avg_ms * 1e-3)
    # FP32 rows of at most 128 floats: the register-resident query kernel
    fwd_kernel = "kde_yres_kernel<gaussian>" if d <= 128 else "kde_tile_kernel<float,gaussian>"
    roof_fwd = {"bound": "mfma", "kernel": fwd_kernel,
                "achieved": fwd_achieved / 1e12, "peak": PEAK_FP32_MFMA / 1e12,
                "unit": "TFLOP/s", "frac": fwd_achieved / PEAK_FP32_MFMA,
                "traffic": measured_traffic(fwd_kernel, workload),
                "flops_per_launch": flops_exact, "kernel_avg_ms": tile_avg_ms,
                "launches_timed": len(tile_ms),
                "note": "exact KDE alone: 2*n*d*q flops per launch / the tile kernel's own "
                        "duration (HIP events recorded by the library around it on its stream)"}
    if fused:
        step_avg_ms = float(np.mean(step_tile_ms))
        achieved = 2.0 * flops_exact / (step_avg_ms * 1e-3)
        roofline = {"bound": "mfma", "kernel": "kde_backward_kernel<gaussian>",
                    "achieved": achieved / 1e12, "peak": PEAK_FP32_MFMA / 1e12,
                    "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_MFMA,
                    "traffic": measured_traffic("kde_backward_kernel<gaussian>", workload),
                    "flops_per_launch": 2.0 * flops_exact, "kernel_avg_ms": step_avg_ms,
                    "launches_timed": len(step_tile_ms),
                    "note": "exact KDE with its gradient (the step's dominant kernel): 4*n*d*q "
                            "flops per launch (distance tile recomputed + W X) / the kernel's own "
                            "duration (HIP events recorded by the library on its stream)"}
    else:
        roofline = roof_fwd
    out = {
        "value": q / (ms_step * 1e-3),
        "ms_per_step": ms_step,
        "config": {"workload": workload, "n": n, "d": d, "q": q, "kernel": KERNEL, "h": h,
                   "k": K_NN, "m": M_SAMPLES, "deann_scan": "bf16", "exact": "fp32",
                   "exact_gradient_in_step": fused},
        "roofline": roofline,
        "roofline_exact_kde": roof_fwd,
        "components_ms": comp_ms,
        "queries_per_s": {
            "step": q / (ms_step * 1e-3),
            "deann_bf16_refine": q / (ms_deann16 * 1e-3),
            "deann_bf16_with_grad": q / (comp_ms["deann_bf16_with_grad"] * 1e-3),
            "deann_fp32": q / (ms_deann32 * 1e-3),
            "deann_permuted_bf16_refine": q / (ms_deannp * 1e-3),
            "deann_permuted_index_bf16_refine": q / (ms_deannp_idx * 1e-3),
            "deann_ivf_fp32": q / (ms_ivf * 1e-3),
            "exact_kde_and_grad_fp32": (q / (comp_ms["exact_kde_and_grad_fp32"] * 1e-3)
                                        if fused else None),
            "kde_exact_fp32": q / (ms_exact_fwd * 1e-3),
            "kde_exact_bf16": q / (ms_exact16 * 1e-3),
            "kde_hybrid_bf16": q / (ms_hyb * 1e-3),
            "kde_hybrid_bf16_given_neighbours": q / (ms_hyb_nn * 1e-3),
            "kde_exact_fp32_split": q / (ms_split * 1e-3) if ms_split else None,
            "exact_kde_and_grad_fp32_split": (q / (ms_split_grad * 1e-3)
                                              if ms_split_grad else None),
            "deann_backward": q / (ms_bwd * 1e-3),
        },
        "accuracy": {
            "deann_bf16_vs_fp32_same_indices": same_idx,
            "deann_bf16_vs_fp32_max_rel": rel_bf16_vs_fp32,
            "deann_with_grad_same_indices_as_deann_query": same_as_step,
            "deann_with_grad_vs_deann_query_max_rel": step_vs_alone,
            "deann_with_grad_same_gradient_as_backward": same_grad_as_step,
            "exact_bf16_vs_fp32_mean_rel": float(rel_exact16.mean()) if keep.any() else None,
            "exact_bf16_vs_fp32_max_rel": float(rel_exact16.max()) if keep.any() else None,
            "hybrid_bf16_vs_fp32_mean_rel": float(rel_hyb.mean()) if keep.any() else None,
            "hybrid_bf16_vs_fp32_max_rel": float(rel_hyb.max()) if keep.any() else None,
            "hybrid_bf16_given_nn_vs_fp32_max_rel": (float(rel_hyb_nn.max()) if keep.any()
                                                     else None),
            "deann_vs_exact_mean_rel": float(rel_deann_vs_exact.mean()) if keep.any() else None,
            "deann_vs_exact_median_rel": float(np.median(rel_deann_vs_exact)) if keep.any() else None,
            "deann_permuted_vs_exact_mean_rel": float(rel_deannp.mean()) if keep.any() else None,
            "exact_split_vs_fp32_max_rel": (float(np.max(np.abs(mus_h - mu_fwd_h)[keep]
                                                         / mu_fwd_h[keep]))
                                            if mus_h is not None and keep.any() else None),
            "exact_and_grad_split_vs_fp32_max_rel": (float(np.max(np.abs(musg_h - mu_h)[keep]
                                                                  / mu_h[keep]))
                                                     if musg_h is not None and keep.any() else None),
            "queries_below_1e-16": int((~keep).sum()),
        },
        "exact_fp32_split": {"kde_exact_ms": ms_split, "split_kernel": split_kernel,
                             "queries_reevaluated": split_refined},
        "step_fp32_split": ({"ms_per_step": ms_step_split,
                             "queries_per_s": q / (ms_step_split * 1e-3),
                             "note": "the same step with the exact KDE (and its gradient, d <= "
                                     "128) from three-part bfloat16 MFMAs (DEANN_FP32_SPLIT, "
                                     "certified to the same 1e-5), outside the timed step above"}
                            if ms_step_split else None),
        "step_prepared": {"ms_per_step": ms_step_prepared,
                          "queries_per_s": q / (ms_step_prepared * 1e-3),
                          "same_outputs_as_step": prepared_same,
                          "note": "the step with X prepared once outside the timed region "
                                  "(deann_prepare: FP32 set for the exact KDE, BF16 set for "
                                  "DEANN); queries prepared per call"},
        "serving_deann_bf16_with_grad": dict(serving, note="batches of the first 128 / 1024 "
                                             "queries, each call timed alone (HIP events, 10 "
                                             "calls); with and without the prepared BF16 set"),
        "mean_shift": {"steps": MEAN_SHIFT_STEPS,
                       "exact_ms": ms_shift_exact,
                       "exact_query_steps_per_s": (q * MEAN_SHIFT_STEPS / (ms_shift_exact * 1e-3)
                                                   if ms_shift_exact else None),
                       "deann_bf16_ms": ms_shift_deann,
                       "deann_bf16_query_steps_per_s": q * MEAN_SHIFT_STEPS
                                                       / (ms_shift_deann * 1e-3),
                       "note": "Gaussian mean shift of all queries; exact: kde_exact_with_grad "
                               "per step (d <= 128 only); DEANN: deann_query_with_grad per step"},
        "permuted_index": {"build_s": perm_build_s, "bytes": perm_bytes,
                           "ms": ms_deannp_idx, "ms_evaluated_permutation": ms_deannp,
                           "same_estimates_as_evaluated": perm_same,
                           "note": "deann_query_permuted with the permuted copy of X (App. G's "
                                   "preprocessing): each query's block read contiguously"},
        "ivf": {"n_clusters": n_clusters, "n_probe": n_probe, "iters": ivf_iters,
                "build_s": t1 - t0, "index_s": t2 - t1, "ms": ms_ivf,
                "queries_per_s": q / (ms_ivf * 1e-3),
                "recall_mean": float(recall.mean()), "recall_min": float(recall.min()),
                "vs_exact_mean_rel": float(rel_ivf.mean()) if keep.any() else None,
                "note": "DEANN with the k nearest rows among the n_probe closest of n_clusters "
                        "k-means clusters (FP32 scan of those clusters); recall against the "
                        "exact k-NN of the step"},
    }

    if with_cpu:
        # about 20 s of oracle work: one query costs about 3 n d FP64 element
        # operations per pass (exact KDE, k-NN) at roughly 4e8 per second
        size = args.cpu_sample or max(2, min(16, int(20.0 / (3e-9 * n * d))))   # ~20 s
        out["cpu_baseline"], out["parity_sample"] = cpu_baseline(
            X, Y, h, size, mu_h, est_h, nn.cpu().numpy(), sm.cpu().numpy(),
            gy.cpu().numpy(), K_NN, M_SAMPLES, fused,
            gye.cpu().numpy() if gye is not None else None)
        if args.all_cores:
            out["cpu_baseline_all_cores"] = cpu_baseline_all_cores(workload, h, K_NN,
                                                                   M_SAMPLES, fused)
    del Xd, Yd
    return out


def cpu_baseline(X, Y, h, size, mu_gpu, est_gpu, nn_gpu, sm_gpu, gy_gpu, K_NN, M_SAMPLES,
                 exact_bwd, gye_gpu=None):
    """The FP64 oracle timed on the host for a few queries of the same workload,
    doing the same per-query work as one step; also checks those queries."""
    import numpy as np

    import oracle
    import synth

    sub = synth.query_subset(Y.shape[0], size, seed=11)
    t0 = time.perf_counter()
    rel_exact, rel_deann, nn_ok, sm_ok, rel_gy, gye_ref = [], [], True, True, [], {}
    excluded = 0
    for j in sub:
        if exact_bwd:   # the KDE and its gradient
            mu, g_ref, _ = oracle.kde_grad(X, Y[j], h, oracle.GAUSSIAN)
            gye_ref[j] = (mu, g_ref)
        else:
            mu = oracle.kde_exact(X, Y[j:j + 1], h, oracle.GAUSSIAN)[0]
        est, nn_ref, s_ref = oracle.deann_estimate(X, Y[j], h, oracle.GAUSSIAN, K_NN, M_SAMPLES,
                                                   0, int(j))
        _, gy_ref, _ = oracle.deann_grad(X, Y[j], h, oracle.GAUSSIAN, nn_ref, s_ref, M_SAMPLES)
        if mu >= 1e-16:
            rel_exact.append(abs(mu_gpu[j] - mu) / mu)
            rel_deann.append(abs(est_gpu[j] - est) / est)
        else:
            excluded += 1
        nn_ok &= bool(np.array_equal(nn_gpu[j], nn_ref))
        sm_ok &= bool(np.array_equal(sm_gpu[j], s_ref))
        nrm = np.linalg.norm(gy_ref)
        if nrm >= 1e-30:   # grad_Y is float32: smaller gradients underflow
            rel_gy.append(float(np.linalg.norm(gy_gpu[j] - gy_ref) / nrm))
    dt = time.perf_counter() - t0
    # exact gradient, normwise against sum_i K_i ||x_i - y|| / (n h^2) (not timed)
    rel_gye = []
    if gye_gpu is not None:
        for j, (mu_j, g_ref) in gye_ref.items():
            if mu_j < 1e-16:   # the paper's exclusion, as for the values
                continue
            d2 = oracle.sq_dists(X, Y[j])
            scale = (oracle.kernel_values(d2, h, oracle.GAUSSIAN) * np.sqrt(d2)).sum() / (
                X.shape[0] * h * h)
            if scale > 0:
                rel_gye.append(float(np.linalg.norm(gye_gpu[j] - g_ref) / scale))
    base = {"value": len(sub) / dt, "unit": "queries/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(sub)} queries of the same workload, full step per query "
                      "(exact KDE" + (" with its gradient" if exact_bwd else "") + ", DEANN, DEANN adjoint"
                      + "), FP64 NumPy, single thread",
            "seconds": dt}
    par = {"queries": [int(j) for j in sub], "nn_equal": nn_ok, "samples_equal": sm_ok,
           "exact_fp32_max_rel": max(rel_exact) if rel_exact else None,
           "deann_max_rel": max(rel_deann) if rel_deann else None,
           "deann_grad_y_max_rel": max(rel_gy) if rel_gy else None,
           "exact_grad_y_max_err_normwise": max(rel_gye) if rel_gye else None,
           "queries_below_1e-16_excluded": excluded}
    return base, par


def sweep_km(args, X, Y, h):
    """Error against the exact KDE and queries/s of DEANN (BF16 scan +
    refinement) over a grid of k and m (powers of 2 times 10), one JSON line."""
    import numpy as np
    import torch

    import paper_2107_02736_amd as dk
    dev = torch.device("cuda:0")
    Xd, Yd = torch.from_numpy(X).to(dev), torch.from_numpy(Y).to(dev)
    q = Y.shape[0]
    mu = dk.kde_exact(Xd, Yd, h, KERNEL, "fp32").cpu().numpy()
    keep = mu >= 1e-16
    rows = []
    for k in (0, 10, 20, 40, 80, 160, 320):
        for m in (0, 10, 40, 160, 640, 2560):
            if k == 0 and m == 0:
                continue
            dk.deann_query(Xd, Yd, h, k, m, KERNEL, seed=0, precision="bf16")
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            a.record()
            for _ in range(3):
                est = dk.deann_query(Xd, Yd, h, k, m, KERNEL, seed=0, precision="bf16")[0]
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / 3
            e = np.abs(est.cpu().numpy()[keep] - mu[keep]) / mu[keep]
            rows.append({"k": k, "m": m, "queries_per_s": q / (ms * 1e-3), "ms": ms,
                         "mean_rel_err": float(e.mean()), "median_rel_err": float(np.median(e)),
                         "p90_rel_err": float(np.percentile(e, 90))})
            print(f"# k={k} m={m}: {ms:.2f} ms, mean rel err {e.mean():.3e}", file=sys.stderr,
                  flush=True)
    print(json.dumps({"sweep": "deann_km", "workload": args.workload, "kernel": KERNEL, "h": h,
                      "scan": "bf16", "queries_excluded_below_1e-16": int((~keep).sum()),
                      "rows": rows}), flush=True)


def sweep_ivf(args, X, Y, h, k_nn, m_samples):
    """Inverted-file DEANN over cluster counts n_l and inspected clusters n_q:
    build time, queries/s, recall against the exact k-NN and error against the
    exact KDE, one JSON line; the exact-k-NN DEANN (BF16 scan) for reference."""
    import numpy as np
    import torch

    import paper_2107_02736_amd as dk
    dev = torch.device("cuda:0")
    Xd, Yd = torch.from_numpy(X).to(dev), torch.from_numpy(Y).to(dev)
    n, q = X.shape[0], Y.shape[0]
    mu = dk.kde_exact(Xd, Yd, h, KERNEL, "fp32").cpu().numpy()
    keep = mu >= 1e-16

    def timed(fn):
        fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(3):
            r = fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / 3, r

    ms, (est, nn, _) = timed(lambda: dk.deann_query(Xd, Yd, h, k_nn, m_samples, KERNEL, seed=0,
                                                    precision="bf16"))
    nn = nn.cpu().numpy()
    e = np.abs(est.cpu().numpy()[keep] - mu[keep]) / mu[keep]
    ref = {"queries_per_s": q / (ms * 1e-3), "ms": ms, "mean_rel_err": float(e.mean())}
    rows = []
    for n_clusters in (256, 1024, 4096):
        if n_clusters > n:
            continue
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        C, a = dk.ivf_build(Xd, n_clusters, iters=4)
        index = dk.IvfIndex(Xd, C, a)
        torch.cuda.synchronize()
        build_s = time.perf_counter() - t0
        for n_probe in (1, 2, 4, 8, 16, 32, 64):
            if n_probe > n_clusters:
                continue
            ms, (est, nni, _) = timed(lambda: dk.deann_ivf_query(
                Xd, Yd, index, n_probe, h, k_nn, m_samples, KERNEL, seed=0))
            nni = nni.cpu().numpy()
            rec = np.array([np.intersect1d(nn[j], nni[j]).size / max(k_nn, 1) for j in range(q)])
            e = np.abs(est.cpu().numpy()[keep] - mu[keep]) / mu[keep]
            rows.append({"n_clusters": n_clusters, "n_probe": n_probe, "build_s": build_s,
                         "queries_per_s": q / (ms * 1e-3), "ms": ms,
                         "recall_mean": float(rec.mean()), "recall_min": float(rec.min()),
                         "mean_rel_err": float(e.mean())})
            print(f"# n_l={n_clusters} n_q={n_probe}: {ms:.2f} ms, recall {rec.mean():.3f}, "
                  f"mean rel err {e.mean():.3e}", file=sys.stderr, flush=True)
        del index, C, a
    print(json.dumps({"sweep": "deann_ivf", "workload": args.workload, "kernel": KERNEL, "h": h,
                      "k": k_nn, "m": m_samples, "exact_knn_bf16": ref,
                      "queries_excluded_below_1e-16": int((~keep).sum()), "rows": rows}),
          flush=True)


def _oracle_shard(workload, h, k_nn, m_samples, exact_bwd, queries):
    """Worker of the all-cores oracle run: regenerates the workload (seeded) and
    times the same per-query oracle work as cpu_baseline on its queries."""
    import oracle
    import synth
    spec, X, Y = synth.workload(workload)
    t0 = time.perf_counter()
    for j in queries:
        if exact_bwd:
            oracle.kde_grad(X, Y[j], h, oracle.GAUSSIAN)
        else:
            oracle.kde_exact(X, Y[j:j + 1], h, oracle.GAUSSIAN)
        est, nn_ref, s_ref = oracle.deann_estimate(X, Y[j], h, oracle.GAUSSIAN, k_nn, m_samples,
                                                   0, int(j))
        oracle.deann_grad(X, Y[j], h, oracle.GAUSSIAN, nn_ref, s_ref, m_samples)
    return time.perf_counter() - t0


def cpu_baseline_all_cores(workload, h, k_nn, m_samples, exact_bwd, per_worker=2):
    """The same oracle work on every host core: one spawned process per core
    (at most 16), each on its own queries; queries/s = all queries over the
    slowest worker's time (data generation excluded)."""
    import concurrent.futures as cf
    import multiprocessing as mp

    import synth
    spec = synth.WORKLOADS[workload]
    # each worker holds the data and FP64 temporaries of about 5x its size
    workers = max(1, min(16, os.cpu_count() or 1, int(150e9 // (5 * spec.n * spec.d * 4))))
    sub = synth.query_subset(spec.q, workers * per_worker, seed=13)
    shards = [[int(j) for j in sub[w::workers]] for w in range(workers)]
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        times = list(ex.map(_oracle_shard, [workload] * workers, [h] * workers,
                            [k_nn] * workers, [m_samples] * workers, [exact_bwd] * workers,
                            shards))
    return {"value": len(sub) / max(times), "unit": "queries/s", "cores": workers,
            "kind": "oracle",
            "sample": f"{len(sub)} queries of the same workload in {workers} processes "
                      f"({per_worker} each), same per-query work as cpu_baseline",
            "seconds": max(times)}


if __name__ == "__main__":
    main()
