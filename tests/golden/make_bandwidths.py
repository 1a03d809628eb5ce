"""Write tests/golden/bandwidths.json: the bandwidth h of every workload.

Calls only the FP64 oracle (and the seeded inputs).  Following the paper's
bandwidth selection (Sec. 5), h is found by bisection so that the exact KDE
averaged over a query set is within 1% of the target; the workloads ask for
the mean rather than the median.  For the large workloads the average runs
over a fixed random subset of the queries (size stated in the output).

Usage:  python tests/golden/make_bandwidths.py [workload ...]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

# (workload, kernel name, target mean KDE, queries averaged over)
JOBS = [
    ("mix10_n1e4_d16", "gaussian", 1e-2, 1000),
    ("mix10_n1e4_d16", "exponential", 1e-2, 1000),
    ("mix100_n1e6_d128", "gaussian", 1e-3, 100),
    ("mix100_n1e6_d128", "exponential", 1e-3, 100),
    ("mix50_n5e5_d64", "gaussian", 1e-3, 100),
    ("mix200_n1e6_d960", "gaussian", 1e-4, 50),
]
KERNELS = {"gaussian": oracle.GAUSSIAN, "exponential": oracle.EXPONENTIAL}


def main(names):
    path = os.path.join(HERE, "bandwidths.json")
    table = json.load(open(path)) if os.path.exists(path) else {}
    cache = {}
    for wl, kname, target, nq in JOBS:
        if names and wl not in names:
            continue
        t0 = time.time()
        if wl not in cache:
            spec, X, Y = synth.workload(wl)
            sub = synth.query_subset(spec.q, nq, seed=7)
            cache.clear()
            cache[wl] = (spec, sub, oracle.pairwise_sq_dists(X, Y[sub]))
            del X, Y
        spec, sub, D2 = cache[wl]
        h = oracle.bisect_h(D2, target, KERNELS[kname], stat="mean")
        table.setdefault(wl, {})[kname] = {
            "h": h, "target_mean_kde": target, "queries_averaged": int(len(sub)),
            "query_subset_seed": 7,
        }
        print(f"{wl} {kname}: h={h!r} ({time.time() - t0:.1f}s)", flush=True)
        with open(path, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:])
