"""Calibrate the epsilon of each synthetic workload with the CPU oracle and
write ``paper_2510_14147_amd/workloads.json``.

For a target mean neighbour count k, S seeded sample rows are measured
against every point in FP64 (``oracle.rows_dist``); with the distances
sorted, eps is the midpoint of the (k*S)-th and (k*S+1)-th smallest
non-self distance, so the sampled rows average about k neighbours.  The
Hamming (eps = 24 bits) and Levenshtein (eps = 6 edits) workloads take
their eps as given.  Run:  python -m oracle.calibrate  [--quick]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import oracle as O                       # noqa: E402
from paper_2510_14147_amd import datagen as G         # noqa: E402

OUT = os.path.join(ROOT, "paper_2510_14147_amd", "workloads.json")


def calibrate(points, metric, targets, samples, seed):
    n = points.shape[0]
    rng = np.random.default_rng(seed)
    rows = np.sort(rng.choice(n, size=min(samples, n), replace=False))
    d = O.rows_dist(points, metric, rows)
    d[np.arange(rows.size), rows] = np.inf          # drop self pairs
    flat = np.sort(d.ravel())
    out = []
    for k in targets:
        i = int(round(k * rows.size))
        i = max(1, min(i, flat.size - 1))
        out.append(float(0.5 * (flat[i - 1] + flat[i])))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true",
                    help="skip the 1M-point and many-cloud calibrations")
    args = ap.parse_args(argv)
    old = json.load(open(OUT)) if os.path.exists(OUT) else {}
    W = dict(old)
    t0 = time.time()

    x = G.c1_clusters()
    (e,) = calibrate(x, O.L2, [20], 2000, 1101)
    W["c1"] = dict(name="c1_clusters_20k_d8", generator="c1_clusters", metric="l2",
                   n=20000, dim=8, seed=1001, eps=e, target_nbrs=20)

    xa = G.angular_dirs()
    (e,) = calibrate(xa, O.ANGULAR, [20], 2000, 1106)
    W["ang"] = dict(name="angular_dirs_20k_d16", generator="angular_dirs",
                    metric="angular", n=20000, dim=16, seed=1006, eps=e,
                    target_nbrs=20)

    xs = G.c2_manifold(n=50_000)
    e70, e500 = calibrate(xs, O.L2, [70, 500], 2000, 1102)
    W["c2_50k"] = dict(name="c2_manifold_50k_d128", generator="c2_manifold",
                       metric="l2", n=50000, dim=128, seed=1002,
                       eps=[e70, e500], target_nbrs=[70, 500])

    W["c3"] = dict(name="c3_hamming_2m_256b", generator="c3_hamming",
                   metric="hamming", n=2_000_000, dim=256, seed=1003, eps=24.0)
    W["c4"] = dict(name="c4_strings_100k_len80_120", generator="c4_strings",
                   metric="levenshtein", n=100_000, dim=128, seed=1004, eps=6.0)

    if not args.quick:
        x2 = G.c2_manifold()
        e70, e500 = calibrate(x2, O.L2, [70, 500], 2000, 1102)
        W["c2"] = dict(name="c2_manifold_1m_d128", generator="c2_manifold",
                       metric="l2", n=1_000_000, dim=128, seed=1002,
                       eps=[e70, e500], target_nbrs=[70, 500])
        del x2
        eps5 = []
        for spec in G.c5_cloud_specs():
            xc = G.c5_cloud(spec)
            (e,) = calibrate(xc, O.L2, [spec["target_nbrs"]],
                             min(500, spec["n"]), 1105 + spec["cloud"])
            eps5.append(e)
        W["c5"] = dict(name="c5_256_clouds", generator="c5_cloud_specs",
                       metric="l2", n_clouds=256, seed=1005, eps=eps5)
    W["_note"] = ("eps calibrated by oracle/calibrate.py: midpoint of the "
                  "(k*S)-th and (k*S+1)-th smallest non-self FP64 distance "
                  "from S seeded sample rows; c3/c4 eps fixed.")
    with open(OUT, "w") as f:
        json.dump(W, f, indent=1, sort_keys=True)
    print("wrote", OUT, "in %.1f s" % (time.time() - t0))


if __name__ == "__main__":
    main()
