"""Benchmark: exact epsilon-graph of the 1M x 128 Euclidean workload on one
MI355X.

A step is the whole hot path on one batch of device-resident synthetic
points: fnn_tree_build (cover tree) + fnn_eps_graph (all-points range query
-> symmetric CSR).  Prints one JSON line (metric: edges/s; distance
evaluations/s and the per-phase split are extra fields), with the roofline of
the dominant kernel and the CPU oracle's rate on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2a]
                    [--precision fp32|bf16|fp8] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2510_14147_amd import datagen as G  # noqa: E402

W = json.load(open(os.path.join(ROOT, "paper_2510_14147_amd", "workloads.json")))

# Published MI355X peaks.
PEAK_HBM_GBS = 8000.0
PEAK_FP32_VEC_TFLOPS = 157.3
PEAK_BF16_TFLOPS = 2500.0
PEAK_FP8_TFLOPS = 5000.0


def workload(name: str):
    """(points, metric, eps, description) of a named workload."""
    if name == "c2a":
        return G.c2_manifold(), "l2", W["c2"]["eps"][0], "c2_manifold_1m_d128_eps70"
    if name == "c2b":
        return G.c2_manifold(), "l2", W["c2"]["eps"][1], "c2_manifold_1m_d128_eps500"
    if name == "c2_50k":
        return (G.c2_manifold(n=50_000), "l2", W["c2_50k"]["eps"][0],
                "c2_manifold_50k_d128_eps70")
    if name == "c1":
        return G.c1_clusters(), "l2", W["c1"]["eps"], "c1_clusters_20k_d8"
    if name == "c3":
        return G.c3_hamming(), "hamming", 24.0, "c3_hamming_2m_256b_eps24"
    if name == "c4":
        return G.c4_strings(), "levenshtein", 6.0, "c4_strings_100k_eps6"
    if name == "ang":
        return G.angular_dirs(), "angular", W["ang"]["eps"], "angular_20k_d16"
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(x, metric, eps, rows: int, seed: int = 7):
    """The FP64 oracle (brute force, as it stands) on a bounded sample of
    rows against all points, on this host's cores."""
    from oracle import oracle as O
    mid = {"l2": 0, "angular": 1, "hamming": 2, "levenshtein": 3}[metric]
    rng = np.random.default_rng(seed)
    sample = np.sort(rng.choice(x.shape[0], size=min(rows, x.shape[0]),
                                replace=False))
    O.lib()
    t0 = time.perf_counter()
    rp, _, _ = O.bruteforce(x, mid, eps, rows=sample)
    dt = time.perf_counter() - t0
    edges = int(rp[-1])
    cores = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp:
        cores = min(cores, int(omp))
    return {"value": edges / dt, "unit": "edges/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{sample.size} seeded rows vs all {x.shape[0]} points, "
                      f"FP64 brute force ({edges} edges in {dt:.2f} s); "
                      f"pair evals/s {sample.size * x.shape[0] / dt:.3e}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2a")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--sched", default="two_pass")
    ap.add_argument("--cpu-rows", type=int, default=1500)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the epsilon-graph path has no "
              "multi-GPU mode; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2510_14147_amd as fnn

    x, metric, eps, desc = workload(args.workload)
    print(f"[bench] workload {desc} n={x.shape[0]} metric={metric} eps={eps}",
          file=sys.stderr, flush=True)
    if metric == "hamming":
        xd = torch.from_numpy(x.view(np.int64)).cuda()
    else:
        xd = torch.from_numpy(x).cuda()
    torch.cuda.synchronize()

    def step():
        tree = fnn.fnn_tree_build(xd, metric)
        g = fnn.fnn_eps_graph(tree, eps, precision=args.precision,
                              sched=args.sched)
        return tree, g

    for i in range(args.warmup):
        tree, g = step()
        print(f"[bench] warmup {i}: nnz={g.nnz} build={tree.stats['build_ms']:.1f} ms "
              f"query={g.stats['total_ms']:.1f} ms", file=sys.stderr, flush=True)
        del tree, g
    torch.cuda.synchronize()
    times, stats = [], []
    t_all = time.perf_counter()
    for i in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tree, g = step()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        times.append(dt)
        stats.append((tree.stats, g.stats, g.nnz))
        print(f"[bench] step {i}: {dt * 1e3:.1f} ms nnz={g.nnz}",
              file=sys.stderr, flush=True)
        del tree, g
    total = time.perf_counter() - t_all
    ms = 1e3 * total / args.steps
    tb, tq, nnz = stats[-1]
    evals = tb["build_dist_evals"] + tq["traverse_tests"] + 2 * tq["tile_pairs"]
    value = nnz / (ms / 1e3)
    dim = x.shape[1] if metric in ("l2", "angular") else None

    # Dominant kernel: the leaf-tile count pass (event-timed in the library
    # on the stream it runs on).  Algorithmic work: 3*d flops per pair
    # (difference, square, accumulate) for the vector metrics.
    roof = None
    if metric in ("l2", "angular") and args.precision != "fp32" and tq["count_ms"] > 0:
        # MFMA Gram filter: 2*k flops per screened pair (k = padded dim)
        kq = -(-dim // 16) * 16 if args.precision == "bf16" else -(-dim // 64) * 64
        flops = 2.0 * kq * tq["filter_pairs"]
        ach = flops / (tq["count_ms"] / 1e3) / 1e12
        peak = PEAK_BF16_TFLOPS if args.precision == "bf16" else PEAK_FP8_TFLOPS
        roof = {"bound": "mfma", "achieved": round(ach, 3), "peak": peak,
                "unit": "TFLOP/s", "frac": round(ach / peak, 4), "traffic": None,
                "kernel": f"k_gram<L2,{args.precision},count>",
                "kernel_ms": round(tq["count_ms"], 3), "flops_per_launch": flops}
    elif metric in ("l2", "angular") and tq["count_ms"] > 0:
        flops = 3.0 * dim * tq["tile_pairs"]
        ach = flops / (tq["count_ms"] / 1e3) / 1e12
        roof = {"bound": "alu", "achieved": round(ach, 3),
                "peak": PEAK_FP32_VEC_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ach / PEAK_FP32_VEC_TFLOPS, 4), "traffic": None,
                "kernel": "k_tile<L2,count>", "kernel_ms": round(tq["count_ms"], 3),
                "flops_per_launch": flops}
    out = {
        "metric": "epsilon-graph edges/s (exact, symmetric CSR)",
        "value": value, "unit": "edges/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": desc, "n": int(x.shape[0]), "dim": dim,
                   "metric": metric, "eps": eps, "precision": args.precision,
                   "sched": args.sched, "nnz": int(nnz),
                   "mean_neighbors": nnz / x.shape[0]},
        "dist_evals_per_s": evals / (ms / 1e3),
        "phases_ms": {"build": tb["build_ms"], "traverse": tq["traverse_ms"],
                      "count": tq["count_ms"], "scan": tq["scan_ms"],
                      "fill": tq["fill_ms"], "sort": tq["sort_ms"]},
        "counters": {k: tq[k] for k in ("interactions", "tile_pairs",
                                        "traverse_tests", "fp64_rechecks",
                                        "filter_pairs", "filter_survivors",
                                        "packs", "nodes")} |
                    {"build_dist_evals": tb["build_dist_evals"],
                     "rounds": tb["rounds"], "netsel_passes": tb["netsel_passes"]},
        "roofline": roof,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(x, metric, eps, args.cpu_rows)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
