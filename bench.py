"""Benchmark: exact epsilon-graph of the 1M x 128 Euclidean workload on one
MI355X.

A step is the whole hot path on one batch of device-resident synthetic
points: fnn_tree_build (cover tree) + fnn_eps_graph (all-points range query
-> symmetric CSR).  Prints one JSON line (metric: edges/s; distance
evaluations/s and the per-phase split are extra fields), with the roofline of
the dominant kernel and the CPU oracle's rate on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2a]
                    [--precision fp32|bf16|fp16|fp8] [--no-cpu]
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
PEAK_INT8_TOPS = 5000.0


def workload(name: str):
    """(points, metric, eps, description) of a named workload."""
    if name == "c2a":
        return G.c2_manifold(), "l2", W["c2"]["eps"][0], "c2_manifold_1m_d128_eps70"
    if name == "c2b":
        return G.c2_manifold(), "l2", W["c2"]["eps"][1], "c2_manifold_1m_d128_eps500"
    if name == "c2_50k":
        return (G.c2_manifold(n=50_000), "l2", W["c2_50k"]["eps"][0],
                "c2_manifold_50k_d128_eps70")
    if name == "c2q":
        # the C2 set as the tree, 100K more draws from the same manifold as
        # queries (prefixes of one seeded stream)
        x = G.c2_manifold(n=1_100_000)
        return (x, "l2", W["c2"]["eps"][0],
                "c2_manifold_1m_d128_eps70_query_100k")
    if name == "c1":
        return G.c1_clusters(), "l2", W["c1"]["eps"], "c1_clusters_20k_d8"
    if name == "c3":
        return G.c3_hamming(), "hamming", 24.0, "c3_hamming_2m_256b_eps24"
    if name == "c4":
        return G.c4_strings(), "levenshtein", 6.0, "c4_strings_100k_eps6"
    if name == "ang":
        return G.angular_dirs(), "angular", W["ang"]["eps"], "angular_20k_d16"
    raise SystemExit(f"unknown workload {name}")


def c5_groups(max_clouds: int | None = None):
    """The many-clouds workload as one batch per dimension (a batch shares
    one row layout): [(points, offsets, eps list, dim)]."""
    specs = G.c5_cloud_specs()
    if max_clouds:
        specs = specs[:max_clouds]
    groups = []
    for d in (3, 16, 64):
        sel = [s for s in specs if s["dim"] == d]
        if not sel:
            continue
        xs = [G.c5_cloud(s) for s in sel]
        off = np.concatenate([[0], np.cumsum([len(x) for x in xs])]).astype(np.int64)
        groups.append((np.concatenate(xs, axis=0), off,
                       [W["c5"]["eps"][s["cloud"]] for s in sel], d))
    return groups


def cpu_baseline_c5(groups, rows: int, seed: int = 7):
    """The FP64 oracle (brute force) on seeded sample rows of the clouds,
    each row against all points of its own cloud."""
    from oracle import oracle as O
    rng = np.random.default_rng(seed)
    O.lib()
    ntot = sum(g[0].shape[0] for g in groups)
    edges, pairs, dt, nrows = 0, 0, 0.0, 0
    for x, off, eps, _ in groups:
        k = max(1, int(round(rows * x.shape[0] / ntot)))
        sample = np.sort(rng.choice(x.shape[0], size=min(k, x.shape[0]), replace=False))
        cl = np.searchsorted(off, sample, side="right") - 1
        for c in np.unique(cl):
            lo, hi = int(off[c]), int(off[c + 1])
            r = sample[cl == c] - lo
            t0 = time.perf_counter()
            rp, _, _ = O.bruteforce(x[lo:hi], 0, eps[c], rows=r)
            dt += time.perf_counter() - t0
            edges += int(rp[-1])
            pairs += r.size * (hi - lo)
            nrows += r.size
    cores = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp:
        cores = min(cores, int(omp))
    return {"value": edges / dt, "unit": "edges/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{nrows} seeded rows, each vs all points of its cloud, "
                      f"FP64 brute force ({edges} edges in {dt:.2f} s); "
                      f"pair evals/s {pairs / dt:.3e}"}


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
    cores = _cores()
    out = {"value": edges / dt, "unit": "edges/s", "cores": cores,
           "kind": "oracle",
           "sample": f"{sample.size} seeded rows vs all {x.shape[0]} points, "
                     f"FP64 brute force ({edges} edges in {dt:.2f} s); "
                     f"pair evals/s {sample.size * x.shape[0] / dt:.3e}",
           "cpu_model": _cpu_model()}
    # one core: the first rows of the same sample, one thread
    k1 = max(1, sample.size // 30)
    if _omp_threads(1):
        try:
            t0 = time.perf_counter()
            rp1, _, _ = O.bruteforce(x, mid, eps, rows=sample[:k1])
            d1 = time.perf_counter() - t0
        finally:
            _omp_threads(None)
        out["single_thread"] = {"edges_per_s": int(rp1[-1]) / d1,
                                "pair_evals_per_s": k1 * x.shape[0] / d1,
                                "rows": int(k1), "s": round(d1, 3)}
    return out


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _omp_threads(k: int | None):
    """Set the OpenMP thread count of the oracle's runtime (None: restore
    the default).  Returns False when the runtime cannot be reached."""
    import ctypes
    try:
        g = ctypes.CDLL("libgomp.so.1")
    except OSError:
        return False
    g.omp_set_num_threads(int(k if k else _cores()))
    return True


def _cores() -> int:
    cores = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp:
        cores = min(cores, int(omp))
    return cores


def cpu_cover_tree(x, metric, eps_scaled, n: int):
    """The oracle's own cover tree (Algorithms 1-3, FP64, as it stands) on
    the first n points: build and all-points query timed apart."""
    from oracle import oracle as O
    mid = {"l2": 0, "angular": 1, "hamming": 2, "levenshtein": 3}[metric]
    xs = np.ascontiguousarray(x[:n])
    t0 = time.perf_counter()
    t = O.tree_build(xs, mid, zeta=64)
    t1 = time.perf_counter()
    rp, _, _ = O.tree_query(xs, mid, eps_scaled, t)
    t2 = time.perf_counter()
    return {"n": int(n), "eps": eps_scaled, "build_s": round(t1 - t0, 3),
            "query_s": round(t2 - t1, 3), "edges": int(rp[-1]),
            "edges_per_s": int(rp[-1]) / (t2 - t0)}


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE measurement (scaled by the
    copy-kernel factors recorded with it), or None when there is none or the
    kernel's source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(f"{kernel}|{workload}")
    if not rec:
        return None
    src = os.path.join(ROOT, rec["source"])
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["source_sha256"]:
        return None
    return rec["bytes_per_launch"]


def roofline(dim, precision, tq, workload=""):
    """Roofline of the dominant kernel of one query: the leaf-tile count pass
    (plain FP32: 3*d flops per pair -- difference, square, accumulate) or the
    MFMA Gram filter (2*k flops per screened pair, k = padded dim; on Hamming
    codes 2*k integer ops, k = code bits), timed with HIP events inside the
    library on the stream it runs on."""
    if tq["count_ms"] <= 0:
        return None
    if precision == "i8":
        ops = 2.0 * dim * tq["filter_pairs"]
        kms = tq["filter_ms"] if tq.get("filter_ms", 0) > 0 else tq["count_ms"]
        ach = ops / (kms / 1e3) / 1e12
        kname = f"k_gram<HAM,i8,k{dim}>"
        return {"bound": "mfma", "achieved": round(ach, 3), "peak": PEAK_INT8_TOPS,
                "unit": "TOP/s", "frac": round(ach / PEAK_INT8_TOPS, 4),
                "traffic": measured_traffic(kname, workload),
                "kernel": kname, "kernel_ms": round(kms, 3),
                "ops_per_launch": ops}
    if precision != "fp32":
        # the MFMA filter kernel alone, event-timed inside the library; k is
        # the padded width it ran on: the leading principal coordinates when
        # the library projected (proj_dim), else the coordinates
        k = tq.get("proj_dim", 0) or dim
        b16 = precision in ("bf16", "fp16")
        kq = -(-k // 16) * 16 if b16 else -(-k // 64) * 64
        flops = 2.0 * kq * tq["filter_pairs"]
        kms = tq["filter_ms"] if tq.get("filter_ms", 0) > 0 else tq["count_ms"]
        ach = flops / (kms / 1e3) / 1e12
        # dense FP16 and BF16 MFMA share one peak
        peak = PEAK_BF16_TFLOPS if b16 else PEAK_FP8_TFLOPS
        if b16 and kq <= 32:
            kname = f"k_gram_direct<L2,{precision},k{kq}>"
        else:
            kname = f"k_gram<L2,{precision},k{kq}>"
        return {"bound": "mfma", "achieved": round(ach, 3), "peak": peak,
                "unit": "TFLOP/s", "frac": round(ach / peak, 4),
                "traffic": measured_traffic(kname, workload),
                "kernel": kname, "kernel_ms": round(kms, 3), "k": kq,
                "flops_per_launch": flops}
    flops = 3.0 * dim * tq["tile_pairs"]
    ach = flops / (tq["count_ms"] / 1e3) / 1e12
    return {"bound": "alu", "achieved": round(ach, 3),
            "peak": PEAK_FP32_VEC_TFLOPS, "unit": "TFLOP/s",
            "frac": round(ach / PEAK_FP32_VEC_TFLOPS, 4),
            "traffic": measured_traffic("k_tile<L2,count>", workload),
            "kernel": "k_tile<L2,count>", "kernel_ms": round(tq["count_ms"], 3),
            "flops_per_launch": flops}


class _Stats:
    """Stands in for the tree of a landmark run (its build happens inside
    the call; the graph's stats carry the build figures)."""

    def __init__(self, st):
        self.stats = st


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2a",
                    help="c2a c2b c2_50k c1 c3 c4 ang | c2q (bichromatic: 100K "
                         "queries against the C2 tree) | c5 (many clouds, one "
                         "batch per dim) | c5_loop (one call per cloud)")
    ap.add_argument("--precision", default="auto",
                    help="auto (the library chooses per query: i8 on Hamming "
                         "codes of <= 256 bits, fp16 on vector data where the "
                         "filter's margin is small against eps^2, else fp32) "
                         "| fp32 | bf16 | fp16 | fp8 | i8 (Hamming codes)")
    ap.add_argument("--sched", default="two_pass")
    ap.add_argument("--proj", type=int, default=0,
                    help="filter on leading principal coordinates: 0 automatic, "
                         "-1 off, else their number (multiple of 16)")
    ap.add_argument("--cpu-rows", type=int, default=1500)
    ap.add_argument("--cpu-tree-n", type=int, default=20000,
                    help="points of the oracle cover-tree timing (0: skip)")
    ap.add_argument("--c5-clouds", type=int, default=0,
                    help="use only the first K clouds of c5 (0: all 256)")
    ap.add_argument("--landmark", type=int, default=0,
                    help="run the landmark mode with this many Voronoi cells "
                         "(single-cloud workloads; 0: the direct build + query)")
    ap.add_argument("--tune", action="store_true",
                    help="autotune every batch first (untimed) and run the "
                         "tuned options")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the plain FP32 comparison steps")
    ap.add_argument("--plain-steps", type=int, default=2,
                    help="timed plain FP32 steps (after one untimed step)")
    ap.add_argument("--no-extra", action="store_true",
                    help="c2a: skip the learned-schedule and ~500-neighbour rows")
    ap.add_argument("--extra-steps", type=int, default=3)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the epsilon-graph path has no "
              "multi-GPU mode; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2510_14147_amd as fnn

    def prec_for(metric, dim):
        if args.precision == "auto":
            return "auto"
        if metric == "hamming":
            # the integer filter covers codes of <= 256 bits
            return "i8" if args.precision == "i8" and dim <= 256 else "fp32"
        if metric == "levenshtein":
            return "fp32"  # no filter precision to choose
        if args.precision == "i8":
            raise SystemExit("--precision i8 applies to Hamming codes only")
        return args.precision

    # jobs: (device points, offsets or None, metric, eps, dim, precision)
    jobs, groups = [], None
    if args.workload in ("c5", "c5_loop"):
        groups = c5_groups(args.c5_clouds or None)
        metric = "l2"
        n_all = sum(g[0].shape[0] for g in groups)
        desc = (f"c5_many_clouds_{sum(len(g[2]) for g in groups)}_sum_n{n_all}_"
                f"d3_16_64_{'batched' if args.workload == 'c5' else 'per_cloud'}")
        for x, off, eps, d in groups:
            xd = torch.from_numpy(x).cuda()
            if args.workload == "c5":
                jobs.append((xd, off, metric, eps, d, prec_for(metric, d)))
            else:
                for c in range(len(eps)):
                    jobs.append((xd[int(off[c]):int(off[c + 1])], None, metric,
                                 eps[c], d, prec_for(metric, d)))
        eps_desc = "per-cloud"
        x = None
    else:
        x, metric, eps, desc = workload(args.workload)
        n_all = x.shape[0]
        if metric == "hamming":
            xd = torch.from_numpy(x.view(np.int64)).cuda()
        else:
            xd = torch.from_numpy(x).cuda()
        # coordinates, or code bits on Hamming
        dim = {"l2": x.shape[1], "angular": x.shape[1],
               "hamming": 64 * x.shape[1]}.get(metric)
        jobs.append((xd, None, metric, eps, dim, prec_for(metric, dim or 0)))
        eps_desc = eps
    print(f"[bench] workload {desc} n={n_all} metric={metric} eps={eps_desc} "
          f"jobs={len(jobs)}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()

    # options per job: defaults with --precision / --sched, or tuned
    opts, tuning = [], []
    for xd, off, m, e, d, p in jobs:
        o = {"precision": p, "sched": args.sched, "proj": args.proj}
        if args.tune:
            t0 = time.perf_counter()
            o2 = off if off is not None else np.array([0, xd.shape[0]], np.int64)
            r = fnn.fnn_autotune(xd, o2, m, e, reps=2)
            o = {k: v for k, v in r["best"].items()
                 if k in ("zeta", "pack", "kmax", "graph_passes", "precision", "sched",
                          "lpt")}
            tuning.append({"dim": d, "best": o, "best_ms": r["best_ms"],
                           "base_ms": r["base_ms"], "candidates": r["ncand"],
                           "tune_s": time.perf_counter() - t0})
            print(f"[bench] tuned dim={d}: {tuning[-1]}", file=sys.stderr, flush=True)
        opts.append(o)
    BUILD_KEYS = ("zeta", "pack", "kmax", "graph_passes")

    INV_PREC = {v: k for k, v in fnn.PRECISIONS.items()}

    def run_job(xd, off, m, e, o, precision):
        """Build + query of one job: (tree, graph)."""
        bo = {k: v for k, v in o.items() if k in BUILD_KEYS}
        if args.landmark > 0 and off is None and args.workload != "c2q":
            g = fnn.fnn_landmark_eps_graph(xd, e, args.landmark, metric=m, seed=1,
                                           precision=precision, sched=o["sched"],
                                           proj=o.get("proj", 0),
                                           **{k: v for k, v in bo.items()
                                              if k in ("zeta", "pack", "kmax")})
            return _Stats(g.stats), g
        if args.workload == "c2q":
            # tree over the first 1M rows, bichromatic query of the rest
            tree = fnn.fnn_tree_build(xd[:1_000_000], m, **bo)
            g = fnn.fnn_eps_query(tree, xd[1_000_000:], e, precision=precision,
                                  proj=o.get("proj", 0))
        elif off is None:
            tree = fnn.fnn_tree_build(xd, m, **bo)
            g = fnn.fnn_eps_graph(tree, e, precision=precision, sched=o["sched"],
                                  proj=o.get("proj", 0), lpt=bool(o.get("lpt", 0)))
        else:
            tree = fnn.fnn_tree_build_batch(xd, off, m, **bo)
            g = fnn.fnn_eps_graph_batch(tree, e, precision=precision, sched=o["sched"],
                                        proj=o.get("proj", 0), lpt=bool(o.get("lpt", 0)))
        return tree, g

    kept = []

    def step(keep=False):
        res = []
        for (xd, off, m, e, d, _), o in zip(jobs, opts):
            tree, g = run_job(xd, off, m, e, o, o["precision"])
            # the precision the query ran with (the library resolves auto)
            used = INV_PREC[int(g.stats["precision_used"])]
            res.append((tree.stats, g.stats, g.nnz, d, used))
            if keep:
                kept.append(g)
            del tree, g
        return res

    for i in range(args.warmup):
        r = step()
        print(f"[bench] warmup {i}: nnz={sum(x[2] for x in r)} "
              f"build={sum(x[0]['build_ms'] for x in r):.1f} ms "
              f"query={sum(x[1]['total_ms'] for x in r):.1f} ms",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    stats = []
    t_all = time.perf_counter()
    for i in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = step(keep=(i == args.steps - 1))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        stats.append(r)
        print(f"[bench] step {i}: {dt * 1e3:.1f} ms nnz={sum(x[2] for x in r)}",
              file=sys.stderr, flush=True)
    total = time.perf_counter() - t_all
    ms = 1e3 * total / args.steps
    last = stats[-1]
    nnz = sum(x[2] for x in last)
    agg = lambda k, j: sum(x[j][k] for x in last)  # noqa: E731
    # every metric evaluation once per unordered pair: build, traversal
    # tests, exact leaf / survivor evaluations; the MFMA filter's screens
    # are reported apart
    evals = agg("build_dist_evals", 0) + agg("traverse_tests", 1) + agg("tile_pairs", 1)
    value = nnz / (ms / 1e3)
    # dominant kernel: that of the job with the longest count pass
    dom = max(last, key=lambda x: x[1]["count_ms"])
    roof = (roofline(dom[3], dom[4], dom[1], desc)
            if metric in ("l2", "angular") or dom[4] == "i8" else None)
    if roof is not None and len(last) > 1:
        roof["job"] = f"dim {dom[3]}, {dom[4]}"
    precs = sorted({x[4] for x in last})
    out = {
        "metric": "epsilon-graph edges/s (exact, symmetric CSR)",
        "value": value, "unit": "edges/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": desc + (f"_landmark{args.landmark}" if args.landmark else ""),
                   "n": int(n_all),
                   "dim": None if groups else jobs[0][4], "metric": metric,
                   "eps": None if groups else eps, "precision": "+".join(precs),
                   "sched": "+".join(sorted({o["sched"] for o in opts})),
                   "filter_proj_dim": sorted({int(x[1].get("proj_dim", 0)) for x in last}),
                   "nnz": int(nnz),
                   "mean_neighbors": nnz / n_all, "calls": len(jobs)},
        "dist_evals_per_s": evals / (ms / 1e3),
        "filter_screens_per_s": agg("filter_pairs", 1) / (ms / 1e3),
        "phases_ms": {"build": agg("build_ms", 0), "traverse": agg("traverse_ms", 1),
                      "count": agg("count_ms", 1), "scan": agg("scan_ms", 1),
                      "fill": agg("fill_ms", 1), "sort": agg("sort_ms", 1)},
        "counters": {k: agg(k, 1) for k in ("interactions", "tile_pairs",
                                            "traverse_tests", "fp64_rechecks",
                                            "filter_pairs", "filter_survivors",
                                            "packs", "nodes")} |
                    {"build_dist_evals": agg("build_dist_evals", 0),
                     "rounds": max(x[0]["rounds"] for x in last),
                     "netsel_passes": agg("netsel_passes", 0)},
        "roofline": roof,
        # launches of one step: kernels launched eagerly, recorded launch
        # sequences replayed, and the kernels those replays ran
        "launches": {"kernels": agg("launches", 0) + agg("launches", 1),
                     "graph_replays": agg("graph_launches", 0) + agg("graph_launches", 1),
                     "graph_kernels": agg("graph_kernels", 0) + agg("graph_kernels", 1)},
    }
    if tuning:
        out["tuned"] = tuning
    out["dtype"] = {"fp32": "f32", "bf16": "bf16 filter + f32", "fp16": "fp16 filter + f32",
                    "fp8": "fp8 filter + f32"}.get(
        "+".join(precs), "+".join(precs))
    if metric == "hamming":
        out["dtype"] = ("i8 MFMA (exact integer Gram)" if "i8" in precs
                        else "u64 (xor + popcount)")
    elif metric == "levenshtein":
        out["dtype"] = "u64 (bit-parallel edit distance)"
    if not args.no_plain and any(p != "fp32" for p in precs):
        # the same workload on the plain FP32 tiles, for the MFMA-vs-plain
        # ratio: one untimed step, then the mean of --plain-steps; the last
        # step's CSRs must equal the MFMA path's entry for entry
        def plain_step(keep=False):
            res, gs = [], []
            for (xd, off, m, e, d, _), o in zip(jobs, opts):
                tree, g = run_job(xd, off, m, e, o, "fp32")
                res.append((tree.stats, g.stats, g.nnz, d, "fp32"))
                if keep:
                    gs.append(g)
                del tree, g
            return res, gs
        plain_step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.plain_steps):
            pres, pgs = plain_step(keep=(i == args.plain_steps - 1))
        torch.cuda.synchronize()
        pms = 1e3 * (time.perf_counter() - t0) / args.plain_steps
        pnnz = sum(x[2] for x in pres)
        for ga, gb in zip(kept, pgs):
            same = (ga.nnz == gb.nnz and torch.equal(ga.row_ptr, gb.row_ptr)
                    and torch.equal(ga.col, gb.col)
                    and torch.equal(ga.dist.view(torch.int32), gb.dist.view(torch.int32)))
            if not same:
                raise SystemExit("plain FP32 and MFMA paths give different CSRs")
        del pgs
        pdom = max(pres, key=lambda x: x[1]["count_ms"])
        out["plain_fp32"] = {"ms_per_step": pms, "value": pnnz / (pms / 1e3),
                             "speedup_of_value": pms / ms, "steps": args.plain_steps,
                             "warmup": 1, "csr_identical": True,
                             "roofline": (roofline(pdom[3], "fp32", pdom[1], desc)
                                          if metric in ("l2", "angular") else None)}
        print(f"[bench] plain fp32 step: {pms:.1f} ms", file=sys.stderr, flush=True)
    kept.clear()
    if args.workload == "c2a" and not args.no_extra:
        # the same points at the ~500-neighbour radius, both schedules, the
        # learned schedule at the headline radius, and the BF16 and FP8
        # filters in place of the automatic choice
        xd, _, m, _, d, p = jobs[0]
        extra = {}
        for key, e, sched, pr in (("c2a_learned", eps, "learned", p),
                                  ("c2b_two_pass", W["c2"]["eps"][1], "two_pass", p),
                                  ("c2b_learned", W["c2"]["eps"][1], "learned", p),
                                  ("c2a_bf16", eps, "two_pass", "bf16"),
                                  ("c2a_fp8", eps, "two_pass", "fp8")):
            o = dict(opts[0], sched=sched, precision=pr)
            run_job(xd, None, m, e, o, pr)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.extra_steps):
                tree, g = run_job(xd, None, m, e, o, pr)
                st, tst, nz = g.stats, tree.stats, g.nnz
                del tree, g
            torch.cuda.synchronize()
            ems = 1e3 * (time.perf_counter() - t0) / args.extra_steps
            used = INV_PREC[int(st["precision_used"])]
            extra[key] = {"eps": e, "sched": sched, "nnz": int(nz),
                          "mean_neighbors": nz / n_all, "ms_per_step": ems,
                          "value": nz / (ems / 1e3), "steps": args.extra_steps,
                          "phases_ms": {"build": tst["build_ms"], "count": st["count_ms"],
                                        "fill": st["fill_ms"], "sort": st["sort_ms"]},
                          "filter_passes": 1 + int(st["overflow_rows"]) if used != "fp32" else 0,
                          "roofline": roofline(d, used, st, desc)}
            if sched == "learned":
                extra[key]["pred_mae_log1p_degree"] = st["pred_mae"]
                extra[key]["pred_sum_ratio"] = st["pred_sum_ratio"]
            print(f"[bench] {key}: {ems:.1f} ms nnz={nz}", file=sys.stderr, flush=True)
        out["extra"] = extra
    if not args.no_cpu:
        if groups:
            out["cpu_baseline"] = cpu_baseline_c5(groups, args.cpu_rows)
        else:
            out["cpu_baseline"] = cpu_baseline(x, metric, eps, args.cpu_rows)
            if args.workload in ("c2a", "c2b") and args.cpu_tree_n > 0:
                # the oracle's cover tree (Algorithms 1-3) on a prefix it
                # finishes in seconds, at the radius calibrated for 50K points
                out["cpu_baseline"]["cover_tree"] = cpu_cover_tree(
                    x, metric, W["c2_50k"]["eps"][0], args.cpu_tree_n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
