"""Autotuner: every candidate option set yields the identical graph (bit for
bit), the tuned options are no slower than the base ones by the tuner's own
timing, and a second call for the same input shape is answered from the
cache."""
import numpy as np
import pytest

from paper_2510_14147_amd import datagen as G

pytestmark = pytest.mark.gpu

MID = {"l2": 0, "angular": 1, "hamming": 2, "levenshtein": 3}
BUILD = ("zeta", "pack", "kmax", "graph_passes")
QUERY = ("precision", "sched", "lpt")


@pytest.fixture(scope="module")
def fnn():
    import torch
    assert torch.cuda.is_available()
    import paper_2510_14147_amd as f
    f.lib()
    return f


def run(fnn, X, off, metric, eps, **opt):
    b = {k: v for k, v in opt.items() if k in BUILD}
    q = {k: v for k, v in opt.items() if k in QUERY}
    if len(off) > 2:
        t = fnn.fnn_tree_build_batch(X, off, metric, **b)
        g = fnn.fnn_eps_graph_batch(t, eps, **q)
    else:
        t = fnn.fnn_tree_build(X, metric, **b)
        g = fnn.fnn_eps_graph(t, eps[0], **q)
    return g.to_numpy()


def same(a, b):
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[2].view(np.uint32), b[2].view(np.uint32))


def check_tuner(fnn, orc, X, off, metric, eps, candidates):
    fnn.fnn_autotune_clear()
    r = fnn.fnn_autotune(X, off, metric, eps, reps=1)
    print(f"[case] tune {metric} n={len(X)} -> {r}", flush=True)
    assert not r["cached"] and r["ncand"] >= 3
    assert r["best_ms"] <= r["base_ms"]
    r2 = fnn.fnn_autotune(X, off, metric, eps, reps=1)
    assert r2["cached"] and r2["best"] == r["best"]
    ref = run(fnn, X, off, metric, eps)
    for opt in candidates + [r["best"]]:
        same(ref, run(fnn, X, off, metric, eps, **opt))
    return ref


def test_tune_batch_l2(fnn, orc):
    specs = [s for s in G.c5_cloud_specs()[:30] if s["dim"] == 16][:6]
    clouds = [G.c5_cloud(s, n_override=min(s["n"], 2500)) for s in specs]
    off = np.concatenate([[0], np.cumsum([len(c) for c in clouds])]).astype(np.int64)
    X = np.concatenate(clouds)
    eps = [0.1 + 0.05 * i for i in range(len(clouds))]
    cands = [dict(precision="bf16"), dict(sched="learned"), dict(zeta=32),
             dict(zeta=128), dict(kmax=32), dict(kmax=128), dict(pack=32),
             dict(graph_passes=2), dict(graph_passes=8), dict(sched="learned", lpt=True)]
    rp, col, dist = check_tuner(fnn, orc, X, off, "l2", eps, cands)
    # and the graph is the oracle's (first cloud)
    n0 = int(off[1])
    ref = orc.bruteforce(clouds[0], 0, eps[0])
    assert np.array_equal(rp[:n0 + 1], ref[0]) and np.array_equal(col[:rp[n0]], ref[1])


def test_tune_single_hamming(fnn, orc):
    x = G.random_codes(6000, 256, seed=8, flip=0.07)
    off = np.array([0, len(x)], np.int64)
    cands = [dict(zeta=32), dict(zeta=128), dict(kmax=32), dict(kmax=128),
             dict(sched="learned"), dict(pack=32), dict(graph_passes=2)]
    rp, col, dist = check_tuner(fnn, orc, x, off, "hamming", [20.0], cands)
    ref = orc.bruteforce(x, MID["hamming"], 20.0)
    assert np.array_equal(rp, ref[0]) and np.array_equal(col, ref[1])


def test_launch_counts_reported(fnn):
    """Stats carry the launches of a call: eager kernels, graph replays and
    the kernels those replays ran."""
    x = G.c1_clusters()
    t = fnn.fnn_tree_build(x, "l2")
    g = fnn.fnn_eps_graph(t, 0.1)
    bs, qs = t.stats, g.stats
    print(f"[launches] build: {bs['launches']} kernels + {bs['graph_launches']} graph "
          f"replays ({bs['graph_kernels']} kernels); query: {qs['launches']} kernels",
          flush=True)
    assert bs["launches"] > 0 and qs["launches"] > 0
    assert bs["graph_launches"] > 0 and bs["graph_kernels"] >= bs["graph_launches"]
