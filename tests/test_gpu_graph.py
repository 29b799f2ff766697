"""Net-selection passes replayed from a recorded hipGraph give the same cover
tree as eager passes (one host check per pass): every exported array is
identical, over several replays interleaved with eager work, for single
trees and for a batch of clouds, and the graphs built on them match the
oracle."""
import numpy as np
import pytest

from paper_2510_14147_amd import datagen as G

pytestmark = pytest.mark.gpu

MID = {"l2": 0, "angular": 1, "hamming": 2, "levenshtein": 3}
KEYS = ("order", "center", "radius", "level", "child_begin", "child_count",
        "pt_begin", "pt_end")


@pytest.fixture(scope="module")
def fnn():
    import torch
    assert torch.cuda.is_available()
    import paper_2510_14147_amd as f
    f.lib()
    return f


def same_tree(a, b):
    assert a["nnodes"] == b["nnodes"]
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), k


CASES = [
    ("l2", lambda: G.c1_clusters(n_centers=10, per_center=600), 0.1),
    ("l2", lambda: G.c2_manifold(n=6000, chunk=6000), 3.0),
    ("hamming", lambda: G.random_codes(4000, 256, seed=5, flip=0.08), 30),
    ("levenshtein", lambda: G.random_strings(1200, seed=6, stride=64,
                                             min_len=20, max_len=60), 7),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_graph_replay_equals_eager(fnn, orc, case):
    import torch
    metric, gen, eps = CASES[case]
    x = gen()
    print(f"[case] graph replay metric={metric} n={len(x)}", flush=True)
    eager = fnn.fnn_tree_export(fnn.fnn_tree_build(x, metric, zeta=8, graph_passes=1))
    for rep, gp in enumerate((4, 2, 6)):
        # eager work on the same stream between the replays
        y = torch.randn(1 << 16, device="cuda").cumsum(0)
        assert torch.isfinite(y).all()
        t = fnn.fnn_tree_build(x, metric, zeta=8, graph_passes=gp)
        same_tree(eager, fnn.fnn_tree_export(t))
        if rep == 0:
            rp, col, dist = fnn.fnn_eps_graph(t, eps).to_numpy()
            ref = orc.bruteforce(x, MID[metric], eps)
            cmp = orc.compare_csr(rp, col, dist, *ref, rtol=1e-5)
            assert cmp["ok"], cmp


def test_graph_replay_batch(fnn):
    import torch
    specs = G.c5_cloud_specs()[:12]
    clouds = [G.c5_cloud(s, n_override=min(s["n"], 2500)) for s in specs if s["dim"] == 16]
    off = np.concatenate([[0], np.cumsum([len(c) for c in clouds])]).astype(np.int64)
    X = np.concatenate(clouds)
    print(f"[case] graph replay batch clouds={len(clouds)} n={len(X)}", flush=True)
    eager = fnn.fnn_tree_export(fnn.fnn_tree_build_batch(X, off, "l2", graph_passes=1))
    for gp in (4, 8):
        torch.cuda.synchronize()
        t = fnn.fnn_tree_build_batch(X, off, "l2", graph_passes=gp)
        same_tree(eager, fnn.fnn_tree_export(t))


TRAV_CASES = [
    ("l2", lambda: G.c1_clusters(n_centers=10, per_center=600), 0.1),
    ("l2", lambda: G.c2_manifold(n=6000, chunk=6000), 3.0),
    ("hamming", lambda: G.random_codes(4000, 256, seed=5, flip=0.08), 30),
    ("levenshtein", lambda: G.random_strings(1200, seed=6, stride=64,
                                             min_len=20, max_len=60), 7),
]


@pytest.mark.parametrize("case", range(len(TRAV_CASES)))
def test_traversal_levels_replayed_equal_eager(fnn, orc, case):
    """Traversal levels replayed from a graph over device-resident frontier
    queues (2, 4, 8 levels per replay), the same with buffers so small that
    the replay stops at its first level and the eager loop finishes, and all
    levels eager: bit-identical CSRs, equal to the oracle's graph."""
    metric, gen, eps = TRAV_CASES[case]
    x = gen()
    print(f"[case] traversal replay metric={metric} n={len(x)}", flush=True)
    t = fnn.fnn_tree_build(x, metric, zeta=8)
    base = fnn.fnn_eps_graph(t, eps, graph_passes=1)
    rp, col, dist = base.to_numpy()
    assert base.stats["traverse_tests"] > 0
    ref = orc.bruteforce(x, MID[metric], eps)
    cmp = orc.compare_csr(rp, col, dist, *ref, rtol=1e-5)
    assert cmp["ok"], cmp
    for kw in (dict(graph_passes=2), dict(graph_passes=4), dict(graph_passes=8),
               dict(graph_passes=4, list_cap=64)):
        g = fnn.fnn_eps_graph(t, eps, **kw)
        r2, c2, d2 = g.to_numpy()
        assert np.array_equal(rp, r2), kw
        assert np.array_equal(col, c2), kw
        assert np.array_equal(dist.view(np.uint32), d2.view(np.uint32)), kw
        assert g.stats["traverse_tests"] == base.stats["traverse_tests"], kw
        assert g.stats["interactions"] == base.stats["interactions"], kw
        if kw.get("list_cap") is None:
            assert g.stats["graph_launches"] > 0, kw


def test_traversal_levels_replayed_forest(fnn):
    """The same over a forest of many clouds (the frontier starts at every
    cloud root) and a bichromatic query."""
    specs = G.c5_cloud_specs()[:16]
    clouds = [G.c5_cloud(s, n_override=min(s["n"], 2500)) for s in specs if s["dim"] == 16]
    off = np.concatenate([[0], np.cumsum([len(c) for c in clouds])]).astype(np.int64)
    X = np.concatenate(clouds)
    eps = [0.4 + 0.05 * i for i in range(len(clouds))]
    print(f"[case] traversal replay forest clouds={len(clouds)} n={len(X)}", flush=True)
    t = fnn.fnn_tree_build_batch(X, off, "l2")
    base = fnn.fnn_eps_graph_batch(t, eps, graph_passes=1).to_numpy()
    for gp in (2, 6):
        g = fnn.fnn_eps_graph_batch(t, eps, graph_passes=gp).to_numpy()
        for a, b in zip(base, g):
            assert np.array_equal(a.view(np.uint32) if a.dtype == np.float32 else a,
                                  b.view(np.uint32) if b.dtype == np.float32 else b), gp
    q = X[::7] + np.float32(0.01)
    t1 = fnn.fnn_tree_build(X, "l2")
    a = fnn.fnn_eps_query(t1, q, 0.5, graph_passes=1).to_numpy()
    assert a[0][-1] > 0
    for gp in (2, 4):
        b = fnn.fnn_eps_query(t1, q, 0.5, graph_passes=gp).to_numpy()
        for u, v in zip(a, b):
            assert np.array_equal(u.view(np.uint32) if u.dtype == np.float32 else u,
                                  v.view(np.uint32) if v.dtype == np.float32 else v), gp
