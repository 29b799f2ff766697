"""Parity at the benchmark sizes (GPU): the full graph is built exactly as the
benchmark builds it; seeded sample rows are checked against the oracle's
exhaustive rows (the oracle cannot do all rows at these sizes), and
properties that hold at any size (symmetry, no self loops, sorted rows,
row_ptr consistency) are checked on the whole graph on the device."""
import json
import os

import numpy as np
import pytest

from paper_2510_14147_amd import datagen as G

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
W = json.load(open(os.path.join(ROOT, "paper_2510_14147_amd", "workloads.json")))
MID = {"l2": 0, "angular": 1, "hamming": 2, "levenshtein": 3}


@pytest.fixture(scope="module")
def fnn():
    import torch
    assert torch.cuda.is_available()
    import paper_2510_14147_amd as f
    f.lib()
    return f


def whole_graph_properties(g):
    """Symmetric (with identical distance bits), no self loops, strictly
    ascending columns, consistent row_ptr -- checked on the device."""
    import torch
    n = g.n
    rp = g.row_ptr
    assert int(rp[0]) == 0 and int(rp[-1]) == g.nnz
    assert bool(torch.all(rp[1:] >= rp[:-1]))
    rows = torch.repeat_interleave(torch.arange(n, device=rp.device),
                                   (rp[1:] - rp[:-1]))
    col = g.col.long()
    assert not bool(torch.any(rows == col))
    same = rows[1:] == rows[:-1]
    assert not bool(torch.any(same & (col[1:] <= col[:-1])))
    fwd = rows * n + col
    bwd = col * n + rows
    sb, ob = torch.sort(bwd)
    # fwd is already sorted (rows ascending, columns ascending)
    assert torch.equal(fwd, sb)
    d = g.dist.view(torch.int32)
    assert torch.equal(d, d[ob])


def sampled_rows(fnn, orc, x, metric, eps, nrows, seed, **kw):
    print(f"[case] scale metric={metric} n={len(x)} eps={eps} {kw}", flush=True)
    tree = fnn.fnn_tree_build(x, metric)
    g = fnn.fnn_eps_graph(tree, eps, **kw)
    whole_graph_properties(g)
    rng = np.random.default_rng(seed)
    rows = np.sort(rng.choice(len(x), size=nrows, replace=False))
    ref = orc.bruteforce(x, MID[metric], eps, rows=rows)
    rp = g.row_ptr.cpu().numpy()
    col = g.col.cpu().numpy()
    dist = g.dist.cpu().numpy()
    for r, i in enumerate(rows):
        a = slice(rp[i], rp[i + 1])
        b = slice(ref[0][r], ref[0][r + 1])
        assert np.array_equal(col[a], ref[1][b]), (i, rp[i + 1] - rp[i],
                                                  ref[0][r + 1] - ref[0][r])
        np.testing.assert_allclose(dist[a], ref[2][b], rtol=1e-5, atol=0)
    return g


def test_c2a_full_size_sampled(fnn, orc):
    x = G.c2_manifold()
    g = sampled_rows(fnn, orc, x, "l2", W["c2"]["eps"][0], 150, 21)
    assert 40 < g.nnz / g.n < 120


def test_c2_50k_full_parity(fnn, orc):
    x = G.c2_manifold(n=30_000)
    eps = W["c2_50k"]["eps"][0]
    tree = fnn.fnn_tree_build(x, "l2")
    g = fnn.fnn_eps_graph(tree, eps)
    ref = orc.bruteforce(x, 0, eps)
    cmp = orc.compare_csr(*g.to_numpy(), *ref, rtol=1e-5)
    assert cmp["ok"], cmp


def test_c3_full_size_sampled(fnn, orc):
    x = G.c3_hamming()
    sampled_rows(fnn, orc, x, "hamming", 24.0, 100, 23)


def test_c4_full_size_sampled(fnn, orc):
    x = G.c4_strings()
    sampled_rows(fnn, orc, x, "levenshtein", 6.0, 100, 24)


def test_c3_full_size_sampled_int8(fnn, orc):
    # the integer MFMA filter on the 2M x 256-bit workload
    x = G.c3_hamming()
    g = sampled_rows(fnn, orc, x, "hamming", 24.0, 100, 25, precision="i8")
    assert g.stats["filter_survivors"] <= g.nnz // 2


def _same_csr_on_device(g1, g2):
    import torch
    assert g1.nnz == g2.nnz
    assert torch.equal(g1.row_ptr, g2.row_ptr)
    assert torch.equal(g1.col, g2.col)
    assert torch.equal(g1.dist.view(torch.int32), g2.dist.view(torch.int32))


def test_c2a_bench_path_sampled(fnn, orc):
    """Exactly what the benchmark times: automatic precision (FP16 filter on
    16 principal coordinates), the closed-form dense pack list, two-pass
    emission; sampled rows against the oracle, and every entry against the
    plain FP32 path on the same tree."""
    x = G.c2_manifold()
    eps = W["c2"]["eps"][0]
    print(f"[case] c2a bench path n={len(x)}", flush=True)
    tree = fnn.fnn_tree_build(x, "l2")
    g = fnn.fnn_eps_graph(tree, eps, precision="auto", sched="two_pass", proj=0)
    st = g.stats
    assert st["precision_used"] == fnn.PRECISIONS["fp16"]
    assert st["proj_dim"] == 16
    # the dense list: every pack against every later pack, no traversal
    assert st["interactions"] == st["packs"] * (st["packs"] + 1) // 2
    assert st["filter_pairs"] == len(x) * (len(x) - 1) // 2
    assert st["overflow_rows"] == 0
    whole_graph_properties(g)
    _check_rows(orc, x, "l2", eps, g, 200, 31)
    g2 = fnn.fnn_eps_graph(tree, eps, precision="fp32")
    _same_csr_on_device(g, g2)


def _check_rows(orc, x, metric, eps, g, nrows, seed):
    rng = np.random.default_rng(seed)
    rows = np.sort(rng.choice(len(x), size=nrows, replace=False))
    ref = orc.bruteforce(x, MID[metric], eps, rows=rows)
    rp = g.row_ptr.cpu().numpy()
    col = g.col.cpu().numpy()
    dist = g.dist.cpu().numpy()
    for r, i in enumerate(rows):
        a = slice(rp[i], rp[i + 1])
        b = slice(ref[0][r], ref[0][r + 1])
        assert np.array_equal(col[a], ref[1][b]), (i, rp[i + 1] - rp[i],
                                                  ref[0][r + 1] - ref[0][r])
        np.testing.assert_allclose(dist[a], ref[2][b], rtol=1e-5, atol=0)


def test_c2b_two_pass_and_learned_sampled(fnn, orc):
    """The ~500-neighbour radius at full size, both schedules: sampled rows
    against the oracle; the learned schedule's CSR equals the two-pass one
    entry for entry."""
    x = G.c2_manifold()
    eps = W["c2"]["eps"][1]
    print(f"[case] c2b n={len(x)} eps={eps}", flush=True)
    tree = fnn.fnn_tree_build(x, "l2")
    g = fnn.fnn_eps_graph(tree, eps, precision="auto", sched="two_pass")
    assert 350 < g.nnz / g.n < 700
    assert g.stats["precision_used"] == fnn.PRECISIONS["fp16"]
    assert g.stats["overflow_rows"] == 0      # one filter pass
    whole_graph_properties(g)
    _check_rows(orc, x, "l2", eps, g, 150, 32)
    print("[case] c2b learned", flush=True)
    gl = fnn.fnn_eps_graph(tree, eps, precision="auto", sched="learned")
    _same_csr_on_device(g, gl)
    assert gl.stats["overflow_rows"] == 0


def test_c5_full_size_sampled(fnn, orc):
    """All 256 clouds at full size (one forest per dimension, as the
    benchmark runs them), automatic precision; two sampled rows per cloud
    against the oracle's rows of that cloud alone."""
    specs = G.c5_cloud_specs()
    rng = np.random.default_rng(33)
    for d in (3, 16, 64):
        sel = [s for s in specs if s["dim"] == d]
        xs = [G.c5_cloud(s) for s in sel]
        off = np.concatenate([[0], np.cumsum([len(v) for v in xs])]).astype(np.int64)
        x = np.concatenate(xs, axis=0)
        eps = [W["c5"]["eps"][s["cloud"]] for s in sel]
        print(f"[case] c5 dim={d} clouds={len(sel)} n={len(x)}", flush=True)
        tree = fnn.fnn_tree_build_batch(x, off, "l2")
        g = fnn.fnn_eps_graph_batch(tree, eps, precision="auto")
        whole_graph_properties(g)
        rp = g.row_ptr.cpu().numpy()
        col = g.col.cpu().numpy()
        dist = g.dist.cpu().numpy()
        for c in range(len(sel)):
            lo, hi = int(off[c]), int(off[c + 1])
            rows = np.sort(rng.choice(hi - lo, size=min(2, hi - lo), replace=False))
            ref = orc.bruteforce(x[lo:hi], 0, eps[c], rows=rows)
            for r, i in enumerate(rows):
                a = slice(rp[lo + i], rp[lo + i + 1])
                b = slice(ref[0][r], ref[0][r + 1])
                assert np.array_equal(col[a] - lo, ref[1][b]), (d, c, i)
                np.testing.assert_allclose(dist[a], ref[2][b], rtol=1e-5, atol=0)
        del tree, g
