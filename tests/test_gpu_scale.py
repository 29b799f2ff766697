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
