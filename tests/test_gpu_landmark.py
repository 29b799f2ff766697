"""Landmark mode on one GPU (Section IV-D Algorithm 5, Section IV-E Lemma 1
and Algorithm 6): the graph assembled from Voronoi cells, their eps-ghosts
and one batched forest over cells + ghosts must equal the oracle's
epsilon-graph exactly and the direct path's CSR bit for bit."""
import json
import math
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


def check(fnn, orc, x, metric, eps, ncells, seed=1, **kw):
    print(f"[case] landmark {metric} n={len(x)} eps={eps} cells={ncells} {kw}", flush=True)
    g = fnn.fnn_landmark_eps_graph(x, eps, ncells, metric=metric, seed=seed, **kw)
    ref = orc.bruteforce(x, MID[metric], eps)
    cmp = orc.compare_csr(*g.to_numpy(), *ref)
    assert cmp["missing"] == 0 and cmp["extra"] == 0, cmp
    assert cmp["ok"], cmp
    st = g.stats
    assert st["landmark_cells"] == min(ncells, len(x))
    assert st["landmark_rows"] >= len(x)
    # bit for bit the direct path's CSR
    tree = fnn.fnn_tree_build(x, metric)
    d = fnn.fnn_eps_graph(tree, eps, **{k: v for k, v in kw.items() if k in ("precision",)})
    for u, v in zip(g.to_numpy(), d.to_numpy()):
        assert np.array_equal(u.view(np.uint8), v.view(np.uint8))
    return g


@pytest.mark.parametrize("ncells", [1, 10, 60])
def test_landmark_c1(fnn, orc, ncells):
    x = G.c1_clusters()
    check(fnn, orc, x, "l2", W["c1"]["eps"], ncells)


def test_landmark_c2_prefix_auto(fnn, orc):
    """The 128-d manifold: nearly every point is a ghost of several cells;
    the per-cell queries run the MFMA filter."""
    x = G.c2_manifold(n=30_000)
    g = check(fnn, orc, x, "l2", W["c2_50k"]["eps"][0], 10, precision="auto")
    print(f"[landmark] c2 30K: rows {g.stats['landmark_rows']} for 30000 points", flush=True)


def test_landmark_random_with_duplicates(fnn, orc):
    x = G.random_points(4000, 5, seed=12, duplicates=200)
    check(fnn, orc, x, "l2", 0.2, 25, seed=7)


def test_landmark_angular(fnn, orc):
    x = G.angular_dirs(n=6000, dim=16)
    check(fnn, orc, x, "angular", W["ang"]["eps"], 12)


def test_landmark_hamming(fnn, orc):
    x = G.random_codes(5000, 256, seed=9, n_centers=16, flip=0.06)
    check(fnn, orc, x, "hamming", 30.0, 16)


def test_landmark_levenshtein(fnn, orc):
    x = G.random_strings(1500, seed=10, n_seeds=15)
    check(fnn, orc, x, "levenshtein", 6.0, 8)


def test_landmark_degenerate(fnn, orc):
    # every point its own cell; a radius that makes every point a ghost of
    # every cell; all points identical
    x = G.random_points(300, 3, seed=13)
    check(fnn, orc, x, "l2", 0.3, 1000)
    check(fnn, orc, x, "l2", 5.0, 7)
    y = np.zeros((200, 4), np.float32)
    check(fnn, orc, y, "l2", 0.5, 5)


def test_landmark_errors(fnn):
    x = G.random_points(100, 3, seed=14)
    with pytest.raises(fnn.FnnError) as e:
        fnn.fnn_landmark_eps_graph(x, 0.2, 0)
    assert e.value.code == -1
    with pytest.raises(fnn.FnnError) as e:
        fnn.fnn_landmark_eps_graph(x, math.nan, 4)
    assert e.value.code == -1
