"""GPU parity of the bichromatic range query (fnn_eps_query): rows of a
query set against a tree's points.  The reference is the oracle's brute
force on the concatenation [tree points; queries], restricted to the query
rows and to the tree's columns."""
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


def query_reference(orc, P, Q, metric, eps):
    X = np.concatenate([P, Q], axis=0)
    nP = len(P)
    rp, col, dist = orc.bruteforce(X, MID[metric], eps, rows=np.arange(nP, nP + len(Q)))
    keep = col < nP
    rows = np.repeat(np.arange(len(Q)), np.diff(rp))
    counts = np.bincount(rows[keep], minlength=len(Q))
    rp2 = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return rp2, col[keep], dist[keep]


def check_query(fnn, orc, P, Q, metric, eps, **kw):
    print(f"[case] query metric={metric} nP={len(P)} nQ={len(Q)} eps={eps} kw={kw}",
          flush=True)
    tree = fnn.fnn_tree_build(P, metric)
    g = fnn.fnn_eps_query(tree, Q, eps, **kw)
    assert g.n == len(Q)
    rp, col, dist = g.to_numpy()
    ref = query_reference(orc, P, Q, metric, eps)
    cmp = orc.compare_csr(rp, col, dist, *ref, rtol=1e-5)
    assert cmp["missing"] == 0 and cmp["extra"] == 0, cmp
    assert cmp["ok"], cmp
    return g


def test_query_l2_with_duplicates(fnn, orc):
    P = G.random_points(3000, 5, seed=41, duplicates=60)
    Q = G.random_points(1000, 5, seed=42)
    Q[:50] = P[100:150]  # queries equal to tree points: distance 0 edges
    check_query(fnn, orc, P, Q, "l2", 0.25)


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp16", "auto"])
def test_query_manifold(fnn, orc, precision):
    X = G.c2_manifold(n=10000)
    g = check_query(fnn, orc, X[:8000], X[8000:], "l2", W["c2_50k"]["eps"][1],
                    precision=precision, validate=precision != "fp32")
    assert g.stats["validate_mismatch"] == 0


def test_query_angular(fnn, orc):
    X = G.angular_dirs(n=6000, dim=16, seed=43)
    check_query(fnn, orc, X[:4500], X[4500:], "angular", W["ang"]["eps"], precision="bf16",
                validate=True)


@pytest.mark.parametrize("precision", ["fp32", "i8"])
def test_query_hamming(fnn, orc, precision):
    X = G.random_codes(4000, 256, seed=44, n_centers=10, flip=0.06)
    check_query(fnn, orc, X[:3000], X[3000:], "hamming", 30, precision=precision)


def test_query_levenshtein(fnn, orc):
    X = G.random_strings(1500, seed=45, n_seeds=30, min_len=30, max_len=80, p_edit=0.04)
    check_query(fnn, orc, X[:1000], X[1000:], "levenshtein", 6)


def test_query_levenshtein_alphabets_differ(fnn, orc):
    """Queries over a smaller alphabet than the tree's, and queries holding a
    symbol the tree never uses: the pair forest takes one alphabet for
    both sets."""
    X = G.random_strings(1200, seed=46, n_seeds=24, min_len=30, max_len=70, p_edit=0.04)
    P, Q = X[:800].copy(), X[800:].copy()
    P[P == 3] = 7                      # tree alphabet {0, 1, 2, 7}: sigma 8
    check_query(fnn, orc, P, Q, "levenshtein", 6)      # queries: sigma 4
    Q2 = Q.copy()
    Q2[Q2 == 2] = 200                  # a symbol the tree lacks
    check_query(fnn, orc, P, Q2, "levenshtein", 6)


def test_levenshtein_large_alphabet(fnn, orc):
    """Symbols up to 254 (0xFF pads the rows)."""
    rng = np.random.default_rng(47)
    X = G.random_strings(1500, seed=47, n_seeds=30, min_len=20, max_len=60, p_edit=0.05)
    lut = rng.permutation(255).astype(np.uint8)
    Y = np.where(X == 0xFF, X, lut[np.minimum(X, 254)]).astype(np.uint8)
    tree = fnn.fnn_tree_build(Y, "levenshtein")
    g = fnn.fnn_eps_graph(tree, 5.0)
    ref = orc.bruteforce(Y, MID["levenshtein"], 5.0)
    cmp = orc.compare_csr(*g.to_numpy(), *ref)
    assert cmp["ok"] and cmp["ref_nnz"] > 1000, cmp


def test_query_edge_cases(fnn, orc):
    P = G.random_points(2000, 3, seed=46)
    check_query(fnn, orc, P, P[7:8].copy(), "l2", 0.2)               # one query
    check_query(fnn, orc, P[:1].copy(), P[:300].copy(), "l2", 0.3)   # one-point tree
    far = P[:40] + 100.0
    g = check_query(fnn, orc, P, far, "l2", 0.2)                     # nothing in range
    assert g.nnz == 0


def test_query_rejects(fnn, orc):
    P = G.random_points(500, 4, seed=47)
    X = np.concatenate([P, P], axis=0)
    forest = fnn.fnn_tree_build_batch(X, np.array([0, 500, 1000]), "l2")
    with pytest.raises(fnn.FnnError) as e:
        fnn.fnn_eps_query(forest, P, 0.3)
    assert e.value.code == fnn.FNN_EUNSUPPORTED
    tree = fnn.fnn_tree_build(P, "l2")
    with pytest.raises(fnn.FnnError) as e:
        fnn.fnn_eps_query(tree, P, 0.3, sched="learned")
    assert e.value.code in (fnn.FNN_EUNSUPPORTED, fnn.FNN_EINVAL)
    with pytest.raises(fnn.FnnError) as e:
        fnn.fnn_eps_query(tree, P, -1.0)
    assert e.value.code == fnn.FNN_EINVAL
