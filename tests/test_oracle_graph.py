"""Pins for the oracle's epsilon-graph (CPU only): closed forms, the
hand-derived worked example, and two independent constructions (exhaustive
pairs vs the cover-tree query of Algorithm 3) agreeing on every metric."""
import json
import math
import os

import numpy as np
import pytest

from paper_2510_14147_amd import datagen as G

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_worked_example_fixture(orc):
    fx = json.load(open(os.path.join(GOLDEN, "worked_example_1d.json")))
    P = np.asarray(fx["points"], np.float32)
    rp, col, dist = orc.bruteforce(P, orc.L2, fx["eps"])
    assert rp.tolist() == fx["csr"]["row_ptr"]
    assert col.tolist() == fx["csr"]["col"]
    assert dist.tolist() == fx["csr"]["dist"]
    t = orc.tree_build(P, orc.L2, zeta=fx["zeta"])
    root = fx["tree"]["root"]
    assert t["center"][0] == root["center"] and t["radius"][0] == root["radius"]
    assert t["level"][0] == root["level"]
    kids = t["center"][t["child_begin"][0]:t["child_begin"][0] + t["child_count"][0]]
    assert kids.tolist() == root["children_centers"]
    hub = fx["tree"]["hub_0_1_3"]
    v = t["child_begin"][0]
    assert t["radius"][v] == hub["radius"] and t["level"][v] == hub["level"]
    assert t["center"][t["child_begin"][v]:t["child_begin"][v] + t["child_count"][v]].tolist() \
        == hub["children_centers"]
    assert sorted(t["order"][t["pt_begin"][v]:t["pt_end"][v]].tolist()) == hub["points"]
    rq = orc.tree_query(P, orc.L2, fx["eps"], t)
    assert rq[0].tolist() == fx["csr"]["row_ptr"] and rq[1].tolist() == fx["csr"]["col"]


@pytest.mark.parametrize("k,D", [(5, 2), (4, 3), (3, 4)])
def test_grid_unit_radius_closed_form(orc, k, D):
    P = G.grid_points(k, D)
    rp, col, dist = orc.bruteforce(P, orc.L2, 1.0)
    assert rp[-1] == 2 * D * k ** (D - 1) * (k - 1)
    assert np.all(dist == 1.0)


def test_grid_eight_neighbourhood_closed_form(orc):
    k = 7
    P = G.grid_points(k, 2)
    rp, col, dist = orc.bruteforce(P, orc.L2, 1.5)
    assert rp[-1] == 4 * k * (k - 1) + 4 * (k - 1) ** 2
    t = orc.tree_build(P, orc.L2, zeta=2)
    rq = orc.tree_query(P, orc.L2, 1.5, t)
    assert np.array_equal(rq[0], rp) and np.array_equal(rq[1], col)


def test_angular_cross_polytope_closed_form(orc):
    D = 5
    P = np.concatenate([np.eye(D), -np.eye(D)]).astype(np.float32)
    rp, _, dist = orc.bruteforce(P, orc.ANGULAR, math.pi / 2 + 0.1)
    assert rp[-1] == 2 * D * (2 * D - 2)
    assert np.allclose(dist, math.pi / 2, atol=1e-15)
    rp, _, _ = orc.bruteforce(P, orc.ANGULAR, math.pi / 2 - 0.1)
    assert rp[-1] == 0
    rp, _, _ = orc.bruteforce(P, orc.ANGULAR, 3.5)      # eps > pi: complete
    assert rp[-1] == 2 * D * (2 * D - 1)


def test_hamming_complete_and_duplicates_only(orc):
    X = G.random_codes(200, 128, seed=4)
    X[150:160] = X[10:20]                       # 10 planted duplicate pairs
    n = X.shape[0]
    rp, _, _ = orc.bruteforce(X, orc.HAMMING, 128.0)
    assert rp[-1] == n * (n - 1)
    rp, col, dist = orc.bruteforce(X, orc.HAMMING, 0.5)
    # ordered duplicate pairs only (the random codes themselves are distinct)
    _, counts = np.unique(X, axis=0, return_counts=True)
    assert rp[-1] == int(np.sum(counts * (counts - 1)))
    assert np.all(dist == 0.0)


def test_levenshtein_length_only_graph(orc):
    # strings a^k: d(a^i, a^j) = |i - j|, so eps = 1 links consecutive lengths
    S = np.full((8, 16), 0xFF, np.uint8)
    for i in range(8):
        S[i, :i] = 2
    rp, col, dist = orc.bruteforce(S, orc.LEVENSHTEIN, 1.0)
    assert rp[-1] == 2 * 7
    assert np.all(dist == 1.0)


def orc_l2():
    return G.random_points(1500, 5, seed=21, duplicates=30), 0.12


def orc_ang():
    return G.angular_dirs(n=1500, dim=6, seed=22), 0.2


def orc_ham():
    return G.random_codes(1500, 192, seed=23, n_centers=12, flip=0.08), 20.0


def orc_lev():
    return G.random_strings(800, seed=24, n_seeds=25, min_len=15,
                            max_len=50, p_edit=0.08), 4.0


@pytest.mark.parametrize("metric", [0, 1, 2, 3])
@pytest.mark.parametrize("zeta", [1, 8, 64])
def test_tree_query_equals_bruteforce(orc, metric, zeta):
    (X, eps) = [orc_l2, orc_ang, orc_ham, orc_lev][metric]()
    ref = orc.bruteforce(X, metric, eps)
    assert ref[0][-1] > 0
    t = orc.tree_build(X, metric, zeta=zeta)
    got = orc.tree_query(X, metric, eps, t)
    cmp = orc.compare_csr(*got, *ref, rtol=0.0)
    assert cmp["ok"], cmp
    assert orc.csr_symmetric(*ref)


def test_bruteforce_rows_subset_matches_full(orc):
    X, eps = orc_l2()
    full = orc.bruteforce(X, 0, eps)
    rows = np.array([5, 0, 1499, 700])
    sub = orc.bruteforce(X, 0, eps, rows=rows)
    for r, i in enumerate(rows):
        a = slice(full[0][i], full[0][i + 1])
        b = slice(sub[0][r], sub[0][r + 1])
        assert np.array_equal(full[1][a], sub[1][b])
        assert np.array_equal(full[2][a], sub[2][b])


def test_planted_mistake_in_tree_radius_is_caught_by_query(orc):
    # shrinking one stored radius makes the pruning test unsafe: the tree
    # query then misses edges, which the exhaustive comparison reports
    X, eps = orc_l2()
    ref = orc.bruteforce(X, 0, eps)
    t = orc.tree_build(X, 0, zeta=8)
    bad = dict(t)
    bad["radius"] = t["radius"] * 0.25
    got = orc.tree_query(X, 0, eps, bad)
    assert orc.compare_csr(*got, *ref)["missing"] > 0
