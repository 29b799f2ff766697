"""GPU parity: the HIP path's epsilon-graph equals the FP64 oracle's exactly
(row_ptr and col identical, zero missing and zero extra edges; distances
within 1e-5 relative of FP64), and the exported GPU cover tree satisfies the
invariants under the oracle's pinned comparisons."""
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
RTOL = 1e-5


@pytest.fixture(scope="module")
def fnn():
    import torch
    assert torch.cuda.is_available()
    import paper_2510_14147_amd as f
    f.lib()
    return f


def gpu_graph(fnn, x, metric, eps, **kw):
    print(f"[case] metric={metric} n={len(x)} eps={eps} kw={kw}", flush=True)
    tree = fnn.fnn_tree_build(x, metric, **{k: v for k, v in kw.items()
                                           if k in ("zeta", "pack", "kmax")})
    g = fnn.fnn_eps_graph(tree, eps, **{k: v for k, v in kw.items()
                                        if k in ("precision", "sched", "validate", "proj")})
    return tree, g


def check(fnn, orc, x, metric, eps, tree_check=True, **kw):
    tree, g = gpu_graph(fnn, x, metric, eps, **kw)
    rp, col, dist = g.to_numpy()
    ref = orc.bruteforce(x, MID[metric], eps)
    cmp = orc.compare_csr(rp, col, dist, *ref, rtol=RTOL)
    assert cmp["missing"] == 0 and cmp["extra"] == 0, cmp
    assert cmp["ok"], cmp
    assert orc.csr_symmetric(rp, col, dist)
    if tree_check:
        t = fnn.fnn_tree_export(tree)
        t["radius"] = t["radius"].astype(np.float64)
        v = orc.check_tree(x, MID[metric], t)
        assert all(c == 0 for c in v.values()), v
    return tree, g, cmp


def test_worked_example(fnn, orc):
    fx = json.load(open(os.path.join(ROOT, "tests", "golden", "worked_example_1d.json")))
    x = np.asarray(fx["points"], np.float32)
    tree, g, _ = check(fnn, orc, x, "l2", fx["eps"], zeta=1)
    rp, col, dist = g.to_numpy()
    assert rp.tolist() == fx["csr"]["row_ptr"] and col.tolist() == fx["csr"]["col"]


@pytest.mark.parametrize("n,d,zeta", [(1000, 3, 8), (3001, 5, 64), (5000, 16, 16)])
def test_l2_random(fnn, orc, n, d, zeta):
    x = G.random_points(n, d, seed=n + d, duplicates=n // 50)
    eps = 0.25 if d <= 5 else 0.9
    check(fnn, orc, x, "l2", eps, zeta=zeta)


def test_c1_full(fnn, orc):
    x = G.c1_clusters()
    check(fnn, orc, x, "l2", W["c1"]["eps"])


def test_angular(fnn, orc):
    x = G.angular_dirs(n=8000, dim=16)
    check(fnn, orc, x, "angular", W["ang"]["eps"])


@pytest.mark.parametrize("bits", [128, 256])
def test_hamming(fnn, orc, bits):
    x = G.random_codes(3000, bits, seed=bits, n_centers=10, flip=0.08)
    check(fnn, orc, x, "hamming", 0.12 * bits)


def test_levenshtein(fnn, orc):
    x = G.random_strings(2000, seed=5, n_seeds=40, min_len=30, max_len=120,
                         p_edit=0.04)
    check(fnn, orc, x, "levenshtein", 6.0)


def test_single_point(fnn, orc):
    x = np.zeros((1, 3), np.float32)
    tree, g = gpu_graph(fnn, x, "l2", 1.0)
    rp, col, dist = g.to_numpy()
    assert rp.tolist() == [0, 0] and g.nnz == 0


def test_all_duplicates(fnn, orc):
    x = np.ones((300, 4), np.float32)
    check(fnn, orc, x, "l2", 1e-3)


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_complete_graph_scatter(fnn, orc, prec):
    # every pair is an edge: whole waves of survivors (or listed tile
    # edges) share one row, so the scatter's slot claims cover full runs,
    # runs across wave boundaries and both directions of every edge
    # (239 neighbours per point: the plain tiles' list holds them all)
    x = np.repeat(G.random_points(3, 16, seed=5), 80, axis=0)
    x += np.float32(1e-3) * G.random_points(240, 16, seed=6)
    check(fnn, orc, x, "l2", 100.0, tree_check=False, precision=prec)


@pytest.mark.parametrize("prec", [None, "fp16"])
def test_row_sort_lengths(fnn, orc, prec):
    # separated tight clusters, complete inside, so a row of a cluster of m
    # points holds m - 1 entries and takes one path of the per-row sort:
    #   0 and 1 entries: no sort (a single point, a pair);
    #   49 / 99 / 199 / 299 entries: one wave, 1 / 2 / 4 / 8 keys per lane
    #   (k_sort_small); 599 and 1099: one wave, 16 and 32 keys per lane
    #   (k_sort_wave); 2099: four waves in registers, the longest strides
    #   through LDS (k_sort_blk<4>); 4199: sixteen waves (k_sort_blk<16>).
    # Rows beyond 16384 entries (k_sort_long) are test_long_rows_sorted's.
    # Default precision: FP32 tiles, row cursors.  FP16: the filter's
    # survivors placed by rank as packed words, which the row sort unpacks
    # (rows of 0 and 1 entries and those handed to the longer sorts too).
    sizes = [1, 2, 50, 100, 200, 300, 600, 1100, 2100, 4200]
    d = 3 if prec is None else 16
    parts = [np.float32(100.0 * k) + G.random_points(m, d, seed=20 + k, scale=0.01)
             for k, m in enumerate(sizes)]
    x = np.concatenate(parts).astype(np.float32)
    x = x[np.random.default_rng(12).permutation(len(x))]
    kw = {} if prec is None else {"precision": prec}
    _, g, _ = check(fnn, orc, x, "l2", 1.0, tree_check=False, **kw)
    if prec is not None:
        assert g.stats["fill_path"] == 2, g.stats["fill_path"]


def test_long_rows_sorted(fnn):
    # one tight cluster of 16500 points: every row holds all 16499 others,
    # longer than the register sorts take.  Too large for the oracle's
    # comparison; checked by what a complete graph fixes: the row offsets,
    # each row strictly increasing without its own id, and sampled distances
    # against FP64
    n = 16500
    x = G.random_points(n, 2, seed=31, scale=0.01)
    _, g = gpu_graph(fnn, x, "l2", 1.0)
    rp, col, dist = g.to_numpy()
    assert np.array_equal(rp, np.arange(n + 1, dtype=np.int64) * (n - 1))
    c = col.reshape(n, n - 1)
    assert (np.diff(c, axis=1) > 0).all()
    assert c.min() >= 0 and c.max() < n
    assert (c != np.arange(n)[:, None]).all()
    x64 = x.astype(np.float64)
    for r in (0, 4321, n - 1):
        ref = np.sqrt(((x64[c[r]] - x64[r]) ** 2).sum(axis=1))
        np.testing.assert_allclose(dist[r * (n - 1):(r + 1) * (n - 1)], ref, rtol=RTOL)


def test_tiny_and_huge_eps(fnn, orc):
    x = G.random_points(700, 3, seed=3)
    check(fnn, orc, x, "l2", 1e-6)
    check(fnn, orc, x, "l2", 10.0)


def test_deterministic(fnn, orc):
    x = G.random_points(4000, 6, seed=11, duplicates=40)
    _, g1 = gpu_graph(fnn, x, "l2", 0.3)
    _, g2 = gpu_graph(fnn, x, "l2", 0.3)
    a, b = g1.to_numpy(), g2.to_numpy()
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


# ---- MFMA Gram filter (BF16 / FP16 / FP8) ----------------------------------

@pytest.mark.parametrize("prec", ["bf16", "fp16", "fp8"])
@pytest.mark.parametrize("case", ["c1", "rand16", "c2_8k", "ang"])
def test_mfma_filter_parity(fnn, orc, prec, case):
    if case == "c1":
        x, eps, metric = G.c1_clusters(), W["c1"]["eps"], "l2"
    elif case == "rand16":
        x, eps, metric = G.random_points(4000, 16, seed=77, duplicates=30), 0.9, "l2"
    elif case == "c2_8k":
        x, eps, metric = G.c2_manifold(n=8000), W["c2_50k"]["eps"][1], "l2"
    else:
        x, eps, metric = G.angular_dirs(n=6000, dim=16), W["ang"]["eps"], "angular"
    tree, g, cmp = check(fnn, orc, x, metric, eps, tree_check=False,
                         precision=prec, validate=True)
    st = g.stats
    assert st["filter_pairs"] > 0
    assert st["validate_mismatch"] == 0
    assert st["max_rel_err"] <= 1e-5


@pytest.mark.parametrize("offset,spread", [(1e6, 1.0), (0.0, 1e4), (0.0, 1e-6), (3.0, 1e-3)])
def test_fp16_filter_scaled_ranges(fnn, orc, offset, spread):
    """The FP16 filter scales the centred rows by a power of two: large
    offsets and spreads must not overflow the format, tiny ones must not lose
    edges to subnormals; zero false negatives and the exact graph."""
    x = (G.random_points(3000, 16, seed=5, duplicates=20).astype(np.float64) * spread
         + offset).astype(np.float32)
    eps = 0.6 * spread
    print(f"[case] fp16 ranges offset={offset} spread={spread}", flush=True)
    tree, g, cmp = check(fnn, orc, x, "l2", eps, tree_check=False, precision="fp16",
                         validate=True)
    assert g.stats["validate_mismatch"] == 0


def test_fp16_filter_narrower_than_bf16(fnn, orc):
    """Same graph from both 16-bit filters; the FP16 margin is eight times
    narrower, so it passes fewer non-edges."""
    x = G.c2_manifold(n=20000)
    eps = W["c2_50k"]["eps"][0]
    _, gb, _ = check(fnn, orc, x, "l2", eps, tree_check=False, precision="bf16")
    _, gh, _ = check(fnn, orc, x, "l2", eps, tree_check=False, precision="fp16")
    assert gh.stats["proj_dim"] == gb.stats["proj_dim"] == 16
    assert gh.nnz // 2 <= gh.stats["filter_survivors"] < gb.stats["filter_survivors"]
    for u, v in zip(gb.to_numpy(), gh.to_numpy()):
        assert np.array_equal(u.view(np.uint8), v.view(np.uint8))


def test_mfma_filter_screens(fnn, orc):
    # without validation the filter must reject most pairs of a 128-d set
    x = G.c2_manifold(n=20000)
    eps = W["c2_50k"]["eps"][0]
    tree, g, cmp = check(fnn, orc, x, "l2", eps, tree_check=False, precision="bf16")
    st = g.stats
    assert st["filter_survivors"] < 0.05 * st["filter_pairs"]
    assert st["filter_survivors"] >= g.nnz // 2


# ---- integer MFMA filter (Hamming codes as bytes) ---------------------------

@pytest.mark.parametrize("bits", [64, 128, 192, 256])
@pytest.mark.parametrize("validate", [False, True])
def test_int8_hamming_parity(fnn, orc, bits, validate):
    # 3001 codes: a ragged last tile; clustered so that the graph is not empty
    x = G.random_codes(3001, bits, seed=900 + bits, n_centers=12, flip=0.08)
    tree, g, cmp = check(fnn, orc, x, "hamming", 0.12 * bits, tree_check=False,
                         precision="i8", validate=validate)
    st = g.stats
    assert st["filter_pairs"] > 0
    assert st["validate_mismatch"] == 0
    # the integer test is exact: every pair it passes is an edge
    assert 0 < st["filter_survivors"] <= g.nnz // 2


@pytest.mark.parametrize("eps", [0.5, 5.5, 1e9])
def test_int8_hamming_edge_radii(fnn, orc, eps):
    # eps < 1 keeps exact duplicates only, a fractional eps rounds down,
    # eps beyond the code length connects every pair
    x = G.random_codes(700, 128, seed=31, n_centers=5, flip=0.03)
    x[100:140] = x[7]
    check(fnn, orc, x, "hamming", eps, tree_check=False, precision="i8", validate=True)


def test_int8_hamming_duplicates(fnn, orc):
    x = np.repeat(G.random_codes(3, 256, seed=8), 150, axis=0)
    check(fnn, orc, x, "hamming", 2.0, tree_check=False, precision="i8")


def test_int8_rejects_other_inputs(fnn, orc):
    x = G.random_points(300, 8, seed=1)
    tree = fnn.fnn_tree_build(x, "l2")
    with pytest.raises(fnn.FnnError) as e:
        fnn.fnn_eps_graph(tree, 0.5, precision="i8")
    assert e.value.code == fnn.FNN_EUNSUPPORTED
    codes = G.random_codes(300, 512, seed=2)
    tree = fnn.fnn_tree_build(codes, "hamming")
    with pytest.raises(fnn.FnnError) as e:
        fnn.fnn_eps_graph(tree, 40, precision="i8")
    assert e.value.code == fnn.FNN_EUNSUPPORTED


# ---- filter on leading principal coordinates ---------------------------------

@pytest.mark.parametrize("prec", ["bf16", "fp16", "fp8"])
@pytest.mark.parametrize("proj", [16, 32, 64])
def test_projected_filter_parity(fnn, orc, prec, proj):
    # a fixed number of principal coordinates: the filter must stay
    # conservative (no false negatives) and the graph exact
    x = G.c2_manifold(n=8000)
    tree, g, cmp = check(fnn, orc, x, "l2", W["c2_50k"]["eps"][1], tree_check=False,
                         precision=prec, validate=True, proj=proj)
    st = g.stats
    assert st["proj_dim"] == proj
    assert 0.0 < st["proj_captured"] <= 1.0 + 1e-9
    assert st["filter_survivors"] < 0.05 * st["filter_pairs"]
    assert st["validate_mismatch"] == 0
    assert st["max_rel_err"] <= 1e-5


def test_projected_filter_auto_and_off(fnn, orc):
    x = G.c2_manifold(n=20000)
    eps = W["c2_50k"]["eps"][0]
    _, ga, _ = check(fnn, orc, x, "l2", eps, tree_check=False, precision="bf16")
    _, go, _ = check(fnn, orc, x, "l2", eps, tree_check=False, precision="bf16", proj=-1)
    # the manifold data puts ~98 % of the variance in 16 coordinates, far
    # more than the automatic rule needs at this eps
    assert ga.stats["proj_dim"] == 16 and 0.97 <= ga.stats["proj_captured"] <= 1.0
    assert go.stats["proj_dim"] == 0
    # the projected filter screens nearly as well as the full one
    assert ga.stats["filter_survivors"] < 3 * go.stats["filter_survivors"]
    for u, v in zip(ga.to_numpy(), go.to_numpy()):
        assert np.array_equal(u, v)


def test_projected_filter_angular(fnn, orc):
    x = G.c2_manifold(n=6000)
    check(fnn, orc, x, "angular", 0.35, tree_check=False, precision="bf16",
          validate=True, proj=16)


def test_projected_filter_rejects_bad_width(fnn, orc):
    x = G.random_points(300, 32, seed=4)
    tree = fnn.fnn_tree_build(x, "l2")
    with pytest.raises(fnn.FnnError) as e:
        fnn.fnn_eps_graph(tree, 0.5, precision="bf16", proj=24)
    assert e.value.code == fnn.FNN_EINVAL


# ---- automatic precision ------------------------------------------------------

@pytest.mark.parametrize("case,want", [("c2_20k", "fp16"), ("rand8", "fp32"),
                                       ("ham256", "i8"), ("ham512", "fp32"),
                                       ("lev", "fp32")])
def test_auto_precision(fnn, orc, case, want):
    # the library picks the filter per query; the graph stays exact
    if case == "c2_20k":
        x, metric, eps = G.c2_manifold(n=20000), "l2", W["c2_50k"]["eps"][0]
    elif case == "rand8":
        x, metric, eps = G.random_points(3000, 8, seed=9), "l2", 0.3
    elif case == "ham256":
        x, metric, eps = G.random_codes(3000, 256, seed=10, flip=0.06), "hamming", 20
    elif case == "ham512":
        x, metric, eps = G.random_codes(1500, 512, seed=11, flip=0.06), "hamming", 40
    else:
        x = G.random_strings(800, seed=12, n_seeds=20, min_len=30, max_len=60)
        metric, eps = "levenshtein", 5
    tree, g, cmp = check(fnn, orc, x, metric, eps, tree_check=False, precision="auto")
    names = {v: k for k, v in fnn.PRECISIONS.items()}
    assert names[int(g.stats["precision_used"])] == want


@pytest.mark.parametrize("n", [2, 63, 64, 65, 129, 1000])
@pytest.mark.parametrize("validate", [False, True])
def test_dense_list_full_packs(fnn, orc, n, validate):
    """One cloud whose pack pairs are all kept takes the closed-form work
    list over full packs of 64 consecutive tree positions (the last one
    ragged); every pair is screened once and the graph is exact, with the
    uniform-pack entry loop (no validation) and the general one (validation)."""
    x = G.random_points(n, 16, seed=300 + n)
    eps = 1.6  # about half the pairs: no pack pair can be pruned
    tree, g, cmp = check(fnn, orc, x, "l2", eps, tree_check=False, precision="fp16",
                         validate=validate)
    st = g.stats
    assert st["filter_pairs"] == n * (n - 1) // 2, st["filter_pairs"]
    if validate:
        assert st["validate_mismatch"] == 0
