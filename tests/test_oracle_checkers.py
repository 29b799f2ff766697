"""Planted-failure pins for the oracle's CSR checkers (CPU only): every kind
of mistake the comparison and the symmetry check exist to catch must make
them fail, and the correct graph must pass."""
import numpy as np
import pytest

from paper_2510_14147_amd import datagen as G


@pytest.fixture(scope="module")
def graph(orc):
    x = G.c1_clusters(n_centers=3, per_center=60, seed=11)
    rp, col, dist = orc.bruteforce(x, orc.L2, 0.12)
    assert rp[-1] > 200
    return rp, col, dist


def _csr_from_pairs(n, pairs, dist):
    """CSR of (row, col) pairs sorted by row then col."""
    pairs = np.asarray(pairs, np.int64)
    o = np.lexsort((pairs[:, 1], pairs[:, 0]))
    pairs, dist = pairs[o], np.asarray(dist)[o]
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, pairs[:, 0] + 1, 1)
    return np.cumsum(rp), pairs[:, 1].copy(), dist


def test_identical_graph_passes(orc, graph):
    rp, col, dist = graph
    cmp = orc.compare_csr(rp, col, dist.astype(np.float32), rp, col, dist)
    assert cmp["ok"] and cmp["missing"] == 0 and cmp["extra"] == 0
    assert orc.csr_symmetric(rp, col, dist.astype(np.float32))


def test_compare_catches_extra_edge(orc, graph):
    rp, col, dist = graph
    n = rp.size - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    have = set(zip(rows.tolist(), col.tolist()))
    a, b = next((i, j) for i in range(n) for j in range(n)
                if i != j and (i, j) not in have)
    pairs = np.concatenate([np.stack([rows, col], 1), [[a, b]]])
    rp2, col2, d2 = _csr_from_pairs(n, pairs, np.concatenate([dist, [1.0]]))
    cmp = orc.compare_csr(rp2, col2, d2, rp, col, dist)
    assert cmp["extra"] == 1 and cmp["missing"] == 0 and not cmp["ok"]
    assert not cmp["row_ptr_equal"]


def test_compare_catches_swapped_column(orc, graph):
    """Same row lengths, one column replaced by another: counts equal, edge
    sets differ."""
    rp, col, dist = graph
    col2 = col.copy()
    r = int(np.argmax(np.diff(rp)))
    k = rp[r]
    taken = set(col[rp[r]:rp[r + 1]].tolist()) | {r}
    col2[k] = next(j for j in range(rp.size - 1) if j not in taken)
    cmp = orc.compare_csr(rp, col2, dist, rp, col, dist)
    assert cmp["row_ptr_equal"] and not cmp["col_equal"]
    assert cmp["extra"] == 1 and cmp["missing"] == 1 and not cmp["ok"]


def test_compare_catches_distance_error(orc, graph):
    rp, col, dist = graph
    d2 = dist.copy()
    d2[5] *= 1 + 2e-5                     # beyond the 1e-5 relative bound
    cmp = orc.compare_csr(rp, col, d2, rp, col, dist)
    assert cmp["col_equal"] and not cmp["dist_ok"] and not cmp["ok"]
    assert 1.9e-5 < cmp["max_rel_err"] < 2.1e-5
    d3 = dist.copy()
    d3[5] *= 1 + 0.5e-5                   # within it
    assert orc.compare_csr(rp, col, d3, rp, col, dist)["ok"]


def test_symmetry_catches_missing_mirror(orc, graph):
    rp, col, dist = graph
    n = rp.size - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    keep = np.ones(col.size, bool)
    keep[7] = False                       # drop (i, j) but keep (j, i)
    rp2, col2, d2 = _csr_from_pairs(n, np.stack([rows[keep], col[keep]], 1), dist[keep])
    assert not orc.csr_symmetric(rp2, col2)


def test_symmetry_catches_self_loop(orc, graph):
    rp, col, dist = graph
    n = rp.size - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    pairs = np.concatenate([np.stack([rows, col], 1), [[3, 3]]])
    rp2, col2, d2 = _csr_from_pairs(n, pairs, np.concatenate([dist, [0.0]]))
    assert not orc.csr_symmetric(rp2, col2)


def test_symmetry_catches_unsorted_row(orc, graph):
    rp, col, dist = graph
    r = int(np.argmax(np.diff(rp)))
    col2 = col.copy()
    col2[rp[r]], col2[rp[r] + 1] = col[rp[r] + 1], col[rp[r]]
    assert not orc.csr_symmetric(rp, col2)


def test_symmetry_catches_duplicate_entry(orc, graph):
    """A row listing a column twice (and its mirror twice) is not a valid
    CSR of a simple graph: columns must be strictly ascending."""
    rp, col, dist = graph
    n = rp.size - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    i, j = int(rows[0]), int(col[0])
    pairs = np.concatenate([np.stack([rows, col], 1), [[i, j], [j, i]]])
    rp2, col2, _ = _csr_from_pairs(n, pairs, np.zeros(pairs.shape[0]))
    assert not orc.csr_symmetric(rp2, col2)


def test_symmetry_catches_asymmetric_distance_bits(orc, graph):
    rp, col, dist = graph
    d32 = dist.astype(np.float32)
    assert orc.csr_symmetric(rp, col, d32)
    d2 = d32.copy()
    d2[4] = np.nextafter(d2[4], np.float32(np.inf))   # one ulp on one side only
    assert not orc.csr_symmetric(rp, col, d2)
