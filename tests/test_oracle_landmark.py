"""Pins for the rule the landmark mode relies on (CPU only, FP64): Lemma 1
of Section IV-E -- if p in V_j has an eps-neighbour in V_i (i != j), then
d(p, c_i) <= d(p, c_j) + 2 eps -- checked on every cross-cell edge of
brute-force graphs, and shown to be tight enough that a smaller slack
(eps instead of 2 eps) would miss edges."""
import numpy as np
import pytest

from paper_2510_14147_amd import datagen as G


def _cells(x, centres):
    D = np.sqrt(((x[:, None, :].astype(np.float64) - x[centres][None, :, :]) ** 2).sum(-1))
    return D, D.argmin(1)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_lemma1_holds_on_every_cross_cell_edge(orc, seed):
    rng = np.random.default_rng(seed)
    x = G.random_points(1500, 4, seed=seed + 40)
    eps = 0.15
    centres = rng.choice(len(x), 12, replace=False)
    D, cell = _cells(x, centres)
    rp, col, _ = orc.bruteforce(x, 0, eps)
    rows = np.repeat(np.arange(len(x)), np.diff(rp))
    cross = cell[rows] != cell[col]
    assert cross.sum() > 100
    p, q = rows[cross], col[cross]
    lhs = D[p, cell[q]]                 # d(p, c_i), q in V_i
    rhs = D[p, cell[p]] + 2 * eps       # d(p, C) + 2 eps
    assert np.all(lhs <= rhs + 1e-12)
    # with eps in place of 2 eps the rule would drop some of these pairs
    assert np.any(lhs > D[p, cell[p]] + eps)


def test_ghost_sets_cover_every_cross_pair(orc):
    """Every cross-cell edge (p, q), p in V_j, q in V_i, has p in G_i and q
    in G_j, so each is found in both cells' augmented sets."""
    rng = np.random.default_rng(5)
    x = G.c1_clusters(n_centers=6, per_center=300, seed=77)
    eps = 0.08
    centres = rng.choice(len(x), 9, replace=False)
    D, cell = _cells(x, centres)
    ghost = D <= D[np.arange(len(x)), cell][:, None] + 2 * eps
    ghost[np.arange(len(x)), cell] = False
    rp, col, _ = orc.bruteforce(x, 0, eps)
    rows = np.repeat(np.arange(len(x)), np.diff(rp))
    cross = cell[rows] != cell[col]
    assert np.all(ghost[rows[cross], cell[col[cross]]])
