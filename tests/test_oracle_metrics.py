"""Pins for the oracle's pinned distance predicates (CPU only).

Each check ties the oracle to something other than its own formula: exact
rational arithmetic, the definition of edit distance as a shortest edit
script, Python's integer popcount, closed-form geometry.
"""
import itertools
import math
from collections import deque
from fractions import Fraction

import numpy as np
import pytest

from paper_2510_14147_amd import datagen as G


def _exact_l2(x, y):
    return sum((Fraction(float(a)) - Fraction(float(b))) ** 2 for a, b in zip(x, y))


def test_l2_sq_within_rounding_bound_of_exact(orc):
    # Higham: a sequential FP64 sum of d nonnegative terms, each a rounded
    # square of an exact difference, is within gamma_{d+1} of the exact value.
    rng = np.random.default_rng(7)
    u = 2.0 ** -53
    for d in (1, 3, 8, 128):
        for _ in range(40):
            x = rng.standard_normal(d).astype(np.float32)
            y = (x + rng.standard_normal(d) * 1e-3).astype(np.float32)
            s = orc.l2_sq(x, y)
            ex = _exact_l2(x, y)
            g = (d + 1) * u / (1 - (d + 1) * u)
            assert abs(Fraction(s) - ex) <= Fraction(g) * ex


def test_l2_predicate_is_inclusive_at_exact_boundary(orc):
    # integer coordinates make s exact: s == eps^2 must be an edge
    x = np.array([0, 0, 0], np.float32)
    y = np.array([1, 2, 2], np.float32)          # s = 9
    assert orc.l2_sq(x, y) == 9.0
    assert orc.eps_param(orc.L2, 3.0) == 9.0
    row_ptr, col, dist = orc.bruteforce(np.stack([x, y]), orc.L2, 3.0)
    assert row_ptr.tolist() == [0, 1, 2] and dist.tolist() == [3.0, 3.0]
    row_ptr, col, dist = orc.bruteforce(np.stack([x, y]), orc.L2,
                                        np.nextafter(3.0, 0.0))
    assert row_ptr.tolist() == [0, 0, 0]


def test_angular_predicate_matches_exact_cosine_away_from_boundary(orc):
    rng = np.random.default_rng(11)
    checked = 0
    for _ in range(400):
        d = int(rng.integers(2, 20))
        x = rng.standard_normal(d).astype(np.float32)
        y = rng.standard_normal(d).astype(np.float32)
        eps = float(rng.uniform(0.05, 3.1))
        C = orc.eps_param(orc.ANGULAR, eps)
        g, a, b = orc.ang_terms(x, y)
        gx = sum(Fraction(float(p)) * Fraction(float(q)) for p, q in zip(x, y))
        ax = sum(Fraction(float(p)) ** 2 for p in x)
        bx = sum(Fraction(float(q)) ** 2 for q in y)
        cos_exact = float(gx) / math.sqrt(float(ax) * float(bx))
        if abs(cos_exact - C) < 1e-9:
            continue
        assert orc.ang_pred(g, a, b, C) == (cos_exact >= C)
        checked += 1
    assert checked > 350


def test_angular_distance_matches_arccos_when_well_conditioned(orc):
    rng = np.random.default_rng(12)
    for _ in range(200):
        d = int(rng.integers(2, 64))
        x = rng.standard_normal(d).astype(np.float32)
        y = rng.standard_normal(d).astype(np.float32)
        gx = sum(Fraction(float(p)) * Fraction(float(q)) for p, q in zip(x, y))
        ax = sum(Fraction(float(p)) ** 2 for p in x)
        bx = sum(Fraction(float(q)) ** 2 for q in y)
        c = float(gx) / math.sqrt(float(ax) * float(bx))
        if abs(c) > 0.95:
            continue
        assert abs(orc.ang_dist(x, y) - math.acos(c)) <= 1e-12


def test_angular_special_cases(orc):
    e = np.eye(4, dtype=np.float32)
    # orthogonal: exactly pi/2; antipodal: pi; identical direction: 0
    assert orc.ang_dist(e[0], e[1]) == pytest.approx(math.pi / 2, abs=1e-15)
    assert orc.ang_dist(e[0], -e[0]) == pytest.approx(math.pi, abs=1e-15)
    assert orc.ang_dist(e[0], 3 * e[0]) == 0.0
    # eps >= pi -> every pair is an edge
    assert orc.eps_param(orc.ANGULAR, 4.0) == -1.0


def test_hamming_matches_integer_popcount(orc):
    rng = np.random.default_rng(3)
    for _ in range(500):
        w = int(rng.integers(1, 6))
        x = rng.integers(0, 2**64, w, dtype=np.uint64)
        y = rng.integers(0, 2**64, w, dtype=np.uint64)
        ref = sum(bin(int(a) ^ int(b)).count("1") for a, b in zip(x, y))
        assert orc.ham(x, y) == ref


def _edit_distances_by_bfs(max_len=4, alphabet=4):
    """Edit distance as its definition: the fewest single-symbol insertions,
    deletions and substitutions turning a into b, by breadth-first search
    over all strings of length <= max_len (an optimal script can delete
    first and insert last, so it never needs a longer string)."""
    strings = [()]
    for L in range(1, max_len + 1):
        strings += list(itertools.product(range(alphabet), repeat=L))
    index = {s: i for i, s in enumerate(strings)}

    def nbrs(s):
        out = set()
        for i in range(len(s)):
            out.add(s[:i] + s[i + 1:])
            for c in range(alphabet):
                if c != s[i]:
                    out.add(s[:i] + (c,) + s[i + 1:])
        if len(s) < max_len:
            for i in range(len(s) + 1):
                for c in range(alphabet):
                    out.add(s[:i] + (c,) + s[i:])
        return out

    adj = [[index[t] for t in nbrs(s)] for s in strings]
    dist = np.full((len(strings), len(strings)), -1, np.int32)
    for src in range(len(strings)):
        dist[src, src] = 0
        q = deque([src])
        while q:
            u = q.popleft()
            for v in adj[u]:
                if dist[src, v] < 0:
                    dist[src, v] = dist[src, u] + 1
                    q.append(v)
    return strings, dist


def test_levenshtein_equals_shortest_edit_script_exhaustive(orc):
    strings, dist = _edit_distances_by_bfs(4, 4)
    assert len(strings) == 341
    lib = orc.lib()
    bufs = [np.ascontiguousarray(np.array(s, np.uint8)) if s else np.zeros(1, np.uint8)
            for s in strings]
    lens = [len(s) for s in strings]
    bad = 0
    for i in range(len(strings)):
        for j in range(len(strings)):
            if lib.orc_lev(bufs[i], lens[i], bufs[j], lens[j]) != dist[i, j]:
                bad += 1
    assert bad == 0


def test_levenshtein_textbook_values(orc):
    def enc(w):
        return np.frombuffer(w.encode(), np.uint8)
    assert orc.lev(enc("kitten"), enc("sitting")) == 3
    assert orc.lev(enc("flaw"), enc("lawn")) == 2
    assert orc.lev(enc("intention"), enc("execution")) == 5
    a = enc("abcdef")
    assert orc.lev(a, np.zeros(0, np.uint8)) == 6
    assert orc.lev(a, a) == 0


def test_levenshtein_band_decides_threshold_exactly(orc):
    rng = np.random.default_rng(5)
    strs = G.random_strings(300, seed=9, n_seeds=10, min_len=20, max_len=60,
                            p_edit=0.1)
    for _ in range(1500):
        i, j = rng.integers(0, len(strs), 2)
        k = int(rng.integers(0, 12))
        full = orc.lev(strs[i], strs[j])
        assert orc.lev_banded(strs[i], strs[j], k) == min(full, k + 1)


def test_levenshtein_properties(orc):
    rng = np.random.default_rng(6)
    strs = G.random_strings(60, seed=10, n_seeds=6, min_len=5, max_len=40)
    lens = (strs != 0xFF).sum(1)
    for _ in range(300):
        i, j, k = rng.integers(0, len(strs), 3)
        dij = orc.lev(strs[i], strs[j])
        assert dij == orc.lev(strs[j], strs[i])
        assert dij >= abs(int(lens[i]) - int(lens[j]))
        assert dij <= orc.lev(strs[i], strs[k]) + orc.lev(strs[k], strs[j])
    # equal length + substitutions only -> Hamming distance of the symbols
    a = rng.integers(0, 4, 50).astype(np.uint8)
    b = a.copy()
    pos = rng.choice(50, 2, replace=False)   # two far-apart substitutions
    pos = np.array([3, 40])
    b[pos] = (b[pos] + 1) % 4
    assert orc.lev(a, b) == 2
