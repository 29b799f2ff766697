"""GPU parity of the many-clouds batch: one forest build and one query over
many independent clouds, each with its own eps.  The expected graph is the
union of the oracle's per-cloud brute-force graphs (block diagonal over the
concatenated rows); each cloud's subtree of the exported forest must satisfy
the cover-tree invariants under the oracle's checker; and the batch must
equal the per-cloud calls bit for bit."""
import numpy as np
import pytest

from paper_2510_14147_amd import datagen as G

pytestmark = pytest.mark.gpu

MID = {"l2": 0, "angular": 1, "hamming": 2, "levenshtein": 3}
RTOL = 1e-5


@pytest.fixture(scope="module")
def fnn():
    import torch
    assert torch.cuda.is_available()
    import paper_2510_14147_amd as f
    f.lib()
    return f


def mixture(n, d, seed, dup=False):
    """One small Gaussian-mixture cloud (the many-clouds recipe, any n)."""
    spec = dict(dim=d, components=int(3 + seed % 7), seed=seed)
    x = G.c5_cloud(spec, n_override=n) if n else np.zeros((0, d), np.float32)
    if dup and n:
        x[:] = x[0]
    return x


def block_reference(orc, clouds, metric, eps):
    """Block-diagonal CSR: the oracle graph of every cloud, shifted by the
    cloud's first global row."""
    rps, cols, dists, base, nnz = [np.zeros(1, np.int64)], [], [], 0, 0
    for x, e in zip(clouds, eps):
        if len(x) == 0:
            continue
        rp, col, dist = orc.bruteforce(x, MID[metric], e)
        rps.append(rp[1:] + nnz)
        cols.append(col.astype(np.int64) + base)
        dists.append(dist)
        base += len(x)
        nnz += int(rp[-1])
    cat = lambda a, t: np.concatenate(a) if a else np.zeros(0, t)  # noqa: E731
    return np.concatenate(rps), cat(cols, np.int64), cat(dists, np.float64)


def subtree(t, root, lo, hi):
    """Cloud [lo, hi) of an exported forest as a stand-alone tree: the
    vertices below ``root`` keep their order (children stay consecutive)."""
    cb, cc = t["child_begin"], t["child_count"]
    keep, stack = [], [root]
    while stack:
        v = stack.pop()
        keep.append(v)
        stack.extend(range(cb[v], cb[v] + cc[v]))
    keep = np.sort(np.asarray(keep, np.int64))
    new = {int(v): i for i, v in enumerate(keep)}
    s = dict(order=t["order"][lo:hi] - lo,
             center=t["center"][keep] - lo,
             radius=t["radius"][keep].astype(np.float64),
             level=t["level"][keep],
             child_count=cc[keep],
             child_begin=np.array([new[int(cb[v])] if cc[v] else 0 for v in keep],
                                  np.int32),
             pt_begin=t["pt_begin"][keep] - lo,
             pt_end=t["pt_end"][keep] - lo,
             nnodes=len(keep))
    return s


def run_batch(fnn, orc, clouds, metric, eps, tree_check=True, per_cloud=True,
              **kw):
    sizes = [len(x) for x in clouds]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    X = np.concatenate([x for x in clouds], axis=0)
    print(f"[case] batch metric={metric} clouds={len(clouds)} n={len(X)} "
          f"kw={kw}", flush=True)
    bkw = {k: v for k, v in kw.items() if k in ("zeta", "pack", "kmax")}
    qkw = {k: v for k, v in kw.items() if k in ("precision", "sched", "validate", "proj")}
    tree = fnn.fnn_tree_build_batch(X, off, metric, **bkw)
    g = fnn.fnn_eps_graph_batch(tree, eps, **qkw)
    rp, col, dist = g.to_numpy()
    ref = block_reference(orc, clouds, metric, eps)
    cmp = orc.compare_csr(rp, col, dist, *ref, rtol=RTOL)
    assert cmp["missing"] == 0 and cmp["extra"] == 0, cmp
    assert cmp["ok"], cmp
    assert orc.csr_symmetric(rp, col, dist)
    nonempty = [c for c, s in enumerate(sizes) if s]
    if tree_check and len(nonempty) > 1:
        t = fnn.fnn_tree_export(tree)
        assert t["child_count"][0] == len(nonempty)
        assert np.isinf(t["radius"][0])
        for k, c in enumerate(nonempty):
            sub = subtree(t, 1 + k, int(off[c]), int(off[c + 1]))
            v = orc.check_tree(clouds[c], MID[metric], sub)
            assert all(x == 0 for x in v.values()), (c, v)
    if per_cloud:
        # the batch equals one call per cloud, bit for bit
        for c in nonempty:
            t1 = fnn.fnn_tree_build(clouds[c], metric, **bkw)
            g1 = fnn.fnn_eps_graph(t1, eps[c], **qkw)
            r1, c1, d1 = g1.to_numpy()
            lo, hi = int(off[c]), int(off[c + 1])
            a, b = rp[lo], rp[hi]
            assert np.array_equal(rp[lo:hi + 1] - a, r1)
            assert np.array_equal(col[a:b] - lo, c1)
            assert np.array_equal(dist[a:b].view(np.uint32), d1.view(np.uint32))
    return tree, g


SIZES = [1, 2, 64, 65, 0, 500, 3000, 1, 130, 2000, 0, 777, 5, 4000]


def eps_for(clouds, seed, lo=0.03, hi=0.12):
    rng = np.random.default_rng(seed)
    return [float(rng.uniform(lo, hi) * np.sqrt(max(1, x.shape[1] if len(x.shape) > 1 else 1)))
            for x in clouds]


@pytest.mark.parametrize("d", [3, 16])
def test_batch_l2(fnn, orc, d):
    clouds = [mixture(n, d, 100 + i, dup=(i == 8)) for i, n in enumerate(SIZES)]
    eps = eps_for(clouds, d)
    run_batch(fnn, orc, clouds, "l2", eps, zeta=16)


def test_batch_l2_default_zeta_no_per_cloud(fnn, orc):
    clouds = [mixture(n, 8, 300 + i) for i, n in enumerate([5000, 1, 3000, 64])]
    eps = [0.05, 1.0, 0.2, 0.3]
    run_batch(fnn, orc, clouds, "l2", eps, per_cloud=False)


def test_batch_single_nonempty_cloud(fnn, orc):
    # empty clouds around one cloud: the forest reduces to an ordinary tree
    clouds = [mixture(0, 4, 1), mixture(2500, 4, 2), mixture(0, 4, 3)]
    run_batch(fnn, orc, clouds, "l2", [0.7, 0.1, 0.9])


def test_batch_angular(fnn, orc):
    clouds = [G.angular_dirs(n=n, dim=16, seed=40 + i) if n else
              np.zeros((0, 16), np.float32)
              for i, n in enumerate([1500, 3, 0, 2500, 700])]
    eps = [0.5, 0.3, 0.4, 0.35, 0.6]
    run_batch(fnn, orc, clouds, "angular", eps, zeta=8)


def test_batch_hamming(fnn, orc):
    clouds = [G.random_codes(n, 128, seed=50 + i, flip=0.06)
              for i, n in enumerate([2000, 1, 900, 3000])]
    eps = [10, 3, 14, 8]
    run_batch(fnn, orc, clouds, "hamming", eps, zeta=8)


def test_batch_hamming_int8(fnn, orc):
    # integer MFMA filter over clouds of 256-bit codes, each with its own
    # radius; groups of packs that span clouds skip the cross-cloud pairs
    clouds = [G.random_codes(n, 256, seed=80 + i, flip=0.06) if n else
              np.zeros((0, 4), np.uint64)
              for i, n in enumerate([2000, 1, 0, 900, 3000, 70])]
    eps = [30, 3, 9, 20, 26, 40]
    run_batch(fnn, orc, clouds, "hamming", eps, zeta=8, precision="i8", validate=1)


def test_batch_levenshtein(fnn, orc):
    clouds = [G.random_strings(n, seed=60 + i, stride=64, min_len=20, max_len=60)
              for i, n in enumerate([400, 2, 700, 300])]
    eps = [6, 2, 9, 4]
    run_batch(fnn, orc, clouds, "levenshtein", eps, zeta=8)


@pytest.mark.parametrize("precision", ["bf16", "fp16", "fp8"])
def test_batch_mfma(fnn, orc, precision):
    # MFMA groups of 4 packs may span clouds: pairs across clouds must be
    # skipped and each pack filtered with its own cloud's eps
    clouds = [mixture(n, 64, 500 + i) for i, n in enumerate([3000, 70, 1, 2500, 900, 130])]
    eps = eps_for(clouds, 9, 0.02, 0.08)
    run_batch(fnn, orc, clouds, "l2", eps, precision=precision, validate=1)


def test_batch_projected_filter(fnn, orc):
    # one principal basis for all clouds; each cloud's filter eps^2 is scaled
    # by the same bound and the survivors decided with the cloud's own eps
    clouds = [mixture(n, 64, 800 + i) for i, n in enumerate([2500, 90, 1, 3000, 700])]
    eps = eps_for(clouds, 13, 0.02, 0.08)
    run_batch(fnn, orc, clouds, "l2", eps, precision="bf16", validate=1, proj=32)


def test_batch_auto_precision(fnn, orc):
    # wide mixture clouds: the filter's margin is large against each cloud's
    # eps, so the automatic choice may fall back to the plain tiles; either
    # way the graph is exact
    clouds = [mixture(n, 64, 900 + i) for i, n in enumerate([2500, 90, 1, 3000, 700])]
    eps = eps_for(clouds, 17, 0.02, 0.08)
    run_batch(fnn, orc, clouds, "l2", eps, precision="auto", per_cloud=False)


def test_batch_learned(fnn, orc):
    clouds = [mixture(n, 16, 700 + i) for i, n in enumerate([4000, 3, 2500, 65, 1800])]
    eps = eps_for(clouds, 11)
    run_batch(fnn, orc, clouds, "l2", eps, sched="learned")


def test_batch_many_clouds_recipe(fnn, orc):
    # the first 40 clouds of the many-clouds recipe, capped at 3000 points,
    # batched per dimension as the benchmark does
    specs = G.c5_cloud_specs()[:40]
    import json
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    W = json.load(open(os.path.join(root, "paper_2510_14147_amd", "workloads.json")))
    for d in (3, 16, 64):
        sel = [s for s in specs if s["dim"] == d]
        clouds = [G.c5_cloud(s, n_override=min(s["n"], 3000)) for s in sel]
        eps = [W["c5"]["eps"][s["cloud"]] for s in sel]
        run_batch(fnn, orc, clouds, "l2", eps, tree_check=(d == 16),
                  per_cloud=False, precision="bf16" if d == 64 else "fp32")
