"""The learned cost model (GPU): forward/backward kernels against the FP64
reference network, training, trace targets, and the learned schedule giving
the same graph as the plain two-pass schedule (including forced overflow)."""
import json
import os

import numpy as np
import pytest

from paper_2510_14147_amd import datagen as G

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
W = json.load(open(os.path.join(ROOT, "paper_2510_14147_amd", "workloads.json")))


@pytest.fixture(scope="module")
def fnn():
    import torch
    assert torch.cuda.is_available()
    import paper_2510_14147_amd as f
    f.lib()
    return f


def _rand(seed):
    from oracle import mlp
    rng = np.random.default_rng(seed)
    th = mlp.init(seed)
    th[-2:] = rng.normal(0, 0.3, 2)
    x = rng.normal(0, 1, (300, 16))
    t = rng.normal(0, 1, (300, 2))
    return th, x, t


def test_forward_matches_fp64_reference(fnn):
    import torch
    from oracle import mlp
    th, x, _ = _rand(1)
    y = fnn.fnn_mlp_forward(torch.tensor(th, dtype=torch.float32).cuda(),
                            torch.tensor(x, dtype=torch.float32).cuda()).cpu().numpy()
    ref, _ = mlp.forward(th.astype(np.float32).astype(np.float64),
                         x.astype(np.float32).astype(np.float64))
    np.testing.assert_allclose(y, ref, rtol=1e-4, atol=1e-5)


def test_gradient_matches_fp64_reference(fnn):
    import torch
    from oracle import mlp
    th, x, t = _rand(2)
    th32, x32, t32 = (a.astype(np.float32) for a in (th, x, t))
    loss, g = fnn.fnn_mlp_loss_grad(torch.from_numpy(th32).cuda(),
                                    torch.from_numpy(x32).cuda(),
                                    torch.from_numpy(t32).cuda())
    d64 = [a.astype(np.float64) for a in (th32, x32, t32)]
    ref_g = mlp.backward(*d64)
    ref_l = mlp.loss(*d64)
    assert abs(loss - ref_l) <= 1e-5 * abs(ref_l)
    g = g.cpu().numpy()
    scale = np.abs(ref_g).max()
    np.testing.assert_allclose(g, ref_g, rtol=1e-4, atol=1e-4 * scale)


def test_training_reduces_loss(fnn):
    import torch
    from oracle import mlp
    rng = np.random.default_rng(3)
    teacher = mlp.init(5)
    x = rng.normal(0, 1, (20000, 16))
    t, _ = mlp.forward(teacher, x)
    th = torch.from_numpy(mlp.init(9).astype(np.float32)).cuda()
    X = torch.from_numpy(x.astype(np.float32)).cuda()
    T = torch.from_numpy(t.astype(np.float32)).cuda()
    l0, _ = fnn.fnn_mlp_loss_grad(th, X, T)
    losses = fnn.fnn_mlp_train(th, X, T, epochs=15, batch=512, lr=3e-3, seed=1)
    l1, _ = fnn.fnn_mlp_loss_grad(th, X, T)
    assert np.all(np.isfinite(losses))
    assert l1 < 0.2 * l0, (l0, l1, losses)


def _model(fnn, x, eps, metric):
    """A model trained here on this set's own trace (kept small)."""
    import torch
    from paper_2510_14147_amd.train_cost_model import init_params
    tree = fnn.fnn_tree_build(x, metric)
    g = fnn.fnn_eps_graph(tree, eps, trace=True)
    th = torch.from_numpy(init_params(3)).cuda()
    fnn.fnn_mlp_train(th, g.features.clone(), g.targets.clone(), epochs=30,
                      batch=256, lr=3e-3, seed=2)
    return th.cpu().numpy(), g


def test_trace_targets_are_degrees(fnn):
    x = G.c1_clusters(n_centers=6, per_center=500)
    tree = fnn.fnn_tree_build(x, "l2")
    g = fnn.fnn_eps_graph(tree, 0.1, trace=True)
    order = fnn.fnn_tree_export(tree)["order"]
    rp = g.row_ptr.cpu().numpy()
    deg = np.diff(rp)[order]
    np.testing.assert_allclose(g.targets[:, 1].cpu().numpy(), np.log1p(deg),
                               rtol=1e-6)
    assert np.all(np.isfinite(g.features.cpu().numpy()))


@pytest.mark.parametrize("case", ["c1", "rand", "ham"])
@pytest.mark.parametrize("slack", [None, -90])
def test_learned_schedule_same_graph(fnn, case, slack):
    if case == "c1":
        x, eps, metric = G.c1_clusters(), W["c1"]["eps"], "l2"
    elif case == "rand":
        x, eps, metric = G.random_points(5000, 6, seed=8, duplicates=50), 0.35, "l2"
    else:
        x, eps, metric = G.random_codes(3000, 128, seed=6, n_centers=12, flip=0.08), 14.0, "hamming"
    th, g_ref = _model(fnn, x, eps, metric)
    fnn.fnn_set_cost_model(th)
    tree = fnn.fnn_tree_build(x, metric)
    g = fnn.fnn_eps_graph(tree, eps, sched="learned", slack_pct=slack)
    a, b = g.to_numpy(), g_ref.to_numpy()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(a[2].view(np.uint32), b[2].view(np.uint32))
    st = g.stats
    assert st["pred_mae"] >= 0.0 and st["pred_sum_ratio"] > 0.0
    if slack == -90:
        # rows outgrow their slots: entries spill, and rows whose spill does
        # not fit are re-done by the restricted fill
        assert st["spilled"] > 0 or st["overflow_rows"] > 0


def test_learned_mfma_same_graph(fnn):
    x = G.c2_manifold(n=12000)
    eps = W["c2_50k"]["eps"][0]
    th, _ = _model(fnn, x, eps, "l2")
    fnn.fnn_set_cost_model(th)
    tree = fnn.fnn_tree_build(x, "l2")
    g1 = fnn.fnn_eps_graph(tree, eps, precision="bf16", sched="learned")
    g2 = fnn.fnn_eps_graph(tree, eps, precision="fp32")
    for u, v in zip(g1.to_numpy()[:2], g2.to_numpy()[:2]):
        assert np.array_equal(u, v)
