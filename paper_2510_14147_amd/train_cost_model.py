"""Train the cost model on traces of the 1M x 128 Euclidean workload.

Runs the query with trace capture at several radii around the calibrated
~70- and ~500-neighbour ones and on a quarter-density prefix, trains the
16-64-64-2 network on the GPU with the library's own backward and Adam
kernels, and writes the parameters and a short report to
``cost_model.json``.  The held-out check (other draws of the same manifold)
is tests/test_gpu_learned.py.

    python -m paper_2510_14147_amd.train_cost_model [--out PATH] [--n N]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import paper_2510_14147_amd as fnn  # noqa: E402
from paper_2510_14147_amd import datagen as G  # noqa: E402

W = json.load(open(os.path.join(HERE, "workloads.json")))


def init_params(seed: int) -> np.ndarray:
    """He-normal weights, zero biases, in the library's parameter layout."""
    rng = np.random.default_rng(seed)
    parts = []
    for rows, cols in ((64, 16), (64, 64), (2, 64)):
        parts.append(rng.normal(0.0, np.sqrt(2.0 / cols), (rows, cols)).ravel())
        parts.append(np.zeros(rows))
    return np.concatenate(parts).astype(np.float32)


def traces(x, eps_list, precision="bf16"):
    import torch
    xd = torch.from_numpy(x).cuda()
    feats, targs = [], []
    for eps in eps_list:
        t0 = time.time()
        tree = fnn.fnn_tree_build(xd, "l2")
        g = fnn.fnn_eps_graph(tree, eps, precision=precision, trace=True)
        feats.append(g.features.clone())
        targs.append(g.targets.clone())
        print(f"[train] trace eps={eps:.4f} nnz={g.nnz} {time.time() - t0:.1f}s",
              flush=True)
        del g, tree
    return torch.cat(feats), torch.cat(targs)


def main(argv=None):
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "cost_model.json"))
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--epochs", type=int, default=12)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=2e-3)
    args = ap.parse_args(argv)
    # several radii and densities, so that no feature value identifies one
    # trace: the 10^6 set at four radii between the ~70- and ~500-neighbour
    # ones (and a little below), and a quarter of it (a quarter of the
    # density) at two larger radii
    x = G.c2_manifold(n=args.n)
    e70, e500 = W["c2"]["eps"]
    radii = [0.9 * e70, e70, (e70 * e500) ** 0.5, e500]
    X1, T1 = traces(x, radii)
    X2, T2 = traces(x[: args.n // 4], [e500, 1.15 * e500])
    X, T = torch.cat([X1, X2]), torch.cat([T1, T2])
    del X1, T1, X2, T2
    th = torch.from_numpy(init_params(7)).cuda()
    t0 = time.time()
    losses = fnn.fnn_mlp_train(th, X, T, epochs=args.epochs, batch=args.batch,
                               lr=args.lr, seed=11)
    torch.cuda.synchronize()
    dt = time.time() - t0
    Y = fnn.fnn_mlp_forward(th, X)
    mae = (Y - T).abs().mean(0).tolist()
    print(f"[train] {X.shape[0]} samples, {args.epochs} epochs in {dt:.2f}s; "
          f"epoch losses {np.round(losses, 4).tolist()}; MAE {mae}", flush=True)
    rep = {"params": th.cpu().numpy().astype(float).tolist(),
           "layout": "W1[64][16] b1[64] W2[64][64] b2[64] W3[2][64] b3[2]",
           "trained_on": f"c2_manifold n={args.n} d=128 at eps={radii}, "
                         f"and its first {args.n // 4} rows at eps={[e500, 1.15 * e500]}",
           "samples": int(X.shape[0]), "epochs": args.epochs,
           "batch": args.batch, "lr": args.lr, "epoch_loss": losses.tolist(),
           "mae_log1p": {"visits": mae[0], "neighbours": mae[1]},
           "train_seconds": dt}
    with open(args.out, "w") as f:
        json.dump(rep, f)
    print("[train] wrote", args.out, flush=True)


if __name__ == "__main__":
    main()
