"""Trains the learned codec selector on the GPU with this project's kernels.

Data: frontiers that the GPU BFS itself produces on seeded R-MAT graphs
(scales 18..22, seeds 1..5, 4 roots each), every level split into 16 equal
and into 256 Zipf(1.2)-sized destination ranges.  Per 128-ID block: the eight
fp16 features (bfsc_features) and the exhaustive choice as the label
(bfsc_select, EXHAUSTIVE).  Training: softmax cross-entropy, Adam, batches
of 8192 (bfsc_mlp_train_step); the network is 8 -> 64 -> 64 -> 35.

    python -m paper_1704_00513_amd.train [--scales 18 19 20 21 22] [--seeds 1 2 3 4 5]

Writes selector_weights.npy (fp32, 7011 values) and selector_weights.json
next to this file.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
WEIGHTS = os.path.join(HERE, "selector_weights.npy")
META = os.path.join(HERE, "selector_weights.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def frontier_batches(ctx, P, torch, g, roots, splits):
    """GPU BFS from each root; yields (ids tensor, n, level) per level."""
    dg = P.DeviceGraph.from_host(g)
    V = g.n_vertices
    level = torch.empty(V, dtype=torch.int32, device="cuda")
    parent = torch.empty(V, dtype=torch.int32, device="cuda")
    fa = torch.empty(V, dtype=torch.int32, device="cuda")
    fb = torch.empty(V, dtype=torch.int32, device="cuda")
    la = torch.zeros(1, dtype=torch.int32, device="cuda")
    lb = torch.zeros(1, dtype=torch.int32, device="cuda")
    ws = ctx.bfs_workspace(dg)
    for root in roots:
        ctx.bfs_init(dg, int(root), level, parent, fa, la, ws)
        L = 0
        while True:
            n = int(la.item())
            if n == 0:
                break
            yield fa, n, L
            ctx.bfs_level(dg, L, fa, la, level, parent, fb, lb, ws)
            fa, fb, la, lb = fb, fa, lb, la
            L += 1


def build_dataset(ctx, P, torch, scales, seeds, n_roots=4, nseg_eq=16, nseg_zipf=256):
    """Features X (u16 [N, 8]) and exhaustive labels y (u8 [N]) on the host."""
    import inputs
    Xs, ys = [], []
    for scale in scales:
        for seed in seeds:
            t0 = time.time()
            g = inputs.Graph(inputs.RMAT, scale, 16, seed)
            roots = inputs.roots(g, n_roots, seed)
            V = g.n_vertices
            splits = [inputs.bounds_equal(V, nseg_eq), inputs.bounds_zipf(V, nseg_zipf, seed)[0]]
            dev_bounds = [torch.from_numpy(b.view(np.int32)).cuda() for b in splits]
            nblk = 0
            for ids, n, L in frontier_batches(ctx, P, torch, g, roots, splits):
                for bh, bd in zip(splits, dev_bounds):
                    R = bh.size - 1
                    seg_off = torch.zeros(R + 1, dtype=torch.int64, device="cuda")
                    n_dev = torch.tensor([n], dtype=torch.int32, device="cuda")
                    ctx.partition(ids, n_dev, bd, seg_off)
                    lev = torch.full((R,), L, dtype=torch.int32, device="cuda")
                    b = P.DeviceBatch(ids, seg_off, bd[:-1].contiguous(), bd[1:].contiguous(), lev,
                                      max_ids=n)
                    feat = torch.zeros((b.n_blocks_max, 8), dtype=torch.int16, device="cuda")
                    cls = torch.zeros(b.n_blocks_max, dtype=torch.uint8, device="cuda")
                    ctx.features(b, feat)
                    ctx.select(b, P.SEL_EXHAUSTIVE, cls)
                    nb = (np.diff(seg_off.cpu().numpy()) + 127) // 128
                    k = int(nb.sum())
                    Xs.append(feat[:k].cpu().numpy().view(np.uint16))
                    ys.append(cls[:k].cpu().numpy())
                    nblk += k
            ctx.sync()
            log("scale %d seed %d: %d blocks (%.1fs)" % (scale, seed, nblk, time.time() - t0))
            del g
    return np.concatenate(Xs), np.concatenate(ys)


def train(ctx, P, torch, X, y, epochs=8, batch=8192, lr=1e-3, seed=1):
    import inputs
    rng = np.random.default_rng(seed)
    perm = rng.permutation(X.shape[0])
    X, y = X[perm], y[perm]
    Xd = torch.from_numpy(np.ascontiguousarray(X).view(np.int16)).cuda()
    yd = torch.from_numpy(np.ascontiguousarray(y)).cuda()
    ctx.mlp_init(seed)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    ws = ctx.workspace(P.OP_MLP, batch, 0, key="mlp")
    N = X.shape[0]
    hist = []
    for ep in range(epochs):
        tot, cnt = 0.0, 0
        for s in range(0, N - batch + 1, batch):
            ctx.mlp_train_step(Xd[s:s + batch], yd[s:s + batch], batch, lr=lr, loss=loss, ws=ws)
            if (s // batch) % 20 == 0:
                tot += float(loss.item())
                cnt += 1
        hist.append(tot / max(1, cnt))
        log("epoch %d: loss %.4f" % (ep, hist[-1]))
    ctx.sync()
    return ctx.mlp_get_weights(), hist


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--scales", type=int, nargs="+", default=[18, 19, 20, 21, 22])
    ap.add_argument("--seeds", type=int, nargs="+", default=[1, 2, 3, 4, 5])
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--out", default=WEIGHTS)
    args = ap.parse_args()
    sys.path.insert(0, ROOT)
    import torch
    import paper_1704_00513_amd as P

    ctx = P.Context(0)
    t0 = time.time()
    X, y = build_dataset(ctx, P, torch, args.scales, args.seeds)
    log("dataset: %d blocks, %d classes present (%.1fs)" % (X.shape[0], np.unique(y).size,
                                                              time.time() - t0))
    w, hist = train(ctx, P, torch, X, y, epochs=args.epochs)
    np.save(args.out, w.astype(np.float32), allow_pickle=False)
    meta = {"shape": [8, 64, 64, 35], "classes": "0 bitmap, 1..33 bit-pack width 0..32, 34 PFOR",
            "features": ["n/128", "bitlen(min d)/32", "bitlen(max d)/32", "bitlen(span/m)/32",
                         "bitlen(span)/32", "n/(span+1)", "min(level,63)/64", "bitlen(seg n)/32"],
            "data": {"graph": "rmat", "scales": args.scales, "seeds": args.seeds, "roots": 4,
                     "splits": ["equal16", "zipf256"], "blocks": int(X.shape[0])},
            "label_hist": {str(int(k)): int(v) for k, v in zip(*np.unique(y, return_counts=True))},
            "train": {"epochs": args.epochs, "batch": 8192, "optimizer": "adam lr 1e-3",
                      "loss_per_epoch": [round(x, 5) for x in hist]}}
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(meta, f, indent=1)
    log("wrote %s (%.1fs total)" % (args.out, time.time() - t0))
    ctx.close()


if __name__ == "__main__":
    main()
