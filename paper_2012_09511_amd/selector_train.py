"""Training of the learned machine-pair selector from logged search nodes.

Data: full-LB2 depth-first searches (pfsp_search with the node log on) on a
set of training instances; every logged node is bounded again with
LB2_FULL and its per-child argmax pairs are turned into a soft target (the
share of children whose LB2 is attained first by each pair).  Features and
targets come from the library's kernels; the training steps (forward,
backward, Adam) run in the library's kernels too.  This module only moves
batches around.

    python -m paper_2012_09511_amd.selector_train --out selector.npy
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import binding, inputs


def collect(ctx, instances, budget_nodes=2_000_000, log_capacity=200_000, log_stride=8,
            max_per_instance=50_000, chunk=65536, seed=0, log=None):
    """Logs nodes of full-LB2 searches and returns (features [N,64], targets [N,190])
    as device tensors, plus per-instance statistics."""
    import torch
    feats, targs, stats = [], [], []
    rng = np.random.default_rng(seed)
    for (n, m, p) in instances:
        ctx.load_instance(p)
        ub0, _ = ctx.neh()
        ctx.set_option("log_capacity", log_capacity)
        ctx.set_option("log_stride", log_stride)
        t0 = time.time()
        r = ctx.search(ub0 + 1, budget_nodes, binding.LB2_FULL)
        perm, d1, d2 = ctx.search_log(log_capacity)
        ctx.set_option("log_capacity", 0)
        if len(perm) > max_per_instance:
            keep = np.sort(rng.choice(len(perm), max_per_instance, replace=False))
            perm, d1, d2 = perm[keep], d1[keep], d2[keep]
        for s in range(0, len(perm), chunk):
            dev = [torch.from_numpy(np.ascontiguousarray(a[s:s + chunk])).to(ctx.device)
                   for a in (perm, d1, d2)]
            _, _, _, ap = ctx.bound_children(*dev, kind=binding.LB2_FULL, want_argpair=True)
            targs.append(ctx.selector_targets(*dev, ap))
            feats.append(ctx.selector_features(*dev))
        stats.append(dict(n=n, m=m, nodes=r["nodes"], logged=len(perm), best=r["best"],
                          proven=r["proven"], seconds=round(time.time() - t0, 3)))
        if log:
            log(json.dumps(stats[-1]))
    X = torch.cat(feats) if feats else None
    T = torch.cat(targs) if targs else None
    return X, T, stats


def train(ctx, X, T, epochs=20, batch=4096, lr=2e-3, seed=0, init=None, log=None):
    """Adam on the soft-target cross-entropy; returns (parameters, loss history)."""
    import torch
    params = init if init is not None else inputs.selector_params(seed)
    ctx.selector_set(params)
    g = torch.Generator(device="cpu").manual_seed(seed)
    N = X.shape[0]
    hist = []
    for ep in range(epochs):
        order = torch.randperm(N, generator=g).to(X.device)
        tot, cnt = 0.0, 0
        for s in range(0, N, batch):
            idx = order[s:s + batch]
            loss, _ = ctx.selector_train_step(X[idx].contiguous(), T[idx].contiguous(), lr)
            tot += loss * len(idx)
            cnt += len(idx)
        hist.append(tot / max(cnt, 1))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.4f}")
    return ctx.selector_get(), hist


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="selector.npy")
    ap.add_argument("--n", type=int, default=50)
    ap.add_argument("--m", type=int, default=20)
    ap.add_argument("--seeds", default="500-531")
    ap.add_argument("--budget", type=int, default=2_000_000)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--lr", type=float, default=2e-3)
    args = ap.parse_args()
    a, b = (int(x) for x in args.seeds.split("-"))
    ctx = binding.Context(0)
    insts = [(args.n, args.m, inputs.instance(args.n, args.m, s)) for s in range(a, b + 1)]
    X, T, stats = collect(ctx, insts, budget_nodes=args.budget,
                          log=lambda s: print(s, flush=True))
    print(json.dumps(dict(records=int(X.shape[0]), instances=stats)), flush=True)
    params, hist = train(ctx, X, T, epochs=args.epochs, lr=args.lr,
                         log=lambda s: print(s, flush=True))
    np.save(args.out, params)
    print(json.dumps(dict(saved=args.out, loss=hist)))


if __name__ == "__main__":
    main()
