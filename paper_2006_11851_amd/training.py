"""Training-data orchestration for the leaf-proposal MLP.

Pairs (PCA query, leaf of the query's exact match) come from the search
method itself: the output windows visited by a plain solve (tree search and
patch blend), each labelled with the leaf that holds its exhaustive
full-dimension nearest neighbour.  Everything here only sequences calls of
the C ABI; every step runs in libpts kernels.
"""
from __future__ import annotations

import torch


def collect_pairs(ctx, x0, w: int, stride: int, iters: int, mode: str = "tree"):
    """Run `iters` search/blend iterations from x0 (not modified); return
    (queries float32 [iters*nq][d], labels int32 [iters*nq])."""
    x = x0.clone()
    qs, ls = [], []
    for _ in range(iters):
        q = ctx.project(x, stride)
        nn_exact, _ = ctx.estep(x, w, stride, mode="exact_full")
        qs.append(q)
        ls.append(ctx.leaf_of(nn_exact))
        nn, dist = ctx.estep(x, w, stride, mode=mode)
        ctx.mstep(nn, dist, x, w, stride)
    return torch.cat(qs), torch.cat(ls)


def train(ctx, q, labels, epochs: float = 4.0, batch: int = 4096, lr: float = 2e-3, seed: int = 0, bf16=True,
          log_every: int = 50):
    steps = max(1, int(epochs * q.shape[0] / batch))
    return ctx.mlp_train(q, labels, steps, batch=batch, lr=lr, seed=seed, bf16=bf16, log_every=log_every)


def collect_pairs_sampled(ctx, x0, w: int, stride: int, iters: int, per_iter: int, seed: int = 0,
                          mode: str = "tree"):
    """As collect_pairs, labelling a seeded random sample of `per_iter` output
    windows per iteration with the exhaustive search of those windows only."""
    x = x0.clone()
    H, W = x.shape[:2]
    nq = ctx.nq(H, W, w, stride)
    g = torch.Generator(device="cpu").manual_seed(seed)
    qs, ls = [], []
    for _ in range(iters):
        qids = torch.randperm(nq, generator=g)[:per_iter].to(torch.int32).to(x.device)
        qp = ctx.project(x, stride)
        nn_exact, _ = ctx.exact_search(x, w, stride, qids)
        qs.append(qp[qids.long()])
        ls.append(ctx.leaf_of(nn_exact))
        nn, dist = ctx.estep(x, w, stride, mode=mode)
        ctx.mstep(nn, dist, x, w, stride)
    return torch.cat(qs).contiguous(), torch.cat(ls).contiguous()
