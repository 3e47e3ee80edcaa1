"""Training-data orchestration for the leaf-proposal MLP.

Pairs (PCA query, leaf of the query's exact match) come from the search
method itself: the output windows visited by a plain solve (tree search and
patch blend), each labelled with the leaf that holds its exhaustive
full-dimension nearest neighbour.  Everything here only sequences calls of
the C ABI; every step runs in libpts kernels.
"""
from __future__ import annotations

import torch

from . import synth


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


def collect_training_pairs(ctx, ex_u8, H: int, W: int, w: int, stride: int, init_seed: int, solve_iters: int = 2,
                           extra_inits: int = 6, per_source: int = 16384, seed: int = 0, guidance: float = 0.5):
    """The training recipe: pairs from `solve_iters` iterations of a plain
    solve started from the initial output of `init_seed`, plus the initial
    outputs of `extra_inits` other seeds (init_seed + 2000 + k), a seeded
    sample of `per_source` queries from each.  The extra initial outputs
    matter: a solve's first iterations move its queries away from those of a
    freshly initialised output, which the network must also serve."""
    src, _ = synth.row_matched_init(init_seed, ex_u8, H, W, w)
    q, lab = collect_pairs_sampled(ctx, ctx.rgbs_from_u8(src, guidance), w, stride, solve_iters, per_source, seed=seed)
    qs, ls = [q], [lab]
    for k in range(extra_inits):
        ik, _ = synth.row_matched_init(init_seed + 2000 + k, ex_u8, H, W, w)
        a, b = collect_pairs_sampled(ctx, ctx.rgbs_from_u8(ik, guidance), w, stride, 1, per_source, seed=seed + 1 + k)
        qs.append(a)
        ls.append(b)
    return torch.cat(qs).contiguous(), torch.cat(ls).contiguous()
