"""The learned-proposal form over a set of seeded exemplars.

For each exemplar (the 256^2 -> 512^2 workload's finest level: 8 x 8
windows on the stride-2 grid, PCA 64, 32-way k-means tree of depth 2 =
1024 leaves): build the index, label sampled queries of two plain
search/blend iterations and of six other initial outputs with the leaf of
their exhaustive full-dimension match (131 072 pairs per exemplar, ~2.1M
over 16 exemplars), train the leaf-proposal MLP on them, then run ten
learned search/blend iterations from another initial output and measure,
at every iterate, the energy gap to exhaustive search on the same image
(G_t = E(x; nn_method) / E(x; nn_exact) - 1): the learned form with an
exact FP32 scan of the proposed leaves (top-8 in PCA space, re-ranked in
full dimension), the same with BF16 scans, the one-pass BF16 scan whose
candidates are the query's 12 smallest class minima, and the plain tree.  Each exemplar's network proposes the leaves
of that exemplar's tree.  Only C-ABI calls are sequenced here.
"""
from __future__ import annotations

import time

import numpy as np

from . import synth, training


def run_exemplar(ctx, wl, seed: int, iters: int = 10, train_iters: int = 2, extra_inits: int = 6,
                 per_source: int = 16384, epochs: float = 16.0, mode: str = "learned", margin: float = 0.2,
                 n_proposals: int = 4, residual: int = 0, class_topk: int = 12, log=None):
    w, s = wl.w[-1], wl.stride[-1]
    H = wl.out_size
    ex = wl.exemplar(seed)
    ctx.set_exemplar_u8(ex, 0.5)
    info = ctx.build_index(w, wl.pca_dims, wl.branching, wl.depth, seed=0, make_bf16=True)
    t0 = time.time()
    q, lab = training.collect_training_pairs(ctx, ex, H, H, w, s, seed, solve_iters=train_iters,
                                             extra_inits=extra_inits, per_source=per_source, seed=seed)
    ctx.mlp_init(info.d, 256, info.n_leaves, seed=seed)
    losses = training.train(ctx, q, lab, epochs=epochs, batch=4096, lr=2e-3, log_every=25)
    prop, _ = ctx.mlp_propose(q, n_proposals)
    recall = float((prop == lab[:, None]).any(dim=1).float().mean())
    train_s = time.time() - t0
    # evaluation from another initial output
    init2, _ = synth.row_matched_init(seed + 1000, ex, H, H, w)
    res = {}
    forms = (("learned", dict(mode=mode, margin=margin, n_proposals=n_proposals, rerank_full=1)),
             ("learned_bf16", dict(mode="learned_bf16", margin=margin, n_proposals=n_proposals, rerank_full=1,
                                   residual=residual)),
             ("learned_bf16_class", dict(mode="learned_bf16_class", margin=margin, n_proposals=n_proposals,
                                         rerank_full=1, residual=residual, topk=class_topk)),
             ("tree", dict(mode="tree")))
    for name, kw in forms:
        x = ctx.rgbs_from_u8(init2, 0.5)
        G, fb = [], []
        for _ in range(iters):
            nn, d, st = ctx.estep(x, w, s, stats=True, **kw)
            _, d_x = ctx.estep(x, w, s, mode="exact_full")
            G.append(ctx.energy(d)[0] / ctx.energy(d_x)[0] - 1.0)
            fb.append(st.fallbacks / st.nq)
            ctx.mstep(nn, d, x, w, s)
        res[name] = dict(gaps=G, max_gap=max(G), last_gap=G[-1], fallback_rate=float(np.mean(fb)))
    out = dict(seed=seed, pairs=int(q.shape[0]), leaves=info.n_leaves, loss_first=float(losses[0]),
               loss_last=float(losses[-1]), top4_train_recall=recall, train_s=train_s, **res)
    if log:
        log(f"seed {seed}: pairs {out['pairs']}, loss {losses[0]:.3f} -> {losses[-1]:.3f}, recall {recall:.3f}, "
            f"learned gap max {res['learned']['max_gap']:.4f} last {res['learned']['last_gap']:.4f} "
            f"(fallbacks {res['learned']['fallback_rate']:.3f}); learned BF16 + full-D re-rank gap max "
            f"{res['learned_bf16']['max_gap']:.4f} last {res['learned_bf16']['last_gap']:.4f}; class candidates "
            f"{res['learned_bf16_class']['max_gap']:.4f} last {res['learned_bf16_class']['last_gap']:.4f}; "
            f"tree gap max {res['tree']['max_gap']:.4f}")
    return out


def run(ctx, seeds=None, **kw):
    wl = synth.workload("ex256_out512_learned")
    seeds = list(wl.extra["exemplar_seeds"]) if seeds is None else list(seeds)
    return [run_exemplar(ctx, wl, sd, **kw) for sd in seeds]
