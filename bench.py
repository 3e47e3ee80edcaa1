"""Benchmark: NN queries/s and ms/iteration, BF16 + learned proposal against
the plain FP32 tree search, at the finest level of a synthetic workload.

One step = one iteration over the whole output image: E-step (projection,
search, winner distance) + M-step (2x2 patch blend) + energy, with inputs
resident in HBM.  Both forms run from the same initial output; the
proposal network is trained on pairs from a plain solve started from
another initial output (held out).  After the timed steps the same
trajectory is replayed untimed (the steps are deterministic; the replay
checks that it reaches the same image) to record, at every iterate, the
energy gap to exhaustive full-dimension search on a fixed random 1/16 of the
queries and the work each scan did.  Prints one JSON line.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--form learned_bf16|brute_bf16]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: dense bf16 MFMA, FP32 matrix (MFMA), FP32 vector (TFLOP/s); HBM (GB/s)
PEAK = {"bf16": 2500.0, "fp32_matrix": 157.3, "fp32_vector": 157.3, "hbm": 8000.0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="ex1024_out2048")
    ap.add_argument("--form", default="learned_bf16", help="learned_bf16 (headline) or brute_bf16 (precision form)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-solve", action="store_true", help="skip the timed multiscale solves")
    ap.add_argument("--no-exact", action="store_true", help="skip the timed exhaustive E-step")
    ap.add_argument("--train-iters", type=int, default=2, help="plain-solve iterations labelled for training")
    ap.add_argument("--train-inits", type=int, default=6, help="other initial outputs labelled for training")
    ap.add_argument("--train-per-iter", type=int, default=65536, help="queries sampled per labelled image")
    ap.add_argument("--epochs", type=float, default=6.0)
    ap.add_argument("--proposals", type=int, default=4)
    ap.add_argument("--margin", type=float, default=0.2)
    ap.add_argument("--residual", type=int, default=0)
    ap.add_argument("--rerank-full", type=int, default=1)
    ap.add_argument("--only", default="", help="run one form only (tree, learned_bf16 or brute_bf16)")
    ap.add_argument("--suite", default="", help="learned_c4: the learned form over the 16 seeded 256^2 exemplars")
    ap.add_argument("--suite-seeds", type=int, default=16)
    ap.add_argument("--class-topk", type=int, default=12,
                    help="class-minimum candidates re-ranked in full D by the reported learned form")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-MiB tensor 3 times (the HBM-counter scale for rocprofv3 --pmc) and exit")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU: --gpus must be 1", "n_gpus": a.gpus}))
        sys.exit(2)
    import torch

    if a.calibrate_copy:
        n = a.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": 4 * n, "launches": 3}))
        return
    if a.suite == "learned_c4":
        return learned_suite(a)
    return headline(a)


def headline(a):
    import torch

    from paper_2006_11851_amd import pts, synth, training

    wl = synth.workload(a.workload)
    ex = wl.exemplar()
    w, s = wl.w[-1], wl.stride[-1]
    Hout = wl.out_size
    ctx = pts.Context(0)
    ctx.set_exemplar_u8(ex, 0.5)
    t0 = time.time()
    info = ctx.build_index(w, wl.pca_dims, wl.branching, wl.depth, seed=0, make_bf16=True)
    build_s = time.time() - t0
    log(f"index: N={info.N} d={info.d} leaves={info.n_leaves} mean leaf {info.leaf_mean:.1f} "
        f"retained {info.retained_variance:.4f} in {build_s:.1f} s")
    init, _ = synth.row_matched_init(wl.init_seed, ex, Hout, Hout, w)
    x0 = ctx.rgbs_from_u8(init, 0.5)
    nq = ctx.nq(Hout, Hout, w, s)
    learned = a.form == "learned_bf16"

    setup = {"index_build_s": build_s}
    if learned:
        # the network learns from held-out images: a plain solve from another
        # initial output and further initial outputs (seeds other than the
        # timed trajectory's)
        torch.cuda.synchronize()
        t0 = time.time()
        q, lab = training.collect_training_pairs(ctx, ex, Hout, Hout, w, s, wl.init_seed + 1,
                                                 solve_iters=a.train_iters, extra_inits=a.train_inits,
                                                 per_source=min(a.train_per_iter, nq), seed=1)
        torch.cuda.synchronize()
        label_s = time.time() - t0
        t0 = time.time()
        ctx.mlp_init(info.d, 256, info.n_leaves, seed=0)
        losses = training.train(ctx, q, lab, epochs=a.epochs, batch=4096, lr=2e-3, log_every=50)
        torch.cuda.synchronize()
        train_s = time.time() - t0
        prop, _ = ctx.mlp_propose(q, a.proposals)
        recall = float((prop == lab[:, None]).any(dim=1).float().mean())
        setup.update(labels_s=label_s, training_s=train_s, mlp_pairs=int(q.shape[0]),
                     mlp_loss_first=float(losses[0]), mlp_loss_last=float(losses[-1]),
                     top_p_train_recall=recall)
        log(f"MLP: {q.shape[0]} pairs labelled in {label_s:.1f} s (held-out images), trained in {train_s:.1f} s, "
            f"loss {losses[0]:.3f} -> {losses[-1]:.3f}, top-{a.proposals} train recall {recall:.3f}")
        del q, lab

    sample = torch.randperm(nq, generator=torch.Generator().manual_seed(16))[: nq // 16].to(torch.int32).cuda()

    def gap(x, dist):
        _, d_ex = ctx.exact_search(x, w, s, sample)
        return ctx.energy(dist[sample.long()].contiguous())[0] / ctx.energy(d_ex)[0] - 1.0

    if learned:
        # headline: one BF16 pass whose candidates are the query's 8 smallest
        # class minima; beside it the exact BF16 top-8 form (two passes)
        exact_kw = dict(mode="learned_bf16", residual=a.residual, rerank_full=a.rerank_full,
                        n_proposals=a.proposals, margin=a.margin)
        method = ("bf16_learned_class", dict(exact_kw, mode="learned_bf16_class", topk=a.class_topk))
        forms = dict([("plain_fp32_tree", dict(mode="tree")), ("bf16_learned_exact_top8", exact_kw), method])
    else:
        method = ("bf16_brute", dict(mode="brute_bf16", residual=a.residual, rerank_full=a.rerank_full, topk=16))
        forms = dict([("plain_fp32_tree", dict(mode="tree")), method])
    if a.only:
        forms = {k: v for k, v in forms.items() if v["mode"] == a.only}
    res = {}
    for name, kw in forms.items():
        res[name] = run_form(ctx, x0, w, s, nq, kw, a, gap)
        r = res[name]
        log(f"{name}: {r['value']:.3e} q/s, {r['ms_per_step']:.3f} ms/step (median {r['ms_per_step_median']:.3f}), "
            f"gap max {r['gap_max']:.4f} (first {r['gaps'][0]:.4f}, last {r['gaps'][-1]:.4f})")

    head = res.get(method[0]) or res["plain_fp32_tree"]
    tree = res.get("plain_fp32_tree")
    if learned and method[0] in res and "bf16_learned_exact_top8" in res:
        # the class-minimum candidates against the exact top-8 on the initial
        # output: identical winners and the energy difference
        nn_c, d_c = ctx.estep(x0, w, s, **method[1])
        nn_e, d_e = ctx.estep(x0, w, s, **forms["bf16_learned_exact_top8"])
        setup["class_vs_exact_top8"] = dict(
            identical_winners=float((nn_c == nn_e).float().mean()),
            energy_ratio=float(ctx.energy(d_c)[0] / ctx.energy(d_e)[0]))
        log(f"class candidates vs exact top-8 at x0: identical winners "
            f"{setup['class_vs_exact_top8']['identical_winners']:.4f}, energy ratio "
            f"{setup['class_vs_exact_top8']['energy_ratio']:.6f}")
    if learned and tree and method[0] in res:
        saving_ms = tree["ms_per_step"] - head["ms_per_step"]
        setup_ms = 1000.0 * (setup["labels_s"] + setup["training_s"])
        setup["break_even_iterations"] = setup_ms / saving_ms if saving_ms > 0 else None
    kern = head["kernels_ms_per_step"]
    rank = sorted(kern, key=lambda k: -kern[k])
    roofs = [roofline(head, info, nq, a, k, a.workload) for k in rank[:4]]
    roofs = [r for r in roofs if r["bound"] is not None] or roofs
    roof = max(roofs, key=lambda r: r["ms_per_launch"])
    roof_next = [r for r in roofs if r is not roof]

    extra = {}
    if not a.no_exact:
        extra["exact_fp32_estep"] = exact_row(ctx, x0, w, s, nq)
        log(f"exact FP32 exhaustive E-step: {extra['exact_fp32_estep']['value']:.3e} q/s")
    if not a.no_solve and a.workload == "ex1024_out2048":
        extra["solve"] = solve_rows(ctx, wl, ex, learned, a)
    cpu = None
    if not a.no_cpu:
        cpu = cpu_baseline(ctx, ex, init, w, s, a.cpu_seconds, threads=1)
        extra["cpu_baseline_all_cores"] = cpu_baseline(ctx, ex, init, w, s, a.cpu_seconds, threads=0)
    if not a.no_solve and a.workload == "ex1024_out2048":
        # last: these replace the context's exemplar and index
        extra["solve_small_workloads"] = small_solve_rows(ctx)
    out = {
        "metric": "NN queries/s + ms/iteration",
        "value": head["value"],
        "unit": "NN queries/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16" if head is not tree else "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{a.workload} finest level: exemplar {wl.ex_size}^2, output {Hout}^2, w={w}, stride={s}, "
                        f"N={info.N}, nq={nq}, PCA {info.d}, k-means tree b{wl.branching} L{wl.depth} "
                        f"({info.n_leaves} leaves)",
            "form": (f"one BF16 MFMA scan of the MLP's top-{a.proposals} leaves (plus the tree's leaf below margin "
                     f"{a.margin}), the {a.class_topk} smallest class minima as candidates (16 classes per leaf: "
                     f"rows i and i + 16 of each 32-row tile), FP32 re-rank" if learned else
                     "BF16 MFMA distances to every exemplar window, exact top-16, FP32 re-rank")
                    + (" in full D" if a.rerank_full else " in PCA space")
                    + (", residual-energy ranking" if a.residual else ""),
        },
        "forms": res,
        "speedup_vs_plain_fp32": (head["value"] / tree["value"]) if (tree and head is not tree) else None,
        "setup": setup,
        "roofline": roof,
        "roofline_next": roof_next,
        "cpu_baseline": cpu,
        **extra,
    }
    print(json.dumps(out))


def run_form(ctx, x0, w, s, nq, kw, a, gap):
    """Timed steps (total and per step), then the untimed replay of the same
    trajectory with the energy gap and the scan statistics at every iterate."""
    import torch

    x = x0.clone()
    nn = torch.empty(nq, dtype=torch.int32, device="cuda")
    dist = torch.empty(nq, dtype=torch.float32, device="cuda")
    # every step records its energy on the device; they are read after the
    # timed region, so the steps are not serialised by host round trips
    Edev = torch.zeros((a.warmup + a.steps, 2), dtype=torch.float32, device="cuda")

    def step(xx, i):
        ctx.estep(xx, w, s, nn=nn, dist=dist, **kw)
        ctx.mstep(nn, dist, xx, w, s)
        ctx.energy_device(dist, Edev[i])

    for i in range(a.warmup):
        step(x, i)
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(a.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for i in range(a.steps):
        step(x, a.warmup + i)
        ev[i + 1].record()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    per_step = [ev[i].elapsed_time(ev[i + 1]) for i in range(a.steps)]
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    E = Edev.double().cpu()
    x_timed = x
    # replay: the same trajectory, untimed, with the gap and statistics per iterate
    xr = x0.clone()
    gaps, stats = [], []
    for i in range(a.warmup + a.steps):
        nn_r, d_r, st = ctx.estep(xr, w, s, stats=True, **kw)
        gaps.append(gap(xr, d_r))
        stats.append(dict(fallbacks=st.fallbacks, scan_overflows=st.scan_overflows, scan_rows=st.scan_rows,
                          collect_rows=st.collect_rows))
        ctx.mstep(nn_r, d_r, xr, w, s)
    same = bool(torch.equal(xr, x_timed))
    timed = stats[a.warmup:]
    return dict(value=nq * a.steps / el, ms_per_step=1000 * el / a.steps,
                ms_per_step_median=float(np.median(per_step)), ms_per_step_events=per_step,
                gaps=gaps, gap_max=max(gaps), gap_first=gaps[0], gap_last=gaps[-1],
                energy_first=float(E[0, 0]), energy_last=float(E[-1, 0]),
                fallback_rate=float(np.mean([t["fallbacks"] for t in timed])) / nq,
                scan_overflow_rate=float(np.mean([t["scan_overflows"] for t in timed])) / nq,
                scan_rows_per_step=float(np.mean([t["scan_rows"] for t in timed])),
                collect_rows_per_step=float(np.mean([t["collect_rows"] for t in timed])),
                replay_identical=same,
                kernels_ms_per_step={k: v[0] / a.steps for k, v in prof.items()},
                launches={k: v[1] for k, v in prof.items()})


def roofline(head, info, nq, a, dom, workload=None):
    """Kernel `dom` of the reported form against its bound: algorithmic work
    per launch (counted on the device for the scans) over the launch's
    average time on the library's stream."""
    kern = head["kernels_ms_per_step"]
    launches = head["launches"]
    per_launch_ms = kern[dom] * a.steps / max(1, launches[dom])
    d, h, L = info.d, 256, info.n_leaves
    dk = -(-d // 32) * 32
    K1 = -(-d // 32) * 32
    if dom == "mlp_propose_mfma":
        # both hidden layers and the output layer (counted once; the queries
        # redone over its list run it again)
        flops = 2.0 * (K1 * h + h * h + h * (-(-L // 32) * 32)) * nq
        bound, peak, unit = "mfma", PEAK["bf16"], "TFLOP/s"
    elif dom in ("leaf_scan_bf16", "leaf_scan_bf16_class"):
        flops = 2.0 * dk * head["scan_rows_per_step"]
        bound, peak, unit = "mfma", PEAK["bf16"], "TFLOP/s"
    elif dom == "leaf_scan_bf16_collect":
        flops = 2.0 * dk * head["collect_rows_per_step"]
        bound, peak, unit = "mfma", PEAK["bf16"], "TFLOP/s"
    elif dom == "brute_bf16_topk":
        flops = 2.0 * dk * info.N * nq
        bound, peak, unit = "mfma", PEAK["bf16"], "TFLOP/s"
    elif dom == "project_queries":
        flops = 2.0 * info.D * d * nq
        bound, peak, unit = "mfma", PEAK["fp32_matrix"], "TFLOP/s"
    elif dom == "leaf_scan_f32":
        flops = 3.0 * d * nq * info.leaf_mean
        bound, peak, unit = "alu", PEAK["fp32_vector"], "TFLOP/s"
    else:
        return {"kernel": dom, "bound": None, "achieved": None, "peak": None, "unit": None, "frac": None,
                "traffic": None, "ms_per_launch": per_launch_ms}
    ach = flops / (per_launch_ms * 1e-3) / 1e12
    return {"kernel": dom, "bound": bound, "achieved": ach, "peak": peak, "unit": unit, "frac": ach / peak,
            "traffic": measured_traffic(dom, workload or a.workload), "ms_per_launch": per_launch_ms,
            "algorithmic_flops_per_launch": flops}


def measured_traffic(label, workload):
    """HBM bytes per full-size launch of the kernel behind `label` on this
    workload, from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary
    (scaled by the copy calibration), or None when there is none or the
    kernel's source file has changed since the counters were taken."""
    import glob
    import hashlib

    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*.md"))):
        for line in open(path):
            f = line.split()
            if len(f) == 6 and f[0] == "traffic:" and f[1] == workload and f[2] == label:
                src = os.path.join(ROOT, "paper_2006_11851_amd", "csrc", f[4])
                if not os.path.exists(src):
                    return None
                digest = hashlib.sha1(open(src, "rb").read()).hexdigest()[:12]
                return float(f[3]) if digest == f[5] else None
    return None


def exact_row(ctx, x0, w, s, nq):
    """The exhaustive FP32 E-step (the exact reference) over every query."""
    import torch

    x = x0.clone()
    ctx.estep(x, w, s, mode="exact_full")  # warm-up (allocations)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    ctx.estep(x, w, s, mode="exact_full")
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    return {"value": nq / (ms * 1e-3), "unit": "NN queries/s", "ms_per_estep": ms,
            "form": "exhaustive full-dimension FP32 search of every query (E-step only)"}


def solve_rows(ctx, wl, ex, learned, a):
    """The whole coarse-to-fine solve (four levels, ten iterations each; tree
    search at the coarse levels; at the finest level the plain tree or the
    learned form with this context's index and network): per level the sum
    of the per-iteration times (search + blend + energy), and the total."""
    import torch

    init0 = wl.initial_output(ex)
    x0 = ctx.rgbs_from_u8(init0, 0.5)
    levels = [dict(w=wl.w[l], stride=wl.stride[l], iters=wl.iters, pca_dims=wl.pca_dims, branching=wl.branching,
                   depth=wl.depth) for l in range(wl.levels)]
    out = {}
    modes = [("plain_fp32_tree", "tree")] + ([("bf16_learned_class", "learned_bf16_class"),
                                              ("bf16_learned_exact_top8", "learned_bf16")] if learned else [])
    for name, mode in modes:
        torch.cuda.synchronize()
        t0 = time.time()
        topk = a.class_topk if mode == "learned_bf16_class" else 8
        _, tr = ctx.solve(x0, levels, mode=mode, coarse_mode="tree", topk=topk, rerank_full=a.rerank_full,
                          n_proposals=a.proposals, margin=a.margin, residual=a.residual, reuse_finest_index=True)
        torch.cuda.synchronize()
        wall = time.time() - t0
        per_level = [float(tr["ms"][tr["level"] == l].sum()) for l in range(wl.levels)]
        out[name] = {"ms_per_level": per_level, "ms_iterations_total": float(sum(per_level)),
                     "wall_s_with_index_builds": wall, "energy_final": float(tr["E"][-1])}
        log(f"solve {name}: iterations {sum(per_level):.1f} ms (per level {['%.1f' % v for v in per_level]}), "
            f"wall {wall:.1f} s with the coarse levels' index builds")
    return out


def small_solve_rows(ctx):
    """The plain tree solve of the two small workloads (64^2 -> 128^2, one
    level of 5 iterations; 256^2 -> 512^2, three levels of 10), every level's
    index built by the solve: the sum of the per-iteration times and the wall
    time with the index builds."""
    import torch

    from paper_2006_11851_amd import synth

    out = {}
    for name in ("ex64_out128", "ex256_out512"):
        wl = synth.workload(name)
        ex = wl.exemplar()
        ctx.set_exemplar_u8(ex, 0.5)
        x0 = ctx.rgbs_from_u8(wl.initial_output(ex), 0.5)
        levels = [dict(w=wl.w[l], stride=wl.stride[l], iters=wl.iters, pca_dims=wl.pca_dims,
                       branching=wl.branching, depth=wl.depth) for l in range(wl.levels)]
        torch.cuda.synchronize()
        t0 = time.time()
        _, tr = ctx.solve(x0, levels, mode="tree", coarse_mode="tree")
        torch.cuda.synchronize()
        wall = time.time() - t0
        out[name] = {"ms_iterations_total": float(np.sum(tr["ms"])), "iterations": int(len(tr["ms"])),
                     "wall_s_with_index_builds": wall, "energy_final": float(tr["E"][-1])}
        log(f"solve {name} (plain tree): iterations {out[name]['ms_iterations_total']:.1f} ms, wall {wall:.2f} s")
    return out


def learned_suite(a):
    """The learned form over seeded exemplars at the 256^2 -> 512^2 workload's
    finest level; one JSON line."""
    from paper_2006_11851_amd import learned_suite as ls
    from paper_2006_11851_amd import pts, synth

    ctx = pts.Context(0)
    wl = synth.workload("ex256_out512_learned")
    seeds = list(wl.extra["exemplar_seeds"])[: a.suite_seeds]
    t0 = time.time()
    rows = ls.run(ctx, seeds, log=log, n_proposals=a.proposals, residual=a.residual)
    keys = [k for k in rows[0] if isinstance(rows[0][k], dict) and "max_gap" in rows[0][k]]
    summary = {}
    for k in keys:
        g = np.array([r[k]["max_gap"] for r in rows])
        summary[f"{k}_max_gap_mean"] = float(g.mean())
        summary[f"{k}_max_gap_max"] = float(g.max())
        summary[f"{k}_last_gap_mean"] = float(np.mean([r[k]["last_gap"] for r in rows]))
    print(json.dumps({
        "suite": "learned_c4", "exemplars": len(rows), "pairs_total": int(sum(r["pairs"] for r in rows)),
        "config": "exemplar 256^2, output 512^2 finest level, w=8, stride 2, PCA 64, tree b32 L2 (1024 leaves), "
                  f"MLP 64-256-256-1024, top-{a.proposals} leaves, tree leaf added below margin 0.2, re-ranked in "
                  "full D: exact top-8 of an FP32 scan ('learned') and of BF16 scans ('learned_bf16'), the 12 "
                  "smallest class minima of one BF16 pass ('learned_bf16_class')",
        **summary,
        "top_p_train_recall_mean": float(np.mean([r["top4_train_recall"] for r in rows])),
        "seconds": time.time() - t0, "per_exemplar": rows}))


def cpu_baseline(ctx, ex, init, w, s, seconds, threads=1):
    """The FP64 oracle's search (projection, tree descent, leaf scan, full-D
    winner distance) on a bounded random sample of the same queries, with the
    GPU's basis and tree.  threads=1: one process with BLAS limited to one
    thread; threads=0: one process per host core over disjoint parts of the
    sample (the oracle's loops are Python, so processes, not BLAS threads)."""
    import multiprocessing as mp

    from oracle import pca, vectors
    from tests import helpers

    g = ctx.export_index()
    t = helpers.dict_to_oracle_tree(g)
    Z = vectors.rgbs(ex)
    X = vectors.rgbs(init)
    Zm = vectors.exemplar_matrix(Z, w)
    Q = vectors.query_matrix(X, w, s)
    Zp = pca.project(Zm, g["mu"], g["basis"])
    order = np.random.default_rng(0).permutation(Q.shape[0])
    global _CPU_STATE
    _CPU_STATE = (g, t, Zm, Q, Zp, order, seconds)
    ncore = os.cpu_count() or 1
    model = _cpu_model()
    if threads == 1:
        done, el = _cpu_worker((0, 1))
        return {"value": done / el, "unit": "NN queries/s", "cores": 1, "kind": "oracle", "cpu_model": model,
                "nproc": ncore,
                "sample": f"{done} random queries of the initial output image, oracle tree search (projection, "
                          f"descent, leaf scan, full-D winner distance) with the GPU-built basis and tree, FP64, one "
                          f"thread, {el:.1f} s"}
    n = ncore
    with mp.get_context("fork").Pool(n) as pool:
        parts = pool.map(_cpu_worker, [(i, n) for i in range(n)])
    done = sum(p[0] for p in parts)
    el = max(p[1] for p in parts)
    return {"value": done / el, "unit": "NN queries/s", "cores": n, "kind": "oracle", "cpu_model": model,
            "nproc": ncore,
            "sample": f"{done} random queries, the same oracle search in {n} processes (one per host core, "
                      f"BLAS one thread each), {el:.1f} s"}


_CPU_STATE = None


def _cpu_worker(arg):
    from threadpoolctl import threadpool_limits

    from oracle import pca, solve, tree

    part, nparts = arg
    g, t, Zm, Q, Zp, order, seconds = _CPU_STATE
    mine = order[part::nparts]
    with threadpool_limits(1):
        done = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < seconds and done < mine.size:
            idx = mine[done : done + 64]
            Qp = pca.project(Q[idx], g["mu"], g["basis"])
            nn, _, _, _ = tree.tree_nn(Qp, Zp, t)
            solve.winner_distance(Q[idx], Zm, nn)
            done += idx.size
        el = time.perf_counter() - t0
    return done, el


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


if __name__ == "__main__":
    main()
