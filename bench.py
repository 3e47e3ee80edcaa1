"""Benchmark: NN queries/s and ms/iteration, BF16 + learned proposal against
the plain FP32 tree search, at the finest level of a synthetic workload.

One step = one iteration over the whole output image: E-step (projection,
search, winner distance) + M-step (2x2 patch blend) + energy, with inputs
resident in HBM.  Both forms run from the same output image; the energy gap
of each to exhaustive full-dimension search is measured on a fixed random
1/16 of the queries before and after the timed steps.  Prints one JSON line.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
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
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--train-iters", type=int, default=6)
    ap.add_argument("--train-per-iter", type=int, default=65536)
    ap.add_argument("--epochs", type=float, default=6.0)
    ap.add_argument("--residual", type=int, default=1)
    ap.add_argument("--rerank-full", type=int, default=1)
    ap.add_argument("--only", default="", help="run one form only (tree or learned_bf16)")
    ap.add_argument("--suite", default="", help="learned_c4: the learned form over the 16 seeded 256^2 exemplars")
    ap.add_argument("--suite-seeds", type=int, default=16)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-MiB tensor 3 times (the HBM-counter scale for rocprofv3 --pmc) and exit")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU: --gpus must be 1", "n_gpus": a.gpus}))
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

    from paper_2006_11851_amd import pts, synth, training

    if a.suite == "learned_c4":
        return learned_suite(a)
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

    # learned proposal: pairs from the plain method, labelled by exhaustive search
    t0 = time.time()
    q, lab = training.collect_pairs_sampled(ctx, x0, w, s, a.train_iters, min(a.train_per_iter, nq), seed=1)
    ctx.mlp_init(info.d, 256, info.n_leaves, seed=0)
    losses = training.train(ctx, q, lab, epochs=a.epochs, batch=4096, lr=2e-3, log_every=50)
    train_s = time.time() - t0
    leaves_hit = None
    prop, _ = ctx.mlp_propose(q, 4)
    leaves_hit = float((prop == lab[:, None]).any(dim=1).float().mean())
    log(f"MLP: {q.shape[0]} pairs, loss {losses[0]:.3f} -> {losses[-1]:.3f}, top-4 train recall {leaves_hit:.3f}, "
        f"{train_s:.1f} s")

    sample = torch.randperm(nq, generator=torch.Generator().manual_seed(16))[: nq // 16].to(torch.int32).cuda()

    def gap(x, nn_dist):
        _, d_ex = ctx.exact_search(x, w, s, sample)
        d_m = nn_dist[sample.long()].contiguous()
        return ctx.energy(d_m)[0] / ctx.energy(d_ex)[0] - 1.0

    forms = {
        "plain_fp32_tree": dict(mode="tree"),
        "bf16_learned": dict(mode="learned_bf16", residual=a.residual, rerank_full=a.rerank_full, n_proposals=4,
                             margin=0.2),
    }
    if a.only:
        forms = {k: v for k, v in forms.items() if v["mode"] == a.only}
    res = {}
    for name, kw in forms.items():
        x = x0.clone()
        nn = torch.empty(nq, dtype=torch.int32, device="cuda")
        dist = torch.empty(nq, dtype=torch.float32, device="cuda")
        ctx.estep(x, w, s, nn=nn, dist=dist, **kw)
        g0 = gap(x, dist)

        # every step records its energy on the device; they are read after the
        # timed region, so the steps are not serialised by host round trips
        Edev = torch.zeros((max(a.steps, a.warmup), 2), dtype=torch.float32, device="cuda")

        def step(i):
            ctx.estep(x, w, s, nn=nn, dist=dist, **kw)
            ctx.mstep(nn, dist, x, w, s)
            ctx.energy_device(dist, Edev[i])

        for i in range(a.warmup):
            step(i)
        torch.cuda.synchronize()
        ctx.profile_enable(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(a.steps):
            step(i)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        E = Edev[: a.steps].double().cpu().tolist()
        prof = ctx.profile_read()
        ctx.profile_enable(False)
        _, _, st = ctx.estep(x, w, s, nn=nn, dist=dist, stats=True, **kw)
        g1 = gap(x, dist)
        res[name] = dict(value=nq * a.steps / el, ms_per_step=1000 * el / a.steps, gap_first=g0, gap_last=g1,
                         fallback_rate=st.fallbacks / nq, energy_last=E[-1][0],
                         kernels_ms_per_step={k: v[0] / a.steps for k, v in prof.items()},
                         launches={k: v[1] for k, v in prof.items()}, x=x)
        log(f"{name}: {res[name]['value']:.3e} q/s, {res[name]['ms_per_step']:.3f} ms/step, gap {g0:.4f} -> {g1:.4f}")

    head = res.get("bf16_learned") or res["plain_fp32_tree"]
    kern = head["kernels_ms_per_step"]
    roof = roofline(ctx, head, info, nq, a, forms)
    # the next kernels by time, for context
    ranked = sorted(kern, key=lambda k: -kern[k])
    roof_next = [roofline(ctx, head, info, nq, a, forms, dom=k) for k in ranked[1:3]]
    cpu = None if a.no_cpu else cpu_baseline(ctx, ex, init, w, s, a.cpu_seconds)
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
        "dtype": "bf16" if "bf16_learned" in res else "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{a.workload} finest level: exemplar {wl.ex_size}^2, output {Hout}^2, w={w}, stride={s}, "
                        f"N={info.N}, nq={nq}, PCA {info.d}, k-means tree b{wl.branching} L{wl.depth} "
                        f"({info.n_leaves} leaves)",
            "form": "BF16 MFMA leaf scans of the MLP's top-4 leaves (plus the tree's leaf below margin 0.2), "
                    "8 class-minimum candidates, FP32 re-rank"
                    + (" in full D" if a.rerank_full else " in PCA space")
                    + (", residual-energy ranking" if a.residual else ""),
        },
        "forms": {k: {kk: vv for kk, vv in v.items() if kk != "x"} for k, v in res.items()},
        "speedup_vs_plain_fp32": (res["bf16_learned"]["value"] / res["plain_fp32_tree"]["value"])
        if len(res) == 2 else None,
        "index_build_s": build_s,
        "mlp_training_s": train_s,
        "mlp_pairs": int(q.shape[0]),
        "mlp_top4_train_recall": leaves_hit,
        "roofline": roof,
        "roofline_next": roof_next,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def learned_suite(a):
    """The learned form (FP32 scan of the proposed leaves) over seeded
    exemplars at the 256^2 -> 512^2 workload's finest level; one JSON line."""
    from paper_2006_11851_amd import learned_suite as ls
    from paper_2006_11851_amd import pts, synth

    ctx = pts.Context(0)
    wl = synth.workload("ex256_out512_learned")
    seeds = list(wl.extra["exemplar_seeds"])[: a.suite_seeds]
    t0 = time.time()
    rows = ls.run(ctx, seeds, log=log)
    lg = np.array([r["learned"]["max_gap"] for r in rows])
    ll = np.array([r["learned"]["last_gap"] for r in rows])
    bg = np.array([r["learned_bf16"]["max_gap"] for r in rows])
    bl = np.array([r["learned_bf16"]["last_gap"] for r in rows])
    tg = np.array([r["tree"]["max_gap"] for r in rows])
    print(json.dumps({
        "suite": "learned_c4", "exemplars": len(rows), "pairs_total": int(sum(r["pairs"] for r in rows)),
        "config": "exemplar 256^2, output 512^2 finest level, w=8, stride 2, PCA 64, tree b32 L2 (1024 leaves), "
                  "MLP 64-256-256-1024, top-4 leaves scanned in FP32, tree leaf added below margin 0.2",
        "learned_max_gap_mean": float(lg.mean()), "learned_max_gap_max": float(lg.max()),
        "learned_last_gap_mean": float(ll.mean()), "learned_last_gap_max": float(ll.max()),
        "learned_bf16_full_rerank_max_gap_mean": float(bg.mean()), "learned_bf16_full_rerank_max_gap_max": float(bg.max()),
        "learned_bf16_full_rerank_last_gap_mean": float(bl.mean()),
        "tree_max_gap_mean": float(tg.mean()),
        "fallback_rate_mean": float(np.mean([r["learned"]["fallback_rate"] for r in rows])),
        "top4_train_recall_mean": float(np.mean([r["top4_train_recall"] for r in rows])),
        "seconds": time.time() - t0, "per_exemplar": rows}))


def roofline(ctx, head, info, nq, a, forms, dom=None):
    """Dominant kernel of the reported form (or kernel `dom`) against its bound."""
    kern = head["kernels_ms_per_step"]
    launches = head["launches"]
    if dom is None:
        dom = max(kern, key=lambda k: kern[k])
    per_launch_ms = kern[dom] * a.steps / max(1, launches[dom])
    d, h, L = info.d, 256, info.n_leaves
    dk = -(-d // 32) * 32
    K1 = -(-d // 32) * 32
    if dom == "mlp_propose_mfma":
        # both hidden layers and the output layer (counted once; its two passes run it twice)
        flops = 2.0 * (K1 * h + h * h + h * (-(-L // 32) * 32)) * nq
        bound, peak, unit = "mfma", PEAK["bf16"], "TFLOP/s"
    elif dom == "leaf_scan_bf16":
        flops = 2.0 * dk * scanned_pairs(ctx, head, info, nq)
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
            "traffic": measured_traffic(dom), "ms_per_launch": per_launch_ms, "algorithmic_flops_per_launch": flops}


def measured_traffic(label):
    """HBM bytes per full-size launch of the kernel behind `label`, from the
    committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary (scaled by the copy
    calibration), or None when there is none or the kernel's source file has
    changed since the counters were taken."""
    import glob
    import hashlib

    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*.md"))):
        for line in open(path):
            f = line.split()
            if len(f) == 5 and f[0] == "traffic:" and f[1] == label:
                src = os.path.join(ROOT, "paper_2006_11851_amd", "csrc", f[3])
                if not os.path.exists(src):
                    return None
                digest = hashlib.sha1(open(src, "rb").read()).hexdigest()[:12]
                return float(f[2]) if digest == f[4] else None
    return None


def scanned_pairs(ctx, head, info, nq):
    """(query, exemplar) pairs the learned BF16 scan visits for the final image."""
    import torch

    x = head["x"]
    g = ctx.export_index()
    sizes = torch.from_numpy(np.diff(g["leaf_off"])).cuda()
    qp = ctx.project(x, 2)
    prop, margin = ctx.mlp_propose(qp, 4)
    dleaf = ctx.descend(qp)
    fb = ~(margin >= 0.2)
    dup = (prop == dleaf[:, None]).any(dim=1)
    tot = sizes[prop.long()].sum(dim=1) + torch.where(fb & ~dup, sizes[dleaf.long()], torch.zeros_like(dleaf))
    return float(tot.sum())


def cpu_baseline(ctx, ex, init, w, s, seconds):
    """The FP64 oracle's search (projection, tree descent, leaf scan, full-D
    winner distance) on a bounded random sample of the same queries, with the
    GPU's basis and tree, BLAS limited to one thread."""
    from threadpoolctl import threadpool_limits

    from oracle import pca, solve, tree, vectors
    from tests import helpers

    g = ctx.export_index()
    t = helpers.dict_to_oracle_tree(g)
    Z = vectors.rgbs(ex)
    X = vectors.rgbs(init)
    Zm = vectors.exemplar_matrix(Z, w)
    Q = vectors.query_matrix(X, w, s)
    with threadpool_limits(1):
        Zp = pca.project(Zm, g["mu"], g["basis"])
        order = np.random.default_rng(0).permutation(Q.shape[0])
        done = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < seconds and done < Q.shape[0]:
            idx = order[done : done + 64]
            Qp = pca.project(Q[idx], g["mu"], g["basis"])
            nn, _, _, _ = tree.tree_nn(Qp, Zp, t)
            solve.winner_distance(Q[idx], Zm, nn)
            done += idx.size
        el = time.perf_counter() - t0
    return {"value": done / el, "unit": "NN queries/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} random queries of the initial output image, oracle tree search (projection, descent, "
                      f"leaf scan, full-D winner distance) with the GPU-built basis and tree, FP64, one thread, "
                      f"{el:.1f} s"}


if __name__ == "__main__":
    main()
