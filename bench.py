"""Benchmark: NN queries/s and ms/iteration of the search + blend hot path.

One step = one iteration at the finest level: E-step (projection, search,
winner distance) + M-step (2x2 patch blend) + energy, over the whole output
image, inputs resident in HBM.  Prints one JSON line.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--form FORM]
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

PEAKS = {  # MI355X published peaks
    "hbm_gbs": 8000.0,
    "bf16_tflops": 2500.0,
    "fp32_vector_tflops": 157.3,
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="ex256_out512")
    ap.add_argument("--form", default="tree", choices=["tree", "exact_pca", "brute_bf16", "learned", "learned_bf16"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    return ap.parse_args()


def kernel_algorithmic(form, name, nq, N, d, D, leaf_mean, w, H, W):
    """(bound, algorithmic units per launch, unit) for the kernels we report."""
    if name == "leaf_scan_f32":
        # 3 flops (sub, mul, add) per (query, member, dimension)
        return "alu", 3.0 * nq * leaf_mean * d, "TFLOP/s"
    if name == "mstep_patch2x2":
        # per pixel: (w/s)^2 covering windows x 16 B gathered + 16 B read/written;
        # per window: 8 B of (id, distance)
        return "hbm", None, "GB/s"
    return None, None, None


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1", "n_gpus": a.gpus}))
        sys.exit(2)
    import torch

    from paper_2006_11851_amd import pts, synth

    wl = synth.workload(a.workload)
    ex = wl.exemplar()
    w, s = wl.w[-1], wl.stride[-1]
    Hout = wl.out_size
    ctx = pts.Context(0)
    ctx.set_exemplar_u8(ex, 0.5)
    t0 = time.time()
    info = ctx.build_index(w, wl.pca_dims, wl.branching, wl.depth, seed=0, make_bf16=True)
    build_s = time.time() - t0
    init, _ = synth.row_matched_init(wl.init_seed, ex, Hout, Hout, w)
    x0 = ctx.rgbs_from_u8(init, 0.5)
    x = x0.clone()
    nq = ctx.nq(Hout, Hout, w, s)
    nn = torch.empty(nq, dtype=torch.int32, device="cuda")
    dist = torch.empty(nq, dtype=torch.float32, device="cuda")

    def step():
        ctx.estep(x, w, s, mode=a.form, nn=nn, dist=dist)
        ctx.mstep(nn, dist, x, w, s)
        return ctx.energy(dist)

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    energies = []
    for _ in range(a.steps):
        energies.append(step())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    ms_per_step = 1000.0 * elapsed / a.steps
    value = nq / (elapsed / a.steps)

    # dominant kernel and its roofline
    kern = {k: v for k, v in prof.items()}
    dom = max(kern, key=lambda k: kern[k][0])
    dom_ms = kern[dom][0] / max(1, kern[dom][1])
    roof = None
    leaf_mean = info.leaf_mean
    if dom == "leaf_scan_f32":
        flops = 3.0 * nq * leaf_mean * info.d
        ach = flops / (dom_ms * 1e-3) / 1e12
        roof = {"kernel": dom, "bound": "alu", "achieved": ach, "peak": PEAKS["fp32_vector_tflops"],
                "unit": "TFLOP/s", "frac": ach / PEAKS["fp32_vector_tflops"], "traffic": None}
    elif dom == "mstep_patch2x2":
        cover = (w // s) ** 2
        byts = Hout * Hout * (cover * 16 + 32) + (Hout * Hout / 4) * cover * 8
        ach = byts / (dom_ms * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": PEAKS["hbm_gbs"], "unit": "GB/s",
                "frac": ach / PEAKS["hbm_gbs"], "traffic": None}
    else:
        roof = {"kernel": dom, "bound": None, "achieved": None, "peak": None, "unit": None, "frac": None,
                "traffic": None}

    cpu = None
    if not a.no_cpu:
        cpu = cpu_baseline(ctx, ex, init, w, s, a.cpu_seconds)

    out = {
        "metric": "NN queries/s + ms/iteration",
        "value": value,
        "unit": "NN queries/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{a.workload} finest level: exemplar {wl.ex_size}^2, output {Hout}^2, "
                               f"w={w}, stride={s}, N={info.N}, nq={nq}, d={info.d}, "
                               f"tree b{wl.branching} L{wl.depth}", "form": a.form},
        "kernels_ms_per_step": {k: v[0] / a.steps for k, v in kern.items()},
        "energy_last": energies[-1][0],
        "index_build_s": build_s,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def cpu_baseline(ctx, ex, init, w, s, seconds):
    """The FP64 oracle's search (PCA projection, tree descent, leaf scan,
    winner distance) timed on a bounded sample of the same queries, with the
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
        r = np.random.default_rng(0)
        order = r.permutation(Q.shape[0])
        done = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < seconds and done < Q.shape[0]:
            idx = order[done : done + 256]
            Qp = pca.project(Q[idx], g["mu"], g["basis"])
            nn, _, _, _ = tree.tree_nn(Qp, Zp, t)
            solve.winner_distance(Q[idx], Zm, nn)
            done += idx.size
        el = time.perf_counter() - t0
    return {"value": done / el, "unit": "NN queries/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} random queries of the same image, oracle tree search (projection, descent, "
                      f"leaf scan, full-D winner distance) with the GPU-built basis and tree, FP64, "
                      f"{el:.1f} s"}


if __name__ == "__main__":
    main()
