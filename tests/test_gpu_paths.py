"""GPU paths the other files do not reach: the caller allocator (PyTorch's
caching allocator, and one that refuses), non-finite inputs, the solve's
guidance channel, both projection kernels at their workload shapes, the
blend at stride 2 for both patch origins, and a free-running coarse-to-fine
solve against the oracle's."""
import numpy as np
import pytest

from oracle import exact, irls, mstep, parity, pca, solve, vectors
from tests import helpers

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def _small_case():
    ex, init, wl = helpers.workload_inputs("ex64_out128")
    return ex, init, wl.w[0], wl.stride[0]


def test_torch_allocator_serves_the_context(gpu_ctx, ptslib):
    """The library's memory comes from PyTorch's caching allocator and the
    results equal those of a context on the library's own allocator."""
    import torch

    pts = ptslib
    ex, init, w, s = _small_case()
    alloc = pts.TorchAllocator(0)
    ctx = pts.Context(0, allocator=alloc)
    ctx.set_exemplar_u8(ex, 0.5)
    ctx.build_index(w, 16, 4, 3, seed=0)
    x = ctx.rgbs_from_u8(init)
    nn, dist = ctx.estep(x, w, s, mode="tree")
    ctx.mstep(nn, dist, x, w, s)
    torch.cuda.synchronize()
    assert alloc.in_use > 0 and len(alloc.sizes) > 0
    gpu_ctx.set_exemplar_u8(ex, 0.5)
    gpu_ctx.build_index(w, 16, 4, 3, seed=0)
    x2 = gpu_ctx.rgbs_from_u8(init)
    nn2, dist2 = gpu_ctx.estep(x2, w, s, mode="tree")
    gpu_ctx.mstep(nn2, dist2, x2, w, s)
    assert np.array_equal(_np(nn), _np(nn2)) and np.array_equal(_np(x), _np(x2))
    ctx.close()
    torch.cuda.synchronize()
    assert alloc.in_use == 0  # everything handed back


def test_refusing_allocator_returns_oom_and_the_context_stays_usable(ptslib):
    import torch

    pts = ptslib
    ex, init, w, s = _small_case()
    alloc = pts.TorchAllocator(0, budget=1 << 20)
    ctx = pts.Context(0, allocator=alloc)
    ctx.set_exemplar_u8(ex, 0.5)  # fits in the budget
    with pytest.raises(pts.PtsError) as e:
        ctx.build_index(w, 16, 4, 3, seed=0)  # needs more than the budget
    assert e.value.code == pts.PTS_ERR_OOM and alloc.refused > 0
    with pytest.raises(pts.PtsError) as e:
        ctx.estep(torch.zeros((128, 128, 4), device="cuda"), w, s, mode="tree")  # no index was kept
    assert e.value.code == pts.PTS_ERR_STATE
    alloc.budget = None
    ctx.build_index(w, 16, 4, 3, seed=0)
    x = ctx.rgbs_from_u8(init)
    nn, dist = ctx.estep(x, w, s, mode="tree")
    assert (_np(nn) >= 0).all() and np.isfinite(_np(dist)).all()


def test_non_finite_inputs_are_refused(gpu_ctx, ptslib):
    import torch

    pts = ptslib
    ex, init, w, s = _small_case()
    gpu_ctx.set_exemplar_u8(ex, 0.5)
    x = gpu_ctx.rgbs_from_u8(init)
    bad = x.clone()
    bad[40, 17, 1] = float("nan")
    with pytest.raises(pts.PtsError) as e:
        gpu_ctx.estep(bad, w, s, mode="exact_full", stats=True)
    assert e.value.code == pts.PTS_ERR_ARG
    z = gpu_ctx.rgbs_from_u8(ex)
    z[3, 3, 0] = float("inf")
    with pytest.raises(pts.PtsError) as e:
        gpu_ctx.set_exemplar(z)
    assert e.value.code == pts.PTS_ERR_ARG
    with pytest.raises(pts.PtsError) as e:
        gpu_ctx.solve(bad, [dict(w=w, stride=s, iters=1)], mode="exact_full", coarse_mode="exact_full")
    assert e.value.code == pts.PTS_ERR_ARG
    # the previous exemplar is still in place and the context works
    nn, dist, st = gpu_ctx.estep(x, w, s, mode="exact_full", stats=True)
    Q, Zm = helpers.query_and_exemplar(vectors.rgbs(init), vectors.rgbs(ex), w, s)
    ok, _, _ = parity.nn_agreement(Q, Zm, _np(nn), exact.exact_nn(Q, Zm)[0])
    assert ok >= 0.999
    torch.cuda.synchronize()


def test_solve_guidance_weight_other_than_the_exemplars(gpu_ctx):
    """Every pyramid level, the finest included, carries the solve's guidance
    weight; a negative weight keeps the exemplar's own guidance channel (blurred
    for the coarser levels like the colours)."""
    ex, init, wl = helpers.workload_inputs("ex256_out512")
    gpu_ctx.set_exemplar_u8(ex, 0.5)
    L = 3
    for gw in (0.25, 0.5):
        for l in range(L):
            z = _np(gpu_ctx.pyramid_level(L, l, gw))
            h = z.shape[0]
            s_ref = gw * (np.arange(h) + 0.5) / h
            assert np.abs(z[..., 3] - s_ref[:, None]).max() <= 1e-6, (gw, l)
    # carried: the finest level is the exemplar's channel, a coarser one its blur
    Z = vectors.rgbs(ex, 0.5)
    fin = _np(gpu_ctx.pyramid_level(L, L - 1, -1.0))
    assert np.abs(fin - Z.astype(np.float32)).max() <= 1e-6
    pyr_o = solve.exemplar_pyramid(np.concatenate([Z[..., :3], Z[..., 3:]], axis=2), L, 0.5)
    coarse = _np(gpu_ctx.pyramid_level(L, 0, -1.0))
    blurred = solve.blur_decimate(solve.blur_decimate(Z[..., 3:4].repeat(3, axis=2)))[..., 0]
    assert np.abs(coarse[..., 3] - blurred).max() <= 1e-5
    assert np.abs(coarse[..., :3] - pyr_o[0][..., :3]).max() <= 1e-5


def test_projection_kernels_at_their_workload_shapes(gpu_ctx):
    """The resident-basis projection (windows up to 8x8; d = 64 as in the
    learned workload) and the streamed-basis MFMA projection (16x16 windows,
    D = 1024, d = 64) against the oracle's FP64 projection with the GPU's
    basis, on sampled windows."""
    for name, d, b, L in (("ex256_out512_learned", 64, 32, 2), ("ex512_out1024_w16", 64, 8, 3)):
        ex, init, wl = helpers.workload_inputs(name)
        w, s = wl.w[-1], wl.stride[-1]
        print(f"case: projection {name} w={w} d={d}", flush=True)
        gpu_ctx.set_exemplar_u8(ex, 0.5)
        gpu_ctx.build_index(w, d, b, L, seed=0, make_bf16=False)
        g = gpu_ctx.export_index()
        H = wl.out_size
        from paper_2006_11851_amd import synth

        init_f, _ = synth.row_matched_init(wl.init_seed, ex, H, H, w)
        x = gpu_ctx.rgbs_from_u8(init_f)
        qp = _np(gpu_ctx.project(x, s)).astype(np.float64)
        X = vectors.rgbs(init_f)
        u, v = vectors.output_grid(H, H, w, s)
        sample = np.sort(np.random.default_rng(3).choice(u.size, 2048, replace=False))
        Q = np.stack([vectors.window(X, int(u[i]), int(v[i]), w, True) for i in sample])
        ref = pca.project(Q, g["mu"], g["basis"])
        scale = np.maximum(1.0, np.abs(ref).max(axis=1, keepdims=True))
        err = (np.abs(qp[sample] - ref) / scale).max()
        print(f"  max scaled error {err:.2e}", flush=True)
        assert err <= 1e-4, err
        # the exemplar side: every window, against the same FP64 projection
        zp = _np(gpu_ctx.exemplar_projection()).astype(np.float64)
        Zm = vectors.exemplar_matrix(vectors.rgbs(ex), w)
        zs = np.sort(np.random.default_rng(4).choice(Zm.shape[0], 2048, replace=False))
        zref = pca.project(Zm[zs], g["mu"], g["basis"])
        zscale = np.maximum(1.0, np.abs(zref).max(axis=1, keepdims=True))
        assert (np.abs(zp[zs] - zref) / zscale).max() <= 1e-4


@pytest.mark.parametrize("o", [0, 1])
def test_mstep_stride2_both_patch_origins(gpu_ctx, o):
    """The blend at the learned workload's finest level (w = 8, s = 2: 16
    windows cover a patch at o = 0, 9 wholly contain one at o = 1, the
    paper's count), teacher-forced with the GPU's tree matches, against the
    oracle's blend over the whole 512^2 image."""
    import torch

    ex, _, wl = helpers.workload_inputs("ex256_out512")
    from paper_2006_11851_amd import synth

    w, s, H = 8, 2, 512
    init, _ = synth.row_matched_init(0, ex, H, H, w)
    gpu_ctx.set_exemplar_u8(ex, 0.5)
    gpu_ctx.build_index(w, 24, 8, 3, seed=0)
    x = gpu_ctx.rgbs_from_u8(init)
    nn, dist = gpu_ctx.estep(x, w, s, mode="tree")
    X = vectors.rgbs(init)
    Z = vectors.rgbs(ex)
    Xo, den = mstep.mstep(X, Z, _np(nn).astype(np.int64), irls.weights(_np(dist).astype(np.float64)), w, s, o)
    gpu_ctx.mstep(nn, dist, x, w, s, 0.8, 1e-3, o)
    err = np.abs(_np(x) - Xo).max()
    print(f"case: mstep w=8 s=2 o={o}: max pixel difference {err:.2e}", flush=True)
    assert err <= 1e-3, err
    pc, _ = mstep.covering_counts(64, 64, w, s, o)
    assert pc[8:56, 8:56].max() == (16 if o == 0 else 9)
    torch.cuda.synchronize()


def test_free_running_multiscale_solve_against_the_oracle(gpu_ctx):
    """A three-level solve (256^2 -> 512^2 workload: windows 32/16/8, strides
    8/4/2), exhaustive search at every level, run free on both sides from the
    same initial output: the energy trajectories of every level agree.  The
    first search of the coarsest level sees identical inputs (1e-5, the
    energy tolerance); afterwards FP32 near-ties between matches may
    resolve differently and each level inherits its predecessor's image, so
    the trajectories are held to 2e-3 relative, and each decreases."""
    ex, init, wl = helpers.workload_inputs("ex256_out512")
    iters = [4, 4, 2]
    levels = [dict(w=w, stride=s, iters=t) for w, s, t in zip(wl.w, wl.stride, iters)]
    print("case: free-running 3-level exact solve ex256_out512", flush=True)
    gpu_ctx.set_exemplar_u8(ex, 0.5)
    x0 = gpu_ctx.rgbs_from_u8(init)
    out, tr = gpu_ctx.solve(x0, levels, mode="exact_full", coarse_mode="exact_full")
    _, otr = solve.multiscale(vectors.rgbs(ex), vectors.rgbs(init), list(wl.w), list(wl.stride), iters,
                              mode="exact")
    E, Eo = np.asarray(tr["E"]), np.asarray(otr.E)
    lv, lvo = np.asarray(tr["level"]), np.asarray(otr.level)
    assert np.array_equal(lv, lvo)
    print("GPU   ", ["%.6g" % v for v in E], flush=True)
    print("oracle", ["%.6g" % v for v in Eo], flush=True)
    assert helpers.rel(E[0], Eo[0]) <= 1e-5
    assert np.all(np.abs(E - Eo) <= 2e-3 * np.abs(Eo)), (E, Eo)
    for l in range(3):
        e = E[lv == l]
        assert np.all(np.diff(e) <= 1e-5 * e[:-1]), (l, e)
