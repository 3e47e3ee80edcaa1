"""The perspective scale map (Methodology 1, Eqs. 1-3) and the scale-matched
initialisation (Section 4, steps 1-3) on the GPU against the oracle: the
guidance channel at the exemplar's size and resampled to other sizes, the
init's tile choices bit for bit, and free-running two-level solves guided
by the map from that init."""
import math

import numpy as np
import pytest

from oracle import scale, solve, vectors
from tests import helpers

pytestmark = pytest.mark.gpu

ANGLES = [(30, 18), (60, 60), (45, 0), (20, 90), (0, 30), (75, 44), (10, 46)]


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("sig,tau", ANGLES)
def test_scale_guidance_against_the_oracle(gpu_ctx, sig, tau):
    import torch

    s, t = math.radians(sig), math.radians(tau)
    for (H, W), ref in (((105, 105), None), ((64, 48), None), ((210, 131), (105, 105)), ((40, 70), (96, 128))):
        x = torch.zeros((H, W, 4), device="cuda")
        gpu_ctx.scale_guidance(x, s, t, 0.5, ref)
        rh, rw = (H, W) if ref is None else ref
        want = scale.output_guidance(s, t, rh, rw, H, W, 0.5)
        got = _np(x)
        err = np.abs(got[..., 3] - want).max()
        print(f"case: scale guidance sigma={sig} tau={tau} {H}x{W} ref={ref}: {err:.2e}", flush=True)
        assert err <= 1e-6, err
        assert np.all(got[..., :3] == 0.0)


def test_scale_map_ranges_are_refused(gpu_ctx, ptslib):
    import torch

    pts = ptslib
    x = torch.zeros((16, 16, 4), device="cuda")
    for slant, tilt, ref in ((math.pi / 2, 0.1, None), (0.3, -0.01, None), (0.3, 1.6, None), (0.3, 0.2, (2, 16)),
                             (float("nan"), 0.2, None)):
        with pytest.raises(pts.PtsError) as e:
            gpu_ctx.scale_guidance(x, slant, tilt, 0.5, ref)
        assert e.value.code == pts.PTS_ERR_ARG
    ex = torch.zeros((8, 8, 4), device="cuda")
    rnd = torch.zeros((2, 2), dtype=torch.int32, device="cuda")
    with pytest.raises(pts.PtsError) as e:
        gpu_ctx.scale_init(ex, 16, 8, 9, rnd, 0.3, 0.2)  # tile larger than the exemplar
    assert e.value.code == pts.PTS_ERR_ARG
    torch.cuda.synchronize()


@pytest.mark.parametrize("sig,tau", ANGLES)
def test_scale_matched_init_against_the_oracle(gpu_ctx, sig, tau):
    """Every tile copies the oracle's window (bit-exact colours: the corner
    is the same FP64 rounding decision on both sides) and the guidance is
    the resampled map; output sides that leave ragged tiles included."""
    import torch

    from paper_2006_11851_amd import synth

    s, t = math.radians(sig), math.radians(tau)
    ex, _, _ = helpers.workload_inputs("ex256_out512")
    Z = vectors.rgbs(ex).astype(np.float32)
    for (hz, wz), (H, W), tile in (((256, 256), (512, 512), 32), ((64, 64), (128, 128), 8),
                                  ((256, 256), (300, 212), 16), ((64, 48), (37, 90), 8)):
        Zs = np.ascontiguousarray(Z[:hz, :wz])
        rnd = synth.tile_draws(sig * 100 + tau, H, W, tile)
        x = gpu_ctx.scale_init(torch.from_numpy(Zs).cuda(), H, W, tile,
                               torch.from_numpy(rnd.view(np.int32)).cuda(), s, t, 0.5)
        want = scale.matched_init(Zs.astype(np.float64), H, W, tile, rnd, s, t, 0.5)
        got = _np(x)
        bad = np.argwhere(np.any(got[..., :3] != want[..., :3], axis=2))
        print(f"case: scale init sigma={sig} tau={tau} ex {hz}x{wz} out {H}x{W} tile {tile}: "
              f"{len(bad)} pixels differ", flush=True)
        assert len(bad) == 0, bad[:5]
        assert np.abs(got[..., 3] - want[..., 3]).max() <= 1e-6


@pytest.mark.parametrize("sig,tau", [(30, 18), (50, 70)])
def test_solve_guided_by_the_scale_map_against_the_oracle(gpu_ctx, sig, tau):
    """Steps 1-4 end to end: the scale-matched init at the coarsest level,
    then a free-running two-level exhaustive solve whose every level is
    guided by the map (each exemplar level its own, each output the
    resample), against the oracle's solve from its own init: first energy
    at 1e-5, trajectories at 2e-3 (FP32 near-ties may resolve differently
    once the images diverge), energy non-increasing per level."""
    import torch

    from paper_2006_11851_amd import synth

    s, t = math.radians(sig), math.radians(tau)
    ex, _, _ = helpers.workload_inputs("ex64_out128")
    L, ws, ss, iters = 2, [8, 8], [4, 4], [3, 2]
    gpu_ctx.set_exemplar_u8(ex, 0.5)
    Z = vectors.rgbs(ex)
    pyr_o = solve.exemplar_pyramid(Z, L, 0.5, (s, t))
    H0 = 128 >> (L - 1)
    rnd = synth.tile_draws(7, H0, H0, ws[0])
    z0 = gpu_ctx.pyramid_level(L, 0, 0.5)
    x0 = gpu_ctx.scale_init(z0, H0, H0, ws[0], torch.from_numpy(rnd.view(np.int32)).cuda(), s, t, 0.5)
    X0 = scale.matched_init(pyr_o[0], H0, H0, ws[0], rnd, s, t, 0.5)
    assert np.abs(_np(x0) - X0).max() <= 1e-5
    levels = [dict(w=w, stride=st, iters=it) for w, st, it in zip(ws, ss, iters)]
    print(f"case: scale-guided 2-level exact solve sigma={sig} tau={tau}", flush=True)
    out, tr = gpu_ctx.solve(x0, levels, mode="exact_full", coarse_mode="exact_full", scale=(s, t))
    Xo, otr = solve.multiscale(Z, X0, ws, ss, iters, mode="exact", scale=(s, t))
    E, Eo = np.asarray(tr["E"]), np.asarray(otr.E)
    lv = np.asarray(tr["level"])
    assert np.array_equal(lv, np.asarray(otr.level))
    print("GPU   ", ["%.6g" % v for v in E], flush=True)
    print("oracle", ["%.6g" % v for v in Eo], flush=True)
    assert helpers.rel(E[0], Eo[0]) <= 1e-5
    assert np.all(np.abs(E - Eo) <= 2e-3 * np.abs(Eo)), (E, Eo)
    for l in range(L):
        e = E[lv == l]
        assert np.all(np.diff(e) <= 1e-5 * e[:-1]), (l, e)
    # the result carries the finest level's output map
    want = scale.output_guidance(s, t, 64, 64, 128, 128, 0.5)
    assert np.abs(_np(out)[..., 3] - want).max() <= 1e-6
    torch.cuda.synchronize()
