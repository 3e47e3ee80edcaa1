"""GPU parity of the histogram matching of Section 3 (Eq. 9: histogram-
weighted blend weights) and Section 4, step 4 (the final histogram match)
against the oracle, teacher-forced on the GPU's matches."""
import numpy as np
import pytest

from oracle import histogram, irls, mstep, vectors
from tests import helpers

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("bins", [16, 64])
def test_histogram_weights_and_blend(gpu_ctx, bins):
    """Eq. 9 weights at 1e-5 relative and the blend they drive at 1e-3, on
    an output several iterations in (blended colours, not only exemplar
    values) at the 256^2 -> 512^2 workload's finest level."""
    ex, _, wl = helpers.workload_inputs("ex256_out512")
    from paper_2006_11851_amd import synth

    w, s, H = 8, 2, 512
    init, _ = synth.row_matched_init(0, ex, H, H, w)
    gpu_ctx.set_exemplar_u8(ex, 0.5)
    gpu_ctx.build_index(w, 24, 8, 3, seed=0)
    x = gpu_ctx.rgbs_from_u8(init)
    for _ in range(2):  # move away from the initial output's exemplar colours
        nn, dist = gpu_ctx.estep(x, w, s, mode="tree")
        gpu_ctx.mstep(nn, dist, x, w, s)
    nn, dist = gpu_ctx.estep(x, w, s, mode="tree")
    X = _np(x).astype(np.float64)
    Z = vectors.rgbs(ex)
    nn_n, d_n = _np(nn).astype(np.int64), _np(dist).astype(np.float64)
    Wo = histogram.weights(irls.weights(d_n), X, Z, nn_n, w, bins)
    Wg = _np(gpu_ctx.irls_weights(nn, dist, x, w, s, hist_bins=bins)).astype(np.float64)
    rel = np.abs(Wg - Wo) / Wo
    base = irls.weights(d_n)
    print(f"bins {bins}: weights changed for {np.mean(Wo < base):.3f} of the windows, "
          f"max relative difference {rel.max():.2e}", flush=True)
    assert np.mean(Wo < base * (1 - 1e-3)) > 0.05  # the modification is not idle here
    assert rel.max() <= 1e-5, rel.max()
    Xo, _ = mstep.mstep(X, Z, nn_n, Wo, w, s, 0)
    gpu_ctx.mstep(nn, dist, x, w, s, hist_bins=bins)
    err = np.abs(_np(x) - Xo).max()
    assert err <= 1e-3, err
    # without the histograms the same call gives the plain weights
    W0 = _np(gpu_ctx.irls_weights(nn, dist, x, w, s)).astype(np.float64)
    assert np.allclose(W0, irls.weights(d_n), rtol=1e-5)


def test_final_histogram_match(gpu_ctx):
    """Rank-for-rank match of R, G, B to the exemplar's distribution: every
    value is an exemplar value, so the GPU result equals the oracle's
    exactly (ties in pixel order on both sides)."""
    import torch

    ex, _, wl = helpers.workload_inputs("ex256_out512")
    from paper_2006_11851_amd import synth

    w, s, H = 8, 2, 512
    init, _ = synth.row_matched_init(0, ex, H, H, w)
    gpu_ctx.set_exemplar_u8(ex, 0.5)
    gpu_ctx.build_index(w, 24, 8, 3, seed=0)
    x = gpu_ctx.rgbs_from_u8(init)
    nn, dist = gpu_ctx.estep(x, w, s, mode="tree")
    gpu_ctx.mstep(nn, dist, x, w, s)
    X = _np(x).astype(np.float64)
    Z = _np(gpu_ctx.rgbs_from_u8(ex)).astype(np.float64)
    gpu_ctx.histogram_match(x)
    Y = histogram.match(X, Z)
    assert np.array_equal(_np(x).astype(np.float64), Y)
    # the matched output's channel histograms are the exemplar's (4x its pixels)
    for j in range(3):
        assert np.array_equal(np.sort(Y[..., j].reshape(-1))[::4], np.sort(Z[..., j].reshape(-1)))
    torch.cuda.synchronize()


def test_solve_with_histogram_weights_and_final_match(gpu_ctx):
    """The solve runs the weighted blend at every level and ends with the
    match; its result carries the exemplar's colour distribution."""
    ex, init, wl = helpers.workload_inputs("ex64_out128")
    gpu_ctx.set_exemplar_u8(ex, 0.5)
    x0 = gpu_ctx.rgbs_from_u8(init)
    out, tr = gpu_ctx.solve(x0, [dict(w=8, stride=4, iters=3)], mode="exact_full", coarse_mode="exact_full",
                            hist_bins=16, final_hist_match=True)
    Y = _np(out).astype(np.float64)
    Z = vectors.rgbs(ex)
    for j in range(3):
        assert np.allclose(np.sort(Y[..., j].reshape(-1))[::4], np.sort(Z[..., j].reshape(-1)), atol=1e-7)
    assert np.isfinite(tr["E"]).all()
