"""Pins of the scale-map oracle (Methodology 1, Eqs. 1-3; Section 4 steps
1-3) against closed forms, hand-computed values and brute force."""
import math

import numpy as np
import pytest

from oracle import scale, solve


def test_eq1_extremes_closed_form():
    smax, smin, sd = scale.extremes(math.radians(60))
    assert abs(smax - 2.0) < 1e-15 and abs(smin - 0.5) < 1e-15 and abs(sd - 1.5) < 1e-15
    assert scale.extremes(0.0) == (1.0, 1.0, 0.0)


def test_eq2_range_closed_form():
    # 105 x 105 (the paper's inputs) at tilt 18 degrees: (105 - 1 - 52.5) (sin + cos)
    ymax, ymin, yd = scale.y_range(math.radians(18), 105, 105)
    want = 51.5 * (math.sin(math.radians(18)) + math.cos(math.radians(18)))
    assert abs(ymax - want) < 1e-12 and ymin == -ymax and abs(yd - 2 * want) < 1e-12


@pytest.mark.parametrize("sig,tau", [(30, 18), (60, 60), (45, 0), (20, 90)])
def test_eq3_ends_and_midpoint(sig, tau):
    """S(Y_min) = S_max, S(Y_max) = S_min (the S_max reading of Eq. 3), the
    top-right pixel (p(Y) = Y_max) holds S_min, and the image centre
    (p(Y) = 0) the mean of the extremes."""
    s, t = math.radians(sig), math.radians(tau)
    h, w = 40, 56
    smax, smin, _ = scale.extremes(s)
    ymax, ymin, _ = scale.y_range(t, h, w)
    assert abs(scale.scale_of(ymin, s, t, h, w) - smax) < 1e-12
    assert abs(scale.scale_of(ymax, s, t, h, w) - smin) < 1e-12
    S = scale.scale_map(s, t, h, w)
    assert abs(S[0, w - 1] - smin) < 1e-12
    # paper point (w/2, h/2) is array row h - 1 - h/2, column w/2
    assert abs(S[h - 1 - h // 2, w // 2] - 0.5 * (smax + smin)) < 1e-12


def test_eq3_gradient_follows_the_tilt():
    """One column right lowers S by sin(tau) S_D / Y_D; one row down (one
    step towards the origin) raises it by cos(tau) S_D / Y_D."""
    s, t = math.radians(30), math.radians(18)
    h, w = 105, 105
    _, _, sd = scale.extremes(s)
    _, _, yd = scale.y_range(t, h, w)
    S = scale.scale_map(s, t, h, w)
    assert np.allclose(S[:, :-1] - S[:, 1:], math.sin(t) * sd / yd, atol=1e-13, rtol=0)
    assert np.allclose(S[1:, :] - S[:-1, :], math.cos(t) * sd / yd, atol=1e-13, rtol=0)
    assert S[-1, 0] == S.max() and S[0, -1] == S.min()  # largest at the origin, smallest top right


def test_zero_tilt_is_the_row_guidance_up_to_an_affine_map():
    """At tau = 0 the normalised map is row / (h - 2): constant along a row
    and affine in the row guidance g = (row + 0.5) / h."""
    h, w = 64, 48
    n = scale.guidance(math.radians(40), 0.0, h, w, 1.0)
    rows = np.arange(h, dtype=np.float64)[:, None]
    assert np.abs(n - rows / (h - 2)).max() < 1e-13
    g = solve.guidance(h, w, 1.0)
    assert np.abs(n - (g * h - 0.5) / (h - 2)).max() < 1e-13


def test_right_angle_tilt_depends_on_the_column_only():
    h, w = 30, 50
    n = scale.guidance(math.radians(50), math.pi / 2, h, w, 1.0)
    cols = np.arange(w, dtype=np.float64)[None, :]
    assert np.abs(n - (w - 1 - cols) / (w - 2)).max() < 1e-12


def test_flat_map_and_ranges():
    assert np.all(scale.guidance(0.0, 0.3, 20, 20, 0.5) == 0.0)
    assert np.all(scale.scale_map(0.0, 0.3, 20, 20) == 1.0)
    for bad in ((math.pi / 2, 0.1, 20, 20), (0.2, -0.1, 20, 20), (0.2, 1.6, 20, 20), (0.2, 0.1, 2, 20)):
        with pytest.raises(ValueError):
            scale.scale_map(*bad)


def test_resample_hand_values():
    """Pixel-centre bilinear resize with clamped edges, one axis at a time."""
    ramp = np.array([[0.0, 1.0, 2.0, 3.0]])
    assert np.allclose(scale.resample(ramp, 1, 2), [[0.5, 2.5]])
    assert np.allclose(scale.resample(np.array([[0.0, 1.0]]), 1, 4), [[0.0, 0.25, 0.75, 1.0]])
    col = np.array([[0.0], [2.0], [4.0]])
    assert np.allclose(scale.resample(col, 2, 1), [[0.5], [3.5]])  # rows at 0.25, 1.75
    rng = np.random.default_rng(0)
    A = rng.normal(size=(7, 9))
    assert np.array_equal(scale.resample(A, 7, 9), A)  # same size: identity
    assert np.allclose(scale.resample(np.full((5, 6), 2.5), 11, 3), 2.5)


def test_resample_of_the_affine_map_is_the_map_at_clamped_points():
    """Bilinear interpolation reproduces an affine field: the resampled map
    equals Eq. 3 evaluated at the clamped source coordinates."""
    s, t = math.radians(35), math.radians(25)
    h, w, H, W = 24, 40, 50, 33
    R = scale.resample(scale.scale_map(s, t, h, w), H, W)
    v = np.clip((np.arange(H) + 0.5) * h / H - 0.5, 0, h - 1)[:, None]
    u = np.clip((np.arange(W) + 0.5) * w / W - 0.5, 0, w - 1)[None, :]
    want = scale.scale_of(scale.projected_y(u, h - 1 - v, t, h, w), s, t, h, w)
    assert np.abs(R - want).max() < 1e-12


def _pY(row, col, tau, h, w):
    return scale.projected_y(col, h - 1 - row, tau, h, w)


@pytest.mark.parametrize("tau", [0, 10, 30, 45, 60, 80, 90])
def test_matched_corners_lie_nearest_the_iso_scale_line(tau):
    """Brute force: along the drawn coordinate, no other corner's window
    centre has a scale closer to the tile's target (equal scale = equal
    p(Y)); the drawn coordinate is the integer drawn modulo the range."""
    t_rad = math.radians(tau)
    h, w, H, W, t = 48, 40, 72, 88, 8
    rng = np.random.default_rng(tau)
    nty, ntx = -(-H // t), -(-W // t)
    rnd = rng.integers(0, 2**32, size=(nty * ntx, 2), dtype=np.uint64)
    cs = scale.matched_corners(t_rad, False, h, w, H, W, t, rnd)
    nu, nv = w - t + 1, h - t + 1
    by_col = math.cos(t_rad) >= math.sin(t_rad)
    for k, (u, v) in enumerate(cs):
        ti, tj = divmod(k, ntx)
        Vc = min(max((ti * t + t / 2 + 0.5) * h / H - 0.5, 0), h - 1)
        Uc = min(max((tj * t + t / 2 + 0.5) * w / W - 0.5, 0), w - 1)
        target = _pY(Vc, Uc, t_rad, h, w)
        if by_col:
            assert u == rnd[k, 0] % nu
            errs = np.abs(_pY(np.arange(nv) + t / 2, u + t / 2, t_rad, h, w) - target)
            assert errs[v] <= errs.min() + 1e-9, (k, v, errs.argmin())
        else:
            assert v == rnd[k, 1] % nv
            errs = np.abs(_pY(v + t / 2, np.arange(nu) + t / 2, t_rad, h, w) - target)
            assert errs[u] <= errs.min() + 1e-9, (k, u, errs.argmin())


def test_matched_corners_same_size_zero_tilt_copy_the_tile_rows():
    """Output and exemplar of one size at tau = 0: tile row ti takes the
    exemplar rows it covers (its centre's scale is exactly available)."""
    h = w = H = W = 64
    t = 8
    rnd = np.arange(2 * 64, dtype=np.uint64).reshape(64, 2) * 7919
    cs = scale.matched_corners(0.0, False, h, w, H, W, t, rnd)
    for k, (u, v) in enumerate(cs):
        assert v == (k // 8) * t and u == int(rnd[k, 0]) % (w - t + 1)


def test_flat_map_draws_both_coordinates_and_init_copies_windows():
    h, w, H, W, t = 32, 36, 40, 50, 8
    rng = np.random.default_rng(5)
    nt = (-(-H // t)) * (-(-W // t))
    rnd = rng.integers(0, 2**32, size=(nt, 2), dtype=np.uint64)
    cs = scale.matched_corners(0.4, True, h, w, H, W, t, rnd)
    assert np.array_equal(cs[:, 0], rnd[:, 0] % (w - t + 1)) and np.array_equal(cs[:, 1], rnd[:, 1] % (h - t + 1))
    Z = rng.random((h, w, 4))
    X = scale.matched_init(Z, H, W, t, rnd, math.radians(30), 0.4, 0.5)
    cs = scale.matched_corners(0.4, False, h, w, H, W, t, rnd)
    ntx = -(-W // t)
    for k, (u, v) in enumerate(cs):
        r0, c0 = (k // ntx) * t, (k % ntx) * t
        hh, ww = min(t, H - r0), min(t, W - c0)
        assert np.array_equal(X[r0:r0 + hh, c0:c0 + ww, :3], Z[v:v + hh, u:u + ww, :3])
    assert np.allclose(X[..., 3], scale.output_guidance(math.radians(30), 0.4, h, w, H, W, 0.5))
    assert np.all(scale.matched_init(Z, H, W, t, rnd, 0.0, 0.4)[..., 3] == 0.0)


def test_solve_with_the_scale_map_wires_each_level():
    """Every exemplar level carries its own size's map; every upsampled
    output the resample of the next exemplar level's map; the colours are
    upsampled as without it."""
    s, t = math.radians(30), math.radians(18)
    rng = np.random.default_rng(1)
    Z = rng.random((32, 32, 4))
    pyr = solve.exemplar_pyramid(Z, 3, 0.5, (s, t))
    for P in pyr:
        assert np.abs(P[..., 3] - scale.guidance(s, t, P.shape[0], P.shape[1], 0.5)).max() < 1e-15
    X = rng.random((12, 10, 4))
    up = solve.upsample2(X, 0.5, (s, t), (16, 16))
    assert np.abs(up[..., 3] - scale.output_guidance(s, t, 16, 16, 24, 20, 0.5)).max() < 1e-15
    assert np.array_equal(up[..., :3], solve.upsample2(X, 0.5)[..., :3])
