"""Perspective scale map (oracle, FP64).  Test infrastructure only.

Methodology 1 (Scale Evaluation), Eqs. 1-3: for a locally planar texture
seen under slant sigma and tilt tau, with the image origin at the
bottom-left corner (the largest texels there):

  Eq. 1   S_max = 1 / cos(sigma),  S_min = cos(sigma),  S_D = S_max - S_min
  Eq. 2   Y_max = (w - 1 - w/2) sin(tau) + (h - 1 - h/2) cos(tau),
          Y_min = -Y_max,  Y_D = Y_max - Y_min
  Eq. 3   p(Y) = (p(x) - w/2) sin(tau) + (p(y) - h/2) cos(tau),
          S(p) = S_max - (p(Y) - Y_min) S_D / Y_D

for an image of width w and height h.  Readings:
* the printed Eq. 3 starts with Y_max; read as S_max (with Y_max, S would
  not even carry the units of a scale, and S(Y_min) = S_max, S(Y_max) =
  S_min hold only with S_max);
* image rows count from the top in the arrays here, so the paper's p(y) is
  h - 1 - row and p(x) the column;
* the guidance channel the search uses is weight * (S - S_min) / S_D, the
  scale normalised to [0, 1] (at zero tilt affine in the row, as the
  default guidance weight * (row + 0.5) / h is, up to an affine map); a
  flat map (sigma = 0, S_D = 0) gives a zero channel;
* tilt in [0, pi/2]: the paper mirrors the input so that the largest texel
  sits at the origin, which leaves only this quadrant;
* step 2 (resample the map to the output size) is bilinear interpolation
  with pixel centres aligned and edge coordinates clamped; step 3 is
  ``matched_corners``.
Scalar trigonometry uses the C library's (``math``), as the library's host
code does, so that both sides round the same decisions from the same inputs.
"""
from __future__ import annotations

import math

import numpy as np


def _check(sigma: float, tau: float, h: int, w: int):
    """The ranges the closed forms need: a slant in [0, pi/2) (S_max
    finite), a tilt in [0, pi/2] (the largest texel at the origin after the
    mirroring the paper assumes) and at least 3 x 3 pixels (Y_D > 0)."""
    if not (0.0 <= sigma < math.pi / 2 and 0.0 <= tau <= math.pi / 2 and h >= 3 and w >= 3):
        raise ValueError("scale map: slant in [0, pi/2), tilt in [0, pi/2], sides >= 3")


def extremes(sigma: float):
    """Eq. 1: (S_max, S_min, S_D)."""
    smax = 1.0 / math.cos(sigma)
    smin = math.cos(sigma)
    return smax, smin, smax - smin


def y_range(tau: float, h: int, w: int):
    """Eq. 2: (Y_max, Y_min, Y_D)."""
    ymax = (w - 1 - w / 2.0) * math.sin(tau) + (h - 1 - h / 2.0) * math.cos(tau)
    return ymax, -ymax, 2.0 * ymax


def projected_y(px, py, tau: float, h: int, w: int):
    """Eq. 3, first line: p(Y) of image points (paper coordinates)."""
    return (np.asarray(px, dtype=np.float64) - w / 2.0) * math.sin(tau) + (
        np.asarray(py, dtype=np.float64) - h / 2.0) * math.cos(tau)


def scale_of(pY, sigma: float, tau: float, h: int, w: int):
    """Eq. 3, second line (S_max reading)."""
    smax, _, sd = extremes(sigma)
    ymax, ymin, yd = y_range(tau, h, w)
    return smax - (np.asarray(pY, dtype=np.float64) - ymin) * sd / yd


def scale_map(sigma: float, tau: float, h: int, w: int) -> np.ndarray:
    """S for every pixel of an h x w image, array rows from the top."""
    _check(sigma, tau, h, w)
    rows, cols = np.mgrid[0:h, 0:w]
    return scale_of(projected_y(cols, h - 1 - rows, tau, h, w), sigma, tau, h, w)


def guidance(sigma: float, tau: float, h: int, w: int, weight: float = 0.5) -> np.ndarray:
    """The guidance channel: weight * (S - S_min) / S_D (zero for a flat map,
    sigma = 0, where S_D = 0)."""
    _, smin, sd = extremes(sigma)
    S = scale_map(sigma, tau, h, w)
    if sd == 0.0:
        return np.zeros_like(S)
    return weight * (S - smin) / sd


def resample(S: np.ndarray, H: int, W: int) -> np.ndarray:
    """Section 4, step 2: the map resized to H x W by bilinear
    interpolation (reading: output pixel (r, c) samples the source at
    ((r + 0.5) h / H - 0.5, (c + 0.5) w / W - 0.5), coordinates clamped to
    the source's edge pixels), one axis after the other."""
    S = np.asarray(S, dtype=np.float64)

    def axis(a: np.ndarray, n_out: int, ax: int) -> np.ndarray:
        n = a.shape[ax]
        t = np.clip((np.arange(n_out) + 0.5) * n / n_out - 0.5, 0.0, n - 1)
        i0 = np.floor(t).astype(np.int64)
        i1 = np.minimum(i0 + 1, n - 1)
        f = t - i0
        lo, hi = np.take(a, i0, axis=ax), np.take(a, i1, axis=ax)
        f = f[:, None] if ax == 0 else f[None, :]
        return (1.0 - f) * lo + f * hi

    return axis(axis(S, H, 0), W, 1)


def output_guidance(sigma: float, tau: float, h: int, w: int, H: int, W: int,
                    weight: float = 0.5) -> np.ndarray:
    """The guidance channel of an H x W output: the h x w exemplar's
    normalised scale map resampled to the output size (steps 1-2)."""
    return resample(guidance(sigma, tau, h, w, weight), H, W)


def matched_corners(tau: float, flat: bool, h: int, w: int, H: int, W: int, t: int,
                    rnd: np.ndarray) -> np.ndarray:
    """Section 4, step 3: the exemplar window (corner (u, v), t x t pixels,
    centre (u + t/2, v + t/2)) copied to each t x t tile of an H x W output.

    Reading: the tile's target scale is that of its nominal centre pixel
    (ti t + t/2, tj t + t/2) on the resampled map, i.e. of the exemplar
    point (Vc, Uc) that pixel samples (step 2's clamped coordinates).  Equal
    scale means equal p(Y) (S is affine and decreasing in it), so the
    candidates lie on the line through (Vc, Uc) along which
    (col) sin(tau) - (row) cos(tau) is constant.  One coordinate of the
    corner is drawn from the tile's pair of uniform 32-bit integers rnd[k]
    (column rnd[k][0] mod (w - t + 1), or row rnd[k][1] mod (h - t + 1)):
    the column when the line is closer to horizontal (cos tau >= sin tau),
    else the row; the other is the nearest to the line, rounded half up
    and clamped into the exemplar.  With a flat map (sigma = 0: every point
    has the same scale) both coordinates are drawn.  Returns int64
    [tiles][2] = (u, v), tiles in row-major order."""
    _check(0.0, tau, h, w)
    if not (1 <= t <= min(h, w) and H >= 1 and W >= 1):
        raise ValueError("matched init: tile side in 1..min(h, w)")
    nty, ntx = -(-H // t), -(-W // t)
    rnd = np.asarray(rnd, dtype=np.uint64).reshape(nty * ntx, 2)
    nu, nv = w - t + 1, h - t + 1
    s, c = math.sin(tau), math.cos(tau)
    out = np.empty((nty * ntx, 2), dtype=np.int64)
    for ti in range(nty):
        Vc = min(max((ti * t + t / 2.0 + 0.5) * h / H - 0.5, 0.0), h - 1.0)
        for tj in range(ntx):
            k = ti * ntx + tj
            Uc = min(max((tj * t + t / 2.0 + 0.5) * w / W - 0.5, 0.0), w - 1.0)
            ru, rv = int(rnd[k, 0] % nu), int(rnd[k, 1] % nv)
            if flat:
                u, v = ru, rv
            elif c >= s:
                u = ru
                row = Vc + (u + t / 2.0 - Uc) * s / c  # the line's row at the centre column
                v = min(max(int(np.floor(row - t / 2.0 + 0.5)), 0), nv - 1)
            else:
                v = rv
                col = Uc + (v + t / 2.0 - Vc) * c / s
                u = min(max(int(np.floor(col - t / 2.0 + 0.5)), 0), nu - 1)
            out[k] = (u, v)
    return out


def matched_init(Z: np.ndarray, H: int, W: int, t: int, rnd: np.ndarray, sigma: float,
                 tau: float, weight: float = 0.5) -> np.ndarray:
    """Steps 1-3: the initial RGBS output.  Each t x t tile takes the colours
    of its matched exemplar window (``matched_corners``; a ragged last tile
    its top-left part) and the guidance channel of the resampled map."""
    Z = np.asarray(Z, dtype=np.float64)
    h, w = Z.shape[:2]
    _, _, sd = extremes(sigma)
    corners = matched_corners(tau, sd == 0.0, h, w, H, W, t, rnd)
    out = np.empty((H, W, 4))
    ntx = -(-W // t)
    for k, (u, v) in enumerate(corners):
        ti, tj = divmod(k, ntx)
        r0, c0 = ti * t, tj * t
        hh, ww = min(t, H - r0), min(t, W - c0)
        out[r0:r0 + hh, c0:c0 + ww, :3] = Z[v:v + hh, u:u + ww, :3]
    out[..., 3] = output_guidance(sigma, tau, h, w, H, W, weight)
    return out
