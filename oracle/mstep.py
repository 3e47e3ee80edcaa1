"""Optimisation phase: 2x2 patch blend (oracle, FP64).  Test infra only.

Methodology 2.1: with the nearest neighbourhoods {z_p} fixed, x is the
continuous vector that minimises sum_p W_p ||x_p - z_p||^2 (Eq. 8).
Methodology 2.2: the sparse grid (interval w/4) and the 2x2 patch: all
points of a patch are processed together from the neighbourhoods that wholly
contain the patch.

For a patch P and a pixel p in P, channel c in R, G, B:

  x_new(p, c) = sum_{q in C(P)} W_q Z_c(e_q + (p - o_q)) / sum_{q in C(P)} W_q

where C(P) is the set of output windows that contain every pixel of P (with
the x wrap), o_q the window's corner and e_q the corner of its matched
exemplar window.  The guidance channel is the fixed target map and is left
unchanged; a pixel whose C(P) is empty keeps its value.

Patches are 2x2 blocks at origin (2a + o, 2b + o), ``patch_offset`` o in
{0, 1}, clipped to the image rows (with o = 1 the first and last rows form
1-pixel-high patches); columns wrap.  With o = 0 and even w and s, C(P) is
the set of windows touching P, and the update is exactly the weighted least
squares minimiser of Eq. 8 (every window pixel is covered).  With o = 1 at
w = 8, s = 2 each patch has 9 covering windows against 16 per single pixel -
the count the paper's 8x8 example gives.
"""
from __future__ import annotations

import numpy as np

from .vectors import exemplar_corner, output_grid


def patch_rows_cols(px, py, H: int, W: int, o: int):
    """Row range (lo, hi) and the two columns of the patch holding (px, py)."""
    r0 = 2 * np.floor_divide(py - o, 2) + o
    c0 = 2 * np.floor_divide(px - o, 2) + o
    lo = np.maximum(r0, 0)
    hi = np.minimum(r0 + 1, H - 1)
    return lo, hi, np.mod(c0, W), np.mod(c0 + 1, W)


def mstep(
    X: np.ndarray,
    Z: np.ndarray,
    nn: np.ndarray,
    Wq: np.ndarray,
    w: int,
    s: int,
    patch_offset: int = 0,
):
    """Return the blended output (float64 [H][W][4]) and the weight sums."""
    H, W = X.shape[:2]
    Hz, Wz = Z.shape[:2]
    if W % 2 or H % 2:
        raise ValueError("2x2 patches need even output sides")
    u, v = output_grid(H, W, w, s)
    ex, ey = exemplar_corner(np.asarray(nn, dtype=np.int64), Hz, Wz, w)
    Wq = np.asarray(Wq, dtype=np.float64)
    num = np.zeros((H, W, 3))
    den = np.zeros((H, W))
    for dy in range(w):
        for dx in range(w):
            py = v + dy
            px = (u + dx) % W
            lo, hi, c0, c1 = patch_rows_cols(px, py, H, W, patch_offset)
            inside = (
                (lo >= v)
                & (hi <= v + w - 1)
                & (np.mod(c0 - u, W) < w)
                & (np.mod(c1 - u, W) < w)
            )
            q = np.nonzero(inside)[0]
            src = Z[ey[q] + dy, ex[q] + dx, :3]
            np.add.at(num, (py[q], px[q]), Wq[q][:, None] * src)
            np.add.at(den, (py[q], px[q]), Wq[q])
    out = np.array(X, dtype=np.float64, copy=True)
    has = den > 0
    out[..., :3][has] = num[has] / den[has][:, None]
    return out, den


def covering_counts(H: int, W: int, w: int, s: int, patch_offset: int):
    """Number of windows in C(P) for every pixel's patch, and per pixel.

    Returns (patch_count [H][W], pixel_count [H][W]): the first is |C(P)| of
    the patch holding each pixel, the second the number of windows that
    contain the pixel itself.
    """
    u, v = output_grid(H, W, w, s)
    pc = np.zeros((H, W), dtype=np.int64)
    xc = np.zeros((H, W), dtype=np.int64)
    yy, xx = np.mgrid[0:H, 0:W]
    lo, hi, c0, c1 = patch_rows_cols(xx, yy, H, W, patch_offset)
    for q in range(u.size):
        rin = (yy >= v[q]) & (yy <= v[q] + w - 1)
        cin = np.mod(xx - u[q], W) < w
        xc += rin & cin
        pin = (lo >= v[q]) & (hi <= v[q] + w - 1) & (np.mod(c0 - u[q], W) < w) & (np.mod(c1 - u[q], W) < w)
        pc += pin
    return pc, xc
