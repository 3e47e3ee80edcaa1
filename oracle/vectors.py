"""Neighbourhood vectors (oracle, FP64).  Test infrastructure only.

Methodology 2.1, text of Eq. 4: x_p is the vector of the pixels of the
neighbourhood N_p of width w in the output X; z_p is a neighbourhood vector
of the exemplar Z.  Section 4 (Synthesis Procedure) adds the scale map as a
fourth channel beside R, G and B.

Readings used here (the paper is silent on them):
* channels are R, G, B = u8 / 255 and S = lambda * (y + 0.5) / H_img with
  lambda = 0.5, the image's own height; at zero tilt the paper's scale map
  (Eq. 3) is affine in the row, so a normalised row coordinate stands in for
  it, weighted by lambda;
* a window at top-left (u, v) is flattened with index (dy * w + dx) * 4 + c;
* exemplar windows: every valid top-left corner at stride 1, id
  e = v * (Wz - w + 1) + u;
* output windows: rows v_i = i * s for i = 0 .. (H - w) / s (clamped, no
  vertical wrap), columns u_j = j * s for j = 0 .. W / s - 1, wrapping in x;
  id q = i * (W / s) + j.
"""
from __future__ import annotations

import numpy as np


def rgbs(u8: np.ndarray, guidance_weight: float = 0.5) -> np.ndarray:
    """u8 [H][W][3] -> float64 [H][W][4] with the weighted row guidance."""
    H, W = u8.shape[:2]
    out = np.empty((H, W, 4), dtype=np.float64)
    out[..., :3] = u8.astype(np.float64) / 255.0
    out[..., 3] = (guidance_weight * (np.arange(H, dtype=np.float64) + 0.5) / H)[:, None]
    return out


def n_exemplar_windows(Hz: int, Wz: int, w: int) -> int:
    return (Hz - w + 1) * (Wz - w + 1)


def exemplar_corner(e, Hz: int, Wz: int, w: int):
    """Exemplar window id -> (u, v) top-left corner."""
    nu = Wz - w + 1
    e = np.asarray(e)
    return e % nu, e // nu


def output_grid(H: int, W: int, w: int, s: int):
    """Top-left corners (u_j, v_i) of the output windows, in id order."""
    if (H - w) % s or W % s or w > H:
        raise ValueError("grid does not tile the output")
    rows = np.arange(0, H - w + 1, s)
    cols = np.arange(0, W, s)
    v = np.repeat(rows, cols.size)
    u = np.tile(cols, rows.size)
    return u, v


def window(img: np.ndarray, u: int, v: int, w: int, wrap_x: bool) -> np.ndarray:
    """One neighbourhood vector of length 4 w^2, index (dy*w+dx)*4+c."""
    Wd = img.shape[1]
    cols = (u + np.arange(w)) % Wd if wrap_x else u + np.arange(w)
    return img[v : v + w][:, cols, :].reshape(-1)


def exemplar_matrix(Z: np.ndarray, w: int) -> np.ndarray:
    """All exemplar windows, [N][D], row e is the window with id e."""
    Hz, Wz = Z.shape[:2]
    nv, nu = Hz - w + 1, Wz - w + 1
    out = np.empty((nv * nu, 4 * w * w), dtype=np.float64)
    for dy in range(w):
        for dx in range(w):
            k = (dy * w + dx) * 4
            out[:, k : k + 4] = Z[dy : dy + nv, dx : dx + nu, :].reshape(-1, 4)
    return out


def query_matrix(X: np.ndarray, w: int, s: int) -> np.ndarray:
    """All output windows on the sparse grid, [nq][D], row q = window q."""
    H, W = X.shape[:2]
    u, v = output_grid(H, W, w, s)
    out = np.empty((u.size, 4 * w * w), dtype=np.float64)
    for dy in range(w):
        for dx in range(w):
            k = (dy * w + dx) * 4
            out[:, k : k + 4] = X[v + dy, (u + dx) % W, :]
    return out
