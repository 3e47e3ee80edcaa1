"""Histogram-weighted blend and final histogram match (oracle, FP64).
Test infrastructure only.

Section 3 (Histogram Matching, Eq. 9): the optimisation phase's weights are
reduced for matched neighbourhoods whose colour is over-represented in the
output:

  W_p' = W_p / (1 + sum_j max[0, H_x,j(b_j(c_p)) - H_z,j(b_j(c_p))])

with H_x,j and H_z,j the j-th histograms of the output and of the exemplar
and b_j(c) the bin of colour c in them.  Readings (the paper's notation is
garbled: it calls k both the number of bins and the number of histograms):

* one histogram per colour channel j in {R, G, B}, ``bins`` equal bins over
  [0, 1] (value v in bin min(floor(v * bins), bins - 1)), counted over every
  pixel of the image and normalised to fractions, so that images of
  different sizes compare;
* c_p, the colour of matched neighbourhood z_p, is the exemplar pixel at its
  centre, offset (w / 2, w / 2) from its top-left corner;
* H_x is the histogram of the output the blend starts from (the current
  iterate), H_z that of the exemplar.

Section 4, step 4: after the optimisation the output's histograms are
matched to the exemplar's.  Reading: per colour channel, exact histogram
specification by rank - the output pixels sorted by value (ties by pixel
index) take the exemplar's sorted values at the same quantile: the i-th
smallest of n takes the exemplar value of rank floor((i + 1/2) n_z / n).
"""
from __future__ import annotations

import numpy as np

from .vectors import exemplar_corner


def bin_of(v, bins: int):
    """Bin index of values in [0, 1] (values outside are clamped into the end bins)."""
    b = np.floor(np.asarray(v, dtype=np.float64) * bins).astype(np.int64)
    return np.clip(b, 0, bins - 1)


def channel_histograms(img, bins: int) -> np.ndarray:
    """[3][bins] fractions of the image's pixels per bin, channels R, G, B."""
    rgb = np.asarray(img, dtype=np.float64)[..., :3].reshape(-1, 3)
    out = np.zeros((3, bins))
    for j in range(3):
        out[j] = np.bincount(bin_of(rgb[:, j], bins), minlength=bins) / rgb.shape[0]
    return out


def window_colours(Z, nn, w: int) -> np.ndarray:
    """Colour (R, G, B) of each matched exemplar window: its centre pixel."""
    Hz, Wz = Z.shape[:2]
    ex, ey = exemplar_corner(np.asarray(nn, dtype=np.int64), Hz, Wz, w)
    return np.asarray(Z, dtype=np.float64)[ey + w // 2, ex + w // 2, :3]


def excess(colours, Hx, Hz, bins: int) -> np.ndarray:
    """sum_j max[0, H_x,j(b_j(c)) - H_z,j(b_j(c))] for every colour c."""
    c = np.asarray(colours, dtype=np.float64)
    total = np.zeros(c.shape[0])
    for j in range(3):
        b = bin_of(c[:, j], bins)
        total += np.maximum(0.0, Hx[j][b] - Hz[j][b])
    return total


def weights(W, X, Z, nn, w: int, bins: int) -> np.ndarray:
    """Eq. 9: the blend weights W of the matched windows nn, divided by one
    plus the histogram excess of their colours (output X, exemplar Z)."""
    Hx = channel_histograms(X, bins)
    Hz = channel_histograms(Z, bins)
    return np.asarray(W, dtype=np.float64) / (1.0 + excess(window_colours(Z, nn, w), Hx, Hz, bins))


def match(X, Z) -> np.ndarray:
    """Section 4, step 4: X with each colour channel's values replaced, rank
    for rank, by the exemplar's (the reading above); the guidance channel
    is kept."""
    X = np.asarray(X, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64)
    out = X.copy()
    n = X.shape[0] * X.shape[1]
    nz = Z.shape[0] * Z.shape[1]
    for j in range(3):
        xv = X[..., j].reshape(-1)
        zs = np.sort(Z[..., j].reshape(-1))
        order = np.lexsort((np.arange(n), xv))  # ascending value, ties by pixel index
        src = np.floor((np.arange(n) + 0.5) * nz / n).astype(np.int64)
        col = np.empty(n)
        col[order] = zs[np.minimum(src, nz - 1)]
        out[..., j] = col.reshape(X.shape[:2])
    return out
