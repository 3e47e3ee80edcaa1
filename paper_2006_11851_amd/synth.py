"""Seeded synthetic inputs for the perspective texture optimisation.

This module only draws random numbers and paints pixels.  It holds none of
the arithmetic of the synthesis method (no neighbourhood vectors, guidance
channel, PCA, search, weights or blending); both the GPU library and the FP64
oracle receive its arrays as inputs.

The paper measures on its own photographs (Figs. 8-10, Table 1), which are
not available.  Seeded perspective exemplars stand in for them: elliptical
texels whose size grows linearly from the top row (far) to the bottom row
(near), over a background whose brightness ramps with the row, so the scale
changes across the image the way a slanted textured plane does (Section 1,
Scale Evaluation, with the tilt fixed at zero).

Recipe (all draws from one ``numpy.random.default_rng(seed)`` stream, PCG64):

* palette: ``n_palette`` colours, uniform in [0, 255]^3;
* background: 255 * L(y) + N(0, bg_noise^2) per pixel and channel, with
  L(y) = 0.6 + 0.4 * y / (H - 1);
* texel centres: uniform candidates in [0, W) x [0, H), accepted with
  probability (r_top / r(y_c))^2, where
  r(y_c) = r_top + (r_bot - r_top) * y_c / (H - 1) is the horizontal
  semi-axis; the vertical semi-axis is 0.6 * r (foreshortening).  Rejection
  sampling gives a texel density proportional to 1 / r^2;
* texel colour: a uniform palette entry plus N(0, jitter^2) per channel;
* painting: far to near (ascending y_c), hard edges tested at pixel centres
  (integer coordinates), values clipped and rounded to uint8.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "perspective_exemplar",
    "row_matched_init",
    "tile_draws",
    "Workload",
    "WORKLOADS",
    "workload",
]


def perspective_exemplar(
    seed: int,
    H: int,
    W: int,
    n_texels: int,
    r_top: float,
    r_bot: float,
    n_palette: int = 6,
    jitter: float = 8.0,
    bg_noise: float = 4.0,
) -> np.ndarray:
    """Return a uint8 [H][W][3] exemplar drawn from ``seed``."""
    if H < 2 or W < 1 or n_texels < 0 or r_top <= 0 or r_bot < r_top:
        raise ValueError("bad exemplar recipe")
    rng = np.random.default_rng(seed)
    palette = rng.uniform(0.0, 255.0, size=(n_palette, 3))
    ramp = 0.6 + 0.4 * np.arange(H, dtype=np.float64) / (H - 1)
    img = 255.0 * ramp[:, None, None] + rng.normal(0.0, bg_noise, size=(H, W, 3))

    # rejection-sampled dart throwing
    xs, ys = [], []
    need = n_texels
    while need > 0:
        batch = max(1024, 4 * need)
        cx = rng.uniform(0.0, W, size=batch)
        cy = rng.uniform(0.0, H, size=batch)
        u = rng.uniform(0.0, 1.0, size=batch)
        r = r_top + (r_bot - r_top) * cy / (H - 1)
        ok = u < (r_top / r) ** 2
        xs.append(cx[ok][:need])
        ys.append(cy[ok][:need])
        need -= int(min(need, ok.sum()))
    cx = np.concatenate(xs) if xs else np.zeros(0)
    cy = np.concatenate(ys) if ys else np.zeros(0)
    pal_idx = rng.integers(0, n_palette, size=cx.size)
    colours = palette[pal_idx] + rng.normal(0.0, jitter, size=(cx.size, 3))

    order = np.argsort(cy, kind="stable")
    yy = np.arange(H, dtype=np.float64)[:, None]
    xx = np.arange(W, dtype=np.float64)[None, :]
    for t in order:
        a = r_top + (r_bot - r_top) * cy[t] / (H - 1)
        b = 0.6 * a
        y0, y1 = int(max(0, np.floor(cy[t] - b))), int(min(H - 1, np.ceil(cy[t] + b)))
        x0, x1 = int(max(0, np.floor(cx[t] - a))), int(min(W - 1, np.ceil(cx[t] + a)))
        sub_y = yy[y0 : y1 + 1]
        sub_x = xx[:, x0 : x1 + 1]
        inside = ((sub_x - cx[t]) / a) ** 2 + ((sub_y - cy[t]) / b) ** 2 <= 1.0
        img[y0 : y1 + 1, x0 : x1 + 1][inside] = colours[t]
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


def row_matched_init(seed: int, ex: np.ndarray, H: int, W: int, w: int):
    """Seeded initial output: exemplar patches of size w x w on a w-grid.

    Tile (ti, tj) covers rows ti*w.., columns tj*w..; its source row in the
    exemplar is the one at the same normalised height,
    ``v = clamp(round(g * Hz - w / 2), 0, Hz - w)`` with
    ``g = (ti * w + w / 2) / H``, and its source column is uniform in
    [0, Wz - w].  Returns ``(init_u8 [H][W][3], corners int32 [tiles][2])``
    where each corner row is (u, v) in exemplar pixels.
    """
    Hz, Wz = ex.shape[:2]
    if w > Hz or w > Wz:
        raise ValueError("window larger than exemplar")
    rng = np.random.default_rng(seed)
    nty = -(-H // w)
    ntx = -(-W // w)
    out = np.empty((H, W, 3), dtype=np.uint8)
    corners = np.empty((nty * ntx, 2), dtype=np.int32)
    us = rng.integers(0, Wz - w + 1, size=nty * ntx)
    for ti in range(nty):
        g = (ti * w + w / 2.0) / H
        v = int(min(max(int(np.floor(g * Hz - w / 2.0 + 0.5)), 0), Hz - w))
        for tj in range(ntx):
            k = ti * ntx + tj
            u = int(us[k])
            corners[k] = (u, v)
            h = min(w, H - ti * w)
            ww = min(w, W - tj * w)
            out[ti * w : ti * w + h, tj * w : tj * w + ww] = ex[v : v + h, u : u + ww]
    return out, corners


def tile_draws(seed: int, H: int, W: int, t: int) -> np.ndarray:
    """Uniform 32-bit integers [tiles][2] for the t x t tiles of an H x W
    output (row-major tiles): the draws a scale-matched initialisation
    consumes, one pair per tile."""
    n = (-(-H // t)) * (-(-W // t))
    return np.random.default_rng(seed).integers(0, 2**32, size=(n, 2), dtype=np.uint64).astype(np.uint32)


@dataclass(frozen=True)
class Workload:
    """One synthetic workload: exemplar recipe plus the solve's level plan.

    Levels are listed coarse to fine; ``ex_sizes``/``out_sizes`` are square
    side lengths per level.
    """

    name: str
    seed: int
    ex_size: int
    out_size: int
    n_texels: int
    r_top: float
    r_bot: float
    w: tuple
    stride: tuple
    pca_dims: int
    branching: int
    depth: int
    iters: int
    init_seed: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def levels(self) -> int:
        return len(self.w)

    def ex_sizes(self):
        L = self.levels
        return [self.ex_size >> (L - 1 - l) for l in range(L)]

    def out_sizes(self):
        L = self.levels
        return [self.out_size >> (L - 1 - l) for l in range(L)]

    def initial_output(self, ex: np.ndarray, seed: int | None = None) -> np.ndarray:
        """uint8 initial output at the coarsest level.

        Row-matched w x w patches (``row_matched_init``) copied from the
        exemplar subsampled by 2^(levels-1), so that the patches have the
        coarsest level's scale; subsampling the uint8 image keeps the initial
        output identical for every consumer.
        """
        f = 1 << (self.levels - 1)
        src = np.ascontiguousarray(ex[::f, ::f])
        out0 = self.out_sizes()[0]
        init, _ = row_matched_init(self.init_seed if seed is None else seed, src, out0, out0, self.w[0])
        return init

    def exemplar(self, seed: int | None = None) -> np.ndarray:
        return perspective_exemplar(
            self.seed if seed is None else seed,
            self.ex_size,
            self.ex_size,
            self.n_texels,
            self.r_top,
            self.r_bot,
        )


# The five workloads: a 64^2 single-level oracle-scale case; a 256^2 -> 512^2
# three-level plain FP32 solve; a 512^2 -> 1024^2 single level at 16x16
# windows for the BF16 brute-force form; the learned-proposal form at the
# second workload's shapes (PCA 64, 32-way tree of depth 2, exemplar seeds
# 100..115); and the 1024^2 -> 2048^2 four-level solve.
WORKLOADS = {
    "ex64_out128": Workload("ex64_out128", 1, 64, 128, 60, 2.0, 8.0, (8,), (4,), 16, 4, 3, 5),
    "ex256_out512": Workload("ex256_out512", 2, 256, 512, 800, 3.0, 24.0, (32, 16, 8), (8, 4, 2), 24, 8, 3, 10),
    "ex512_out1024_w16": Workload(
        "ex512_out1024_w16", 3, 512, 1024, 3000, 3.0, 40.0, (16,), (4,), 64, 8, 3, 10
    ),
    "ex256_out512_learned": Workload(
        "ex256_out512_learned", 100, 256, 512, 800, 3.0, 24.0, (32, 16, 8), (8, 4, 2), 64, 32, 2, 10,
        extra={"exemplar_seeds": tuple(range(100, 116))},
    ),
    "ex1024_out2048": Workload(
        "ex1024_out2048", 5, 1024, 2048, 12000, 4.0, 64.0, (32, 32, 16, 8), (8, 8, 4, 2), 64, 32, 2, 10
    ),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]
