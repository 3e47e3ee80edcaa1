"""Search/optimisation alternation and coarse-to-fine solve (oracle, FP64).

Test infrastructure only.

Methodology 2.1: the output is refined by alternating a search phase (find
z_p for every sparse-grid neighbourhood) and an optimisation phase (solve
Eq. 8 for x with the z_p fixed) until the set {z_p} stops changing; a
coarse-resolution result is upsampled by interpolation to initialise the
next resolution.

Readings where the paper is silent:
* iteration t: nn^t = search(x^{t-1}); E_t = E(x^{t-1}; nn^t) is recorded;
  W from the full-dimension distances; x^t = patch blend.  A fixed count T
  of iterations per level; the number of changed matches is reported;
* the weights and the energy always use the full-dimension distance of the
  chosen match, whichever search space found it;
* exemplar pyramid: separable [1 4 6 4 1] / 16 blur with mirrored borders
  (edge sample not repeated) and 2x decimation keeping even samples, on
  R, G, B; the guidance channel is recomputed for each level's size;
* upsampling: bilinear on R, G, B at coarse position
  ((x + 0.5) / 2 - 0.5, (y + 0.5) / 2 - 0.5), wrapping in x and clamping in
  y; the guidance channel is recomputed at the finer size;
* with a perspective scale map (slant, tilt; Methodology 1) in place of the
  row guidance, each exemplar level's guidance is the normalised map of its
  own size and each output level's the resample of its exemplar level's
  map (Section 4, steps 1-2).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import exact, irls, mstep as mstep_mod, pca as pca_mod, scale as scale_mod, tree as tree_mod
from .vectors import exemplar_matrix, query_matrix, rgbs

_BLUR = np.array([1.0, 4.0, 6.0, 4.0, 1.0]) / 16.0


def guidance(H: int, W: int, weight: float = 0.5) -> np.ndarray:
    return np.broadcast_to((weight * (np.arange(H) + 0.5) / H)[:, None], (H, W)).copy()


def blur_decimate(rgb: np.ndarray) -> np.ndarray:
    """[H][W][C] -> [H/2][W/2][C]: 5-tap binomial blur, keep even samples."""
    p = np.pad(rgb, ((2, 2), (0, 0), (0, 0)), mode="reflect")
    t = sum(_BLUR[k] * p[k : k + rgb.shape[0]] for k in range(5))
    p = np.pad(t, ((0, 0), (2, 2), (0, 0)), mode="reflect")
    t = sum(_BLUR[k] * p[:, k : k + rgb.shape[1]] for k in range(5))
    return t[0::2, 0::2]


def _level_guidance(h: int, w: int, weight: float, scale):
    if scale is None:
        return guidance(h, w, weight)
    return scale_mod.guidance(scale[0], scale[1], h, w, weight)


def exemplar_pyramid(Z: np.ndarray, levels: int, weight: float = 0.5, scale=None):
    """Coarse-to-fine list of RGBS exemplars; the last is Z itself.  A
    negative weight keeps Z's own guidance channel (a scale map) and blurs
    it like the colours; otherwise each level's guidance is recomputed (the
    row guidance, or with scale = (slant, tilt) the level's scale map)."""
    out = [np.array(Z, dtype=np.float64)]
    if weight >= 0:
        out[0][..., 3] = _level_guidance(Z.shape[0], Z.shape[1], weight, scale)
    for _ in range(levels - 1):
        if weight < 0:
            out.insert(0, blur_decimate(out[0]))
            continue
        rgb = blur_decimate(out[0][..., :3])
        img = np.empty(rgb.shape[:2] + (4,))
        img[..., :3] = rgb
        img[..., 3] = _level_guidance(rgb.shape[0], rgb.shape[1], weight, scale)
        out.insert(0, img)
    return out


def upsample2(X: np.ndarray, weight: float = 0.5, scale=None, ref=None) -> np.ndarray:
    """2x bilinear upsampling; with scale = (slant, tilt) the new guidance is
    the map of an exemplar of size ref = (h, w) resampled to the new size."""
    Hc, Wc = X.shape[:2]
    H, W = 2 * Hc, 2 * Wc
    yc = (np.arange(H) + 0.5) / 2.0 - 0.5
    xc = (np.arange(W) + 0.5) / 2.0 - 0.5
    y0 = np.floor(yc).astype(np.int64)
    x0 = np.floor(xc).astype(np.int64)
    fy = (yc - y0)[:, None, None]
    fx = (xc - x0)[None, :, None]
    ya, yb = np.clip(y0, 0, Hc - 1), np.clip(y0 + 1, 0, Hc - 1)
    xa, xb = np.mod(x0, Wc), np.mod(x0 + 1, Wc)
    ch = X if weight < 0 else X[..., :3]  # a negative weight interpolates the guidance too
    top = (1 - fx) * ch[ya][:, xa] + fx * ch[ya][:, xb]
    bot = (1 - fx) * ch[yb][:, xa] + fx * ch[yb][:, xb]
    out = np.empty((H, W, 4))
    out[..., : ch.shape[2]] = (1 - fy) * top + fy * bot
    if weight >= 0:
        if scale is None:
            out[..., 3] = guidance(H, W, weight)
        else:
            out[..., 3] = scale_mod.output_guidance(scale[0], scale[1], ref[0], ref[1], H, W, weight)
    return out


@dataclass
class Index:
    """PCA basis plus search tree for one exemplar level."""

    w: int
    mu: np.ndarray
    B: np.ndarray
    Zp: np.ndarray
    tree: tree_mod.Tree | None
    retained: float = 1.0


def build_index(Z: np.ndarray, w: int, d: int, branching: int, depth: int, seed: int = 0) -> Index:
    Zm = exemplar_matrix(Z, w)
    mu, B, _, ret = pca_mod.basis(Zm, d)
    Zp = pca_mod.project(Zm, mu, B)
    t = tree_mod.build(Zp, branching, depth, seed) if depth > 0 else None
    return Index(w, mu, B, Zp, t, ret)


def winner_distance(Q: np.ndarray, Zm: np.ndarray, nn: np.ndarray) -> np.ndarray:
    diff = Q - Zm[nn]
    return np.sqrt(np.einsum("ij,ij->i", diff, diff))


def estep(X: np.ndarray, Z: np.ndarray, w: int, s: int, mode: str = "exact", index: Index | None = None):
    """Search phase: returns (nn [nq] exemplar ids, full-D distance [nq])."""
    Q = query_matrix(X, w, s)
    Zm = exemplar_matrix(Z, w)
    if mode == "exact":
        nn = exact.exact_nn(Q, Zm)[0]
    elif mode == "pca":
        Qp = pca_mod.project(Q, index.mu, index.B)
        nn = exact.topk(Qp, index.Zp, 1)[0][:, 0]
    elif mode == "tree":
        Qp = pca_mod.project(Q, index.mu, index.B)
        nn = tree_mod.tree_nn(Qp, index.Zp, index.tree)[0]
    else:
        raise ValueError(mode)
    return nn, winner_distance(Q, Zm, nn)


@dataclass
class Trace:
    E: list = field(default_factory=list)
    E2: list = field(default_factory=list)
    changes: list = field(default_factory=list)
    level: list = field(default_factory=list)


def iterate(X, Z, w, s, T, mode="exact", index=None, r=irls.R_DEFAULT, delta=irls.DELTA_DEFAULT,
            patch_offset=0, trace: Trace | None = None, level: int = 0, search=None):
    """T search/blend iterations at one level; returns the final x.

    ``search`` optionally replaces the search phase (callable X -> nn) so a
    caller can teacher-force another searcher's matches.
    """
    prev = None
    X = np.array(X, dtype=np.float64, copy=True)
    for _ in range(T):
        if search is None:
            nn, d = estep(X, Z, w, s, mode, index)
        else:
            nn = np.asarray(search(X), dtype=np.int64)
            d = winner_distance(query_matrix(X, w, s), exemplar_matrix(Z, w), nn)
        E, E2 = irls.energy(d, r, delta)
        if trace is not None:
            trace.E.append(E)
            trace.E2.append(E2)
            trace.changes.append(int(nn.size if prev is None else np.count_nonzero(nn != prev)))
            trace.level.append(level)
        prev = nn
        X, _ = mstep_mod.mstep(X, Z, nn, irls.weights(d, r, delta), w, s, patch_offset)
    return X


def multiscale(Z_fine, X0, ws, ss, Ts, mode="exact", pca_dims=0, branching=4, depth=0, seed=0,
               r=irls.R_DEFAULT, delta=irls.DELTA_DEFAULT, patch_offset=0, weight=0.5, scale=None):
    """Coarse-to-fine solve; X0 is the RGBS initial output at the coarsest
    level; scale = (slant, tilt) selects the scale-map guidance."""
    L = len(ws)
    pyr = exemplar_pyramid(Z_fine, L, weight, scale)
    X = np.array(X0, dtype=np.float64, copy=True)
    trace = Trace()
    for l in range(L):
        idx = None
        if mode in ("pca", "tree"):
            idx = build_index(pyr[l], ws[l], pca_dims, branching, depth if mode == "tree" else 0, seed)
        X = iterate(X, pyr[l], ws[l], ss[l], Ts[l], mode, idx, r, delta, patch_offset, trace, l)
        if l + 1 < L:
            X = upsample2(X, weight, scale, pyr[l + 1].shape[:2])
    return X, trace


__all__ = ["rgbs", "estep", "iterate", "multiscale", "build_index", "exemplar_pyramid",
           "upsample2", "blur_decimate", "winner_distance", "Index", "Trace"]
