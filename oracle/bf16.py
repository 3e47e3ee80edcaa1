"""BF16 distance form with top-k re-rank (oracle, FP64).  Test infra only.

The precision form of the search: the PCA-space vectors are rounded to
bfloat16 (round to nearest, ties to even, from their float32 values), all
exemplar distances are ranked on the rounded vectors, the k best candidates
(k = 8) are kept, and those k are re-ranked with the unrounded vectors; the
winner is the re-ranked minimum (ties to the lowest exemplar id).

The oracle evaluates the distances of the rounded vectors exactly in FP64,
i.e. the value the BF16 computation approximates; the GPU accumulates the
same products in FP32.
"""
from __future__ import annotations

import numpy as np

from . import exact


def round_bf16(a) -> np.ndarray:
    """float32 values rounded to the nearest bfloat16 (ties to even), as float64."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> np.uint64(16)) & np.uint64(1)
    rounded = ((bits + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return rounded.astype(np.uint32).view(np.float32).astype(np.float64)


def brute_topk(Qp, Zp, k: int = 8, offset=None):
    """Top-k exemplar ids per query by the distance of the bf16-rounded
    vectors (plus an optional per-exemplar offset, see ``residual``)."""
    return exact.topk(round_bf16(Qp), round_bf16(Zp), k, offset=offset)


def residual(Zm, mu, Zp):
    """Energy of each exemplar window outside the PCA subspace,
    ||z - mu||^2 - ||z'||^2 (>= 0).  Adding it to the PCA-space distance
    ranks candidates by an estimate of the full-dimension distance that is
    unbiased when the two windows' residuals are uncorrelated (the query's
    own residual energy is a constant per query)."""
    A = np.asarray(Zm, dtype=np.float64) - np.asarray(mu, dtype=np.float64)
    P = np.asarray(Zp, dtype=np.float64)
    return np.maximum(np.einsum("ij,ij->i", A, A) - np.einsum("ij,ij->i", P, P), 0.0)


def rerank(Q, Z, cand, offset=None):
    """Re-rank candidate ids with unrounded vectors; returns (nn, d2)."""
    Q = np.asarray(Q, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64)
    nq = Q.shape[0]
    nn = np.empty(nq, dtype=np.int64)
    d2 = np.empty(nq)
    for q in range(nq):
        c = np.asarray(cand[q], dtype=np.int64)
        diff = Z[c] - Q[q][None, :]
        dd = np.einsum("ij,ij->i", diff, diff)
        if offset is not None:
            dd = dd + np.asarray(offset, dtype=np.float64)[c]
        o = np.lexsort((c, dd))[0]
        nn[q] = c[o]
        d2[q] = dd[o]
    return nn, d2


def brute_nn(Qp, Zp, k: int = 8, Q_full=None, Z_full=None, offset=None):
    """BF16 top-k then FP64 re-rank in PCA space (or full D if given)."""
    cand, _ = brute_topk(Qp, Zp, k, offset=offset)
    if Q_full is not None:
        return rerank(Q_full, Z_full, cand)[0], cand
    return rerank(Qp, Zp, cand, offset=offset)[0], cand


def class_candidates(q, Zrows, offset=None):
    """Candidate rule of a BF16 scan over an ordered list of rows (a leaf's
    members in leaf order): with i the position of a row in the scan, the
    rows fall into 16 classes by i % 16 and into 32-row tiles by i // 32;
    each class's score is its minimum over the rows (ties to the earliest
    tile), the 4 classes with the smallest scores are kept, and each
    contributes the two rows of its tile in that class (i and i + 16 within
    the tile).  Scores are exact distances of the bf16-rounded vectors (plus
    the optional per-row offset).  Returns (positions into Zrows [<=8],
    scores [<=8]) with both rows of a class sharing the class score.
    """
    qb = round_bf16(np.asarray(q)[None, :])[0]
    Zb = round_bf16(Zrows)
    d = np.einsum("ij,ij->i", Zb - qb[None, :], Zb - qb[None, :])
    if offset is not None:
        d = d + np.asarray(offset, dtype=np.float64)
    m = d.size
    best = []
    for b in range(16):
        bv, bt = np.inf, -1
        for t in range((m + 31) // 32):
            rows = [i for i in (32 * t + b, 32 * t + b + 16) if i < m]
            if not rows:
                continue
            v = min(d[i] for i in rows)
            if v < bv:
                bv, bt = v, t
        if bt >= 0:
            best.append((bv, b, bt))
    best.sort(key=lambda e: (e[0], e[1]))
    pos, sc = [], []
    for v, b, t in best[:4]:
        for i in (32 * t + b, 32 * t + b + 16):
            if i < m:
                pos.append(i)
                sc.append(v)
    return np.asarray(pos, dtype=np.int64), np.asarray(sc)
