"""BF16 distance form with top-k re-rank (oracle, FP64).  Test infra only.

The precision form of the search: the PCA-space vectors are rounded to
bfloat16 (round to nearest, ties to even, from their float32 values), the
exemplar distances are ranked on the rounded vectors, the k best candidates
(k = 8) are kept, and those k are re-ranked with the unrounded vectors; the
winner is the re-ranked minimum (ties to the lowest exemplar id).  The
brute-force form ranks every exemplar window (``brute_topk``); the learned
form ranks only the members of the leaves it scans (``scan_topk``): the same
definition over a smaller set.

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


def scan_topk(Qp, Zp, members, k: int = 8, offset=None):
    """The k best exemplar ids of each query among ``members[i]`` (the union
    of the members of the leaves scanned for query i; repeated ids count
    once), ranked like :func:`brute_topk`: squared distance of the
    bf16-rounded vectors plus the optional per-exemplar offset, ties to the
    lowest id.  Returns (list of id arrays [<= k], list of score arrays)."""
    Qb = round_bf16(Qp)
    Zb = round_bf16(Zp)
    off = None if offset is None else np.asarray(offset, dtype=np.float64)
    ids_out, sc_out = [], []
    for i in range(Qb.shape[0]):
        ids = np.unique(np.asarray(members[i], dtype=np.int64))
        diff = Zb[ids] - Qb[i][None, :]
        d = np.einsum("ij,ij->i", diff, diff)
        if off is not None:
            d = d + off[ids]
        o = np.lexsort((ids, d))[:k]
        ids_out.append(ids[o])
        sc_out.append(d[o])
    return ids_out, sc_out


def scan_scores(q, Zp_rows, offset_rows=None):
    """Scores of one query against listed exemplar rows, as ranked by
    :func:`scan_topk` (bf16-rounded vectors, FP64 arithmetic)."""
    qb = round_bf16(np.asarray(q)[None, :])[0]
    diff = round_bf16(Zp_rows) - qb[None, :]
    d = np.einsum("ij,ij->i", diff, diff)
    if offset_rows is not None:
        d = d + np.asarray(offset_rows, dtype=np.float64)
    return d


def fp32_score_tolerance(q, Zp_rows, d: int, offset_rows=None, Zm_rows=None, mu=None) -> float:
    """Bound on how far two scores of one query can be reordered when the
    score ||z||^2 - 2 q.z (+ offset) of bf16 operands is evaluated in FP32
    instead of exactly: each evaluation errs by at most
    gamma * (||z||^2 + 2 |q.z|) <= gamma * (||q||^2 + 3 ||z||^2) with
    gamma = (d + 4) u, u = 2^-24 (the standard bound for a length-d sum
    started at the norm, plus the norm's own rounding), and an offset computed
    in FP32 from the D full-dimension entries errs by at most
    (D + d + 4) u ||z - mu||^2; two scores together by twice the largest.
    The rows are the ones the query scans."""
    u = 2.0 ** -24
    qb = round_bf16(np.asarray(q)[None, :])[0]
    zb = round_bf16(Zp_rows)
    zn = np.einsum("ij,ij->i", zb, zb)
    t = (d + 4) * u * (float(qb @ qb) + 3.0 * float(zn.max(initial=0.0)))
    if offset_rows is not None and Zm_rows is not None:
        A = np.asarray(Zm_rows, dtype=np.float64) - np.asarray(mu, dtype=np.float64)[None, :]
        D = A.shape[1]
        t += (D + d + 4) * u * float(np.einsum("ij,ij->i", A, A).max(initial=0.0))
    return 2.0 * t
