"""Parity judging helpers (test infrastructure only).

A search result differs from the oracle's only where it may: a returned id
that is not the oracle's is excused when its squared distance, evaluated by
the oracle in FP64, exceeds the oracle's by less than a relative 1e-4 (ties
and near-ties that rounding can reorder).
"""
from __future__ import annotations

import numpy as np


def sqdist_rows(Q, Z, ids):
    Q = np.asarray(Q, dtype=np.float64)
    diff = Q - np.asarray(Z, dtype=np.float64)[np.asarray(ids, dtype=np.int64)]
    return np.einsum("ij,ij->i", diff, diff)


def nn_agreement(Q, Z, nn_test, nn_ref, rel: float = 1e-4):
    """(fraction equal-or-excused, fraction exactly equal, excused mask)."""
    nn_test = np.asarray(nn_test, dtype=np.int64)
    nn_ref = np.asarray(nn_ref, dtype=np.int64)
    same = nn_test == nn_ref
    dt = sqdist_rows(Q, Z, nn_test)
    dr = sqdist_rows(Q, Z, nn_ref)
    excused = (~same) & (dt - dr <= rel * np.maximum(dr, 1e-300))
    ok = same | excused
    return float(ok.mean()), float(same.mean()), excused


def topk_rerank_valid(ids, score, rdist, winner, k: int = 8, tol_score: float = 0.0, rel: float = 1e-4) -> bool:
    """Whether ``winner`` is what a top-k-then-re-rank search may return when
    its ranking scores are only known to within ``tol_score`` (the scores of a
    query's scanned exemplars, evaluated by the oracle exactly, against a
    search that evaluates them in lower precision).

    ids, score, rdist: the scanned exemplar ids, their ranking scores and their
    re-rank distances (FP64).  A valid candidate set holds every id scored
    below s_k - tol (s_k = the k-th smallest score) and completes it to k ids
    from those within tol of s_k; the search returns the smallest re-rank
    distance of its set (a difference within ``rel`` relative is a tie).  The
    winner is valid if some valid set has it as that minimum."""
    ids = np.asarray(ids, dtype=np.int64)
    score = np.asarray(score, dtype=np.float64)
    rdist = np.asarray(rdist, dtype=np.float64)
    w = np.nonzero(ids == int(winner))[0]
    if w.size == 0:
        return False
    rg = rdist[w[0]]
    lo = rg * (1.0 - rel)
    if ids.size <= k:
        return bool(np.all(rdist >= lo))
    sk = np.sort(score)[k - 1]
    must = score < sk - tol_score
    may = (~must) & (score <= sk + tol_score)
    if not (must[w[0]] or may[w[0]]):
        return False
    if np.any(rdist[must] < lo):
        return False
    need = k - int(must.sum()) - (1 if may[w[0]] else 0)
    others = may.copy()
    others[w[0]] = False
    return int(np.count_nonzero(others & (rdist >= lo))) >= need
