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
